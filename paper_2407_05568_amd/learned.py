"""Learned warm start for the mesh redistribution (Section 4): data generation from the
scheme's own runs, training with the library's MFMA forward/backward and Adam kernels, and
the comparison with the plain iteration at the same final residual.

A frame is a state (U^n, x^n) of a moving-mesh run of the method (its usual fixed sweep
count): its inputs are the node features written by ``mlp_features`` and its target is the
converged (pre-limiter) displacement (x^[mu] - x^n) / dxi per component of the redistribution
of that state solved to the tolerance mesh_tol.  The
network sees only the 5 x 5 stencil of features around a node; the plain Jacobi iteration
always finishes the solve from x^n + warm_dx to the same tolerance, so the final mesh
residual does not depend on the network.

Run as a module for the full-size experiment (prints one JSON line, progress on stderr):
    python -m paper_2407_05568_amd.learned --size 1024
(frames every 5 steps of the method's own runs from 6 training seeds, 3 frames each of 2
held-out seeds for the comparison).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import synth
from .esvdw import MLP_NPARAM, Context, mlp_adam


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def init_params(seed):
    """He-style initialisation in the library's packing (W[k][j] maps input k to output j):
    W1 64 x 64 (rows 50..63 zero), b1, W2 64 x 64, b2, W3 64 x 16 (columns 2..15 zero), b3."""
    rng = np.random.default_rng(seed)
    P = np.zeros(MLP_NPARAM, np.float32)
    P[0:50 * 64] = rng.normal(scale=np.sqrt(2.0 / 50), size=50 * 64)
    P[4160:4160 + 4096] = rng.normal(scale=np.sqrt(2.0 / 64), size=4096)
    W3 = np.zeros((64, 16), np.float32)
    W3[:, :2] = rng.normal(scale=np.sqrt(1.0 / 64), size=(64, 2))
    P[8320:8320 + 1024] = W3.ravel()
    return P


def tol_problem(p, tol):
    """The same problem with the Jacobi iteration taken to the tolerance tol (largest node
    update), the setting in which a warm start can shorten the solve."""
    q = dict(p)
    q.update(fixed_mu=0, mu=50_000_000, mesh_tol=tol)
    return q


class Run:
    """A moving-mesh run of one problem on the GPU: it advances with the method's own step
    (redistribution with the problem's fixed sweep count, then three RK stages), and at frames
    solves the redistribution of the current state to the tolerance with a second context."""

    def __init__(self, torch, p, prim, tol=1e-8, stream=None):
        self.torch, self.p = torch, p
        self.ctx = Context(p)
        self.ctx_tol = Context(tol_problem(p, tol))
        self.stream = stream or torch.cuda.current_stream()
        n = p["n"][:p["dim"]]
        shape = tuple(reversed(n))
        f64 = dict(dtype=torch.float64, device="cuda")
        self.N = int(np.prod(n))
        self.dxi = torch.tensor([(p["hi"][k] - p["lo"][k]) / p["n"][k] for k in range(p["dim"])], **f64)
        self.x = torch.empty((p["dim"],) + shape, **f64)
        self.J = torch.empty(shape, **f64)
        self.JU = torch.empty((p["dim"] + 2,) + shape, **f64)
        self.xdot = torch.empty_like(self.x)
        self.xmu = torch.empty_like(self.x)
        self.dt = torch.zeros(1, **f64)
        self.dt_step = torch.zeros(1, **f64)
        self.res = torch.zeros(1, **f64)
        self.sweeps = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.ctx.init_mesh(self.x, self.J, 1, self.stream)
        self.ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), self.J, self.JU, self.stream)

    def features(self, out):
        self.ctx.mlp_features(self.JU, self.J, out, self.stream)

    def solve(self, warm=None):
        """Redistribution of the current state to the tolerance, from x^n (+ warm);
        returns (sweeps, final residual, ms)."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.ctx_tol.redistribute_mesh(self.JU, self.J, self.x, warm, self.xdot, self.dt, self.res, self.sweeps,
                                       self.stream)
        e1.record(self.stream)
        torch.cuda.synchronize()
        return int(self.sweeps.item()), float(self.res.item()), e0.elapsed_time(e1)

    def target(self, out):
        """(x^[mu] - x^n) / dxi of the last tolerance solve, as FP32 (dim fields)."""
        self.ctx_tol.mesh_converged(self.xmu, self.stream)
        d = self.p["dim"]
        out.copy_(((self.xmu - self.x) / self.dxi.view((d,) + (1,) * d)).float())

    def advance(self, steps):
        """`steps` steps of the method (fixed sweep count); raises if the scheme flags a state."""
        for _ in range(steps):
            self.ctx.step(self.JU, self.J, self.x, 1, self.dt_step, self.stream)
        st = self.ctx.status()
        if st:
            raise RuntimeError("scheme raised status flags %d" % st)


def generate(torch, p, prims, frames, every, tol=1e-8, tag=""):
    """Frames from runs of the method: for each initial state in `prims`, `frames` frames taken
    every `every` steps (features and the converged displacement / dxi, FP32 [F][2][N]).
    Returns (feats, tgts, per-frame statistics)."""
    shape = tuple(reversed(p["n"][:2]))
    F = frames * len(prims)
    feats = torch.empty((F, 2) + shape, dtype=torch.float32, device="cuda")
    tgts = torch.empty_like(feats)
    stats = []
    f = 0
    for r, prim in enumerate(prims):
        run = Run(torch, p, prim, tol)
        for k in range(frames):
            run.features(feats[f])
            sw, res, ms = run.solve()
            run.target(tgts[f])
            stats.append(dict(run=r, frame=k, sweeps=sw, resid=res, ms=ms))
            _log("%srun %d frame %d: %d sweeps, residual %.2e, %.1f ms, |target|max %.2f dxi" % (
                tag, r, k, sw, res, ms, float(tgts[f].abs().max())))
            f += 1
            run.advance(every)
        del run
    return feats, tgts, stats


def train(torch, ctx, feats, tgts, iters=2000, batch=8192, lr=1e-3, seed=0, log_every=250):
    """Adam on the mean squared displacement error over random (frame, node) samples, with the
    library's gradient and Adam kernels.  Returns the FP32 parameters (device) and the loss
    history."""
    F = feats.shape[0]
    N = feats[0, 0].numel()
    P = torch.from_numpy(init_params(seed)).cuda()
    grad = torch.zeros_like(P)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    samples = torch.empty((batch, 2), dtype=torch.int32, device="cuda")
    hist = []
    for it in range(1, iters + 1):
        samples[:, 0] = torch.randint(0, F, (batch,), generator=gen, device="cuda", dtype=torch.int32)
        samples[:, 1] = torch.randint(0, N, (batch,), generator=gen, device="cuda", dtype=torch.int32)
        ctx.mlp_grad(feats, tgts, samples, batch, 1.0 / batch, P, grad, loss)
        mlp_adam(P, grad, m, v, it, lr)
        if it % log_every == 0 or it == 1:
            hist.append((it, float(loss.item())))
            _log("  iter %d loss %.4e" % hist[-1])
    return P, hist


def heldout_error(torch, ctx, P, feats, tgts, dxi):
    """Relative L2 error of the network's displacement on frames, against the zero predictor."""
    shape = feats.shape[2:]
    warm = torch.empty((2,) + tuple(shape), dtype=torch.float64, device="cuda")
    num = den = 0.0
    for f in range(feats.shape[0]):
        ctx.mlp_infer(feats[f], P, warm)
        y = warm / dxi.view(2, 1, 1)
        num += float(((y - tgts[f].double()) ** 2).sum())
        den += float((tgts[f].double() ** 2).sum())
    return (num / den) ** 0.5 if den > 0 else 0.0


def compare(torch, run, P, frames, every, tag=""):
    """At `frames` frames of `run`, `every` steps apart: time the plain solve (x^[0] = x^n) and
    the warm-started one (features + inference + the same iteration from x^n + warm_dx), both
    to the tolerance.  The run advances with the method's own step between frames."""
    shape = tuple(reversed(run.p["n"][:2]))
    feat = torch.empty((2,) + shape, dtype=torch.float32, device="cuda")
    warm = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
    out = []
    for k in range(frames):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        run.features(feat)
        run.ctx.mlp_infer(feat, P, warm, run.stream)
        e1.record(run.stream)
        sw_w, res_w, ms_w = run.solve(warm)
        torch.cuda.synchronize()
        ms_inf = e0.elapsed_time(e1)
        sw_p, res_p, ms_p = run.solve()
        rec = dict(plain_sweeps=sw_p, plain_resid=res_p, plain_ms=ms_p, warm_sweeps=sw_w, warm_resid=res_w,
                   warm_ms=ms_w + ms_inf, infer_ms=ms_inf)
        out.append(rec)
        _log("%sframe %d: plain %d sweeps %.1f ms (res %.1e) | warm %d sweeps %.1f ms (+%.2f ms net, res %.1e)" % (
            tag, k, sw_p, ms_p, res_p, sw_w, ms_w, ms_inf, res_w))
        run.advance(every)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--train-seeds", default="0,4,5,11,13,14")
    ap.add_argument("--test-seeds", default="2,19")
    ap.add_argument("--frames", type=int, default=6)
    ap.add_argument("--test-frames", type=int, default=3)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the learned warm start runs on the GPU"
    n = args.size
    p = synth.problem(2, [n, n], bc="outflow")
    seeds = [int(v) for v in args.train_seeds.split(",")]
    tests = [int(v) for v in args.test_seeds.split(",")]
    t0 = time.time()
    prims = [synth.quadrants_2d(p, synth.quadrant_states(p, sd)) for sd in seeds]
    feats, tgts, gstats = generate(torch, p, prims, args.frames, args.every, args.tol, "train ")
    t_gen = time.time() - t0
    ctx = Context(p)
    dxi = torch.tensor([1.0 / n, 1.0 / n], dtype=torch.float64, device="cuda")
    t0 = time.time()
    P, hist = train(torch, ctx, feats, tgts, args.iters, args.batch, args.lr, seeds[0])
    torch.cuda.synchronize()
    t_train = time.time() - t0
    err_train = heldout_error(torch, ctx, P, feats, tgts, dxi)
    _log("training frames: relative displacement error %.3f" % err_train)
    del feats, tgts
    recs = []
    for sd in tests:
        run = Run(torch, p, synth.quadrants_2d(p, synth.quadrant_states(p, sd)), args.tol)
        recs += compare(torch, run, P, args.test_frames, args.every, "held-out seed %d " % sd)
        del run
    ps, ws = sum(r["plain_ms"] for r in recs), sum(r["warm_ms"] for r in recs)
    out = dict(size=n, tol=args.tol, train_seeds=seeds, test_seeds=tests, frames_per_run=args.frames,
               every=args.every, iters=args.iters, batch=args.batch, gen_s=t_gen, train_s=t_train, loss=hist,
               train_rel_err=err_train, plain_ms=ps, warm_ms=ws, speedup=ps / ws if ws > 0 else None,
               plain_sweeps=sum(r["plain_sweeps"] for r in recs), warm_sweeps=sum(r["warm_sweeps"] for r in recs),
               max_final_resid=max(max(r["plain_resid"], r["warm_resid"]) for r in recs), frames=recs, gen=gstats)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
