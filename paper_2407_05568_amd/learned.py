"""Learned warm start for the mesh redistribution (Section 4): data generation from the
scheme's own runs, training with the library's MFMA forward/backward and Adam kernels, and
the comparison with the plain iteration at the same final residual.

A frame is the state (U^n, x^n) of a moving-mesh run with the Jacobi iteration taken to the
tolerance mesh_tol: its inputs are the node features written by ``mlp_features`` and its
target is the converged (pre-limiter) displacement (x^[mu] - x^n) / dxi per component.  The
network sees only the 5 x 5 stencil of features around a node; the plain Jacobi iteration
always finishes the solve from x^n + warm_dx to the same tolerance, so the final mesh
residual does not depend on the network.

Run as a module for the full-size experiment (prints one JSON line, progress on stderr):
    python -m paper_2407_05568_amd.learned --size 1024 --train-steps 16 --test-steps 4
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


class Run:
    """A moving-mesh run of one problem on the GPU, one redistribution per step in tolerance
    mode (the Jacobi iteration runs until the largest node update is below mesh_tol)."""

    def __init__(self, torch, p, prim, stream=None):
        self.torch, self.p = torch, p
        self.ctx = Context(p)
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
        self.stage = [torch.empty_like(self.JU) for _ in range(2)]
        self.stageJ = [torch.empty_like(self.J) for _ in range(2)]
        self.dt = torch.zeros(1, **f64)
        self.res = torch.zeros(1, **f64)
        self.sweeps = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.ctx.init_mesh(self.x, self.J, 1, self.stream)
        self.ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), self.J, self.JU, self.stream)

    def features(self, out):
        self.ctx.mlp_features(self.JU, self.J, out, self.stream)

    def redistribute(self, warm=None):
        """Redistribution from the current state; returns (sweeps, final residual, ms)."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.ctx.redistribute_mesh(self.JU, self.J, self.x, warm, self.xdot, self.dt, self.res, self.sweeps,
                                   self.stream)
        e1.record(self.stream)
        torch.cuda.synchronize()
        return int(self.sweeps.item()), float(self.res.item()), e0.elapsed_time(e1)

    def advance(self):
        """Three SSP-RK3 stages with the mesh velocity of the last redistribution."""
        c, s = self.ctx, self.stream
        c.rk_stage(0, self.dt, self.JU, self.J, self.JU, self.J, self.x, self.xdot, self.stage[0], self.stageJ[0],
                   None, s)
        c.rk_stage(1, self.dt, self.JU, self.J, self.stage[0], self.stageJ[0], self.x, self.xdot, self.stage[1],
                   self.stageJ[1], None, s)
        c.rk_stage(2, self.dt, self.JU, self.J, self.stage[1], self.stageJ[1], self.x, self.xdot, self.JU, self.J,
                   self.x, s)

    def target(self, out):
        """(x^[mu] - x^n) / dxi of the last redistribution, as FP32 (dim fields)."""
        self.ctx.mesh_converged(self.xmu, self.stream)
        d = self.p["dim"]
        out.copy_(((self.xmu - self.x) / self.dxi.view((d,) + (1,) * d)).float())


def generate(torch, p, prim, steps, tag=""):
    """Frames of a run: features and targets (FP32, [steps][2][N]) and per-step statistics."""
    run = Run(torch, p, prim)
    shape = tuple(reversed(p["n"][:2]))
    feats = torch.empty((steps, 2) + shape, dtype=torch.float32, device="cuda")
    tgts = torch.empty_like(feats)
    stats = []
    for s in range(steps):
        run.features(feats[s])
        sw, res, ms = run.redistribute()
        run.target(tgts[s])
        run.advance()
        st = run.ctx.status()
        stats.append(dict(sweeps=sw, resid=res, ms=ms, flags=st))
        _log("%sframe %d: %d sweeps, residual %.2e, %.1f ms, |target|max %.2f dxi" % (
            tag, s, sw, res, ms, float(tgts[s].abs().max())))
        if st:
            raise RuntimeError("scheme raised status flags %d while generating frames" % st)
    return run, feats, tgts, stats


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


def compare(torch, run, P, steps, tag=""):
    """Advance `run` by `steps` steps; at each, time the plain redistribution (x^[0] = x^n)
    and the warm-started one (features + inference + the same iteration from x^n + warm_dx),
    both to mesh_tol.  The run itself advances with the plain result."""
    shape = tuple(reversed(run.p["n"][:2]))
    feat = torch.empty((2,) + shape, dtype=torch.float32, device="cuda")
    warm = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
    out = []
    for s in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        run.features(feat)
        run.ctx.mlp_infer(feat, P, warm, run.stream)
        e1.record(run.stream)
        sw_w, res_w, ms_w = run.redistribute(warm)
        torch.cuda.synchronize()
        ms_inf = e0.elapsed_time(e1)
        sw_p, res_p, ms_p = run.redistribute()
        run.advance()
        st = run.ctx.status()
        if st:
            raise RuntimeError("scheme raised status flags %d during the comparison run" % st)
        rec = dict(plain_sweeps=sw_p, plain_resid=res_p, plain_ms=ms_p, warm_sweeps=sw_w, warm_resid=res_w,
                   warm_ms=ms_w + ms_inf, infer_ms=ms_inf)
        out.append(rec)
        _log("%sstep %d: plain %d sweeps %.1f ms (res %.1e) | warm %d sweeps %.1f ms (+%.2f ms net, res %.1e)" % (
            tag, s, sw_p, ms_p, res_p, sw_w, ms_w, ms_inf, res_w))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--train-steps", type=int, default=16)
    ap.add_argument("--test-steps", type=int, default=4)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--test-seed", type=int, default=2)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the learned warm start runs on the GPU"
    n = args.size
    p = synth.problem(2, [n, n], bc="outflow", fixed_mu=0, mu=50_000_000, mesh_tol=args.tol)
    t0 = time.time()
    prim = synth.quadrants_2d(p, synth.quadrant_states(p, args.seed))
    run, feats, tgts, gstats = generate(torch, p, prim, args.train_steps, "train ")
    t_gen = time.time() - t0
    t0 = time.time()
    P, hist = train(torch, run.ctx, feats, tgts, args.iters, args.batch, args.lr, args.seed)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    err_train = heldout_error(torch, run.ctx, P, feats, tgts, run.dxi)
    _log("training frames: relative displacement error %.3f" % err_train)
    # same run, later steps (in distribution) and a run from other quadrant states
    same = compare(torch, run, P, args.test_steps, "same-run ")
    prim2 = synth.quadrants_2d(p, synth.quadrant_states(p, args.test_seed))
    run2 = Run(torch, p, prim2)
    other = compare(torch, run2, P, args.test_steps, "other-run ")

    def agg(recs):
        ps, ws = sum(r["plain_ms"] for r in recs), sum(r["warm_ms"] for r in recs)
        return dict(plain_ms=ps, warm_ms=ws, speedup=ps / ws if ws > 0 else None,
                    plain_sweeps=sum(r["plain_sweeps"] for r in recs), warm_sweeps=sum(r["warm_sweeps"] for r in recs),
                    max_final_resid=max(max(r["plain_resid"], r["warm_resid"]) for r in recs))
    out = dict(size=n, tol=args.tol, train_steps=args.train_steps, iters=args.iters, batch=args.batch,
               gen_s=t_gen, train_s=t_train, loss=hist, train_rel_err=err_train,
               same_run=agg(same), other_run=agg(other), steps_same=same, steps_other=other, gen=gstats)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
