"""Learned warm start for the mesh redistribution (Section 4): data generation from the
scheme's own runs, training with the library's MFMA forward/backward and Adam kernels, and
the comparison with the plain iteration at the same final residual.

A frame is a state (U^n, x^n) of a moving-mesh run of the method (its usual fixed sweep
count): its inputs are the node features written by ``mlp_features`` and its target is the
converged (pre-limiter) displacement (x* - x^n) / dxi per component, x* the solution of the
discretised mesh equations for the monitor of that state.  The network sees only the 5 x 5
stencil of features around a node.

Every solve is finished by a plain iteration to the same final residual (the largest node
update one Jacobi sweep would make), so the final mesh residual does not depend on the
network.  Two finishers: the method's Jacobi iteration (tolerance mode of redistribute_mesh)
and red-black SOR (`mesh_sor`, Gauss-Seidel for relax 1).  The SOR comparison starts the warm
solve with a few Gauss-Seidel sweeps, which damp the pointwise error of the network's output
(over-relaxed SOR damps every mode at the same slow rate, so pointwise noise would otherwise
cost as many sweeps as a smooth error of the same size).

Run as a module for the full-size experiment (prints one JSON line, progress on stderr):
    python -m paper_2407_05568_amd.learned --size 1024 [--save weights.npz]
(frames every 5 steps of the method's own runs from 6 training seeds, 3 frames each of 2
held-out seeds for the comparison).
"""
import argparse
import json
import math
import os
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
        self.torch, self.p, self.tol = torch, p, tol
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


def default_relax(n):
    """Over-relaxation factor for an n x n grid, 2 / (1 + c pi / n) with c = 0.42, fitted to the
    best factor of the 64^2 and 128^2 quadrant frames (the variable monitor makes the
    iteration slower than for the plain Laplacian, whose optimum has c = 1)."""
    return 2.0 / (1.0 + 0.42 * math.pi / n)


class SorSolver:
    """Red-black SOR to a Jacobi-residual tolerance on the mesh of a `Run`: `check` sweeps at a
    time, then the largest node update one Jacobi sweep would make is measured; the solve stops
    once it is below the tolerance (checks included in the time)."""

    def __init__(self, torch, run, relax=None, check=50):
        self.torch, self.run = torch, run
        self.relax = relax or default_relax(max(run.p["n"][:2]))
        self.check = check
        self.omega = torch.empty_like(run.J)
        self.x = torch.empty_like(run.x)
        self.xc = torch.empty_like(run.x)
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")

    def residual(self, x):
        """Largest node update of one Jacobi sweep from x (x is not changed)."""
        run = self.run
        self.xc.copy_(x)
        run.ctx.mesh_jacobi(self.omega, self.xc, 1, self.res, run.stream)
        return float(self.res.item())

    def solve(self, tol, warm=None, start=None, presmooth=0, max_sweeps=10_000_000):
        """Solve from x^n (+ warm, a displacement), or from the mesh `start`; `presmooth`
        Gauss-Seidel sweeps first.  Returns (sweeps, final residual, ms); the mesh is left in
        self.x."""
        torch, run = self.torch, self.run
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run.stream)
        run.ctx.mesh_monitor(run.JU, run.J, self.omega, run.stream)
        if start is not None:
            self.x.copy_(start)
        elif warm is not None:
            torch.add(run.x, warm, out=self.x)
        else:
            self.x.copy_(run.x)
        sweeps = 0
        if presmooth:
            run.ctx.mesh_sor(self.omega, self.x, presmooth, 1.0, None, run.stream)
            sweeps += presmooth
        res = self.residual(self.x)
        while res >= tol and sweeps < max_sweeps:
            run.ctx.mesh_sor(self.omega, self.x, self.check, self.relax, None, run.stream)
            sweeps += self.check
            res = self.residual(self.x)
        e1.record(run.stream)
        torch.cuda.synchronize()
        return sweeps, res, e0.elapsed_time(e1)


def generate(torch, p, prims, frames, every, tol=1e-10, tag=""):
    """Frames from runs of the method: for each initial state in `prims`, `frames` frames taken
    every `every` steps (features and the converged displacement / dxi, FP32 [F][2][N], the
    mesh equations solved by SOR to the residual tol).  Returns (feats, tgts, statistics)."""
    shape = tuple(reversed(p["n"][:2]))
    F = frames * len(prims)
    feats = torch.empty((F, 2) + shape, dtype=torch.float32, device="cuda")
    tgts = torch.empty_like(feats)
    stats = []
    f = 0
    d = p["dim"]
    for r, prim in enumerate(prims):
        run = Run(torch, p, prim, tol)
        sor = SorSolver(torch, run)
        for k in range(frames):
            run.features(feats[f])
            sw, res, ms = sor.solve(tol)
            tgts[f].copy_(((sor.x - run.x) / run.dxi.view((d,) + (1,) * d)).float())
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


def warm_start(torch, run, P, feat, warm):
    """Features and inference for the current state of `run` into warm (2 fields, displacement
    in domain units); returns the GPU ms they took."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(run.stream)
    run.features(feat)
    run.ctx.mlp_infer(feat, P, warm, run.stream)
    e1.record(run.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def compare(torch, run, P, frames, every, tag="", finisher="sor", presmooth=8, previous=True):
    """At `frames` frames of `run`, `every` steps apart, the redistribution solved to the
    tolerance three ways: plain (x^[0] = x^n), warm (features + inference + the same iteration
    from x^n + warm_dx, with `presmooth` Gauss-Seidel sweeps first for the SOR finisher), and,
    for the SOR finisher with previous=True, from the converged mesh of the step before (a
    non-learned warm start, for reference).  With the SOR finisher the warm start is also tried
    clipped with the movement limiter's bound: x^n + Delta_gamma warm_dx, Delta_gamma the
    limiter factor of the move x^n -> x^n + warm_dx (Section 4).  finisher "sor" (red-black
    SOR) or "jacobi" (the method's iteration).  The run advances with the method's own step
    between frames."""
    shape = tuple(reversed(run.p["n"][:2]))
    feat = torch.empty((2,) + shape, dtype=torch.float32, device="cuda")
    warm = torch.empty((2,) + shape, dtype=torch.float64, device="cuda")
    gam = torch.zeros(1, dtype=torch.float64, device="cuda")
    sor = SorSolver(torch, run) if finisher == "sor" else None
    xprev = torch.empty_like(run.x) if (sor and previous) else None
    out = []
    for k in range(frames):
        if xprev is not None:  # the converged mesh of the step before the frame
            sor.solve(1e-10)
            xprev.copy_(sor.x)
            run.advance(1)
        ms_inf = warm_start(torch, run, P, feat, warm)
        if sor is not None:
            tol = run.tol
            sw_w, res_w, ms_w = sor.solve(tol, warm=warm, presmooth=presmooth)
            sw_p, res_p, ms_p = sor.solve(tol)
        else:
            sw_w, res_w, ms_w = run.solve(warm)
            sw_p, res_p, ms_p = run.solve()
        rec = dict(plain_sweeps=sw_p, plain_resid=res_p, plain_ms=ms_p, warm_sweeps=sw_w, warm_resid=res_w,
                   warm_ms=ms_w + ms_inf, infer_ms=ms_inf)
        line = "%sframe %d: plain %d sweeps %.1f ms (res %.1e) | warm %d sweeps %.1f ms (+%.2f ms net, res %.1e)" % (
            tag, k, sw_p, ms_p, res_p, sw_w, ms_w, ms_inf, res_w)
        if sor is not None:  # the warm start clipped with the limiter's bound
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(run.stream)
            sor.xc.copy_(run.x).add_(warm)
            run.ctx.mesh_limiter(run.x, sor.xc, gam, run.stream)
            warm.mul_(gam)
            e1.record(run.stream)
            torch.cuda.synchronize()
            sw_l, res_l, ms_l = sor.solve(run.tol, warm=warm, presmooth=presmooth)
            ms_l += ms_inf + e0.elapsed_time(e1)
            rec.update(limited_sweeps=sw_l, limited_resid=res_l, limited_ms=ms_l, gamma=float(gam.item()))
            line += " | limited (gamma %.3g) %d sweeps %.1f ms" % (float(gam.item()), sw_l, ms_l)
        if xprev is not None:
            sw_q, res_q, ms_q = sor.solve(run.tol, start=xprev)
            rec.update(prev_sweeps=sw_q, prev_resid=res_q, prev_ms=ms_q)
            line += " | previous mesh %d sweeps %.1f ms" % (sw_q, ms_q)
        out.append(rec)
        _log(line)
        run.advance(every - 1 if xprev is not None else every)
    return out


def save_params(path, P, meta):
    """FP32 parameters and a description of how they were made (npz, no pickled objects)."""
    np.savez(path, params=P.detach().cpu().numpy().astype(np.float32), meta=np.array(json.dumps(meta)))


def load_params(path):
    d = np.load(path)
    return d["params"].astype(np.float32), json.loads(str(d["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--train-seeds", default="0,4,5,11,13,14")
    ap.add_argument("--test-seeds", default="2,19")
    ap.add_argument("--frames", type=int, default=6)
    ap.add_argument("--test-frames", type=int, default=3)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--iters", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--presmooth", type=int, default=8)
    ap.add_argument("--jacobi", action="store_true", help="also compare with the Jacobi finisher (slow)")
    ap.add_argument("--save", default=None, help="write the trained parameters (npz)")
    ap.add_argument("--load", default=None, help="compare with these parameters (npz) instead of training")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the learned warm start runs on the GPU"
    n = args.size
    p = synth.problem(2, [n, n], bc="outflow")
    seeds = [int(v) for v in args.train_seeds.split(",")]
    tests = [int(v) for v in args.test_seeds.split(",")]
    if args.load:
        Pl, meta = load_params(args.load)
        if meta.get("size") != n:
            raise ValueError("%s was trained at %s^2, not %d^2" % (args.load, meta.get("size"), n))
        P = torch.from_numpy(Pl).cuda()
        seeds, t_gen, t_train, hist, gstats = meta.get("train_seeds", seeds), 0.0, 0.0, [], None
        err_train = meta.get("train_rel_err")
    else:
        t0 = time.time()
        prims = [synth.quadrants_2d(p, synth.quadrant_states(p, sd)) for sd in seeds]
        feats, tgts, gstats = generate(torch, p, prims, args.frames, args.every, 1e-10, "train ")
        t_gen = time.time() - t0
        ctx = Context(p)
        dxi = torch.tensor([1.0 / n, 1.0 / n], dtype=torch.float64, device="cuda")
        t0 = time.time()
        P, hist = train(torch, ctx, feats, tgts, args.iters, args.batch, args.lr, seeds[0], log_every=1000)
        torch.cuda.synchronize()
        t_train = time.time() - t0
        err_train = heldout_error(torch, ctx, P, feats, tgts, dxi)
        _log("training frames: relative displacement error %.3f" % err_train)
        del feats, tgts
    if args.save and not args.load:
        save_params(args.save, P, dict(size=n, train_seeds=seeds, frames=args.frames, every=args.every,
                                       iters=args.iters, batch=args.batch, lr=args.lr, train_rel_err=err_train,
                                       command="python -m paper_2407_05568_amd.learned --size %d --iters %d --save PATH" % (n, args.iters)))
    out = dict(size=n, tol=args.tol, train_seeds=seeds, test_seeds=tests, frames_per_run=args.frames,
               every=args.every, iters=args.iters, batch=args.batch, gen_s=t_gen, train_s=t_train, loss=hist,
               train_rel_err=err_train, presmooth=args.presmooth, gen=gstats)
    for fin in (["sor", "jacobi"] if args.jacobi else ["sor"]):
        recs = []
        for sd in tests:
            run = Run(torch, p, synth.quadrants_2d(p, synth.quadrant_states(p, sd)), args.tol)
            recs += compare(torch, run, P, args.test_frames, args.every, "%s held-out seed %d " % (fin, sd), fin,
                            args.presmooth)
            del run
        ps, ws = sum(r["plain_ms"] for r in recs), sum(r["warm_ms"] for r in recs)
        res = dict(plain_ms=ps, warm_ms=ws, speedup=ps / ws if ws > 0 else None,
                   plain_sweeps=sum(r["plain_sweeps"] for r in recs), warm_sweeps=sum(r["warm_sweeps"] for r in recs),
                   max_final_resid=max(max(r["plain_resid"], r["warm_resid"]) for r in recs), frames=recs)
        if fin == "sor":
            qs = sum(r["prev_ms"] for r in recs)
            res.update(previous_ms=qs, previous_speedup=ps / qs if qs > 0 else None,
                       previous_sweeps=sum(r["prev_sweeps"] for r in recs))
            ls = sum(r["limited_ms"] for r in recs)
            res.update(limited_ms=ls, limited_speedup=ps / ls if ls > 0 else None,
                       limited_sweeps=sum(r["limited_sweeps"] for r in recs),
                       gammas=[r["gamma"] for r in recs])
        out[fin] = res
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
