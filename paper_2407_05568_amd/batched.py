"""Many independent 2D problems advanced together (esvdw_batch_*): set-up of a batch from
problem dicts, the tile autotuner, and a throughput run.

The library offers two launch modes over the same work lists and device code: a persistent
kernel (one launch per RK stage, grid barriers between its phases) and phased kernels (CFL,
node data, fluxes and update as separate launches, each at its own occupancy).  Variants
0 .. V/2 - 1 are the persistent kernel with each tile set, V/2 .. V - 1 the phased kernels.  The
autotuner times every variant on the batch it will run (a few full steps each, from the same
initial state, HIP events on the launch stream) and keeps the fastest; the variants compute
identical results, so the choice only moves speed.

Run as a module for the 256-instance batch (prints one JSON line, progress on stderr):
    python -m paper_2407_05568_amd.batched --count 256 --steps 10 [--moving]
With --moving a step is the mesh redistribution of every instance (monitor, 5 filter passes,
10 Jacobi sweeps, limiter, CFL) followed by the three RK stages on the moving meshes.
"""
import argparse
import json
import sys

import numpy as np

from . import synth
from .esvdw import Batch


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


class BatchRun:
    """A batch with its pooled device arrays (uniform meshes, initial states from prims)."""

    def __init__(self, torch, problems, prims, stream=None):
        self.torch = torch
        self.B = Batch(problems)
        self.off = self.B.off
        self.stream = stream or torch.cuda.current_stream()
        f64 = dict(dtype=torch.float64, device="cuda")
        tot = self.B.total
        self.x = torch.zeros(2 * tot, **f64)
        self.J = torch.zeros(tot, **f64)
        self.JU = torch.zeros(4 * tot, **f64)
        self.dt = torch.zeros(len(problems), **f64)
        self.xdot = torch.zeros(2 * tot, **f64)
        self.moving = False
        pool = np.zeros(4 * tot)
        for i, pr in enumerate(prims):
            pool[4 * self.off[i]:4 * self.off[i + 1]] = np.asarray(pr, dtype=np.float64).reshape(-1)
        self.B.init_mesh(self.x, self.J, self.stream)
        self.B.init_state(torch.from_numpy(pool).cuda(), self.J, self.JU, self.stream)
        torch.cuda.synchronize()
        self.JU0, self.J0, self.x0 = self.JU.clone(), self.J.clone(), self.x.clone()

    def reset(self):
        self.JU.copy_(self.JU0)
        self.J.copy_(self.J0)
        self.x.copy_(self.x0)

    def step(self, stream=None):
        st = stream or self.stream
        if self.moving:
            self.B.redistribute(self.JU, self.J, self.x, self.xdot, self.dt, st)
            self.B.step(self.JU, self.J, self.x, self.xdot, self.dt, st)
        else:
            self.B.step(self.JU, self.J, self.x, None, self.dt, st)

    def time_steps(self, steps):
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(steps):
            self.step()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps


def autotune(run, steps=2):
    """Times each tile variant (from the initial state, one untimed step first) and selects the
    fastest.  Returns (best variant, {variant: ms per step})."""
    times = {}
    for v in range(run.B.variants()):
        run.B.set_variant(v)
        run.reset()
        run.step()
        times[v] = run.time_steps(steps)
        _log("  variant %d: %.3f ms/step" % (v, times[v]))
    best = min(times, key=times.get)
    run.B.set_variant(best)
    run.reset()
    return best, times


def launches_per_step(B, v, moving=False, n_filter=5, mu=10):
    """Kernel launches of one step: 3 for the persistent kernel, 2 + 3 x 3 for the phased ones,
    plus 9 + n_filter + mu for the redistribution of a moving step."""
    n = 3 if v < B.variants() // 2 else 11
    return n + (9 + n_filter + mu if moving else 0)


def batch_problems(seed, count):
    inst = synth.batch_instances(seed, count)
    return [p for p, _ in inst], [synth.quadrants_2d(p, st) for p, st in inst]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--moving", action="store_true")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the batched run needs a GPU"
    problems, prims = batch_problems(args.seed, args.count)
    run = BatchRun(torch, problems, prims)
    run.moving = args.moving
    nodes = run.B.total
    _log("batch: %d instances, %d nodes" % (args.count, nodes))
    best, times = (0, {}) if args.no_tune else autotune(run)
    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    # one step captured in a HIP graph, replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            run.step(stream=s)
    torch.cuda.synchronize()
    # replay() launches on the current stream: time it there
    cur = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for _ in range(args.steps):
        g.replay()
    e1.record(cur)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flags = run.B.status()
    out = {"metric": "FP64 node-stage updates/s, batched independent 2D problems%s" % (
               " (moving meshes)" if args.moving else ""), "value": 3 * nodes / (ms / 1e3),
           "unit": "node-stages/s", "ms_per_step": ms, "steps": args.steps, "instances": args.count, "nodes": nodes,
           "variant": best, "mode": "persistent" if best < run.B.variants() // 2 else "phased",
           "variant_ms": times, "launches_per_step": launches_per_step(run.B, best, args.moving), "moving": args.moving,
           "status_flags": flags}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
