"""Solving the mesh equations to a tolerance: the method's Jacobi iteration against red-black SOR
(`mesh_sor`), at equal final residual, on frames of the 2D four-quadrant problem.

The residual of a mesh is what one Jacobi sweep would still move it: the largest node update of
that sweep (the method's own stopping quantity).  The Jacobi solve is the method's tolerance
mode (`redistribute_mesh` with mesh_tol), which stops once its own last update is below the
tolerance.  The SOR solve runs `check` sweeps at a time and stops once the Jacobi residual of
its mesh is below the same tolerance; its time includes those checks.  Both start from x^n with
the same monitor.  A third, tightly converged solve (SOR to a residual of 1e-12, not timed) is
the reference both are measured against: with the Jacobi iteration's slow modes a small last
update does not mean a small error, so the two meshes that meet the same tolerance need not be
equally close to the solution.

    python -m paper_2407_05568_amd.meshsolve --size 1024 [--relax R]

prints one JSON line (per frame: sweeps, GPU ms, final residual and distance to the reference of
each solve; totals and the speed-up).  The frames are those of the learned warm-start
comparison: held-out initial states, taken every 5 steps of the method's own run.
"""
import argparse
import json
import sys

from . import synth
from .learned import Run, SorSolver, default_relax


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def compare(torch, run, frames, every, relax, tol, check, tag=""):
    sor = SorSolver(torch, run, relax, check)
    out = []
    for k in range(frames):
        sw_j, res_j, ms_j = run.solve()
        xj = torch.empty_like(run.x)
        run.ctx_tol.mesh_converged(xj, run.stream)
        sw_s, res_s, ms_s = sor.solve(tol)
        xs = sor.x.clone()
        sor.solve(1e-12)
        ref = sor.x
        err_j = float((xj - ref).abs().max())
        err_s = float((xs - ref).abs().max())
        rec = dict(jacobi_sweeps=sw_j, jacobi_resid=res_j, jacobi_ms=ms_j, jacobi_err=err_j,
                   sor_sweeps=sw_s, sor_resid=sor.residual(xs), sor_ms=ms_s, sor_err=err_s)
        out.append(rec)
        _log("%sframe %d: Jacobi %d sweeps %.1f ms (err %.1e) | SOR %d sweeps %.1f ms (residual %.1e, err %.1e)" % (
            tag, k, sw_j, ms_j, err_j, sw_s, ms_s, rec["sor_resid"], err_s))
        run.advance(every)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--seeds", default="2,19")
    ap.add_argument("--frames", type=int, default=3)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--relax", type=float, default=0.0, help="0: default_relax(size)")
    ap.add_argument("--check", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the comparison runs on the GPU"
    n = args.size
    relax = args.relax or default_relax(n)
    p = synth.problem(2, [n, n], bc="outflow")
    recs = []
    for sd in [int(v) for v in args.seeds.split(",")]:
        run = Run(torch, p, synth.quadrants_2d(p, synth.quadrant_states(p, sd)), args.tol)
        recs += compare(torch, run, args.frames, args.every, relax, args.tol, args.check, "seed %d " % sd)
        del run
    js, ss = sum(r["jacobi_ms"] for r in recs), sum(r["sor_ms"] for r in recs)
    out = dict(size=n, tol=args.tol, relax=relax, check=args.check, jacobi_ms=js, sor_ms=ss, speedup=js / ss,
               jacobi_sweeps=sum(r["jacobi_sweeps"] for r in recs), sor_sweeps=sum(r["sor_sweeps"] for r in recs),
               max_jacobi_err=max(r["jacobi_err"] for r in recs), max_sor_err=max(r["sor_err"] for r in recs),
               frames=recs)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
