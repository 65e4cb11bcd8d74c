"""Flow over a backward-facing step (Example 5.5, Table 5.4: TD1, TD2) on the adaptive moving mesh:
MM / MM1 / UM runs with timing, and the density along the line from (0.6, 0.55) to (2, 0.55).

The paper gives the states, the shock Mach numbers, the final times, the cut line and the grids
(200 x 100 cells for MM, 600 x 300 for the fine UM) but not the domain or the step.  Chosen
here: the domain [0, 2] x [0, 1] with the solid step [0, 0.6] x [0, 0.5] (its corner at the cut
line's start), a planar shock at x_1 = 0.3 in the channel above the step with Table 5.4's state
`left` behind it and `right` ahead and in the lower region, the left face (above the step) an
inflow face holding the state `left`, the right face outflow, the floor, the ceiling and both
faces of the step reflecting walls.  Velocities are read in the paper's unit (reduced ones
sqrt(8/3) larger) and times likewise (final times sqrt(3/8) of the printed ones), as for
Table 5.3; delta = 0.0125.  Monitor of Example 5.5: kappa = 2 with rho and G, alpha =
(1200, 1200) (MM1: alpha_2 = 0); 5 filter passes, mu = 10, CFL 0.4.

    python -m paper_2407_05568_amd.backstep --case TD1

prints one JSON line: per run (MM 200x100, MM1 200x100, UM 200x100, UM 600x300) the steps, GPU
time, status, and rho sampled along the cut; and the L1 distance of each run's cut from the
fine UM run's.
"""
import argparse
import json
import math
import sys

import numpy as np

from . import runner, synth
from .esvdw import Context

LX, LY = 2.0, 1.0
STEP_X, STEP_Y = 0.6, 0.5
SHOCK_X = 0.3
CUT_Y, CUT_X0, CUT_X1 = 0.55, 0.6, 2.0


def problem(case, n0, n1, alpha2=1200.0):
    s0, s1 = int(round(STEP_X / LX * n0)), int(round(STEP_Y / LY * n1))
    return synth.problem(2, [n0, n1], bc="outflow", lo=[0.0, 0.0], hi=[LX, LY], walls=[(1, "lo"), (1, "hi")],
                         step=[s0, s1], inflow=list(synth.step_state(case, "left")), kappa=2, mon_var=["rho", "G"],
                         alpha=[1200.0, alpha2, 0.0])


def t_end(case):
    return synth.TABLE_5_4[case]["t_end"] * math.sqrt(3.0 / 8.0)


def fluid(p):
    m = np.ones((p["n"][1], p["n"][0]), bool)
    m[:p["step"][1], :p["step"][0]] = False
    return m


def cut(rho, x, p, npts=281):
    """rho along the cut line, linearly interpolated from the fluid nodes (scattered: the mesh
    moves)."""
    from scipy.interpolate import griddata
    fl = fluid(p)
    xs = np.linspace(CUT_X0, CUT_X1, npts)
    pts = np.stack([x[0][fl], x[1][fl]], axis=1)
    if not (np.isfinite(pts).all() and np.isfinite(rho[fl]).all()):
        return xs, np.full_like(xs, np.nan)  # a failed run: no cut
    return xs, griddata(pts, rho[fl], (xs, np.full_like(xs, CUT_Y)), method="linear")


def run(torch, case, n0, n1, moving=True, alpha2=1200.0, log=None):
    p = problem(case, n0, n1, alpha2)
    ctx = Context(p)
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty((2, n1, n0), **f64)
    J = torch.empty((n1, n0), **f64)
    JU = torch.empty((4, n1, n0), **f64)
    st = torch.cuda.current_stream()
    ctx.init_mesh(x, J, 1, st)
    ctx.init_state(torch.from_numpy(synth.backward_step(p, case, shock=SHOCK_X)).cuda(), J, JU, st)
    te = t_end(case)
    r = runner.advance_to(torch, ctx, p, JU, J, x, moving, te, log=log)
    rho = (JU[0] / J).cpu().numpy()
    xs = x.cpu().numpy()
    fl = fluid(p)
    out = dict(case=case, n=[n0, n1], moving=moving, alpha2=alpha2, steps=r["steps"], t=r["t"], t_end=te,
               gpu_ms=r["gpu_ms"], ms_per_step=r["gpu_ms"] / max(r["steps"], 1), graph_steps=r["graph_steps"],
               flags=r["flags"], rho_min=float(rho[fl].min()), rho_max=float(rho[fl].max()),
               min_J=float(J.cpu().numpy()[fl].min()))
    return out, rho, xs, p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="TD1", choices=sorted(synth.TABLE_5_4))
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the example runs on the GPU"
    log = lambda m: print(m, file=sys.stderr, flush=True)
    runs = [("MM 200x100", 200, 100, True, 1200.0), ("MM1 200x100", 200, 100, True, 0.0),
            ("UM 200x100", 200, 100, False, 1200.0), ("UM 600x300", 600, 300, False, 1200.0)]
    res, cuts = {}, {}
    for name, n0, n1, moving, a2 in runs:
        log("%s %s" % (args.case, name))
        r, rho, xs, p = run(torch, args.case, n0, n1, moving, a2, log=log)
        xc, rc = cut(rho, xs, p)
        r["cut_rho"] = [round(float(v), 6) if np.isfinite(v) else None for v in rc]
        res[name], cuts[name] = r, rc
        log("  %d steps, %.2f s GPU, flags %d" % (r["steps"], r["gpu_ms"] / 1e3, r["flags"]))
    ref = cuts["UM 600x300"]
    for name in res:
        ok = np.isfinite(cuts[name]) & np.isfinite(ref)
        res[name]["cut_l1_vs_um600"] = (float(np.mean(np.abs(cuts[name][ok] - ref[ok])) * (CUT_X1 - CUT_X0))
                                        if ok.any() else None)
    out = dict(case=args.case, cut_x=[round(float(v), 4) for v in np.linspace(CUT_X0, CUT_X1, 281)], runs=res)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
