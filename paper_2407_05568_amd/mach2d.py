"""2D Mach reflection (Example 5.4) on the adaptive moving mesh: an oblique shock (Table 5.3's
P1 or D1) reflecting off a slip wall, MM / MM1 / UM runs with timing, and their density errors
against a fine uniform-mesh run.

The paper gives the domain [0,1] x [0,0.5], the states, the incidence angle and the Mach number
but not the boundary conditions, the initial shock position or a final time consistent with
the data (P1's shock, 15.5 reduced units per unit time, would cross the domain many times by its
t = 1.0).  Chosen here: the shock's normal points along (cos theta, -sin theta) toward the wall
x_2 = 0 (a reflecting wall); its foot starts at x_1 = 0.1; the other faces are outflow
(zero-gradient) boundaries; the run stops when the foot has moved 0.6 along the wall.  Monitor
of Example 5.4: kappa = 1 with rho, alpha_1 = 1200 and alpha_2 = 500 on |Delta G|^2 (MM1:
alpha_2 = 0); 5 filter passes, mu = 10, CFL 0.4; reduced units with delta = gamma - 1.

    python -m paper_2407_05568_amd.mach2d --case P1 [--ref 2400]

prints one JSON line: per run (MM 200x100, MM1 200x100, UM 200x100, UM 600x300) the steps,
GPU time, status and the area-weighted L1 error of rho against UM at ref x ref/2.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import runner, synth
from .esvdw import Context

FOOT, TRAVEL = 0.1, 0.6


def problem(case, n0, n1, alpha2=500.0):
    c = synth.TABLE_5_3[case]
    return synth.problem(2, [n0, n1], bc="outflow", walls=[(1, "lo")], lo=[0.0, 0.0], hi=[1.0, 0.5],
                         delta=c["gamma"] - 1.0, kappa=1, mon_var=["rho"], alpha=[1200.0, alpha2, 0.0])


def t_end(case):
    """Time for the shock's foot to travel TRAVEL along the wall: shock speed from the mass balance
    rho_r S = rho_l (S - u_l) across the front, foot speed S / cos(theta)."""
    c = synth.TABLE_5_3[case]
    u = c["left"][1] * math.sqrt(8.0 / 3.0)
    S = c["left"][0] * u / (c["left"][0] - c["right"][0])
    return TRAVEL * math.cos(math.radians(c["theta"])) / abs(S)


def run(torch, case, n0, n1, moving=True, alpha2=500.0, log=None):
    p = problem(case, n0, n1, alpha2)
    ctx = Context(p)
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty((2, n1, n0), **f64)
    J = torch.empty((n1, n0), **f64)
    JU = torch.empty((4, n1, n0), **f64)
    st = torch.cuda.current_stream()
    ctx.init_mesh(x, J, 1, st)
    ctx.init_state(torch.from_numpy(synth.mach_reflection(p, case, foot=FOOT)).cuda(), J, JU, st)
    te = t_end(case)
    r = runner.advance_to(torch, ctx, p, JU, J, x, moving, te, log=log)
    rho = (JU[0] / J).cpu().numpy()
    return dict(case=case, n=[n0, n1], moving=moving, alpha2=alpha2, steps=r["steps"], t=r["t"], t_end=te,
                gpu_ms=r["gpu_ms"], ms_per_step=r["gpu_ms"] / max(r["steps"], 1), graph_steps=r["graph_steps"],
                flags=r["flags"], min_J=float(J.min())), rho, x.cpu().numpy(), J.cpu().numpy()


def l1_error(rho, x, J, ref, dxi_area):
    """Area-weighted L1 difference of rho at the run's nodes from the reference (uniform grid on
    [0,1] x [0,0.5], bilinear interpolation at the nodes' positions)."""
    ny, nx = ref.shape
    hx, hy = 1.0 / nx, 0.5 / ny
    fx = np.clip(x[0] / hx - 0.5, 0.0, nx - 1.000001)
    fy = np.clip(x[1] / hy - 0.5, 0.0, ny - 1.000001)
    i0, j0 = np.floor(fx).astype(int), np.floor(fy).astype(int)
    ax, ay = fx - i0, fy - j0
    r = ((1 - ax) * (1 - ay) * ref[j0, i0] + ax * (1 - ay) * ref[j0, i0 + 1] + (1 - ax) * ay * ref[j0 + 1, i0] +
         ax * ay * ref[j0 + 1, i0 + 1])
    return float(np.sum(np.abs(rho - r) * J) * dxi_area / 0.5)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="P1", choices=sorted(synth.TABLE_5_3))
    ap.add_argument("--ref", type=int, default=2400)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the example runs on the GPU"
    log = lambda m: print(m, file=sys.stderr, flush=True)
    w0 = time.time()
    info_ref, ref, _, _ = run(torch, args.case, args.ref, args.ref // 2, moving=False, log=log)
    log("reference %dx%d: %d steps, %.1f s" % (args.ref, args.ref // 2, info_ref["steps"], info_ref["gpu_ms"] / 1e3))
    runs = []
    for n0, n1, moving, a2, name in ((200, 100, True, 500.0, "MM"), (200, 100, True, 0.0, "MM1"),
                                     (200, 100, False, 500.0, "UM"), (600, 300, False, 500.0, "UM")):
        info, rho, x, J = run(torch, args.case, n0, n1, moving, a2, log)
        info["name"] = name
        info["l1_rho"] = l1_error(rho, x, J, ref, (1.0 / n0) * (0.5 / n1))
        log("%s %dx%d: %d steps, %.2f s, L1 %.3e, flags %d" % (name, n0, n1, info["steps"], info["gpu_ms"] / 1e3,
                                                           info["l1_rho"], info["flags"]))
        runs.append(info)
    out = dict(case=args.case, reference=info_ref, runs=runs, wall_s=time.time() - w0)
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
