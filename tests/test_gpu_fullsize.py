"""The benchmark workload at its full size (2D four-quadrant problem, 1024^2, moving mesh, the
step replayed from a HIP graph as the benchmark times it), and the 512^2 configuration of the
same problem, against the oracle over every node:
one whole step (redistribution, CFL, three RK stages).  Bar: 1e-12 per field and node, or 8 times
the oracle's own change at that node under 1-ulp perturbations of the initial state where that
is larger (tests/parity.py); the mesh to 1e-13 and dt to 1e-13 relative.  The oracle takes a few
seconds per step at this size."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
import parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [512, 1024])
def test_bench_workload_full_step_matches_oracle(orc, n):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd.esvdw import Context
    p = bench.make_problem("2d-quadrants", n)
    prim = bench.initial_prim("2d-quadrants", p, 0)
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    JU = o.init_state(prim, J)
    JU1, J1, x1, dt1 = o.step(JU, J, x, moving=True)
    U1 = JU1 / J1[None]
    pert = []
    for sd in (1, 2, 3):
        JUq, Jq, _, _ = o.step(parity.perturb(JU, sd), J, x, moving=True)
        pert.append(JUq / Jq[None])
    ctx = Context(p)
    f64 = dict(dtype=torch.float64, device="cuda")
    xg = torch.from_numpy(x).cuda()
    Jg = torch.empty((n, n), **f64)
    ctx.init_mesh(xg, Jg, 1)
    JUg = torch.empty((4, n, n), **f64)
    ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), Jg, JUg)
    dtg = torch.zeros(1, **f64)
    # one step captured into a graph on a side stream and replayed once, as the benchmark does
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.step(JUg, Jg, xg, 1, dtg, s)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    Ug = (JUg / Jg[None]).cpu().numpy()
    ex = np.abs(xg.cpu().numpy() - x1).max()
    edt = abs(float(dtg.item()) - dt1) / dt1
    print("%d^2 step: x err %.2e, dt rel err %.2e" % (n, ex, edt))
    parity.check("moving step 2D quadrants %dx%d (graph)" % (n, n), Ug, U1, pert, 1e-12)
    assert ex < 1e-13 and edt < 1e-13
    assert ctx.status() == 0 and o.flags() == 0


def test_quadrants_512_two_hundred_steps():
    """The 512^2 four-quadrant configuration run for its 200 RK steps on the GPU (graph-replayed
    steps): no status flag (every node state admissible, every mean state within Theorem 3.1's
    condition, no NaN), positive densities below 1/b, the mesh inside the box and every cell
    positively oriented (J > 0)."""
    import torch
    from paper_2407_05568_amd.esvdw import Context
    n = 512
    p = bench.make_problem("2d-quadrants", n)
    prim = bench.initial_prim("2d-quadrants", p, 0)
    ctx = Context(p)
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty((2, n, n), **f64)
    J = torch.empty((n, n), **f64)
    ctx.init_mesh(x, J, 1)
    JU = torch.empty((4, n, n), **f64)
    ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), J, JU)
    dt = torch.zeros(1, **f64)
    ctx.step(JU, J, x, 1, dt)
    torch.cuda.synchronize()
    t = float(dt.item())
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.step(JU, J, x, 1, dt, s)
    torch.cuda.synchronize()
    for _ in range(199):
        g.replay()
        torch.cuda.synchronize()
        t += float(dt.item())
    assert ctx.status() == 0
    rho = (JU[0] / J).cpu().numpy()
    r0 = prim[0]
    print("512^2, 200 steps: t = %.4f, rho in [%.4f, %.4f] (data [%.4f, %.4f]), J in [%.3e, %.3e]" % (
        t, rho.min(), rho.max(), r0.min(), r0.max(), float(J.min()), float(J.max())))
    assert np.isfinite(JU.cpu().numpy()).all()
    assert 0.0 < rho.min() and rho.max() < 1.0 / p["b"]
    assert float(J.min()) > 0.0
    xx = x.cpu().numpy()
    assert xx.min() > 0.0 and xx.max() < 1.0
