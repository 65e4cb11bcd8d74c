"""The fused kernels of the moving step against the library's separate building blocks, bit for
bit: `esvdw_step` (in 2D the node kernel forms each stage's mesh x^n + c_s dt xdot in its tile,
and the redistribution forms the monitor terms and the CFL maxima in one pass) must give exactly
what `redistribute_mesh` followed by three `rk_stage` calls gives (those materialise each stage
mesh), and the redistribution's time step must equal `cfl_dt` on the same state.  Outflow
quadrants, a periodic smooth flow, slip walls and the backward-facing step, on ragged grids."""
import numpy as np
import pytest

from paper_2407_05568_amd import backstep, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd import esvdw
    esvdw.lib()
    return torch


def _case(kind):
    if kind == "quadrants":
        p = synth.problem(2, [70, 45], bc="outflow")
        prim = synth.quadrants_2d(p, synth.quadrant_states(p, 2))
    elif kind == "walls":
        p = synth.problem(2, [66, 40], bc="outflow", walls=[(1, "lo"), (0, "hi")])
        prim = synth.quadrants_2d(p, synth.quadrant_states(p, 5))
    elif kind == "step":
        p = backstep.problem("TD1", 44, 22)
        prim = synth.backward_step(p, "TD1", shock=0.5)
    else:
        p = synth.problem(2, [64, 38], bc="periodic")
        prim = synth.smooth_state(p, 4)
    return p, prim


@pytest.mark.parametrize("kind", ["quadrants", "periodic", "walls", "step"])
def test_fused_step_equals_building_blocks(torch_dev, kind):
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    p, prim = _case(kind)
    n0, n1 = p["n"][0], p["n"][1]
    f64 = dict(dtype=torch.float64, device="cuda")
    ctx = Context(p)
    x = torch.empty((2, n1, n0), **f64)
    J = torch.empty((n1, n0), **f64)
    JU = torch.empty((4, n1, n0), **f64)
    ctx.init_mesh(x, J, 1)
    ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), J, JU)
    dt = torch.zeros(1, **f64)
    for _ in range(3):  # move the mesh away from uniform first
        ctx.step(JU, J, x, 1, dt)
    torch.cuda.synchronize()
    assert ctx.status() == 0 and bool(torch.isfinite(JU).all())
    a = [t.clone() for t in (JU, J, x)]
    b = [t.clone() for t in (JU, J, x)]
    # the fused step
    dta = torch.zeros(1, **f64)
    ctx.step(a[0], a[1], a[2], 1, dta)
    # the building blocks
    dtb = torch.zeros(1, **f64)
    dtc = torch.zeros(1, **f64)
    ctx.cfl_dt(b[0], b[1], b[2], dtc)
    xdot = torch.empty_like(b[2])
    ctx.redistribute_mesh(b[0], b[1], b[2], None, xdot, dtb)
    s1U, s1J = torch.empty_like(b[0]), torch.empty_like(b[1])
    s2U, s2J = torch.empty_like(b[0]), torch.empty_like(b[1])
    oU, oJ = torch.empty_like(b[0]), torch.empty_like(b[1])
    xn = torch.empty_like(b[2])
    ctx.rk_stage(0, dtb, b[0], b[1], b[0], b[1], b[2], xdot, s1U, s1J)
    ctx.rk_stage(1, dtb, b[0], b[1], s1U, s1J, b[2], xdot, s2U, s2J)
    ctx.rk_stage(2, dtb, b[0], b[1], s2U, s2J, b[2], xdot, oU, oJ, xn)
    torch.cuda.synchronize()
    assert float(dta.item()) == float(dtb.item()) == float(dtc.item())
    assert torch.equal(a[0], oU) and torch.equal(a[1], oJ)
    assert torch.equal(a[2], xn)
    assert ctx.status() == 0 and bool(torch.isfinite(oU).all())
