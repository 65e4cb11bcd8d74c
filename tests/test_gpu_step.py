"""The backward-facing step (Example 5.5) and the inflow face on the GPU against the oracle: the
step's faces, its corner and the inflow face, on the uniform mesh (UM) and the adaptive moving
mesh (MM), whole steps at the per-node bar of the other multi-step cases (max(1e-9, 8 kappa),
tests/parity.py); and a closed L-shaped box's mass on the GPU.  Small grids of the example's
geometry (backstep.problem), with the shock started next to the corner so that it diffracts
within the run."""
import numpy as np
import pytest

import parity
from paper_2407_05568_amd import backstep, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd import esvdw
    esvdw.lib()
    return torch


def gpu_run(torch, p, prim, steps, moving):
    from paper_2407_05568_amd.esvdw import Context
    n0, n1 = p["n"][0], p["n"][1]
    ctx = Context(p)
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty((2, n1, n0), **f64)
    J = torch.empty((n1, n0), **f64)
    JU = torch.empty((4, n1, n0), **f64)
    dt = torch.zeros(1, **f64)
    ctx.init_mesh(x, J, 1)
    ctx.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), J, JU)
    for _ in range(steps):
        ctx.step(JU, J, x, int(moving), dt)
    torch.cuda.synchronize()
    return (JU / J).cpu().numpy(), x.cpu().numpy(), J.cpu().numpy(), JU.cpu().numpy(), ctx.status()


def oracle_run(orc, p, prim, steps, moving, perturb=None):
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    JU = o.init_state(prim, J)
    if perturb is not None:
        JU = parity.perturb(JU, perturb)
    for _ in range(steps):
        JU, J, x, _ = o.step(JU, J, x, moving=moving)
    return JU / J, x, o.flags()


@pytest.mark.parametrize("case,moving,steps", [("TD1", False, 12), ("TD1", True, 8), ("TD2", True, 6)])
def test_backward_step_matches_oracle(torch_dev, orc, case, moving, steps):
    p = backstep.problem(case, 40, 20)
    prim = synth.backward_step(p, case, shock=0.5)
    Ug, xg, _, _, st = gpu_run(torch_dev, p, prim, steps, moving)
    Uo, xo, fo = oracle_run(orc, p, prim, steps, moving)
    assert st == fo == 0
    fl = backstep.fluid(p)
    pr = [oracle_run(orc, p, prim, steps, moving, sd) for sd in (1, 2, 3)]
    name = "backward step %s %s 40x20, %d steps" % (case, "MM" if moving else "UM", steps)
    parity.check(name + " U", Ug[:, fl], Uo[:, fl], [r[0][:, fl] for r in pr], 1e-9)
    parity.check(name + " x", xg, xo, [r[1] for r in pr], 1e-12)
    if moving:
        assert np.abs(xo - orc.Oracle(p).uniform_mesh()).max() > 1e-3  # the mesh moved


def test_closed_l_box_mass_on_gpu(torch_dev, orc):
    walls = [(0, "lo"), (0, "hi"), (1, "lo"), (1, "hi")]
    p = synth.problem(2, [32, 32], bc="outflow", walls=walls, step=[10, 12])
    X, Y = synth.nodes_xi(p)
    g = np.exp(-((X - 0.7) ** 2 + (Y - 0.6) ** 2) / 0.02)
    prim = np.stack([0.8 + 0.15 * g, 0.1 * np.sin(2 * np.pi * Y), 0.05 * np.cos(2 * np.pi * X), 1.4 + 0.2 * g])
    Ug, xg, Jg, JUg, st = gpu_run(torch_dev, p, prim, 20, True)
    assert st == 0
    fl = np.ones((32, 32), bool)
    fl[:12, :10] = False
    o = orc.Oracle(p)
    x0 = o.uniform_mesh()
    JU0 = o.init_state(prim, o.jacobian(x0))
    for v in (0, 3):
        assert abs(JUg[v][fl].sum() - JU0[v][fl].sum()) <= 1e-13 * abs(JU0[v][fl].sum())
    Uo, xo, fo = oracle_run(orc, p, prim, 20, True)
    pr = [oracle_run(orc, p, prim, 20, True, sd) for sd in (1, 2, 3)]
    parity.check("closed L-shaped box 32x32 MM, 20 steps U", Ug[:, fl], Uo[:, fl], [r[0][:, fl] for r in pr], 1e-9)
    parity.check("closed L-shaped box 32x32 MM, 20 steps x", xg, xo, [r[1] for r in pr], 1e-12)
