"""Reflecting walls on the GPU against the oracle: closed boxes and a half-open channel with a
wall below (the boundary of Examples 5.4-5.5), many moving-mesh steps each, and the mass of a
closed box kept on the GPU.  Bar: max(1e-9, 8 kappa) per field after the run (kappa: the oracle's
own change under a 1-ulp perturbation of its initial state), as for the other multi-step runs."""
import os
import sys

import numpy as np
import pytest

from paper_2407_05568_amd import synth

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_walls import smooth_even_odd  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd import esvdw
    esvdw.lib()
    return torch


def relerr(g, r):
    g = np.asarray(g).reshape(np.shape(g)[0], -1)
    r = np.asarray(r).reshape(g.shape)
    return max(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300) for a, b in zip(g, r))


CASES = {
    "box1d": (1, [60], [(0, "lo"), (0, "hi")], "smooth", 40),
    "box2d": (2, [40, 36], [(0, "lo"), (0, "hi"), (1, "lo"), (1, "hi")], "smooth", 30),
    "channel2d": (2, [48, 40], [(1, "lo")], "quadrants", 30),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_walls_match_oracle(orc, torch_dev, case):
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    dim, n, walls, kind, steps = CASES[case]
    p = synth.problem(dim, n, bc="outflow", walls=walls)
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    prim = smooth_even_odd(x, dim) if kind == "smooth" else synth.quadrants_2d(p, synth.quadrant_states(p, 0))
    JU = o.init_state(prim, J)
    ctx = Context(p)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xg = T(x)
    Jg = torch.empty(o.shape, dtype=torch.float64, device="cuda")
    ctx.init_mesh(xg, Jg, 1)
    JUg = torch.empty((dim + 2,) + o.shape, dtype=torch.float64, device="cuda")
    ctx.init_state(T(prim), Jg, JUg)
    m0 = float(JUg[0].sum())
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    perturbed = []
    for seed in (7, 8):  # kappa: the larger of two 1-ulp perturbations
        rng = np.random.default_rng(seed)
        perturbed.append([JU * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=JU.shape)), J.copy(), x.copy()])
    for _ in range(steps):
        JU, J, x, _ = o.step(JU, J, x, moving=True)
        for q in perturbed:
            q[0], q[1], q[2], _ = o.step(q[0], q[1], q[2], moving=True)
        ctx.step(JUg, Jg, xg, 1, dtg)
    torch.cuda.synchronize()
    kappa = max(max(relerr(q[0] / q[1][None], JU / J[None]), np.abs(q[2] - x).max()) for q in perturbed)
    tol = max(1e-9, 8 * kappa)
    eu = relerr((JUg / Jg[None]).cpu().numpy(), JU / J[None])
    ex = np.abs(xg.cpu().numpy() - x).max()
    print("%s, %d steps: U rel err %.3e x err %.3e kappa %.3e tol %.3e" % (case, steps, eu, ex, kappa, tol))
    assert eu < tol and ex < tol
    assert ctx.status() == 0 and o.flags() == 0
    if len(walls) == 2 * dim:  # closed box: no mass crosses a wall
        assert abs(float(JUg[0].sum()) - m0) <= 1e-13 * m0
