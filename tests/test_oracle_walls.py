"""Reflecting (slip) walls, the boundary of Examples 5.4-5.5: pins of the oracle.

A box [0,1]^d with walls on every face is the restriction of the periodic problem on [-1,1]^d
whose data are extended evenly (rho, p) and oddly (the velocity component normal to each face)
about every face: mirror symmetry makes the walls exact.  Both are run with the moving mesh and
compared (rounding only).  A closed box conserves mass exactly and keeps a fluid at rest at rest
on any moving mesh."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth


def smooth_even_odd(x, dim):
    """rho, p even about x_k = 0 and x_k = 1; v_k odd about those faces, even across the others;
    supercritical (T about 1.18 T_c, reduced units) so that no state nears the spinodal."""
    if dim == 1:
        X = x[0]
        return np.array([0.8 + 0.1 * np.cos(np.pi * X), 0.1 * np.sin(np.pi * X), 1.5 + 0.1 * np.cos(np.pi * X)])
    X, Y = x[0], x[1]
    c = np.cos(np.pi * X) * np.cos(np.pi * Y)
    return np.array([0.8 + 0.1 * c, 0.1 * np.sin(np.pi * X) * np.cos(np.pi * Y),
                     0.1 * np.cos(np.pi * X) * np.sin(np.pi * Y), 1.5 + 0.1 * c])


def box(dim, n):
    walls = [(k, s) for k in range(dim) for s in ("lo", "hi")]
    return synth.problem(dim, [n] * dim, bc="outflow", walls=walls, lo=[0.0] * dim, hi=[1.0] * dim)


def run(orc, p, steps, prim=None, x=None):
    o = orc.Oracle(p)
    x = o.uniform_mesh() if x is None else x
    J = o.jacobian(x)
    JU = o.init_state(smooth_even_odd(x, p["dim"]) if prim is None else prim, J)
    m0 = JU[0].sum()
    for _ in range(steps):
        JU, J, x, _ = o.step(JU, J, x, moving=True)
    assert o.flags() == 0
    return JU, J, x, m0


@pytest.mark.parametrize("dim,n", [(1, 20), (2, 12)])
def test_wall_box_equals_symmetric_periodic_extension(orc, dim, n):
    JUb, Jb, xb, _ = run(orc, box(dim, n), 5)
    pp = synth.problem(dim, [2 * n] * dim, bc="periodic", lo=[-1.0] * dim, hi=[1.0] * dim)
    JUp, Jp, xp, _ = run(orc, pp, 5)
    half = (slice(n, 2 * n),) * dim
    Ub, Up = JUb / Jb, (JUp / Jp)[(slice(None),) + half]
    for v in range(dim + 2):
        assert np.abs(Ub[v] - Up[v]).max() <= 1e-10 * np.abs(Up[v]).max(), v
    assert np.abs(xb - xp[(slice(None),) + half]).max() < 1e-12


def test_closed_box_conserves_mass_and_keeps_rest(orc):
    p = box(2, 14)
    JU, J, x, m0 = run(orc, p, 6)
    assert abs(JU[0].sum() - m0) <= 1e-14 * m0
    # a fluid at rest on a moving, non-uniform mesh stays at rest
    o = orc.Oracle(p)
    x = synth.smooth_mesh(p, 3, amp=0.03)
    prim = synth.uniform_state(p, v=[0.0, 0.0])
    JU, J, x, m0 = run(orc, p, 6, prim=prim, x=x)
    U = JU / J
    assert np.abs(U[1:3]).max() < 1e-13
    assert abs(JU[0].sum() - m0) <= 1e-14 * m0
    assert np.abs(x - synth.smooth_mesh(p, 3, amp=0.03)).max() > 1e-4  # the mesh did move


def test_walls_only_on_outflow_directions(orc):
    p = synth.problem(2, [8, 8], bc="periodic", walls=[(0, "lo")])
    with pytest.raises(ValueError):
        orc.Oracle(p)
