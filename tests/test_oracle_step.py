"""The backward-facing step (Example 5.5) and the inflow face: pins of the oracle.

The step is a solid block of nodes in the lower-left corner of a 2D grid; its two faces are
reflecting walls.  Seen along a direction, the solid nodes next to a face stand for the mirror
images of the fluid nodes across it (per direction: the corner block holds a different image
along each).  What the mathematics fixes, and what a mistake in the images, their signs or the
mesh treatment near the corner breaks:
  * a fluid at rest stays at rest on the adaptive moving mesh (the discrete metric identities
    hold at every fluid node only if the metrics of the images equal the metrics of the imaged
    mesh, which the mirror-symmetric lattice of the 6 x 6 nodes around the corner provides);
  * on a perturbed mesh, the RHS of a fluid at rest is that state times the VCL's dJ (the
    momentum RHS is minus the pressure times the metric identities);
  * a closed L-shaped box conserves mass and energy on the moving mesh;
  * a square L-shaped box is symmetric under transposition (x <-> y, v_1 <-> v_2): the images
    along the two directions are built alike;
  * the flux through the step's face equals the interface flux of the explicit mirrored
    stencil, and the flux through the inflow face that of the stencil with the inflow state in
    its three ghost nodes (both built here by hand from the node states and metrics);
  * a uniform stream entering through the inflow face stays uniform."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth

WALLS = [(0, "lo"), (0, "hi"), (1, "lo"), (1, "hi")]


def fluid_mask(p):
    m = np.ones(tuple(reversed(p["n"][:2])), bool)
    s0, s1 = p["step"]
    m[:s1, :s0] = False
    return m


def blob(p):
    """Smooth supercritical data (T about 1.2 T_c) with a density and pressure bump and a
    divergence-free-ish velocity."""
    X, Y = synth.nodes_xi(p)
    g = np.exp(-((X - 0.7) ** 2 + (Y - 0.6) ** 2) / 0.02)
    prim = np.zeros((4,) + X.shape)
    prim[0] = 0.8 + 0.15 * g
    prim[1] = 0.1 * np.sin(2 * np.pi * Y)
    prim[2] = 0.05 * np.cos(2 * np.pi * X)
    prim[3] = 1.4 + 0.2 * g
    return prim


def run(orc, p, prim, steps, moving, x=None):
    o = orc.Oracle(p)
    x = o.uniform_mesh() if x is None else x
    J = o.jacobian(x)
    JU = o.init_state(prim, J)
    for _ in range(steps):
        JU, J, x, _ = o.step(JU, J, x, moving=moving)
    assert o.flags() == 0
    return o, JU, J, x


def test_rest_stays_at_rest_on_moving_mesh(orc):
    p = synth.problem(2, [30, 24], bc="outflow", walls=WALLS, step=[10, 9])
    prim = np.zeros((4, 24, 30))
    prim[0], prim[3] = 0.8, 1.2
    o, JU, J, x = run(orc, p, prim, 6, True)
    U = JU / J
    fl = fluid_mask(p)
    assert np.abs(U[1:3][:, fl]).max() < 1e-13
    assert np.abs(U[0][fl] - U[0][fl][0]).max() < 1e-13
    assert np.abs(x - o.uniform_mesh()).max() > 1e-3  # the rounding-level monitor moved the mesh


def test_rest_state_rhs_vanishes_on_perturbed_mesh(orc):
    p = synth.problem(2, [30, 24], bc="outflow", walls=WALLS, step=[10, 9])
    o = orc.Oracle(p)
    x = synth.smooth_mesh(p, 3, amp=0.03)
    o.step_fill_mesh(x)
    J = o.jacobian(x)
    prim = np.zeros((4, 24, 30))
    prim[0], prim[3] = 0.8, 1.2  # at rest: the momentum RHS is -p times the metric identities
    JU = o.init_state(prim, J)
    met, _ = o.metrics(x)
    dJU, dJ = o.rhs(JU, J, met, None)
    fl = fluid_mask(p)
    assert np.abs((dJU - JU / J * dJ)[:, fl]).max() < 1e-12


def test_closed_l_box_conserves_mass_and_energy(orc):
    p = synth.problem(2, [24, 24], bc="outflow", walls=WALLS, step=[8, 8])
    prim = blob(p)
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    JU0 = o.init_state(prim, o.jacobian(x))
    fl = fluid_mask(p)
    o, JU, J, x = run(orc, p, prim, 6, True)
    for v in (0, 3):
        assert abs(JU[v][fl].sum() - JU0[v][fl].sum()) <= 1e-14 * abs(JU0[v][fl].sum())
    assert np.abs(x - o.uniform_mesh()).max() > 1e-2


def test_corner_block_moves_as_a_mirror_symmetric_lattice(orc):
    """The 6 x 6 nodes around the corner: after moving-mesh steps with a density bump at the
    corner, x_1 depends on the column only and x_2 on the row only, the columns s0 + m and
    s0 - 1 - m (rows s1 + m and s1 - 1 - m) lie at equal distances on both sides of the face, and
    the block has moved."""
    p = synth.problem(2, [24, 24], bc="outflow", walls=WALLS, step=[8, 8])
    X, Y = synth.nodes_xi(p)
    g = np.exp(-((X - 0.36) ** 2 + (Y - 0.38) ** 2) / 0.004)
    prim = blob(p)
    prim[0] += 0.2 * g
    prim[3] += 0.3 * g
    o, JU, J, x = run(orc, p, prim, 6, True)
    s0, s1 = p["step"]
    fx, fy = s0 / 24.0, s1 / 24.0
    bx, by = x[0][s1 - 3:s1 + 3, s0 - 3:s0 + 3], x[1][s1 - 3:s1 + 3, s0 - 3:s0 + 3]
    assert np.abs(bx - bx[0]).max() == 0.0 and np.abs(by - by[:, :1]).max() == 0.0
    assert np.abs((bx[0, 3:] - fx) - (fx - bx[0, 2::-1])).max() < 1e-15
    assert np.abs((by[3:, 0] - fy) - (fy - by[2::-1, 0])).max() < 1e-15
    u = o.uniform_mesh()
    assert np.abs(bx - u[0][s1 - 3:s1 + 3, s0 - 3:s0 + 3]).max() > 1e-3 / 24


def test_square_l_box_is_transposition_symmetric(orc):
    p = synth.problem(2, [24, 24], bc="outflow", walls=WALLS, step=[8, 8])
    prim = blob(p)
    primT = np.ascontiguousarray(np.stack([prim[0].T, prim[2].T, prim[1].T, prim[3].T]))
    _, JU, J, _ = run(orc, p, prim, 5, False)
    _, JUT, JT, _ = run(orc, p, primT, 5, False)
    U, UT = JU / J, JUT / JT
    back = np.stack([UT[0].T, UT[2].T, UT[1].T, UT[3].T])
    fl = fluid_mask(p)
    for v in range(4):
        assert np.abs(U[v] - back[v])[fl].max() <= 1e-10 * np.abs(U[v]).max(), v


def _stencil(o, U, met, k, i0, i1, image=None, ghost=None):
    """The 6-node stencil of the face between node (i0, i1) and the next along k, built by hand:
    image(j) -> (source index along k) for nodes standing for mirror images; ghost: a fixed
    conserved state for nodes before index 0."""
    st, mx, mt = np.zeros((6, 4)), np.zeros((6, 2)), np.zeros(6)
    for s in range(6):
        j = (i0 if k == 0 else i1) + s - 2
        src, sg = j, 1.0
        if image is not None and image(j) is not None:
            src, sg = image(j), -1.0
        a0, a1 = (src, i1) if k == 0 else (i0, src)
        if ghost is not None and j < 0:
            # the fixed state; metrics of the mesh's mirror image across the face (as outflow)
            st[s] = ghost
            a0, a1 = (-1 - j, i1) if k == 0 else (i0, -1 - j)
            msrc = [met[k * 2 + jj][a1, a0] * (-1.0 if jj != k else 1.0) for jj in range(2)]
        else:
            st[s] = U[:, a1, a0]
            if sg < 0:
                st[s][1 + k] = -st[s][1 + k]
            msrc = [met[k * 2 + jj][a1, a0] * (sg if jj != k else 1.0) for jj in range(2)]
        mx[s] = msrc
    return o.interface_flux(st.ravel(), mx.ravel(), mt)


def test_step_face_flux_is_the_mirrored_stencil(orc):
    p = synth.problem(2, [24, 20], bc="outflow", walls=WALLS, step=[8, 10])
    prim = blob(p)
    o = orc.Oracle(p)
    x = synth.smooth_mesh(p, 5, amp=0.02)
    o.step_fill_mesh(x)
    J = o.jacobian(x)
    JU = o.init_state(prim, J)
    met, _ = o.metrics(x)
    recs, _, _ = o.rhs_record(JU, J, met)
    U = JU / J
    s0, s1 = p["step"]
    # vertical face, row 4: interface index s0 along x (left node s0 - 1 is an image)
    F = recs[0]["F"][:, 4, s0]
    ref = _stencil(o, U, met, 0, s0 - 1, 4, image=lambda j: 2 * s0 - 1 - j if j < s0 else None)["F"]
    assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max()
    # horizontal face, column 3
    F = recs[1]["F"][:, s1, 3]
    ref = _stencil(o, U, met, 1, 3, s1 - 1, image=lambda j: 2 * s1 - 1 - j if j < s1 else None)["F"]
    assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max()
    # interfaces inside the solid block carry no flux into the fluid, and the solid does not evolve
    dJU, dJ = o.rhs(JU, J, met)
    assert np.abs(dJU[:, :s1, :s0]).max() == 0.0 and np.abs(dJ[:s1, :s0]).max() == 0.0


def test_inflow_face_flux_uses_the_inflow_state(orc):
    inflow = [0.85, 0.64 * np.sqrt(8.0 / 3.0), 0.0, 1.01]
    p = synth.problem(2, [20, 16], bc="outflow", inflow=inflow)
    prim = blob(p)
    o = orc.Oracle(p)
    x = synth.smooth_mesh(p, 2, amp=0.02)
    J = o.jacobian(x)
    JU = o.init_state(prim, J)
    met, _ = o.metrics(x)
    recs, _, _ = o.rhs_record(JU, J, met)
    U = JU / J
    Uin = o.prim_to_cons(inflow)
    for row in (0, 7, 15):
        F = recs[0]["F"][:, row, 0]
        ref = _stencil(o, U, met, 0, -1, row, ghost=Uin)
        assert np.abs(F - ref["F"]).max() <= 1e-13 * np.abs(ref["F"]).max(), row


def test_uniform_stream_through_the_inflow_face_stays_uniform(orc):
    inflow = [0.8, 0.3, 0.0, 1.3]
    p = synth.problem(2, [24, 12], bc="outflow", inflow=inflow)
    prim = np.zeros((4, 12, 24))
    for v in range(4):
        prim[v] = inflow[v]
    o, JU, J, x = run(orc, p, prim, 8, True)
    U0 = o.prim_to_cons(inflow)
    U = JU / J
    for v in range(4):
        assert np.abs(U[v] - U0[v]).max() <= 1e-13 * max(1.0, abs(U0[v])), v


def test_step_and_inflow_configuration_checks(orc):
    with pytest.raises(ValueError):
        orc.Oracle(synth.problem(2, [16, 16], bc="periodic", step=[4, 4]))
    with pytest.raises(ValueError):
        orc.Oracle(synth.problem(2, [16, 16], bc="outflow", step=[14, 4]))
    with pytest.raises(ValueError):
        orc.Oracle(synth.problem(2, [16, 16], bc="outflow", step=[2, 4]))
    with pytest.raises(ValueError):
        orc.Oracle(synth.problem(2, [16, 16], bc="outflow", walls=[(0, "lo")], inflow=[1, 0, 0, 1]))
    with pytest.raises(ValueError):
        orc.Oracle(synth.problem(2, [16, 16], bc="outflow", step=[4, 4], fixed_mu=0))
