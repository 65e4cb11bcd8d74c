"""Red-black SOR for the mesh equations (`mesh_sor`), GPU against the oracle: the sweeps
themselves at ragged sizes in 1D/2D/3D with outflow and periodic boundaries, the rejection of
odd periodic node counts, and a solve to a tolerance on a four-quadrant frame against the
Jacobi iteration (same fixed point, fewer sweeps, closer to the converged mesh)."""
import numpy as np
import pytest

from paper_2407_05568_amd import esvdw, meshsolve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd import esvdw
    esvdw.lib()
    return torch


CASES = [(1, "outflow", [701]), (2, "outflow", [151, 37]), (2, "periodic", [130, 34]), (3, "outflow", [19, 9, 7]),
         (3, "periodic", [18, 10, 6])]


@pytest.mark.parametrize("dim,bc,n", CASES)
@pytest.mark.parametrize("relax,nsweep", [(1.0, 1), (1.7, 3), (1.95, 8)])
def test_sor_sweeps_match_oracle(orc, torch_dev, dim, bc, n, relax, nsweep):
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    p = synth.problem(dim, n, bc=bc)
    o = orc.Oracle(p)
    rng = np.random.default_rng(dim * 10 + nsweep)
    omega = 1.0 + 3.0 * rng.random(o.shape)
    x0 = synth.smooth_mesh(p, 2, amp=0.02)
    want, res_want = o.sor(omega, x0, nsweep, relax)
    ctx = Context(p)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xg = T(x0)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.mesh_sor(T(omega), xg, nsweep, relax, res)
    torch.cuda.synchronize()
    err = np.abs(xg.cpu().numpy() - want).max()
    print("%dD %s %s relax %.2f x %d: x err %.2e, resid %.6e / %.6e" % (dim, bc, n, relax, nsweep, err,
                                                                       float(res.item()), res_want))
    assert err < 1e-13
    # the residual is a difference of O(1) coordinates: rounding is absolute, ~1e-16
    assert abs(float(res.item()) - res_want) <= 1e-14
    assert ctx.status() == 0


@pytest.mark.parametrize("n,nsweep", [([151, 37], 7), ([64, 64], 4), ([9, 200], 5)])
def test_multi_sweep_sor_equals_single_sweeps(orc, torch_dev, n, nsweep):
    """On 2D outflow grids mesh_sor runs up to two sweeps per launch from an LDS tile; nsweep
    sweeps in one call must equal nsweep calls of one sweep bit for bit (the residual too), and
    the oracle to rounding."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    p = synth.problem(2, n, bc="outflow")
    ctx = Context(p)
    rng = np.random.default_rng(n[0] * 7 + nsweep)
    shape = (n[1], n[0])
    omega = 1.0 + 3.0 * rng.random(shape)
    x0 = synth.smooth_mesh(p, 5, amp=0.02)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    om = T(omega)
    xa, xb = T(x0), T(x0)
    ra = torch.zeros(1, dtype=torch.float64, device="cuda")
    rb = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.mesh_sor(om, xa, nsweep, 1.9, ra)
    for _ in range(nsweep):
        ctx.mesh_sor(om, xb, 1, 1.9, rb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    assert float(ra.item()) == float(rb.item())
    want, res_want = orc.Oracle(p).sor(omega, x0, nsweep, 1.9)
    assert np.abs(xa.cpu().numpy() - want).max() < 1e-13
    assert abs(float(ra.item()) - res_want) <= 1e-14
    assert ctx.status() == 0


def test_sor_rejects_odd_periodic_and_bad_relax(torch_dev):
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    ctx = Context(synth.problem(2, [13, 10], bc="periodic"))
    om = torch.ones((10, 13), dtype=torch.float64, device="cuda")
    x = torch.zeros((2, 10, 13), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        ctx.mesh_sor(om, x, 1, 1.0)
    ctx2 = Context(synth.problem(2, [12, 10], bc="outflow"))
    x2 = torch.zeros((2, 10, 12), dtype=torch.float64, device="cuda")
    for bad in (0.0, 2.0, -1.0):
        with pytest.raises(esvdw.LibError):
            ctx2.mesh_sor(om[:, :12].contiguous(), x2, 1, bad)


def test_sor_solve_beats_jacobi_at_equal_residual(orc, torch_dev):
    """96^2 four-quadrant frame (oracle state after 3 moving-mesh steps, its monitor): the Jacobi
    iteration to a last update below 1e-8 and SOR (default factor) to a Jacobi residual below 1e-8,
    both on the GPU from x^n.  SOR needs under 1/20 of the sweeps, and its mesh is closer to the
    oracle's converged mesh (SOR to a residual of 1e-13) than the Jacobi one."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    n, tol = 96, 1e-8
    p = synth.problem(2, [n, n], bc="outflow")
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    JU = o.init_state(synth.quadrants_2d(p, synth.quadrant_states(p, 2)), J)
    for _ in range(3):
        JU, J, x, _ = o.step(JU, J, x, moving=True)
    om = o.monitor(JU, J)
    ref, res_ref = o.sor(om, x, 6000, meshsolve.default_relax(n))
    assert o.jacobi(om, ref, 1)[2] < 1e-13
    ctx = Context(p)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    omg = T(om)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    xj = T(x)
    sweeps_j = 0
    while True:
        ctx.mesh_jacobi(omg, xj, 100, res)
        sweeps_j += 100
        if float(res.item()) < tol or sweeps_j > 2_000_000:
            break
    xs = T(x)
    sweeps_s = 0
    while True:
        ctx.mesh_sor(omg, xs, 10, meshsolve.default_relax(n), None)
        sweeps_s += 10
        xc = xs.clone()
        ctx.mesh_jacobi(omg, xc, 1, res)
        if float(res.item()) < tol or sweeps_s > 200_000:
            break
    err_j = np.abs(xj.cpu().numpy() - ref).max()
    err_s = np.abs(xs.cpu().numpy() - ref).max()
    print("96^2: Jacobi %d sweeps (err %.2e), SOR %d sweeps (err %.2e)" % (sweeps_j, err_j, sweeps_s, err_s))
    assert sweeps_s * 20 < sweeps_j
    assert err_s < err_j
    assert err_s < 1e-6


@pytest.mark.parametrize("n,nsweep", [([37, 29], 10), ([1024, 1024], 10), ([100, 7], 7), ([33, 17], 2), ([130, 96], 5)])
def test_multi_sweep_jacobi_equals_single_sweeps(orc, torch_dev, n, nsweep):
    """On 2D outflow grids mesh_jacobi runs up to five sweeps per launch from an LDS tile; it must
    equal nsweep single-sweep calls bit for bit (and the oracle to rounding)."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    p = synth.problem(2, n, bc="outflow")
    ctx = Context(p)
    rng = np.random.default_rng(n[0] + nsweep)
    shape = (n[1], n[0])
    omega = 1.0 + 3.0 * rng.random(shape)
    x0 = synth.smooth_mesh(p, 4, amp=0.02)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    om = T(omega)
    xa, xb = T(x0), T(x0)
    ra = torch.zeros(1, dtype=torch.float64, device="cuda")
    rb = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.mesh_jacobi(om, xa, nsweep, ra)
    for _ in range(nsweep):
        ctx.mesh_jacobi(om, xb, 1, rb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    # the residual |v - x| may be formed with or without rounding v first (FMA contraction)
    assert abs(float(ra.item()) - float(rb.item())) <= 1e-15
    if n[0] * n[1] <= 20000:
        o = orc.Oracle(p)
        xr, _, rr = o.jacobi(omega, x0, nsweep)
        assert np.abs(xa.cpu().numpy() - xr).max() < 1e-14
    assert ctx.status() == 0


@pytest.mark.parametrize("n,nf", [([37, 29], 5), ([120, 30], 7), ([55, 13], 20), ([6, 6], 2), ([300, 200], 5)])
def test_multi_pass_filter_matches_oracle(orc, torch_dev, n, nf):
    """On 2D outflow grids the monitor's low-pass filter runs up to five passes per launch; the
    filtered monitor must equal the oracle's (the one its redistribution uses) to rounding."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    p = synth.problem(2, n, bc="outflow", n_filter=nf)
    o = orc.Oracle(p)
    x = synth.smooth_mesh(p, 2, amp=0.02)
    J = o.jacobian(x)
    JU = o.init_state(synth.quadrants_2d(p, synth.quadrant_states(p, 2)), J)
    want = o.redistribute(JU, J, x)["omega"]
    ctx = Context(p)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    om = torch.empty(o.shape, dtype=torch.float64, device="cuda")
    ctx.mesh_monitor(T(JU), T(J), om)
    torch.cuda.synchronize()
    err = np.abs(om.cpu().numpy() - want).max() / np.abs(want).max()
    print("%s n_filter %d: omega rel err %.2e" % (n, nf, err))
    assert err < 1e-14
    assert ctx.status() == 0
