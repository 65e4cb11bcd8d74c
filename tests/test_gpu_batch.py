"""GPU parity of the batched persistent stage kernel (independent 2D problems of uneven size,
each with its own a, b and boundary conditions, one launch per SSP-RK3 stage).

Bars (tests/parity.py, per field and node): against the oracle, 1e-12 for one step, or 8 times
the oracle's own change at a node under 1-ulp perturbations of its input where that is larger.
Against the single-problem GPU path the device functions are the same, but the batched kernel
forms the stage mesh x + c dt xdot at each stencil point where the single path rounds it into a
buffer first, a 1-ulp difference of the mesh that the nonlinear weights amplify like any other:
1e-13, or 8 times the single path's own change under 1-ulp perturbations.  Across tile variants
the interface arithmetic is identical, so they agree to 1e-15 relative."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth

import parity

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


def pack(torch, arrays, nf, off):
    """Per-instance arrays of shape (nf, ny, nx) -> one pooled device array."""
    pool = np.zeros(nf * off[-1])
    for i, a in enumerate(arrays):
        pool[nf * off[i]:nf * off[i + 1]] = np.asarray(a, dtype=np.float64).reshape(-1)
    return torch.from_numpy(pool).cuda()


def unpack(t, nf, off, shapes):
    a = t.cpu().numpy()
    return [a[nf * off[i]:nf * off[i + 1]].reshape((nf,) + s) for i, s in enumerate(shapes)]


def _single_step(c, torch, U0, J0, X0, XD, dti):
    """One SSP-RK3 step through rk_stage of the single-problem path; returns (JU, J, x)."""
    aU, aJ = torch.empty_like(U0), torch.empty_like(J0)
    bU, bJ = torch.empty_like(U0), torch.empty_like(J0)
    oU, oJ, ox = torch.empty_like(U0), torch.empty_like(J0), X0.clone()
    c.rk_stage(0, dti, U0, J0, U0, J0, X0, XD, aU, aJ, None)
    c.rk_stage(1, dti, U0, J0, aU, aJ, X0, XD, bU, bJ, None)
    c.rk_stage(2, dti, U0, J0, bU, bJ, X0, XD, oU, oJ, ox if XD is not None else None)
    return oU.cpu().numpy(), oJ.cpu().numpy(), ox.cpu().numpy()


def _single_perturbed(c, torch, U0, J0, X0, XD, dti):
    """The single path's step from U0 perturbed by one unit in the last place (three seeds)."""
    out = []
    for sd in (1, 2, 3):
        pert = torch.from_numpy(parity.perturb(U0.cpu().numpy(), sd)).cuda()
        out.append(_single_step(c, torch, pert, J0, X0, XD, dti)[0])
    return out


def _problems():
    """Five instances: uneven sizes (down to the 6-node minimum, ragged against every tile),
    per-instance (a, b) in the batched sampling ranges, both boundary types."""
    specs = [((24, 20), "outflow", 2.1, 0.22), ((33, 17), "periodic", 3.9, 0.38), ((40, 41), "outflow", 3.0, 1 / 3),
             ((6, 9), "periodic", 2.6, 0.3), ((70, 7), "outflow", 3.4, 0.25)]
    out = []
    for k, (n, bc, a, b) in enumerate(specs):
        p = synth.problem(2, list(n), bc=bc, a=a, b=b)
        if bc == "periodic":
            prim = synth.smooth_state(p, 40 + k)
        else:
            prim = synth.quadrants_2d(p, synth.quadrant_states(p, 40 + k))
        out.append((p, prim))
    return out


def _batch(torch, probs):
    from paper_2407_05568_amd.esvdw import Batch
    B = Batch([p for p, _ in probs])
    off = B.off
    shapes = [tuple(reversed(p["n"][:2])) for p, _ in probs]
    x = torch.zeros(2 * B.total, dtype=torch.float64, device="cuda")
    J = torch.zeros(B.total, dtype=torch.float64, device="cuda")
    JU = torch.zeros(4 * B.total, dtype=torch.float64, device="cuda")
    B.init_mesh(x, J)
    B.init_state(pack(torch, [pr for _, pr in probs], 4, off), J, JU)
    return B, off, shapes, x, J, JU


def test_batch_step_matches_oracle(orc, torch_dev):
    torch = torch_dev
    probs = _problems()
    B, off, shapes, x, J, JU = _batch(torch, probs)
    dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    J0 = unpack(J, 1, off, shapes)
    JU0 = unpack(JU, 4, off, shapes)
    x0 = unpack(x, 2, off, shapes)
    B.step(JU, J, x, None, dt)
    assert B.status() == 0
    JU1, J1, dts = unpack(JU, 4, off, shapes), unpack(J, 1, off, shapes), dt.cpu().numpy()
    for i, (p, prim) in enumerate(probs):
        o = orc.Oracle(p)
        xr = o.uniform_mesh()
        assert np.abs(x0[i] - xr).max() <= 1e-15
        Jr = o.jacobian(xr)
        JUr = o.init_state(prim, Jr)
        assert relerr(JU0[i], JUr) < 1e-14
        a, Ja, _, dtr = o.step(JUr, Jr, xr, moving=False)
        assert abs(dts[i] - dtr) <= 1e-14 * dtr
        pert = [o.step(parity.perturb(JUr, sd), Jr, xr, moving=False)[0] for sd in (1, 2, 3, 4)]
        parity.check("batched step vs oracle, instance %d %s %s a=%.2f b=%.2f" % (
            i, "x".join(map(str, p["n"][:2])), p["bc"][0], p["a"], p["b"]), JU1[i], a, pert, 1e-12)
        assert relerr(J1[i], Ja[None]) < 1e-13
        assert o.flags() == 0


# launch variants: 0 the persistent stage kernel, 5 and 6 the phased launches (the direction-0
# fluxes fused into the update, with the stage-2 mesh advance)
@pytest.mark.parametrize("variant", [0, 5, 6])
def test_batch_moving_mesh_matches_single_path(torch_dev, variant):
    """Stage meshes x + c_s dt xdot and the mesh advance, against rk_stage of the single-problem
    library path on each instance."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    probs = _problems()
    B, off, shapes, x, J, JU = _batch(torch, probs)
    B.set_variant(variant)
    xs = [synth.smooth_mesh(p, 60 + i, amp=0.02) for i, (p, _) in enumerate(probs)]
    xds = [synth.smooth_velocity(p, 70 + i, amp=0.1) for i, (p, _) in enumerate(probs)]
    x = pack(torch, xs, 2, off)
    xd = pack(torch, xds, 2, off)
    # Jacobians and states on the curvilinear meshes, from the single-problem path
    Js, JUs = [], []
    for i, (p, prim) in enumerate(probs):
        c = Context(p)
        Ji = torch.empty(shapes[i], dtype=torch.float64, device="cuda")
        c.init_mesh(torch.from_numpy(xs[i]).cuda(), Ji, 0)
        JUi = torch.empty((4,) + shapes[i], dtype=torch.float64, device="cuda")
        c.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), Ji, JUi)
        Js.append(Ji.cpu().numpy())
        JUs.append(JUi.cpu().numpy())
    J = pack(torch, Js, 1, off)
    JU = pack(torch, JUs, 4, off)
    dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    B.step(JU, J, x, xd, dt)
    assert B.status() == 0
    gJU, gJ, gx = unpack(JU, 4, off, shapes), unpack(J, 1, off, shapes), unpack(x, 2, off, shapes)
    dts = dt.cpu().numpy()
    for i, (p, _) in enumerate(probs):
        c = Context(p)
        U0 = torch.from_numpy(JUs[i]).cuda()
        J0 = torch.from_numpy(Js[i]).cuda()
        X0 = torch.from_numpy(xs[i]).cuda()
        XD = torch.from_numpy(xds[i]).cuda()
        dti = torch.zeros(1, dtype=torch.float64, device="cuda")
        c.cfl_dt(U0, J0, X0, dti)
        assert abs(dti.item() - dts[i]) <= 1e-14 * dts[i]
        oU, oJ, ox = _single_step(c, torch, U0, J0, X0, XD, dti)
        assert c.status() == 0
        parity.check("batched moving stages vs single path, instance %d" % i, gJU[i], oU,
                     _single_perturbed(c, torch, U0, J0, X0, XD, dti), 1e-13)
        assert relerr(gJ[i], oJ[None]) < 1e-13
        assert np.abs(gx[i] - ox).max() <= 1e-15


def test_batch_variants_agree(torch_dev):
    torch = torch_dev
    probs = _problems()
    ref = None
    from paper_2407_05568_amd.esvdw import Batch
    nvar = Batch([probs[0][0]]).variants()
    for v in range(nvar):
        B, off, shapes, x, J, JU = _batch(torch, probs)
        B.set_variant(v)
        dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
        for _ in range(2):
            B.step(JU, J, x, None, dt)
        assert B.status() == 0
        out = JU.cpu().numpy()
        if ref is None:
            ref = out
        else:
            assert np.abs(out - ref).max() <= 1e-15 * np.abs(ref).max(), v


def test_batch_full_size_sampled(orc, torch_dev):
    """The 256-instance batch (n ~ U{64..384}, a ~ U[2, 4], b ~ U[0.2, 0.4]), one step captured in
    a HIP graph and replayed; three instances (smallest, largest, one more) against the
    single-problem GPU path and against the oracle, every instance finite."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Batch, Context
    inst = synth.batch_instances(0)
    probs = [(p, synth.quadrants_2d(p, st)) for p, st in inst]
    B, off, shapes, x, J, JU = _batch(torch, probs)
    dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    JU0 = JU.clone()
    J0 = J.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            B.step(JU, J, x, None, dt, s)
    torch.cuda.synchronize()
    # the capture did not run the step: reset the state, replay once
    JU.copy_(JU0)
    J.copy_(J0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert B.status() == 0
    assert bool(torch.isfinite(JU).all())
    sizes = [p["n"][0] for p, _ in probs]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17})
    gJU = unpack(JU, 4, off, shapes)
    for i in pick:
        p, _ = probs[i]
        c = Context(p)
        U = JU0[4 * off[i]:4 * off[i + 1]].view((4,) + shapes[i]).clone()
        Ji = J0[off[i]:off[i + 1]].view(shapes[i]).clone()
        xi = x[2 * off[i]:2 * off[i + 1]].view((2,) + shapes[i]).clone()
        dti = torch.zeros(1, dtype=torch.float64, device="cuda")
        c.cfl_dt(U, Ji, xi, dti)
        assert abs(dti.item() - dt[i].item()) <= 1e-14 * dti.item()
        oU = _single_step(c, torch, U, Ji, xi, None, dti)[0]
        assert c.status() == 0
        parity.check("256-instance batch, instance %d (n = %d) vs single path" % (i, p["n"][0]), gJU[i], oU,
                     _single_perturbed(c, torch, U, Ji, xi, None, dti), 1e-13)
        # and against the oracle's step of the same instance
        o = orc.Oracle(p)
        Un, Jn, xn = U.cpu().numpy(), Ji.cpu().numpy(), xi.cpu().numpy()
        ref, _, _, dtr = o.step(Un, Jn, xn, moving=False)
        assert abs(dti.item() - dtr) <= 1e-14 * dtr
        pert = [o.step(parity.perturb(Un, sd), Jn, xn, moving=False)[0] for sd in (1, 2, 3)]
        parity.check("256-instance batch, instance %d (n = %d) vs oracle" % (i, p["n"][0]), gJU[i], ref, pert, 1e-12)
        assert o.flags() == 0


def _moving_setup(torch, probs):
    """Curvilinear meshes (smooth, seeded) with J and JU from the single-problem path."""
    from paper_2407_05568_amd.esvdw import Context
    xs, Js, JUs = [], [], []
    for i, (p, prim) in enumerate(probs):
        c = Context(p)
        x = synth.smooth_mesh(p, 80 + i, amp=0.02)
        shape = tuple(reversed(p["n"][:2]))
        Ji = torch.empty(shape, dtype=torch.float64, device="cuda")
        c.init_mesh(torch.from_numpy(x).cuda(), Ji, 0)
        JUi = torch.empty((4,) + shape, dtype=torch.float64, device="cuda")
        c.init_state(torch.from_numpy(np.ascontiguousarray(prim)).cuda(), Ji, JUi)
        xs.append(x)
        Js.append(Ji.cpu().numpy())
        JUs.append(JUi.cpu().numpy())
    return xs, Js, JUs


def test_batch_redistribute_matches_single_path_and_oracle(orc, torch_dev):
    """Monitor with per-instance maxima, filter, mu Jacobi sweeps, limiter, CFL and xdot of every
    instance: against redistribute_mesh of the single-problem path (same device functions; maxima
    and minima are exact in any order) and against the oracle (the next mesh x + dt xdot to
    1e-13 in domain units, dt to 1e-14 relative)."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    probs = _problems()
    B, off, shapes, _, _, _ = _batch(torch, probs)
    xs, Js, JUs = _moving_setup(torch, probs)
    x, J, JU = pack(torch, xs, 2, off), pack(torch, Js, 1, off), pack(torch, JUs, 4, off)
    xd = torch.zeros_like(x)
    dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    B.redistribute(JU, J, x, xd, dt)
    assert B.status() == 0
    gxd, dts = unpack(xd, 2, off, shapes), dt.cpu().numpy()
    assert np.array_equal(unpack(x, 2, off, shapes)[0], xs[0])  # x is not modified
    for i, (p, _) in enumerate(probs):
        c = Context(p)
        sxd = torch.zeros((2,) + shapes[i], dtype=torch.float64, device="cuda")
        sdt = torch.zeros(1, dtype=torch.float64, device="cuda")
        c.redistribute_mesh(torch.from_numpy(JUs[i]).cuda(), torch.from_numpy(Js[i]).cuda(),
                            torch.from_numpy(xs[i]).cuda(), None, sxd, sdt)
        s = sxd.cpu().numpy()
        assert abs(sdt.item() - dts[i]) <= 1e-15 * dts[i]
        assert np.abs(gxd[i] - s).max() <= 1e-13 * max(np.abs(s).max(), 1e-300), i
        r = orc.Oracle(p).redistribute(JUs[i], Js[i], xs[i])
        assert abs(dts[i] - r["dt"]) <= 1e-14 * r["dt"]
        nx_g = xs[i] + dts[i] * gxd[i]
        nx_o = xs[i] + r["dt"] * r["xdot"]
        print("instance %d: next-mesh difference to the oracle %.2e" % (i, np.abs(nx_g - nx_o).max()))
        assert np.abs(nx_g - nx_o).max() <= 1e-13


@pytest.mark.parametrize("variant", [0, 6])
def test_batch_moving_step_matches_single_path(torch_dev, variant):
    """A full moving-mesh step of every instance (esvdw_batch_redistribute + esvdw_batch_step)
    against esvdw_step(moving) of the single-problem path, at the conditioning bar."""
    torch = torch_dev
    from paper_2407_05568_amd.esvdw import Context
    probs = _problems()
    B, off, shapes, _, _, _ = _batch(torch, probs)
    B.set_variant(variant)
    xs, Js, JUs = _moving_setup(torch, probs)
    x, J, JU = pack(torch, xs, 2, off), pack(torch, Js, 1, off), pack(torch, JUs, 4, off)
    xd = torch.zeros_like(x)
    dt = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    B.redistribute(JU, J, x, xd, dt)
    B.step(JU, J, x, xd, dt)
    assert B.status() == 0
    gJU, gx = unpack(JU, 4, off, shapes), unpack(x, 2, off, shapes)
    for i, (p, _) in enumerate(probs):
        c = Context(p)

        def single(U0):
            U, Jc, X = U0.clone(), torch.from_numpy(Js[i]).cuda(), torch.from_numpy(xs[i]).cuda()
            c.step(U, Jc, X, 1, torch.zeros(1, dtype=torch.float64, device="cuda"))
            return U.cpu().numpy(), X.cpu().numpy()
        U0 = torch.from_numpy(JUs[i]).cuda()
        ref, refx = single(U0)
        assert c.status() == 0
        pert = [single(torch.from_numpy(parity.perturb(JUs[i], sd)).cuda())[0] for sd in (1, 2, 3)]
        parity.check("batched moving step vs single path, instance %d" % i, gJU[i], ref, pert, 1e-13)
        assert np.abs(gx[i] - refx).max() <= 1e-13
