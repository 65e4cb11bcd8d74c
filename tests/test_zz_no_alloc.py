"""GPU check of cfl_dt_noalloc, the CFL step for callers that cannot allocate: against cfl_dt of a
context (same kernels, same reduction order, so bit-identical dt), on two calls in a row, the
second on a smaller grid than the first (the shared static scratch keeps the first call's
partials), and the rejection of grids beyond its scratch."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(torch, p, seed):
    from paper_2407_05568_amd.esvdw import Context
    ctx = Context(p)
    d = p["dim"]
    shape = tuple(reversed(p["n"][:d]))
    x = torch.from_numpy(synth.smooth_mesh(p, seed, amp=0.02)).cuda()
    J = torch.empty(shape, dtype=torch.float64, device="cuda")
    ctx.init_mesh(x, J, 0)
    if d == 2:
        prim = synth.quadrants_2d(p, synth.quadrant_states(p, seed))
    else:
        prim = synth.smooth_state(p, seed)
    JU = torch.empty((d + 2,) + shape, dtype=torch.float64, device="cuda")
    ctx.init_state(torch.from_numpy(prim).cuda(), J, JU)
    return ctx, JU, J, x


def test_noalloc_cfl_matches_context_path():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_05568_amd import esvdw
    cases = [synth.problem(2, [301, 203], bc="outflow"), synth.problem(2, [37, 29], bc="periodic"),
             synth.problem(1, [400], bc="outflow")]
    for i, p in enumerate(cases):
        print("cfl_dt_noalloc case %d: dim %d n %s" % (i, p["dim"], p["n"][:p["dim"]]), flush=True)
        ctx, JU, J, x = _inputs(torch, p, 5 + i)
        ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        got = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        ctx.cfl_dt(JU, J, x, ref)
        esvdw.cfl_dt_noalloc(p, JU, J, x, got)
        torch.cuda.synchronize()
        assert float(ref.cpu()[0]) > 0.0
        assert float(got.cpu()[0]) == float(ref.cpu()[0]), (i, float(got.cpu()[0]), float(ref.cpu()[0]))
        assert ctx.status() == 0
    # a fixed time step is passed through
    p = dict(cases[1], dt_fixed=1.25e-3)
    ctx, JU, J, x = _inputs(torch, p, 9)
    got = torch.zeros(1, dtype=torch.float64, device="cuda")
    esvdw.cfl_dt_noalloc(p, JU, J, x, got)
    torch.cuda.synchronize()
    assert float(got.cpu()[0]) == 1.25e-3


def test_noalloc_rejects_grids_beyond_its_scratch():
    """65536 tiles of 64 x 16 nodes at most: a 16384 x 16400 grid needs 262400 and is refused
    before any launch (the arrays are never touched, so small ones suffice)."""
    import torch
    from paper_2407_05568_amd import esvdw
    p = synth.problem(2, [16384, 16400], bc="outflow")
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(esvdw.LibError, match="static scratch"):
        esvdw.cfl_dt_noalloc(p, t, t, t, t)
    with pytest.raises(esvdw.LibError, match="invalid"):
        esvdw.cfl_dt_noalloc(synth.problem(3, [8, 8, 8], bc="periodic"), t, t, t, t)
