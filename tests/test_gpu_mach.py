"""Example 5.4's oblique shock reflecting off a slip wall (Table 5.3's P1 and D1) on the moving
mesh, run to the final time at 64 x 32: no status flags, the final time reached exactly, the
density inside the range the two states and the reflection allow, and mass changed only
through the open faces (the wall keeps none from leaving: the change stays far below the mass
the open faces could carry)."""
import pytest

from paper_2407_05568_amd import mach2d, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2407_05568_amd import esvdw
    esvdw.lib()
    return torch


@pytest.mark.parametrize("case", ["P1", "D1"])
def test_mach_reflection_runs(torch_dev, case):
    info, rho, x, J = mach2d.run(torch_dev, case, 64, 32, moving=True)
    c = synth.TABLE_5_3[case]
    lo, hi = min(c["left"][0], c["right"][0]), max(c["left"][0], c["right"][0])
    print("%s 64x32: %d steps, t %.5f of %.5f, rho [%.4f, %.4f], min J %.3f" % (
        case, info["steps"], info["t"], info["t_end"], rho.min(), rho.max(), info["min_J"]))
    assert info["flags"] == 0
    assert abs(info["t"] - info["t_end"]) <= 1e-12 * info["t_end"]
    assert 0.5 * lo < rho.min() and rho.max() < 2.5 * hi
    assert info["min_J"] > 0.0
    # the mesh stays inside the box and on it: the wall row's normal coordinates are mirrored, not moved out
    assert x[0].min() > 0.0 and x[0].max() < 1.0 and x[1].min() > 0.0 and x[1].max() < 0.5
