"""The scheme on Table 5.1's shock tubes (Example 5.2) measured against the stored 10 000-cell
finite-volume reference solutions: the L1 density error of the moving mesh with N = 100 (MM,
monitor with rho and G; MM1, rho only) and of the uniform mesh with N = 100 and 300 (UM), all
run by the oracle to the exact final time.

The paper reports (from plots) that MM with 100 cells is better than UM with 300 near the waves.
What is asserted: the moving mesh halves the uniform mesh's error at the same N, and stays
within 15% of the uniform mesh with three times the cells; every run stays admissible."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth

from test_fv_reference import load_reference

T_END = {"rp1": 0.15, "rp2": 0.45, "rp3": 0.2}
ALPHA = {"rp1": [1200.0, 3000.0, 5000.0], "rp2": [1200.0, 3000.0, 5000.0], "rp3": [1200.0, 1200.0, 1200.0]}


def run_to(orc, name, n, mode):
    alpha = ALPHA[name] if mode == "MM" else [ALPHA[name][0], 0.0, 0.0]
    kappa = 2 if mode == "MM" else 1
    p = synth.problem(1, [n], bc="outflow", alpha=alpha, kappa=kappa)
    o = orc.Oracle(p)
    x = o.uniform_mesh()
    J = o.jacobian(x)
    rp = synth.TABLE_5_1[name.upper()]
    JU = o.init_state(synth.riemann_1d(p, rp[0], rp[1]), J)
    t, t_end, moving = 0.0, T_END[name], mode != "UM"
    while t < t_end - 1e-14:
        JU1, J1, x1, dt = o.step(JU, J, x, moving)
        if t + dt > t_end:  # repeat the last step with the remaining time
            q = dict(p)
            q["dt_fixed"] = t_end - t
            JU1, J1, x1, dt = orc.Oracle(q).step(JU, J, x, moving)
        JU, J, x = JU1, J1, x1
        t += dt
    assert o.flags() == 0
    return x[0], JU[0] / J


@pytest.mark.parametrize("name", ["rp1", "rp2", "rp3"])
def test_moving_mesh_error_against_reference(orc, name):
    xr, rr, _, _ = load_reference(name)
    err = {}
    for n, mode in ((100, "MM"), (100, "MM1"), (100, "UM"), (300, "UM")):
        x, rho = run_to(orc, name, n, mode)
        err[(mode, n)] = float(np.mean(np.abs(np.interp(xr, x, rho) - rr)))
    print(name, {"%s-%d" % k: "%.2e" % v for k, v in err.items()})
    assert err[("MM", 100)] < 0.6 * err[("UM", 100)]
    assert err[("MM1", 100)] < 0.6 * err[("UM", 100)]
    assert err[("MM", 100)] < 1.15 * err[("UM", 300)]
    assert err[("UM", 300)] < 8e-3
