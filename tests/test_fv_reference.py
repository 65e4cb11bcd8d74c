"""Pins of the second-order finite-volume reference solver (oracle/fv_reference.py): Sod's
problem for an ideal gas (a = b = 0) against the exact Riemann solution, the van der Waals sound
speed against the isentropic derivative of p, a spherical fluid at rest kept at rest, and
conservation; then the stored 10 000-cell reference solutions of Table 5.1's shock tubes used to
measure the scheme (oracle) on them."""
import math
import os

import numpy as np
import pytest

from oracle import fv_reference as fv
from paper_2407_05568_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_sod(gamma, left, right, x, t, x0=0.5):
    """Exact solution of the ideal-gas Riemann problem (the two-shock/rarefaction pressure
    function solved by bisection, then sampled at (x - x0)/t)."""
    (rl, ul, pl), (rr, ur, pr) = left, right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def fK(p, rK, pK, cK):
        if p > pK:
            A, B = 2.0 / ((gamma + 1.0) * rK), (gamma - 1.0) / (gamma + 1.0) * pK
            return (p - pK) * math.sqrt(A / (p + B))
        return 2.0 * cK / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)

    lo, hi = 1e-12, 10.0 * max(pl, pr)
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if fK(m, rl, pl, cl) + fK(m, rr, pr, cr) + ur - ul > 0.0:
            hi = m
        else:
            lo = m
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (fK(ps, rr, pr, cr) - fK(ps, rl, pl, cl))
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((3, len(x)))
    for i, xi in enumerate(x):
        s = (xi - x0) / t
        if s < us:  # left of the contact
            if ps > pl:
                rs = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                S = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
                out[:, i] = (rl, ul, pl) if s < S else (rs, us, ps)
            else:
                rs = rl * (ps / pl) ** (1.0 / gamma)
                cs = cl * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                if s < ul - cl:
                    out[:, i] = (rl, ul, pl)
                elif s > us - cs:
                    out[:, i] = (rs, us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cl + (gamma - 1.0) / 2.0 * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (gamma - 1.0))
                    out[:, i] = (r, 2.0 / (gamma + 1.0) * (cl + (gamma - 1.0) / 2.0 * ul + s), pl * (c / cl) ** (
                        2.0 * gamma / (gamma - 1.0)))
        else:  # right of the contact
            if ps > pr:
                rs = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                S = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
                out[:, i] = (rr, ur, pr) if s > S else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / gamma)
                cs = cr * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                if s > ur + cr:
                    out[:, i] = (rr, ur, pr)
                elif s < us + cs:
                    out[:, i] = (rs, us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cr - (gamma - 1.0) / 2.0 * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (gamma - 1.0))
                    out[:, i] = (r, 2.0 / (gamma + 1.0) * (-cr + (gamma - 1.0) / 2.0 * ur + s), pr * (c / cr) ** (
                        2.0 * gamma / (gamma - 1.0)))
    return out


def test_exact_sod_reference_values():
    """The exact solver on Sod's problem reproduces the textbook star state (p* = 0.30313,
    u* = 0.92745, rho*L = 0.42632, rho*R = 0.26557 for gamma = 1.4)."""
    x = np.array([0.55, 0.7])
    out = exact_sod(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), x, 0.2)
    assert out[2, 0] == pytest.approx(0.30313, abs=1e-5) and out[1, 0] == pytest.approx(0.92745, abs=1e-5)
    assert out[0, 0] == pytest.approx(0.42632, abs=1e-5) and out[0, 1] == pytest.approx(0.26557, abs=1e-5)


def test_fv_sod_ideal_gas_converges_to_exact():
    eos = fv.VdW(1.0, 1.0 / 0.4, 0.0, 0.0)  # gamma = 1 + R/c_v = 1.4
    errs = {}
    for n in (400, 1600):
        x, rho, v, p = fv.riemann(eos, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.2, n=n)
        ex = exact_sod(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), x, 0.2)
        errs[n] = float(np.mean(np.abs(rho - ex[0])))
        assert np.mean(np.abs(p - ex[2])) < 3 * errs[n] + 1e-3
    assert errs[1600] < 2.5e-3
    assert errs[400] / errs[1600] > 2.5


def test_vdw_sound_speed_is_isentropic_derivative():
    """c^2 = dp/drho at constant entropy s = c_v ln T + R ln(1/rho - b), by central differences."""
    u = synth.units("reduced")
    eos = fv.VdW(u["R"], u["cv"], u["a"], u["b"])
    for rho0, T0 in ((0.5, 1.2), (1.3, 1.05), (0.8, 0.99)):
        def p_isentrope(rho):
            T = T0 * ((1.0 / rho - eos.b) / (1.0 / rho0 - eos.b)) ** (-eos.R / eos.cv)
            return rho * eos.R * T / (1.0 - eos.b * rho) - eos.a * rho * rho
        h = 1e-5 * rho0
        fd = (p_isentrope(rho0 + h) - p_isentrope(rho0 - h)) / (2.0 * h)
        assert eos.c2(rho0, T0) == pytest.approx(fd, rel=1e-7)


def test_fv_spherical_rest_state_and_conservation():
    u = synth.units("reduced")
    eos = fv.VdW(u["R"], u["cv"], u["a"], u["b"])
    s = fv.FV1D(eos, 200, 0.0, 2.0, "spherical")
    U = s.init(0.8, 0.0, 1.1)
    U1, _ = s.run(U, 0.05)
    assert np.abs(U1[1]).max() < 1e-12
    assert np.abs(U1[0] - U[0]).max() < 1e-12
    # a sphere of dense gas: mass conserved while the waves stay inside
    U = s.init(np.where(s.x < 0.5, 1.818, 0.275), 0.0, np.where(s.x < 0.5, 3.0, 0.575))
    m0 = s.mass(U)
    U1, _ = s.run(U, 0.1)
    assert abs(s.mass(U1) - m0) < 1e-13 * m0
    planar = fv.FV1D(eos, 300, 0.0, 1.0)
    U = planar.init(np.where(planar.x < 0.5, 1.818, 0.275), 0.0, np.where(planar.x < 0.5, 3.0, 0.575))
    m0 = planar.mass(U)
    U1, _ = planar.run(U, 0.1)
    assert abs(planar.mass(U1) - m0) < 1e-13 * m0


def load_reference(name):
    a = np.loadtxt(os.path.join(GOLDEN, "fv_%s.txt" % name))
    return a[:, 0], a[:, 1], a[:, 2], a[:, 3]


@pytest.mark.parametrize("name", ["rp1", "rp2", "rp3"])
def test_stored_references_are_shock_tubes(name):
    """The stored 10 000-cell solutions (every 10th cell) keep the data's end states and the
    density range of Table 5.1's shock tubes."""
    x, rho, v, p = load_reference(name)
    (rl, _, pl), (rr, _, pr) = synth.TABLE_5_1[name.upper()]
    assert len(x) == 1000
    assert rho[0] == pytest.approx(rl, abs=1e-9) and rho[-1] == pytest.approx(rr, abs=1e-9)
    assert p[0] == pytest.approx(pl, abs=1e-9) and p[-1] == pytest.approx(pr, abs=1e-9)
    assert min(rl, rr) - 1e-6 < rho.min() and rho.max() < max(rl, rr) + 1e-6
