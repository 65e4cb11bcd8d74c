"""Pins of the dissipation's sign matrix Y at one interface (Section 3.3, eq. HOstable): Y_m = 1
exactly where the plain jump [W_m] and the reconstructed jump [W_m]^WENO have the same strict
sign, else 0; a plain jump at the rounding level of the vector W (2^-40 of the magnitude of all
the terms that form its components at the two nodes) counts as zero.

The oracle reports, per interface, Y, [W]^WENO, the plain jump before its zero test and the
test's scale (orc_interface_flux).  Independent checks: with dissipation off the same call
gives the entropy-conservative flux F_EC, so F_ES - F_EC is the dissipation alone; its entropy
production (F_ES - F_EC) . [V], with [V] from the separately pinned entropy variables, must be
<= 0 for any jump (the scheme's entropy stability) and equals 0 when Y = 0."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth


def _cons(o, p, rho, v, T):
    pr = rho * p["R"] * T / (1.0 - p["b"] * rho) - p["a"] * rho * rho
    return o.prim_to_cons([rho] + list(v) + [pr])


def _case(orc, states, dim=2, metric=(0.9, 0.2), mt=0.05):
    """Interface along xi_1 with the same metrics at the six nodes; states: six (rho, v, T)."""
    p = synth.problem(dim, [8] * dim, bc="periodic")
    o = orc.Oracle(p)
    oe = orc.Oracle(dict(p, dissipation=0))
    st = np.array([_cons(o, p, r, v, T) for r, v, T in states])
    mx = np.tile(np.array(metric[:dim]), (6, 1))
    mtv = np.full(6, mt)
    es = o.interface_flux(st, mx, mtv)
    ec = oe.interface_flux(st, mx, mtv)
    dV = o.entropy_vars(st[3]) - o.entropy_vars(st[2])
    return o, st, mx, mtv, es, ec, dV


BASE = [(0.8, (0.10, -0.05), 1.20), (0.85, (0.12, -0.04), 1.22), (0.9, (0.15, -0.02), 1.25),
        (0.9, (0.15, -0.02), 1.25), (1.1, (0.05, 0.03), 1.30), (1.2, (0.02, 0.05), 1.33)]


def test_zero_plain_jump_gives_no_dissipation(orc):
    """Nodes i and i+1 equal (an exactly zero [W]) while the stencil around them varies, so the
    reconstructed jump is not zero: Y = 0 in every component and F_ES = F_EC bit for bit."""
    o, st, mx, mt, es, ec, dV = _case(orc, BASE)
    assert np.all(es["j0"] == 0.0)
    assert np.abs(es["jw"]).max() > 1e-9  # the reconstruction does see a jump
    assert np.all(es["Y"] == 0.0)
    assert np.array_equal(es["F"], ec["F"])


def test_jump_below_the_rounding_scale_is_zero(orc):
    """Node i+1 one unit in the last place away from node i (the density): every |[W_m]| is at or
    below 2^-40 of its scale, so Y = 0 and F_ES = F_EC exactly."""
    st = list(BASE)
    r, v, T = st[3]
    st[3] = (np.nextafter(r, 2.0), v, T)
    o, s, mx, mt, es, ec, dV = _case(orc, st)
    assert np.any(es["j0"] != 0.0)
    assert np.all(np.abs(es["j0"]) <= np.ldexp(es["scale"], -40))
    assert np.all(es["Y"] == 0.0)
    assert np.array_equal(es["F"], ec["F"])


@pytest.mark.parametrize("eta", [1e-7, 1e-6, 1e-5])
def test_jump_above_the_scale_keeps_the_sign_rule(orc, eta):
    """A plain jump well above the zero test's scale (relative changes of density, velocity and
    temperature of size eta at node i+1, of either sign): Y_m = 1 exactly where [W_m] and
    [W_m]^WENO have the same strict sign; where it is on, dissipation acts (F_ES != F_EC) and
    produces entropy: (F_ES - F_EC) . [V] < 0."""
    for sgn in (1.0, -1.0):
        st = list(BASE)
        r, v, T = st[3]
        st[3] = (r * (1 + sgn * eta), (v[0] + sgn * eta, v[1] - sgn * eta), T * (1 - sgn * 0.5 * eta))
        o, s, mx, mt, es, ec, dV = _case(orc, st)
        j0, jw = es["j0"], es["jw"]
        assert np.all(np.abs(j0) > np.ldexp(es["scale"], -40))
        rule = ((j0 > 0) & (jw > 0)) | ((j0 < 0) & (jw < 0))
        assert np.array_equal(es["Y"] == 1.0, rule)
        assert np.any(rule)
        assert not np.array_equal(es["F"], ec["F"])
        prod = np.dot(es["F"] - ec["F"], dV)
        assert prod < 0.0, prod


def test_step_jump_dissipates_in_every_component(orc):
    """A jump between two constant states (i-2..i left, i+1..i+3 right): the reconstructions from
    each side stay close to that side's value, so [W]^WENO has the sign of [W] in every
    component and Y = 1 throughout; the production is strictly negative.  Reversing the jump
    keeps Y = 1."""
    L, R = (0.7, (0.2, 0.0), 1.20), (1.15, (-0.1, 0.1), 1.32)
    for a, b in ((L, R), (R, L)):
        o, st, mx, mt, es, ec, dV = _case(orc, [a, a, a, b, b, b])
        assert np.all(es["Y"] == 1.0), es
        assert np.dot(es["F"] - ec["F"], dV) < 0.0


def test_disagreeing_signs_switch_the_component_off(orc):
    """Random stencils with a small plain jump at the interface (relative 1e-6, above the zero
    test): wherever it and the reconstructed jump disagree in sign, Y_m = 0 (and such cases
    occur), while agreeing components are on; the production stays < 0 where anything is on."""
    rng = np.random.default_rng(21)
    seen_off = seen_on = 0
    for trial in range(200):
        st = [(rng.uniform(0.7, 1.2), tuple(rng.uniform(-0.2, 0.2, size=2)), rng.uniform(1.15, 1.35))
              for _ in range(6)]
        r, v, T = st[2]
        sg = rng.choice([-1.0, 1.0])
        st[3] = (r * (1 + sg * 1e-6), (v[0] - sg * 1e-6, v[1] + sg * 1e-6), T * (1 + sg * 1e-6))
        o, s, mx, mt, es, ec, dV = _case(orc, st)
        off = es["j0"] * es["jw"] < 0
        on = es["j0"] * es["jw"] > 0
        assert np.all(es["Y"][off] == 0.0) and np.all(es["Y"][on] == 1.0)
        seen_off += int(off.sum())
        seen_on += int(on.sum())
        if on.any():
            assert np.dot(es["F"] - ec["F"], dV) < 0.0
    assert seen_off >= 5 and seen_on >= 50, (seen_off, seen_on)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_production_nonpositive_across_the_threshold(orc, dim):
    """Sweeping the plain jump through the zero test's scale (relative changes 1e-16 .. 1e-9,
    either sign) on random stencils: the interface never produces entropy,
    (F_ES - F_EC) . [V] <= 0 to the rounding of the flux difference, and at every point Y
    follows the rule above with the scale test applied."""
    rng = np.random.default_rng(7 + dim)
    metric = (0.9, 0.2, -0.1)
    for trial in range(20):
        base = [(rng.uniform(0.7, 1.2), tuple(rng.uniform(-0.2, 0.2, size=dim)), rng.uniform(1.15, 1.35))
                for _ in range(6)]
        for eta in (1e-16, 1e-14, 1e-13, 1e-12, 1e-11, 1e-9):
            sgn = rng.choice([-1.0, 1.0])
            st = list(base)
            r, v, T = st[2]
            st[3] = (r * (1 + sgn * eta), v, T * (1 + sgn * eta))
            o, s, mx, mt, es, ec, dV = _case(orc, st, dim=dim, metric=metric)
            j0, jw, sc = es["j0"], es["jw"], es["scale"]
            zero = np.abs(j0) <= np.ldexp(sc, -40)
            rule = ~zero & (((j0 > 0) & (jw > 0)) | ((j0 < 0) & (jw < 0)))
            assert np.array_equal(es["Y"] == 1.0, rule)
            dF = es["F"] - ec["F"]
            prod = np.dot(dF, dV)
            assert prod <= 1e-12 * np.abs(dF).dot(np.abs(dV)) + 1e-300, (trial, eta, prod)
