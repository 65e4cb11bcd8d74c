"""Oracle pins: two-point entropy-conservative flux (Section 3.1), eigen-structure
(Section 3.3) and the coefficients alpha_{w,m} (eq. ECFlux_curv_2p conditions)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2407_05568_amd import synth


def _pairs(o, p, rng, count, dim, margin=0.02):
    """Random admissible state pairs whose mean satisfies Theorem 3.1's constraint with margin."""
    rc, Tc, pc = synth._critical(p)
    a, b, R = p["a"], p["b"], p["R"]
    out = []
    while len(out) < count:
        rho = rng.uniform(0.3, 1.8, size=2) * rc
        T = rng.uniform(0.95, 1.6, size=2) * Tc
        if not all(o.admissible(rho[i], T[i]) for i in range(2)):
            continue
        rm, Tm = rho.mean(), T.mean()
        if b > 0 and R * Tm - 2 * a * rm * (1 - b * rm) ** 2 < margin * R * Tm:
            continue
        v = rng.uniform(-0.8, 0.8, size=(2, dim)) * math.sqrt(pc / rc)
        U = [o.prim_to_cons(np.array([rho[i], *v[i], synth._p_of(p, rho[i], T[i])])) for i in range(2)]
        out.append(U)
    return out


CASES = [("reduced", None), ("paper", None), ("reduced", (2.2, 0.37)), ("ideal", None)]


@pytest.mark.parametrize("unit,ab", CASES)
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_jump_identity(orc, unit, ab, dim):
    """eq. ECCondition_comp: [V].U~ = [phi], [V].F~_j = [psi_j] on random admissible pairs.

    Normalised by the sum of the magnitudes of the terms, 99.9% of the pairs satisfy it to
    1e-13 and all to 5e-13; the residual is the rounding of [V] itself (large c_v ln T terms
    cancel in [V_1]): normalised by the magnitudes (|V_l| + |V_r|).|U~| + |phi_l| + |phi_r| it stays below 5e-14."""
    kw = {} if ab is None else dict(a=ab[0], b=ab[1])
    p = synth.problem(dim, [8] * dim, unit=unit, **kw)
    o = orc.Oracle(p)
    rng = np.random.default_rng(10 + dim)
    rel_terms, rel_mag = [], []
    for Ul, Ur in _pairs(o, p, rng, 1000, dim):
        Ut, Ft = o.ec_pair(Ul, Ur)
        Vl, Vr = o.entropy_vars(Ul), o.entropy_vars(Ur)
        dV = Vr - Vl
        phl, psl = o.potentials(Ul)
        phr, psr = o.potentials(Ur)
        rows = [(Ut, phr, phl)] + [(Ft[j], psr[j], psl[j]) for j in range(dim)]
        for q, qr, ql in rows:
            res = abs(dV @ q - (qr - ql))
            rel_terms.append(res / (np.abs(dV * q).sum() + abs(qr - ql)))
            rel_mag.append(res / ((np.abs(Vl) + np.abs(Vr)) @ np.abs(q) + abs(qr) + abs(ql)))
    assert o.flags() == 0
    rel_terms = np.array(rel_terms)
    assert np.percentile(rel_terms, 99.9) < 1e-13, np.percentile(rel_terms, 99.9)
    assert rel_terms.max() < 5e-13, rel_terms.max()
    assert max(rel_mag) < 5e-14, max(rel_mag)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_symmetry_and_consistency(orc, dim):
    """U~(l, r) = U~(r, l), F~(l, r) = F~(r, l); U~(U, U) = U and F~_j(U, U) = F_j(U)
    (Remark after the explicit flux; F_j from eq. ConserLaw3)."""
    p = synth.problem(dim, [8] * dim, unit="reduced")
    o = orc.Oracle(p)
    rng = np.random.default_rng(20)
    for Ul, Ur in _pairs(o, p, rng, 100, dim):
        a1, b1 = o.ec_pair(Ul, Ur)
        a2, b2 = o.ec_pair(Ur, Ul)
        assert np.allclose(a1, a2, rtol=1e-14, atol=1e-14 * np.abs(a1).max())
        assert np.allclose(b1, b2, rtol=1e-14, atol=1e-14 * np.abs(b1).max())
        Ut, Ft = o.ec_pair(Ul, Ul)
        assert np.allclose(Ut, Ul, rtol=1e-13, atol=1e-13 * np.abs(Ul).max())
        for j in range(dim):
            F = o.phys_flux(Ul, j)
            assert np.allclose(Ft[j], F, rtol=1e-13, atol=1e-13 * np.abs(F).max())


def test_printed_paper_flux(orc):
    """In the paper's units the oracle's closed form reproduces the printed U~_1, U~_m, U~_5,
    F~_{1,1}, F~_{1,2}, F~_{1,m}, F~_{1,5} (Section 3.1), transcribed literally below."""
    p = synth.problem(3, [8] * 3, unit="paper")
    o = orc.Oracle(p)
    delta = synth.DELTA
    rng = np.random.default_rng(30)

    def L(a, b):
        return (b - a) / (math.log(b) - math.log(a))

    def M(f, zl, zr):
        return 0.5 * (f(zl) + f(zr))

    for Ul, Ur in _pairs(o, p, rng, 100, 3):
        zl = o.cons_to_prim(Ul)
        zr = o.cons_to_prim(Ur)
        zl = [zl[0], zl[1], zl[2], zl[3], zl[5]]  # z = (rho, v, T)
        zr = [zr[0], zr[1], zr[2], zr[3], zr[5]]
        if abs(zl[0] - zr[0]) < 1e-3 or abs(zl[4] - zr[4]) < 1e-3:
            continue  # the literal log mean needs distinct arguments
        z1m = M(lambda z: z[0], zl, zr)
        z5m = M(lambda z: z[4], zl, zr)
        Dn = 1 / L(zl[0], zr[0]) + 1 / L(3 - zl[0], 3 - zr[0]) + 3 / ((3 - zl[0]) * (3 - zr[0])) - 9 / (4 * z5m)
        g = M(lambda z: -9 / 8 * z[0] / z[4] + 3 / (3 - z[0]), zl, zr)
        c3 = -9 / 8 / z5m + 3 / ((3 - zl[0]) * (3 - zr[0]))
        U1 = (z1m * c3 + g) / Dn
        Um = [M(lambda z, m=m: z[m], zl, zr) * U1 for m in (1, 2, 3)]
        Kp = 0.5 * sum(M(lambda z, m=m: z[m] ** 2 / z[4], zl, zr) for m in (1, 2, 3)) \
            - z5m / (delta * L(zl[4], zr[4])) + 9 / 4 * M(lambda z: z[0] / z[4], zl, zr)
        U5 = (-Kp * U1 + sum(M(lambda z, m=m: z[m] / z[4], zl, zr) * Um[m - 1] for m in (1, 2, 3))
              + 9 / 8 * z1m * M(lambda z: z[0] / z[4], zl, zr)) / M(lambda z: 1 / z[4], zl, zr)
        z12 = M(lambda z: z[0] * z[1], zl, zr)
        F11 = (z12 * c3 + g * M(lambda z: z[1], zl, zr)) / Dn
        F12 = z1m * z5m * g + M(lambda z: z[1], zl, zr) * F11
        F1m = [M(lambda z, m=m: z[m], zl, zr) * F11 for m in (2, 3)]
        Fv = [F12] + F1m
        F15 = (-Kp * F11 + sum(M(lambda z, m=m: z[m] / z[4], zl, zr) * Fv[m - 1] for m in (1, 2, 3))
               + 9 * z12 / 8 * M(lambda z: z[0] / z[4], zl, zr)) / M(lambda z: 1 / z[4], zl, zr)
        Ut, Ft = o.ec_pair(Ul, Ur)
        want_U = np.array([U1, *Um, U5])
        want_F = np.array([F11, F12, *F1m, F15])
        assert np.allclose(Ut, want_U, rtol=1e-11, atol=1e-11 * np.abs(want_U).max())
        assert np.allclose(Ft[0], want_F, rtol=1e-11, atol=1e-11 * np.abs(want_F).max())


def test_ideal_gas_limit(orc):
    """a = b = 0: the flux reduces to the ideal-gas EC flux in the same parameter vector,
    U~_rho = L(rho), F~_{j,rho} = L(rho){v_j}, pressure term {rho}{T} R."""
    p = synth.problem(2, [8, 8], unit="ideal")
    o = orc.Oracle(p)
    rng = np.random.default_rng(40)
    for Ul, Ur in _pairs(o, p, rng, 100, 2):
        Ut, Ft = o.ec_pair(Ul, Ur)
        zl, zr = o.cons_to_prim(Ul), o.cons_to_prim(Ur)
        Lr = (zr[0] - zl[0]) / (math.log(zr[0]) - math.log(zl[0]))
        assert abs(Ut[0] - Lr) < 1e-13 * Lr
        for j in range(2):
            vm = 0.5 * (zl[1 + j] + zr[1 + j])
            assert abs(Ft[j][0] - Lr * vm) < 1e-13 * (abs(Lr * vm) + 1e-3)
            pres = 0.5 * (zl[0] + zr[0]) * 0.5 * (zl[4] + zr[4]) * p["R"]
            assert abs(Ft[j][1 + j] - (vm * Ft[j][0] + pres)) < 1e-13 * (abs(pres) + 1)


def test_unit_invariance(orc):
    """Paper units (R, c_v, a) = (1, 1/delta, 9/8) and reduced units (8/3 of each) describe the
    same gas with velocities scaled by sqrt(8/3): U~ and F~ map with the same scaling."""
    pr = synth.problem(2, [8, 8], unit="reduced")
    pp = synth.problem(2, [8, 8], unit="paper")
    o_r, o_p = orc.Oracle(pr), orc.Oracle(pp)
    k = 8.0 / 3.0
    sk = math.sqrt(k)
    rng = np.random.default_rng(50)
    for Ul, Ur in _pairs(o_p, pp, rng, 50, 2):
        ql, qr = o_p.cons_to_prim(Ul), o_p.cons_to_prim(Ur)
        Ul2 = o_r.prim_to_cons(np.array([ql[0], ql[1] * sk, ql[2] * sk, ql[3] * k]))
        Ur2 = o_r.prim_to_cons(np.array([qr[0], qr[1] * sk, qr[2] * sk, qr[3] * k]))
        Ut_p, Ft_p = o_p.ec_pair(Ul, Ur)
        Ut_r, Ft_r = o_r.ec_pair(Ul2, Ur2)
        su = np.array([1, sk, sk, k])
        assert np.allclose(Ut_r, su * Ut_p, rtol=1e-13, atol=1e-13 * np.abs(Ut_r).max())
        sf = np.array([sk, k, k, k * sk])
        for j in range(2):
            assert np.allclose(Ft_r[j], sf * Ft_p[j], rtol=1e-13, atol=1e-13 * np.abs(Ft_r[j]).max())


def test_alpha_coefficients(orc):
    """alpha_{3,m} solve sum m alpha = 1, sum m^3 alpha = sum m^5 alpha = 0 (exact rationals)."""
    A = [[Fraction(m) ** (2 * s - 1) for m in (1, 2, 3)] for s in (1, 2, 3)]
    rhs = [Fraction(1), Fraction(0), Fraction(0)]
    # Gaussian elimination in exact arithmetic
    n = 3
    M = [row[:] + [r] for row, r in zip(A, rhs)]
    for i in range(n):
        piv = M[i][i]
        M[i] = [v / piv for v in M[i]]
        for r in range(n):
            if r != i:
                f = M[r][i]
                M[r] = [a - f * b for a, b in zip(M[r], M[i])]
    exact = [float(M[i][n]) for i in range(n)]
    assert np.allclose(orc.alpha(), exact, rtol=0, atol=1e-16)


@pytest.mark.parametrize("unit,ab", [("reduced", None), ("paper", None), ("reduced", (2.2, 0.37))])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_scaled_eigenvectors(orc, unit, ab, dim):
    """eq. eigen: R R^T = dU/dV and (dF_1/dU) R = R diag(lambda), with dU/dV and dF_1/dU
    from finite differences of the oracle's entropy variables and physical flux."""
    kw = {} if ab is None else dict(a=ab[0], b=ab[1])
    p = synth.problem(dim, [8] * dim, unit=unit, **kw)
    o = orc.Oracle(p)
    rng = np.random.default_rng(60 + dim)
    nv = dim + 2
    rc, Tc, pc = synth._critical(p)
    count = 0
    while count < 8:
        rho = rng.uniform(0.3, 1.8) * rc
        T = rng.uniform(1.0, 1.6) * Tc
        if not o.admissible(rho, T):
            continue
        count += 1
        u = rng.uniform(-0.6, 0.6, size=dim) * math.sqrt(pc / rc)
        pr = synth._p_of(p, rho, T)
        U = o.prim_to_cons(np.array([rho, *u, pr]))
        Rm, lam, ok = o.eigen(rho, u, pr)
        assert ok
        dVdU = np.zeros((nv, nv))
        A = np.zeros((nv, nv))
        for i in range(nv):
            h = 1e-6 * max(abs(U[i]), 1e-2)
            Up, Um = U.copy(), U.copy()
            Up[i] += h
            Um[i] -= h
            dVdU[:, i] = (o.entropy_vars(Up) - o.entropy_vars(Um)) / (2 * h)
            A[:, i] = (o.phys_flux(Up, 0) - o.phys_flux(Um, 0)) / (2 * h)
        dUdV = np.linalg.inv(dVdU)
        rel = np.abs(Rm @ Rm.T - dUdV).max() / np.abs(dUdV).max()
        assert rel < 1e-6, rel
        res = np.abs(A @ Rm - Rm @ np.diag(lam)).max() / np.abs(A @ Rm).max()
        assert res < 1e-6, res
