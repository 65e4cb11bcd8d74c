"""Closed-form pins of the oracle's CFL step (eq. cfl), monitor (eq. van der Waalsmonitor and eq.
van der Waalssinmonitor), movement limiter and low-pass filter (Section 4).

Each expected value below is derived from the paper's definition on data where the discrete
operators have a known closed form (uniform or separable sine meshes, sinusoidal fields whose
central differences are exact multiples of their derivatives, single moved nodes, unit
impulses), so that a plausible mistake in the oracle (a wrong grid spacing, a dropped
normalisation, a swapped term or weight, a Laplacian instead of the vector of pure second
derivatives, a full instead of a half gap) changes the result by far more than rounding."""
import numpy as np
import pytest

from paper_2407_05568_amd import synth


def _eos(p, rho, T):
    """van der Waals pressure and squared sound speed in general units (Section 2):
    p = rho R T/(1 - b rho) - a rho^2, c^2 = (1 + delta) R T/(1 - b rho)^2 - 2 a rho."""
    R, a, b = p["R"], p["a"], p["b"]
    d = R / p["cv"]
    ob = 1.0 - b * rho
    return rho * R * T / ob - a * rho * rho, (1.0 + d) * R * T / ob ** 2 - 2.0 * a * rho


def _random_state(p, rng, shape):
    """Admissible supercritical states: rho in [0.7, 1.3], T in [1.15, 1.35] (critical point
    (1, 1) in reduced units), |v_k| <= 0.4."""
    rho = rng.uniform(0.7, 1.3, size=shape)
    T = rng.uniform(1.15, 1.35, size=shape)
    v = rng.uniform(-0.4, 0.4, size=(p["dim"],) + shape)
    pr, c2 = _eos(p, rho, T)
    return np.concatenate([rho[None], v, pr[None]]), rho, T, v, np.sqrt(c2)


# --- CFL (eq. cfl) --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,bc,lo,hi,n", [
    (1, "outflow", [0.0], [3.0], [37]),
    (2, "outflow", [0.0, 0.0], [2.0, 0.5], [20, 12]),
    (3, "periodic", [0.0, 0.0, 0.0], [1.0, 2.0, 0.5], [10, 8, 6]),
])
def test_cfl_uniform_mesh_closed_form(orc, dim, bc, lo, hi, n):
    """On the uniform mesh x = xi of a box with unequal spacings the metrics are the identity and
    J = 1, so dt = CFL / max_i sum_k (|v_k| + c)_i / dxi_k exactly (spacing dxi_k = (hi_k - lo_k)/n_k)."""
    p = synth.problem(dim, n, bc=bc, lo=lo, hi=hi)
    o = orc.Oracle(p)
    rng = np.random.default_rng(11 + dim)
    prim, rho, T, v, c = _random_state(p, rng, o.shape)
    x = o.uniform_mesh()
    J = np.ones(o.shape)
    JU = o.init_state(prim, J)
    dxi = [(hi[k] - lo[k]) / n[k] for k in range(dim)]
    rate = sum((np.abs(v[k]) + c) / dxi[k] for k in range(dim))
    want = p["cfl"] / rate.max()
    got = o.cfl_dt(JU, J, x)
    assert abs(got - want) <= 1e-13 * want, (got, want)


def test_cfl_stretched_mesh_closed_form(orc):
    """Separable stretched mesh x_k = xi_k + eps sin(2 pi xi_k) on [0,1]^2 (consistent with the
    outflow mirror: odd about both faces).  The sixth-order difference of sin(2 pi xi) is
    cos(2 pi xi) sum_m alpha_m sin(2 pi m h), so g_k = delta_k[x_k]/dxi_k is known in closed form;
    the metrics are diagonal (J xi_1/x_1 = g_2, J xi_2/x_2 = g_1) and, with J = g_1 g_2,
    rho_k/J = (|v_k| + c)/g_k: dt = CFL / max sum_k (|v_k| + c)/(g_k dxi_k)."""
    n = [24, 18]
    p = synth.problem(2, n, bc="outflow")
    o = orc.Oracle(p)
    rng = np.random.default_rng(5)
    prim, rho, T, v, c = _random_state(p, rng, o.shape)
    xi = synth.nodes_xi(p)
    eps = 0.04
    x = xi + eps * np.sin(2 * np.pi * xi)
    alpha = (1.5, -0.3, 1.0 / 30.0)  # exact rationals pinned in test_oracle_flux
    g = []
    for k in range(2):
        h = 1.0 / n[k]
        S = sum(alpha[m - 1] * np.sin(2 * np.pi * m * h) for m in (1, 2, 3))
        g.append(1.0 + eps * np.cos(2 * np.pi * xi[k]) * S / h)
    J = g[0] * g[1]
    JU = o.init_state(prim, J)
    rate = sum((np.abs(v[k]) + c) / (g[k] / n[k]) for k in range(2))
    want = p["cfl"] / rate.max()
    got = o.cfl_dt(JU, J, x)
    assert abs(got - want) <= 1e-12 * want, (got, want)
    # the wrong spacing (direction 1's for both) or a missing 1/J would move dt by O(1)
    assert abs(p["cfl"] / sum((np.abs(v[k]) + c) * n[0] for k in range(2)).max() - want) > 1e-3 * want


# --- monitor (Section 4) --------------------------------------------------------------------

def _T_for_G(p, rho, G):
    """Temperature at which the fundamental derivative of the vdW gas takes the value G at density
    rho: from G = [(1 + d)(2 + d) R T/(1 - b rho)^3 - 6 a rho] / (2 c^2) (eq. fundamental), linear
    in T:  T = a rho (4 G - 6) / (K (2 G - (2 + d)/(1 - b rho))),  K = (1 + d) R/(1 - b rho)^2."""
    R, a, b = p["R"], p["a"], p["b"]
    d = R / p["cv"]
    ob = 1.0 - b * rho
    K = (1.0 + d) * R / ob ** 2
    return a * rho * (4.0 * G - 6.0) / (K * (2.0 * G - (2.0 + d) / ob))


def _sine_fields(p, shape):
    """rho and G on a periodic [0,1]^2 grid as sums of one sine per direction (wave numbers 1
    and 2), with the central first and pure second differences of each in closed form:
    (f(x+h) - f(x-h))/(2h) = A cos(phase) sin(k h)/h, (f(x+h) - 2 f + f(x-h))/h^2 =
    -A sin(phase) (2 - 2 cos k h)/h^2."""
    xi = synth.nodes_xi(p)
    h = [1.0 / p["n"][k] for k in range(2)]
    specs = {"rho": (0.5, [(0.06, 1, 0.3), (0.04, 2, 1.1)]), "G": (0.8, [(0.1, 1, 2.0), (-0.08, 2, 0.4)])}
    out = {}
    for name, (base, modes) in specs.items():
        f = np.full(shape, base)
        d1, d2 = [], []
        for k, (A, m, ph) in enumerate(modes):
            kk = 2 * np.pi * m
            phase = kk * xi[k] + ph
            f = f + A * np.sin(phase)
            d1.append(A * np.cos(phase) * np.sin(kk * h[k]) / h[k])
            d2.append(-A * np.sin(phase) * (2.0 - 2.0 * np.cos(kk * h[k])) / h[k] ** 2)
        out[name] = (f, d1, d2)
    return out


def _monitor_case(orc, **kw):
    n = [16, 12]
    p = synth.problem(2, n, bc="periodic", **kw)
    o = orc.Oracle(p)
    fl = _sine_fields(p, o.shape)
    rho = fl["rho"][0]
    T = _T_for_G(p, rho, fl["G"][0])
    pr, c2 = _eos(p, rho, T)
    assert np.all(T > 1.0) and np.all(c2 > 0)  # supercritical, hyperbolic
    v = np.stack([np.full(o.shape, 0.2), np.full(o.shape, -0.1)])
    prim = np.concatenate([rho[None], v, pr[None]])
    J = np.ones(o.shape)
    JU = o.init_state(prim, J)
    return o, o.monitor(JU, J), fl


@pytest.mark.parametrize("alpha", [(7.0, 0.0, 0.0), (0.0, 5.0, 0.0), (0.0, 0.0, 3.0), (7.0, 5.0, 3.0)])
def test_vdw_monitor_terms_closed_form(orc, alpha):
    """eq. van der Waalsmonitor with kappa = 2, delta_1 = rho, delta_2 = G: omega^2 = 1 +
    alpha_1 |grad rho|^2/max + alpha_2 |grad G|^2/max + alpha_3 |Delta_xi G|^2/max, with Delta_xi G
    the vector of pure second derivatives (G_{xi1 xi1}, G_{xi2 xi2}), each term by second-order
    central differences (exact closed forms on sinusoids) and normalised by its maximum over
    the nodes.  One term at a time, then all three with distinct weights."""
    o, w, fl = _monitor_case(orc, kappa=2, mon_var=["rho", "G"], alpha=list(alpha))
    _, r1, _ = fl["rho"]
    _, g1, g2 = fl["G"]
    terms = [r1[0] ** 2 + r1[1] ** 2, g1[0] ** 2 + g1[1] ** 2, g2[0] ** 2 + g2[1] ** 2]
    want = np.sqrt(1.0 + sum(a * t / t.max() for a, t in zip(alpha, terms)))
    assert np.abs(w - want).max() < 1e-10, np.abs(w - want).max()
    # the Laplacian in place of the vector of pure second derivatives would differ
    if alpha[2]:
        lap = (g2[0] + g2[1]) ** 2
        assert np.abs(np.sqrt(1.0 + alpha[2] * lap / lap.max()) - np.sqrt(1.0 + alpha[2] * terms[2] / terms[2].max())).max() > 0.1


def test_vdw_monitor_variable_order(orc):
    """mon_var = (G, rho): the first gradient term is |grad G|^2 with alpha_1, the second
    |grad rho|^2 with alpha_2 (the alpha_k go with the delta_k in the order given)."""
    o, w, fl = _monitor_case(orc, kappa=2, mon_var=["G", "rho"], alpha=[4.0, 9.0, 0.0])
    _, r1, _ = fl["rho"]
    _, g1, _ = fl["G"]
    tg, tr = g1[0] ** 2 + g1[1] ** 2, r1[0] ** 2 + r1[1] ** 2
    want = np.sqrt(1.0 + 4.0 * tg / tg.max() + 9.0 * tr / tr.max())
    assert np.abs(w - want).max() < 1e-10


def test_sine_monitor_closed_form(orc):
    """eq. van der Waalssinmonitor: omega^2 = 1 + alpha_1 |grad rho|/max + alpha_2 |Delta_xi rho|/max
    (norms, not squares)."""
    o, w, fl = _monitor_case(orc, monitor="sine", kappa=0, alpha=[20.0, 15.0, 0.0])
    _, r1, r2 = fl["rho"]
    t1 = np.sqrt(r1[0] ** 2 + r1[1] ** 2)
    t2 = np.sqrt(r2[0] ** 2 + r2[1] ** 2)
    want = np.sqrt(1.0 + 20.0 * t1 / t1.max() + 15.0 * t2 / t2.max())
    assert np.abs(w - want).max() < 1e-10


# --- movement limiter (Section 4) -----------------------------------------------------------

def _stretched(p, seed):
    """A non-uniform, monotone mesh: unequal left and right gaps at every node."""
    xi = synth.nodes_xi(p)
    rng = np.random.default_rng(seed)
    x = xi.copy()
    for k in range(p["dim"]):
        x[k] = xi[k] + 0.3 / p["n"][k] * np.sin(2 * np.pi * xi[k] + rng.uniform(0, 6))
    return x


def test_limiter_single_node_closed_form(orc):
    """Delta_gamma = min(1, min over nodes and directions of the bound): moving one node along
    +x_1 by d > half the gap to its right neighbour (in x^n) gives exactly gap/(2 d); along -x_2,
    half the gap to its lower neighbour over |d|; a move below half the gap gives 1; two moved
    nodes give the smaller bound; only the coordinate's own direction constrains it."""
    n = [14, 11]
    p = synth.problem(2, n, bc="outflow")
    o = orc.Oracle(p)
    xn = _stretched(p, 2)
    i, j = 6, 4  # node (i0, i1) = (6, 4); arrays are [coord][i1][i0]
    gap_r = xn[0, j, i + 1] - xn[0, j, i]
    gap_l = xn[0, j, i] - xn[0, j, i - 1]
    gap_d = xn[1, j, i] - xn[1, j - 1, i]
    assert abs(gap_r - gap_l) > 1e-3 * gap_r  # the two sides differ
    d = 0.9 * gap_r
    xm = xn.copy()
    xm[0, j, i] += d
    assert o.limiter(xn, xm) == pytest.approx(gap_r / (2 * d), rel=1e-14)
    xm = xn.copy()
    xm[0, j, i] -= 1.3 * gap_l
    assert o.limiter(xn, xm) == pytest.approx(gap_l / (2 * 1.3 * gap_l), rel=1e-14)
    xm = xn.copy()
    xm[1, j, i] -= 0.8 * gap_d
    assert o.limiter(xn, xm) == pytest.approx(gap_d / (2 * 0.8 * gap_d), rel=1e-14)
    xm = xn.copy()
    xm[0, j, i] += 0.49 * gap_r
    assert o.limiter(xn, xm) == 1.0
    # a move of x_1 is not bounded by the x_2 gaps: a large x_1 gap, a tiny x_2 gap
    xm = xn.copy()
    xm[0, j, i] += 0.45 * gap_r
    xm[1, 2, 3] += 0.7 * (xn[1, 3, 3] - xn[1, 2, 3])
    assert o.limiter(xn, xm) == pytest.approx(1.0 / 1.4, rel=1e-14)


def test_limiter_at_the_wall(orc):
    """At an outflow face the neighbour across it is the mirror image of the node (x(-1) =
    2 lo - x(0)), so node 0 moving toward the face by d has the bound (x(0) - lo)/d: the node may
    reach the wall but not cross it."""
    p = synth.problem(1, [12], bc="outflow")
    o = orc.Oracle(p)
    xn = _stretched(p, 3)
    d = 1.6 * (xn[0, 0] - 0.0)
    xm = xn.copy()
    xm[0, 0] -= d
    assert o.limiter(xn, xm) == pytest.approx((xn[0, 0] - 0.0) / d, rel=1e-14)


# --- low-pass filter (Section 4) ------------------------------------------------------------

@pytest.mark.parametrize("dim", [1, 2, 3])
def test_filter_impulse_response(orc, dim):
    """One pass on a unit impulse (periodic grid, away from the wrap) returns the filter's own
    weights (1/2)^(|j|_1 + d) at offset j in {-1, 0, 1}^d and zero elsewhere; two passes return
    the weights convolved with themselves (the filter is linear and shift invariant)."""
    n = [9, 8, 7][:dim]
    p = synth.problem(dim, n, bc="periodic")
    o = orc.Oracle(p)
    w = np.zeros(o.shape)
    c = tuple(s // 2 for s in o.shape)
    w[c] = 1.0
    got = o.filter(w, 1)
    want = np.zeros(o.shape)
    for off in np.ndindex(*(3,) * dim):
        j = np.array(off) - 1
        want[tuple(np.array(c) + j)] = 0.5 ** (np.abs(j).sum() + dim)
    assert np.abs(got - want).max() == 0.0
    # two passes: the 1D weights (1/4, 1/2, 1/4) per direction convolved: (1, 4, 6, 4, 1)/16
    got2 = o.filter(w, 2)
    k1 = np.array([1, 4, 6, 4, 1]) / 16.0
    want2 = np.zeros(o.shape)
    for off in np.ndindex(*(5,) * dim):
        j = np.array(off) - 2
        want2[tuple(np.array(c) + j)] = np.prod([k1[q + 2] for q in j])
    assert np.abs(got2 - want2).max() < 1e-16


def test_filter_outflow_replicates_the_boundary_value(orc):
    """Outflow boundaries replicate the first node into the ghost layer (reading of the silent
    boundary treatment): an impulse on node 0 of a 1D grid gives 3/4 there (1/2 + 1/4 from its
    replicated ghost) and 1/4 on node 1."""
    p = synth.problem(1, [10], bc="outflow")
    o = orc.Oracle(p)
    w = np.zeros(10)
    w[0] = 1.0
    got = o.filter(w, 1)
    want = np.zeros(10)
    want[0], want[1] = 0.75, 0.25
    assert np.abs(got - want).max() == 0.0
