"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module only *draws* inputs: problem descriptions (grid sizes, constants, scheme
options), primitive fields (rho, v, p), meshes and mesh velocities.  It holds none of the
scheme's arithmetic.  The one exception is a two-line evaluation of the van der Waals
temperature and admissibility conditions (Remark 2.1 of the paper) that the samplers use to
*define their sampling domain* (rejection of inadmissible draws); both the GPU library
and the oracle convert the primitive fields to conserved variables with their own code.

Units: ``reduced`` = (R, c_v, a, b) = (8/3, (8/3)/delta, 3, 1/3), in which the critical point
is rho_c = T_c = p_c = 1 and the flux pressure equals the paper's dimensionless p_*;
``paper`` = (1, 1/delta, 9/8, 1/3), the paper's own scaling, where the flux pressure is
3/8 p_* (Section 2).
"""
import math

import numpy as np

DELTA = 0.0125


def units(name="reduced", delta=DELTA, a=None, b=None):
    if name == "reduced":
        R = 8.0 / 3.0
        aa, bb = 3.0, 1.0 / 3.0
    elif name == "paper":
        R = 1.0
        aa, bb = 9.0 / 8.0, 1.0 / 3.0
    elif name == "ideal":
        R = 1.0
        aa, bb = 0.0, 0.0
    else:
        raise ValueError(name)
    if a is not None:
        aa = a
    if b is not None:
        bb = b
    return dict(R=R, cv=R / delta, a=aa, b=bb)


def problem(dim, n, bc="outflow", lo=None, hi=None, unit="reduced", delta=DELTA, **kw):
    """Problem/scheme description used by both the GPU binding and the oracle.

    Defaults follow the paper's Section 5: MR-WENO linear weights (0.95, 0.045, 0.005),
    CFL 0.4 (1D/2D) or 0.3 (3D), mu = 10 Jacobi sweeps, vdW monitor with (rho, G),
    5 filter passes."""
    n = list(n) + [1] * (3 - len(n))
    bcs = [bc] * 3 if isinstance(bc, str) else list(bc) + ["periodic"] * (3 - len(bc))
    p = dict(dim=dim, n=n, lo=list(lo or [0.0] * 3), hi=list(hi or [1.0] * 3), bc=bcs,
             dissipation=1, weno_lin=[0.95, 0.045, 0.005], weno_eps=1e-10,
             cfl=0.4 if dim < 3 else 0.3, dt_fixed=0.0,
             monitor="vdw", kappa=2, mon_var=["rho", "G"], alpha=[1200.0, 1200.0, 0.0],
             n_filter=5, mu=10, mesh_tol=1e-8, fixed_mu=1)
    p.update(units(unit, delta))
    for k in ("R", "cv", "a", "b"):
        if k in kw:
            p[k] = kw.pop(k)
    p.update(kw)
    p["lo"] = (p["lo"] + [0.0] * 3)[:3]
    p["hi"] = (p["hi"] + [1.0] * 3)[:3]
    return p


def shape(p):
    return tuple(int(p["n"][k]) for k in reversed(range(p["dim"])))


def nodes_xi(p):
    """Cell-centred computational coordinates xi_k (d, *shape)."""
    d = p["dim"]
    axes = []
    for k in range(d):
        h = (p["hi"][k] - p["lo"][k]) / p["n"][k]
        axes.append(p["lo"][k] + (np.arange(p["n"][k]) + 0.5) * h)
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # z, y, x order
    return np.stack(list(reversed(grids)), axis=0)


# --- sampling-domain helpers (input definition only) --------------------------------

def _T_of(p, rho, pr):
    return (pr + p["a"] * rho * rho) * (1.0 - p["b"] * rho) / (rho * p["R"])


def _p_of(p, rho, T):
    return rho * p["R"] * T / (1.0 - p["b"] * rho) - p["a"] * rho * rho


def _admissible(p, rho, T):
    a, b, R = p["a"], p["b"], p["R"]
    ok = rho > 0
    if b > 0:
        ok = ok and rho < 1.0 / b and T > a / (4.0 * R * b)
    else:
        ok = ok and T > 0
    return bool(ok and R * T - 2.0 * a * rho * (1.0 - b * rho) ** 2 > 0)


def _mean_ok(p, s1, s2):
    a, b, R = p["a"], p["b"], p["R"]
    rm = 0.5 * (s1[0] + s2[0])
    Tm = 0.5 * (s1[1] + s2[1])
    return R * Tm - 2.0 * a * rm * (1.0 - b * rm) ** 2 > 0


def _logmean(u, v):
    return u if abs(u - v) <= 1e-12 * abs(u) else (u - v) / (math.log(u) - math.log(v))


def _avg_ok(p, s1, s2):
    """The interface-averaged state of the dissipation (log-mean density, pressure
    L(rho)/L(rho/p), Section 3.3) of two states (rho, T, p) is admissible."""
    rb = _logmean(s1[0], s2[0])
    pb = rb / _logmean(s1[0] / s1[2], s2[0] / s2[2])
    return _admissible(p, rb, _T_of(p, rb, pb))


# --- meshes ------------------------------------------------------------------------

def smooth_mesh(p, seed, amp=0.02):
    """x = xi + amp * (smooth periodic displacement); a valid, non-orthogonal mesh.

    For periodic directions the displacement is periodic, so x(xi + P e_k) = x(xi) + P e_k.
    For outflow directions the normal displacement vanishes at the walls."""
    rng = np.random.default_rng(seed)
    d = p["dim"]
    xi = nodes_xi(p)
    x = xi.copy()
    for j in range(d):
        disp = np.zeros_like(xi[0])
        for _ in range(3):
            kv = rng.integers(1, 3, size=d)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(2 * math.pi * kv[k] * (xi[k] - p["lo"][k]) / (p["hi"][k] - p["lo"][k]) for k in range(d))
            disp += rng.uniform(-1, 1) * np.sin(arg + ph)
        if p["bc"][j] == "outflow":
            L = p["hi"][j] - p["lo"][j]
            disp *= np.sin(math.pi * (xi[j] - p["lo"][j]) / L)
        x[j] += amp * (p["hi"][j] - p["lo"][j]) * disp / 3.0
    return np.ascontiguousarray(x)


def smooth_velocity(p, seed, amp=0.1):
    """A smooth periodic mesh-velocity field (d, *shape)."""
    rng = np.random.default_rng(seed + 7919)
    d = p["dim"]
    xi = nodes_xi(p)
    v = np.zeros_like(xi)
    for j in range(d):
        for _ in range(2):
            kv = rng.integers(1, 3, size=d)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(2 * math.pi * kv[k] * (xi[k] - p["lo"][k]) / (p["hi"][k] - p["lo"][k]) for k in range(d))
            v[j] += rng.uniform(-1, 1) * np.sin(arg + ph)
        if p["bc"][j] == "outflow":
            L = p["hi"][j] - p["lo"][j]
            v[j] *= np.sin(math.pi * (xi[j] - p["lo"][j]) / L)
    return np.ascontiguousarray(amp * v)


# --- primitive fields (rho, v_1..v_d, p) -----------------------------------------------

def uniform_state(p, rho=0.8, v=None, T=1.2):
    d = p["dim"]
    v = list(v if v is not None else [0.3, -0.2, 0.1][:d])
    sh = shape(p)
    prim = np.zeros((d + 2,) + sh)
    prim[0] = rho
    for m in range(d):
        prim[1 + m] = v[m]
    prim[d + 1] = _p_of(p, rho, T)
    return prim


def smooth_state(p, seed, x=None):
    """Smooth admissible random fields on the node coordinates x (default: uniform mesh).

    rho in [0.55, 1.45] rho_c, T in [1.1, 1.3] T_c (so every mean state satisfies the
    mean-value constraint of Theorem 3.1), |v| <= 0.6 in units of sqrt(p_c/rho_c)."""
    rng = np.random.default_rng(seed)
    d = p["dim"]
    x = nodes_xi(p) if x is None else x
    rc, Tc, pc = _critical(p)
    def field(amp):
        f = np.zeros_like(x[0])
        for _ in range(3):
            kv = rng.integers(1, 3, size=d)
            ph = rng.uniform(0, 2 * math.pi)
            f += rng.uniform(-1, 1) * np.sin(sum(2 * math.pi * kv[k] * x[k] for k in range(d)) + ph)
        return amp * f / 3.0
    rho = rc * (1.0 + field(0.45))
    T = Tc * (1.2 + field(0.1))
    prim = np.zeros((d + 2,) + rho.shape)
    prim[0] = rho
    vs = math.sqrt(pc / rc)
    for m in range(d):
        prim[1 + m] = vs * field(0.6 / math.sqrt(d))
    prim[d + 1] = _p_of(p, rho, T)
    return np.ascontiguousarray(prim)


def _critical(p):
    """(rho_c, T_c, p_c) of the van der Waals gas (eq. vdwconstant); ideal gas: (1, 1, 1)."""
    a, b, R = p["a"], p["b"], p["R"]
    if a == 0 or b == 0:
        return 1.0, 1.0, 1.0
    return 1.0 / (3.0 * b), 8.0 * a / (27.0 * R * b), a / (27.0 * b * b)


def sine_wave(p, x, t, case):
    """Exact smooth solutions of the accuracy tests (constant v and p, so rho is advected):
    case 1 (Ex. 5.1): (0.5 + 0.2 sin 2pi(x - t), 1, 1);  case 2 (Ex. 5.3):
    (0.5 + 0.2 sin 2pi(x1 + x2 - t), 0.5, 0.5, 1);  case 3 (Ex. 5.6):
    (0.5 + 0.2 sin 2pi(x1 + x2 + x3 - 0.9 t), 0.3, 0.3, 0.3, 1).  Values are dimensionless
    and p = 1 is taken as the flux pressure of the unit system in use: rho is advected
    exactly for any constant v and p, so the choice does not affect the test."""
    d = p["dim"]
    if case == 1:
        ph, v = x[0] - t, [1.0]
    elif case == 2:
        ph, v = x[0] + x[1] - t, [0.5, 0.5]
    else:
        ph, v = x[0] + x[1] + x[2] - 0.9 * t, [0.3, 0.3, 0.3]
    prim = np.zeros((d + 2,) + x[0].shape)
    prim[0] = 0.5 + 0.2 * np.sin(2 * math.pi * ph)
    for m in range(d):
        prim[1 + m] = v[m]
    prim[d + 1] = 1.0
    return np.ascontiguousarray(prim)


# Table 5.1 of the paper: (rho, v1, p)_l, (rho, v1, p)_r in dimensionless units
TABLE_5_1 = {
    "RP1": ((1.818, 0.0, 3.000), (0.275, 0.0, 0.575)),
    "RP2": ((0.879, 0.0, 1.090), (0.562, 0.0, 0.885)),
    "RP3": ((0.879, 0.0, 1.090), (0.275, 0.0, 0.575)),
}


def riemann_1d(p, left, right, x0=0.5, x=None):
    """1D shock tube: primitive (rho, v, p) left of x0 and right of it (reduced units)."""
    x = nodes_xi(p) if x is None else x
    prim = np.zeros((3,) + x[0].shape)
    for i in range(3):
        prim[i] = np.where(x[0] < x0, left[i], right[i])
    return prim


def riemann_1d_random(p, seed):
    """A 1D Riemann problem near the critical point in the non-classical region (G < 0):
    rho_l, rho_r ~ U[0.6, 0.85] rho_c with |rho_l - rho_r| >= 0.15 rho_c, T ~ U[0.99, 1.015] T_c,
    v = 0.  In reduced units with delta = 0.0125 this box lies inside the admissible set and
    inside G < 0, and every mean state satisfies Theorem 3.1's constraint."""
    rng = np.random.default_rng(seed)
    rc, Tc, pc = _critical(p)
    while True:
        r = rng.uniform(0.6, 0.85, size=2)
        if abs(r[0] - r[1]) >= 0.15:
            break
    T = rng.uniform(0.99, 1.015, size=2)
    left = (r[0] * rc, 0.0, _p_of(p, r[0] * rc, T[0] * Tc))
    right = (r[1] * rc, 0.0, _p_of(p, r[1] * rc, T[1] * Tc))
    return left, right


def quadrant_states(p, seed, rho=(0.5, 1.5), pr=(0.8, 1.6), vmax=0.5, strict=False, Tmin=0.0):
    """Four quadrant states of a 2D Riemann problem, drawn in reduced form:
    rho ~ U[0.5, 1.5] rho_c, p ~ U[0.8, 1.6] p_c, v_i ~ U[-0.5, 0.5] sqrt(p_c/rho_c) with |v| <= 0.5;
    inadmissible states and tuples whose edge-adjacent pairs break the mean-value constraint
    are redrawn; with strict=True also tuples where the dissipation's averaged state of an
    edge-adjacent pair is inadmissible; states colder than Tmin T_c are redrawn too.  Returns a
    list of 4 tuples (rho, v1, v2, p) for quadrants 1 (x>1/2, y>1/2), 2 (x<1/2, y>1/2),
    3 (x<1/2, y<1/2), 4 (x>1/2, y<1/2)."""
    rng = np.random.default_rng(seed)
    rc, Tc, pc = _critical(p)
    vs = math.sqrt(pc / rc)
    while True:
        states = []
        for _ in range(4):
            while True:
                r = rng.uniform(*rho) * rc
                q = rng.uniform(*pr) * pc
                v = rng.uniform(-vmax, vmax, size=2)
                if np.hypot(*v) > vmax:
                    continue
                T = _T_of(p, r, q)
                if _admissible(p, r, T) and T >= Tmin * Tc:
                    states.append((r, v[0] * vs, v[1] * vs, q, T))
                    break
        ok = all(_mean_ok(p, (states[i][0], states[i][4]), (states[(i + 1) % 4][0], states[(i + 1) % 4][4]))
                 for i in range(4))
        if ok and strict:
            ok = all(_avg_ok(p, (states[i][0], states[i][4], states[i][3]),
                             (states[(i + 1) % 4][0], states[(i + 1) % 4][4], states[(i + 1) % 4][3]))
                     for i in range(4))
        if ok:
            return [s[:4] for s in states]


def quadrants_2d(p, states, x=None, xc=0.5, yc=0.5):
    x = nodes_xi(p) if x is None else x
    prim = np.zeros((4,) + x[0].shape)
    right = x[0] >= xc
    top = x[1] >= yc
    masks = [right & top, ~right & top, ~right & ~top, right & ~top]
    for s, m in zip(states, masks):
        for i in range(4):
            prim[i][m] = s[i]
    return np.ascontiguousarray(prim)


def smooth_3d(p, seed, x=None):
    """rho = 1 + 0.2 sum_{m=1..4} sin(2pi k_m.x + phi_m) with one integer wavevector per shell
    |k_m|_inf = m, v = (0.3, 0.2, 0.1), p = 1.2 (reduced units)."""
    rng = np.random.default_rng(seed)
    x = nodes_xi(p) if x is None else x
    rho = np.ones_like(x[0])
    for m in range(1, 5):
        while True:
            kv = rng.integers(-m, m + 1, size=3)
            if np.max(np.abs(kv)) == m:
                break
        rho += 0.2 * np.sin(2 * math.pi * sum(kv[k] * x[k] for k in range(3)) + rng.uniform(0, 2 * math.pi))
    prim = np.zeros((5,) + x[0].shape)
    prim[0] = rho
    prim[1], prim[2], prim[3] = 0.3, 0.2, 0.1
    prim[4] = 1.2
    return np.ascontiguousarray(prim)


def spherical_shock_3d(p, x=None, r0=0.5, inside=None, outside=None, width=0.0):
    """3D spherically symmetric shock tube (Example 5.7): the RP1 states of Table 5.1 inside and
    outside the sphere |x| < r0 centred at the origin (v = 0; rho and p are the same in paper
    and reduced units).  width > 0 replaces the jump by the profile
    outside + (inside - outside) (1 - tanh((|x| - r0)/width))/2 (used to adapt an initial mesh).
    x may be a numpy array or a torch tensor (then the fields are built with the same arithmetic
    on its device)."""
    x = nodes_xi(p) if x is None else x
    inside = inside or (TABLE_5_1["RP1"][0][0], TABLE_5_1["RP1"][0][2])
    outside = outside or (TABLE_5_1["RP1"][1][0], TABLE_5_1["RP1"][1][2])
    if isinstance(x, np.ndarray):
        r = np.sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
        prim = np.zeros((5,) + x[0].shape)
        if width > 0.0:
            s = 0.5 * (1.0 - np.tanh((r - r0) / width))
            prim[0] = outside[0] + (inside[0] - outside[0]) * s
            prim[4] = outside[1] + (inside[1] - outside[1]) * s
        else:
            prim[0] = np.where(r < r0, inside[0], outside[0])
            prim[4] = np.where(r < r0, inside[1], outside[1])
        return np.ascontiguousarray(prim)
    import torch
    r = torch.sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
    prim = torch.zeros((5,) + tuple(x.shape[1:]), dtype=torch.float64, device=x.device)
    if width > 0.0:
        s = 0.5 * (1.0 - torch.tanh((r - r0) / width))
        prim[0] = outside[0] + (inside[0] - outside[0]) * s
        prim[4] = outside[1] + (inside[1] - outside[1]) * s
        return prim
    # fill, then overwrite inside (torch.where on two Python scalars would round them to FP32)
    inner = r < r0
    prim[0].fill_(outside[0]).masked_fill_(inner, inside[0])
    prim[4].fill_(outside[1]).masked_fill_(inner, inside[1])
    return prim


# Table 5.3 of the paper (Example 5.4): gamma, (rho, v1, v2, p) behind and ahead of the shock;
# velocities in the paper's unit (reduced velocities are sqrt(8/3) times larger), incidence
# angle theta (degrees) and shock Mach number as printed
TABLE_5_3 = {
    "P1": dict(gamma=1.4, left=(0.033, 5.016, 0.0, 3.001), right=(0.0156, 0.0, 0.0, 1.0), theta=20.0, mach=1.65),
    "D1": dict(gamma=1.0125, left=(0.629, -0.135, 0.0, 0.983), right=(0.879, 0.0, 0.0, 1.09), theta=30.0, mach=1.05),
}


def mach_reflection(p, case, x=None, foot=0.1):
    """Example 5.4's oblique shock in reduced units: a planar shock whose normal points along
    (cos theta, -sin theta) toward the wall x_2 = 0, its foot on the wall at x_1 = foot; behind it
    the state `left` of Table 5.3 moving along that normal with speed |v1| sqrt(8/3) (signed as
    printed), ahead of it the state `right` at rest."""
    c = TABLE_5_3[case]
    x = nodes_xi(p) if x is None else x
    th = math.radians(c["theta"])
    n0, n1 = math.cos(th), -math.sin(th)
    behind = (x[0] - foot) * n0 + x[1] * n1 < 0.0
    u = c["left"][1] * math.sqrt(8.0 / 3.0)
    prim = np.zeros((4,) + x[0].shape)
    prim[0] = np.where(behind, c["left"][0], c["right"][0])
    prim[1] = np.where(behind, u * n0, 0.0)
    prim[2] = np.where(behind, u * n1, 0.0)
    prim[3] = np.where(behind, c["left"][3], c["right"][3])
    return np.ascontiguousarray(prim)


# Table 5.4 of the paper (Example 5.5, flow over a backward step): (rho, v1, v2, p)_l, (..)_r
# in the paper's dimensionless units (velocities sqrt(3/8) of the reduced ones), with the
# printed shock Mach numbers and final times
TABLE_5_4 = {
    "TD1": dict(left=(0.85, 0.64, 0.0, 1.01), right=(0.28, 0.0, 0.0, 0.58), mach=1.23, t_end=0.55),
    "TD2": dict(left=(0.62, -0.14, 0.0, 0.98), right=(0.88, 0.0, 0.0, 1.09), mach=1.05, t_end=1.5),
}


def step_state(case, side):
    """State `side` ("left" | "right") of Table 5.4 in reduced units: (rho, v1 sqrt(8/3), v2, p)."""
    rho, u, v, pr = TABLE_5_4[case][side]
    return (rho, u * math.sqrt(8.0 / 3.0), v * math.sqrt(8.0 / 3.0), pr)


def backward_step(p, case, x=None, shock=0.3):
    """Example 5.5's initial data: the state `left` of Table 5.4 behind a planar shock at
    x_1 = shock (in the channel above the step), the state `right` everywhere else (the solid
    nodes included)."""
    x = nodes_xi(p) if x is None else x
    left, right = step_state(case, "left"), step_state(case, "right")
    behind = x[0] < shock
    prim = np.zeros((4,) + x[0].shape)
    for v in range(4):
        prim[v] = np.where(behind, left[v], right[v])
    return np.ascontiguousarray(prim)


def batch_instances(seed, count=256, nmin=64, nmax=384):
    """Independent 2D Riemann instances: n ~ U{nmin..nmax} (square grids), a ~ U[2, 4],
    b ~ U[0.2, 0.4], R = 8/3, c_v = R/0.0125; quadrant states drawn in reduced form and
    scaled by the instance's critical values (corresponding states).  The states are kept
    supercritical (T >= 1.05 T_c) with admissible averaged interface states: subcritical states
    of the (rho, p) box near the spinodal curve send the first rarefactions of a quarter of the
    instances out of the admissible set within one step."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        a = float(rng.uniform(2.0, 4.0))
        b = float(rng.uniform(0.2, 0.4))
        p = problem(2, [n, n], bc="outflow", a=a, b=b)
        st = quadrant_states(p, int(rng.integers(0, 2**31 - 1)), strict=True, Tmin=1.05)
        out.append((p, st))
    return out
