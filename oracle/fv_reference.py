"""Second-order finite-volume reference solver for 1D planar and spherically symmetric flows of
the van der Waals gas: the kind of solver the paper uses for its reference solutions (10 000
cells; Example 5.2 in planar, Example 5.7 in spherical geometry).

TEST INFRASTRUCTURE, like the oracle: only tests, the scripts that write stored reference
solutions under tests/golden/, and analysis of measured runs may use it.  It shares no code with
the GPU library or with the oracle's C code.

Scheme (textbook; the paper does not describe its own): cell averages of U = (rho, rho v, E);
piecewise-linear reconstruction of the primitive variables (rho, v, p) with minmod-limited
slopes; HLL fluxes with Davis' wave-speed bounds min/max(v -+ c) over the two reconstructed
states; SSP-RK2 (Heun) in time at a CFL number of 0.4.  Spherical geometry: volumes
(r+^3 - r-^3)/3 and areas r^2, with the pressure part of the momentum flux balanced by the source
p (A+ - A-)/V, so that a fluid at rest stays at rest; reflection at r = 0.  Outer boundaries
copy the last cell.

EOS in general units: p = rho R T/(1 - b rho) - a rho^2, e = c_v T - a rho; the squared sound
speed follows from p(rho, e) as c^2 = R T (1 + R/c_v)/(1 - b rho)^2 - 2 a rho.
"""
import numpy as np


class VdW:
    def __init__(self, R, cv, a, b):
        self.R, self.cv, self.a, self.b = float(R), float(cv), float(a), float(b)

    def T_from_rho_p(self, rho, p):
        return (p + self.a * rho * rho) * (1.0 - self.b * rho) / (rho * self.R)

    def energy(self, rho, p, v):
        """E = rho e + rho v^2 / 2 from (rho, p, v)."""
        T = self.T_from_rho_p(rho, p)
        return rho * (self.cv * T - self.a * rho) + 0.5 * rho * v * v

    def prim(self, U):
        rho, m, E = U
        v = m / rho
        e = E / rho - 0.5 * v * v
        T = (e + self.a * rho) / self.cv
        p = rho * self.R * T / (1.0 - self.b * rho) - self.a * rho * rho
        return rho, v, p, T

    def c2(self, rho, T):
        return self.R * T * (1.0 + self.R / self.cv) / (1.0 - self.b * rho) ** 2 - 2.0 * self.a * rho


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


class FV1D:
    """n cells on [lo, hi]; geometry "planar" or "spherical" (then lo must be 0)."""

    def __init__(self, eos, n, lo, hi, geometry="planar", cfl=0.4):
        assert geometry in ("planar", "spherical")
        assert geometry == "planar" or lo == 0.0
        self.eos, self.n, self.lo, self.hi, self.geometry, self.cfl = eos, n, lo, hi, geometry, cfl
        self.h = (hi - lo) / n
        self.xf = lo + self.h * np.arange(n + 1)          # faces
        self.x = 0.5 * (self.xf[1:] + self.xf[:-1])       # centres
        if geometry == "spherical":
            self.A = self.xf ** 2
            self.V = (self.xf[1:] ** 3 - self.xf[:-1] ** 3) / 3.0
        else:
            self.A = np.ones(n + 1)
            self.V = np.full(n, self.h)

    def init(self, rho, v, p):
        rho, v, p = (np.broadcast_to(np.asarray(q, dtype=np.float64), (self.n,)).copy() for q in (rho, v, p))
        return np.array([rho, rho * v, self.eos.energy(rho, p, v)])

    def _ghosts(self, W):
        """Two ghost cells per side on primitive fields W = (rho, v, p)."""
        if self.geometry == "spherical":
            left = W[:, [1, 0]].copy()                     # reflection at the centre
            left[1] = -left[1]
        else:
            left = W[:, [0, 0]].copy()
        right = W[:, [-1, -1]].copy()
        return np.concatenate([left, W, right], axis=1)

    def _flux(self, rho, v, p):
        E = self.eos.energy(rho, p, v)
        return np.array([rho * v, rho * v * v + p, (E + p) * v]), np.array([rho, rho * v, E])

    def rhs(self, U):
        eos = self.eos
        rho, v, p, _ = eos.prim(U)
        W = self._ghosts(np.array([rho, v, p]))            # n + 4 cells
        dW = _minmod(W[:, 1:-1] - W[:, :-2], W[:, 2:] - W[:, 1:-1])   # slopes of cells 1 .. n+2
        WL = W[:, 1:-2] + 0.5 * dW[:, :-1]                 # left state at faces 0 .. n
        WR = W[:, 2:-1] - 0.5 * dW[:, 1:]                  # right state at faces 0 .. n
        FL, UL = self._flux(*WL)
        FR, UR = self._flux(*WR)
        cL = np.sqrt(eos.c2(WL[0], eos.T_from_rho_p(WL[0], WL[2])))
        cR = np.sqrt(eos.c2(WR[0], eos.T_from_rho_p(WR[0], WR[2])))
        SL = np.minimum(WL[1] - cL, WR[1] - cR)
        SR = np.maximum(WL[1] + cL, WR[1] + cR)
        Fh = np.where(SL >= 0.0, FL, np.where(SR <= 0.0, FR,
                                                (SR * FL - SL * FR + SL * SR * (UR - UL)) / np.where(SR > SL, SR - SL, 1.0)))
        AF = Fh * self.A
        dU = -(AF[:, 1:] - AF[:, :-1]) / self.V
        if self.geometry == "spherical":
            dU[1] += p * (self.A[1:] - self.A[:-1]) / self.V
        smax = float(np.max(np.maximum(np.abs(SL), np.abs(SR))))
        return dU, smax

    def dt(self, U):
        rho, v, p, T = self.eos.prim(U)
        return self.cfl * self.h / float(np.max(np.abs(v) + np.sqrt(self.eos.c2(rho, T))))

    def run(self, U, t_end, max_steps=10_000_000):
        """Advances to exactly t_end (the last step shortened); returns (U, steps)."""
        t, steps = 0.0, 0
        while t < t_end and steps < max_steps:
            dt = min(self.dt(U), t_end - t)
            k1, _ = self.rhs(U)
            U1 = U + dt * k1
            k2, _ = self.rhs(U1)
            U = 0.5 * (U + U1 + dt * k2)
            t += dt
            steps += 1
        return U, steps

    def mass(self, U):
        return float(np.sum(U[0] * self.V))


def riemann(eos, left, right, t_end, n=10000, lo=0.0, hi=1.0, x0=0.5, geometry="planar"):
    """Reference solution of a shock tube: left/right = (rho, v, p).  Returns (x, rho, v, p)."""
    s = FV1D(eos, n, lo, hi, geometry)
    inside = s.x < x0
    U = s.init(np.where(inside, left[0], right[0]), np.where(inside, left[1], right[1]),
               np.where(inside, left[2], right[2]))
    U, _ = s.run(U, t_end)
    rho, v, p, _ = eos.prim(U)
    return s.x, rho, v, p
