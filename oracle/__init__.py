"""ctypes access to the plain FP64 C oracle of the entropy-stable moving-mesh scheme.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the GPU library;
both sides receive the same seeded inputs from ``paper_2407_05568_amd.synth``.

Every array is float64, C-contiguous, field-major ``f[var][z][y][x]`` over the interior
nodes (x fastest), the same layout the GPU library uses.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esvdw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_libs = {}

BC = {"periodic": 0, "outflow": 1}
MONITOR = {"vdw": 0, "sine": 1}
MONVAR = {"rho": 0, "G": 1}
FLAGS = {"INADMISSIBLE": 1, "MEANCONSTRAINT": 2, "NAN": 4, "NOTCONVERGED": 8}


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force=True):
    """Compile the oracle (plain -O2, no FMA contraction, no fast-math), and the same source
    with OpenMP for the multi-core CPU baseline (identical arithmetic; the tests use the
    single-thread build)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    base = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared", "-Wall"]
    subprocess.check_call(base + ["-Wno-unknown-pragmas", "-o", _LIB + ".tmp", _SRC, "-lm"])
    os.replace(_LIB + ".tmp", _LIB)
    subprocess.check_call(base + ["-fopenmp", "-o", _LIB_OMP + ".tmp", _SRC, "-lm"])
    os.replace(_LIB_OMP + ".tmp", _LIB_OMP)
    return _LIB


class Cfg(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
        ("R", ctypes.c_double), ("cv", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("dissipation", ctypes.c_int), ("weno_lin", ctypes.c_double * 3), ("weno_eps", ctypes.c_double),
        ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double),
        ("monitor_kind", ctypes.c_int), ("kappa", ctypes.c_int), ("mon_var", ctypes.c_int * 2),
        ("alpha", ctypes.c_double * 3), ("n_filter", ctypes.c_int), ("mu", ctypes.c_int),
        ("mesh_tol", ctypes.c_double), ("fixed_mu", ctypes.c_int), ("walls", ctypes.c_int),
        ("step", ctypes.c_int * 2), ("inflow", ctypes.c_int), ("inflow_prim", ctypes.c_double * 4),
    ]


def make_cfg(p):
    """Build the oracle's parameter struct from a problem dict (see synth.problem)."""
    c = Cfg()
    d = int(p["dim"])
    c.dim = d
    for k in range(3):
        c.n[k] = int(p["n"][k]) if k < d else 1
        c.lo[k] = float(p["lo"][k]) if k < d else 0.0
        c.hi[k] = float(p["hi"][k]) if k < d else 1.0
        c.bc[k] = BC[p["bc"][k]] if k < d else 0
        if k < d and c.n[k] < 6:
            raise ValueError("the oracle needs at least 6 nodes per active direction")
    c.R, c.cv, c.a, c.b = (float(p[k]) for k in ("R", "cv", "a", "b"))
    c.dissipation = int(p["dissipation"])
    for i in range(3):
        c.weno_lin[i] = float(p["weno_lin"][i])
        c.alpha[i] = float(p["alpha"][i]) if i < len(p["alpha"]) else 0.0
    c.weno_eps = float(p["weno_eps"])
    c.cfl = float(p["cfl"])
    c.dt_fixed = float(p.get("dt_fixed", 0.0))
    c.monitor_kind = MONITOR[p["monitor"]]
    c.kappa = int(p["kappa"])
    for i in range(2):
        c.mon_var[i] = MONVAR[p["mon_var"][i]] if i < len(p["mon_var"]) else 0
    c.n_filter = int(p["n_filter"])
    c.mu = int(p["mu"])
    c.mesh_tol = float(p["mesh_tol"])
    c.fixed_mu = int(p["fixed_mu"])
    walls = 0
    for k, side in p.get("walls", ()):
        if BC[p["bc"][int(k)]] != BC["outflow"]:
            raise ValueError("walls are faces of outflow directions")
        walls |= 1 << (2 * int(k) + (1 if side == "hi" else 0))
    c.walls = walls
    step = p.get("step")
    if step:
        if d != 2 or any(BC[p["bc"][k]] != BC["outflow"] for k in range(2)):
            raise ValueError("the step needs a 2D problem with outflow-type directions")
        if not (3 <= step[0] and 3 <= step[1] and step[0] + 3 <= c.n[0] and step[1] + 3 <= c.n[1]):
            raise ValueError("the step needs 3 solid nodes and 3 fluid nodes beyond it in each direction")
        if not int(p["fixed_mu"]):
            raise ValueError("the step takes the fixed sweep count of the mesh iteration")
        c.step[0], c.step[1] = int(step[0]), int(step[1])
    inflow = p.get("inflow")
    if inflow is not None:
        if d != 2 or BC[p["bc"][0]] != BC["outflow"] or (walls & 1):
            raise ValueError("the inflow face is the lo face of an outflow direction 0 (2D)")
        c.inflow = 1
        for i in range(4):
            c.inflow_prim[i] = float(inflow[i])
    return c


_D = ctypes.POINTER(ctypes.c_double)
_CP = ctypes.POINTER(Cfg)


def lib(omp=False):
    """The oracle library; omp=True: the OpenMP build of the same source (CPU baseline only)."""
    if omp not in _libs:
        path = _LIB_OMP if omp else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(path)
        sig = {
            "orc_get_flags": (ctypes.c_uint, [ctypes.c_int]),
            "orc_threads": (ctypes.c_int, [ctypes.c_int]),
            "orc_T_from_rho_p": (ctypes.c_double, [_CP, ctypes.c_double, ctypes.c_double]),
            "orc_admissible": (ctypes.c_int, [_CP, ctypes.c_double, ctypes.c_double]),
            "orc_eos_state": (None, [_CP, ctypes.c_double, ctypes.c_double, _D]),
            "orc_prim_to_cons": (None, [_CP, _D, _D]),
            "orc_cons_to_prim": (None, [_CP, _D, _D]),
            "orc_entropy": (ctypes.c_double, [_CP, _D]),
            "orc_entropy_vars": (None, [_CP, _D, _D]),
            "orc_potentials": (None, [_CP, _D, _D, _D]),
            "orc_phys_flux": (None, [_CP, _D, ctypes.c_int, _D]),
            "orc_logmean": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
            "orc_ec_pair": (None, [_CP, _D, _D, _D, _D]),
            "orc_alpha": (None, [_D]),
            "orc_mrweno5": (ctypes.c_double, [_CP] + [ctypes.c_double] * 5),
            "orc_eigen": (ctypes.c_int, [_CP, ctypes.c_double, _D, ctypes.c_double, _D, _D]),
            "orc_metrics": (None, [_CP, _D, _D, _D, _D]),
            "orc_jacobian": (None, [_CP, _D, _D]),
            "orc_uniform_mesh": (None, [_CP, _D]),
            "orc_rhs": (None, [_CP, _D, _D, _D, _D, _D, _D, _D]),
            "orc_rhs_record": (None, [_CP, _D, _D, _D, _D, _D, _D, _D]),
            "orc_interface_flux": (None, [_CP, _D, _D, _D, _D, _D, _D, _D]),
            "orc_rk_stage": (None, [_CP, ctypes.c_int, ctypes.c_double, _D, _D, _D, _D, _D, _D, _D, _D]),
            "orc_cfl_dt": (ctypes.c_double, [_CP, _D, _D, _D]),
            "orc_monitor": (None, [_CP, _D, _D, _D]),
            "orc_filter": (None, [_CP, _D, ctypes.c_int]),
            "orc_jacobi": (ctypes.c_int, [_CP, _D, _D, ctypes.c_int, ctypes.c_double, _D]),
            "orc_sor": (ctypes.c_int, [_CP, _D, _D, ctypes.c_int, ctypes.c_double, _D]),
            "orc_limiter": (ctypes.c_double, [_CP, _D, _D]),
            "orc_redistribute": (None, [_CP, _D, _D, _D, _D, _D, _D, _D, _D,
                                        ctypes.POINTER(ctypes.c_int), _D, _D]),
            "orc_step": (ctypes.c_double, [_CP, _D, _D, _D, ctypes.c_int]),
            "orc_init_state": (None, [_CP, _D, _D, _D]),
            "orc_total_entropy": (ctypes.c_double, [_CP, _D, _D]),
            "orc_step_fill_state": (None, [_CP, _D, _D]),
            "orc_step_fill_scalar": (None, [_CP, _D]),
            "orc_step_fill_mesh": (None, [_CP, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[omp] = L
    return _libs[omp]


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


class Oracle:
    """Oracle bound to one problem configuration (dict from synth.problem)."""

    def __init__(self, p, omp=False):
        self.p = dict(p)
        self.c = make_cfg(p)
        self.L = lib(omp)
        self.d = int(p["dim"])
        self.nv = self.d + 2
        self.shape = tuple(int(p["n"][k]) for k in reversed(range(self.d)))  # (z, y, x)
        self.N = int(np.prod(self.shape))

    def _cp(self):
        return ctypes.byref(self.c)

    # --- pointwise functions -------------------------------------------------
    def flags(self, clear=True):
        return int(self.L.orc_get_flags(int(clear)))

    def T_from_rho_p(self, rho, p):
        return self.L.orc_T_from_rho_p(self._cp(), rho, p)

    def admissible(self, rho, T):
        return bool(self.L.orc_admissible(self._cp(), rho, T))

    def eos_state(self, rho, T):
        out = np.zeros(5)
        self.L.orc_eos_state(self._cp(), rho, T, _p(out))
        return dict(zip(("p", "e", "c2", "G", "s"), out))

    def prim_to_cons(self, prim):
        U = np.zeros(self.nv)
        self.L.orc_prim_to_cons(self._cp(), _p(_arr(prim, self.nv)), _p(U))
        return U

    def cons_to_prim(self, U):
        out = np.zeros(self.nv + 1)
        self.L.orc_cons_to_prim(self._cp(), _p(_arr(U, self.nv)), _p(out))
        return out  # rho, v..., p, T

    def entropy(self, U):
        return self.L.orc_entropy(self._cp(), _p(_arr(U, self.nv)))

    def entropy_vars(self, U):
        V = np.zeros(self.nv)
        self.L.orc_entropy_vars(self._cp(), _p(_arr(U, self.nv)), _p(V))
        return V

    def potentials(self, U):
        phi = np.zeros(1)
        psi = np.zeros(3)
        self.L.orc_potentials(self._cp(), _p(_arr(U, self.nv)), _p(phi), _p(psi))
        return phi[0], psi[: self.d].copy()

    def phys_flux(self, U, j):
        F = np.zeros(self.nv)
        self.L.orc_phys_flux(self._cp(), _p(_arr(U, self.nv)), int(j), _p(F))
        return F

    def ec_pair(self, Ul, Ur):
        Ut = np.zeros(self.nv)
        Ft = np.zeros(15)
        self.L.orc_ec_pair(self._cp(), _p(_arr(Ul, self.nv)), _p(_arr(Ur, self.nv)), _p(Ut), _p(Ft))
        return Ut, Ft.reshape(3, 5)[: self.d, : self.nv].copy()

    def mrweno5(self, w):
        return self.L.orc_mrweno5(self._cp(), *[float(v) for v in w])

    def eigen(self, rho, u, p):
        Rm = np.zeros(25)
        lam = np.zeros(5)
        ok = self.L.orc_eigen(self._cp(), rho, _p(_arr(u, self.d)), p, _p(Rm), _p(lam))
        return Rm.reshape(5, 5)[: self.nv, : self.nv].copy(), lam[: self.nv].copy(), bool(ok)

    # --- field functions -----------------------------------------------------
    def uniform_mesh(self):
        x = np.zeros((self.d,) + self.shape)
        self.L.orc_uniform_mesh(self._cp(), _p(x))
        return x

    def jacobian(self, x):
        J = np.zeros(self.shape)
        self.L.orc_jacobian(self._cp(), _p(_arr(x)), _p(J))
        return J

    def metrics(self, x, xdot=None):
        met = np.zeros((self.d * self.d,) + self.shape)
        xit = np.zeros((self.d,) + self.shape)
        self.L.orc_metrics(self._cp(), _p(_arr(x)), _p(None if xdot is None else _arr(xdot)), _p(met), _p(xit))
        return met, xit

    def step_fill_state(self, JU, J):
        """Images of the state at the solid nodes next to the step (in place)."""
        self.L.orc_step_fill_state(self._cp(), _p(JU), _p(J))

    def step_fill_scalar(self, w):
        self.L.orc_step_fill_scalar(self._cp(), _p(w))

    def step_fill_mesh(self, x):
        """Images of the mesh at the solid nodes, uniform positions at the held nodes (in place)."""
        self.L.orc_step_fill_mesh(self._cp(), _p(x))

    def init_state(self, prim, J):
        JU = np.zeros((self.nv,) + self.shape)
        self.L.orc_init_state(self._cp(), _p(_arr(prim)), _p(_arr(J)), _p(JU))
        return JU

    def rhs(self, JU, J, met, xit=None, want_prod=False):
        dJU = np.zeros((self.nv,) + self.shape)
        dJ = np.zeros(self.shape)
        prod = np.zeros(1)
        self.L.orc_rhs(self._cp(), _p(_arr(JU)), _p(_arr(J)), _p(_arr(met)),
                       _p(None if xit is None else _arr(xit)), _p(dJU), _p(dJ), _p(prod))
        return (dJU, dJ, prod[0]) if want_prod else (dJU, dJ)

    def rhs_record(self, JU, J, met, xit=None):
        """Per-interface records behind rhs(): a list over directions k of dicts with arrays of
        shape (nv,) + interface grid (n_k + 1 along k): F (entropy-stable flux), gcl (shape of the
        grid), Y (sign matrix), jw ([W]^WENO), j0 (plain jump before its zero test), scale (the
        zero test's rounding scale).  Also returns (dJU, dJ)."""
        d, nv = self.d, self.nv
        n = [int(self.p["n"][k]) for k in range(d)]
        sizes = []
        for k in range(d):
            e = list(n)
            e[k] += 1
            sizes.append(tuple(reversed(e)))
        tot = sum((5 * nv + 1) * int(np.prod(s)) for s in sizes)
        rec = np.zeros(tot)
        dJU = np.zeros((nv,) + self.shape)
        dJ = np.zeros(self.shape)
        self.L.orc_rhs_record(self._cp(), _p(_arr(JU)), _p(_arr(J)), _p(_arr(met)),
                              _p(None if xit is None else _arr(xit)), _p(dJU), _p(dJ), _p(rec))
        out, o = [], 0
        for s in sizes:
            m = int(np.prod(s))
            r = rec[o:o + (5 * nv + 1) * m].reshape((5 * nv + 1,) + s)
            o += (5 * nv + 1) * m
            out.append(dict(F=r[:nv], gcl=r[nv], Y=r[nv + 1:2 * nv + 1], jw=r[2 * nv + 1:3 * nv + 1],
                            j0=r[3 * nv + 1:4 * nv + 1], scale=r[4 * nv + 1:5 * nv + 1]))
        return out, dJU, dJ

    def interface_flux(self, st, mx, mt):
        """One interface from its 6-node stencil: st (6, nv) conserved states of nodes i-2..i+3,
        mx (6, d) their J xi_k/x_j, mt (6,) their J xi_k/t.  Returns dict(F, gcl, prod, Y, jw, j0,
        scale)."""
        nv = self.nv
        F = np.zeros(nv)
        g, pr = np.zeros(1), np.zeros(1)
        dg = np.zeros(4 * nv)
        self.L.orc_interface_flux(self._cp(), _p(_arr(st, 6 * nv)), _p(_arr(mx, 6 * self.d)), _p(_arr(mt, 6)),
                                  _p(F), _p(g), _p(pr), _p(dg))
        dg = dg.reshape(4, nv)
        return dict(F=F, gcl=g[0], prod=pr[0], Y=dg[0], jw=dg[1], j0=dg[2], scale=dg[3])

    def rk_stage(self, s, dt, JU0, J0, JUs, Js, xn, xdot=None):
        JUo = np.zeros((self.nv,) + self.shape)
        Jo = np.zeros(self.shape)
        self.L.orc_rk_stage(self._cp(), int(s), float(dt), _p(_arr(JU0)), _p(_arr(J0)), _p(_arr(JUs)),
                            _p(_arr(Js)), _p(_arr(xn)), _p(None if xdot is None else _arr(xdot)), _p(JUo), _p(Jo))
        return JUo, Jo

    def cfl_dt(self, JU, J, x):
        return self.L.orc_cfl_dt(self._cp(), _p(_arr(JU)), _p(_arr(J)), _p(_arr(x)))

    def monitor(self, JU, J):
        w = np.zeros(self.shape)
        self.L.orc_monitor(self._cp(), _p(_arr(JU)), _p(_arr(J)), _p(w))
        return w

    def filter(self, omega, npass):
        w = _arr(omega).copy()
        self.L.orc_filter(self._cp(), _p(w), int(npass))
        return w

    def jacobi(self, omega, x, nsweep, tol=0.0):
        xx = _arr(x).copy()
        res = np.zeros(1)
        it = self.L.orc_jacobi(self._cp(), _p(_arr(omega)), _p(xx), int(nsweep), float(tol), _p(res))
        return xx, it, res[0]

    def sor(self, omega, x, nsweep, relax=1.0):
        """Red-black SOR sweeps (Gauss-Seidel for relax = 1); returns (x, resid).  Raises for a
        periodic direction with an odd node count."""
        xx = _arr(x).copy()
        res = np.zeros(1)
        it = self.L.orc_sor(self._cp(), _p(_arr(omega)), _p(xx), int(nsweep), float(relax), _p(res))
        if it < 0:
            raise ValueError("red-black ordering needs an even node count in periodic directions")
        return xx, res[0]

    def limiter(self, xn, xmu):
        return self.L.orc_limiter(self._cp(), _p(_arr(xn)), _p(_arr(xmu)))

    def redistribute(self, JU, J, xn, warm_dx=None):
        xdot = np.zeros((self.d,) + self.shape)
        dt, gam, res = np.zeros(1), np.zeros(1), np.zeros(1)
        sw = ctypes.c_int(0)
        omega = np.zeros(self.shape)
        xmu = np.zeros((self.d,) + self.shape)
        self.L.orc_redistribute(self._cp(), _p(_arr(JU)), _p(_arr(J)), _p(_arr(xn)),
                                _p(None if warm_dx is None else _arr(warm_dx)), _p(xdot), _p(dt), _p(gam),
                                _p(res), ctypes.byref(sw), _p(omega), _p(xmu))
        return dict(xdot=xdot, dt=dt[0], gamma=gam[0], resid=res[0], sweeps=sw.value, omega=omega, xmu=xmu)

    def step(self, JU, J, x, moving=True):
        """One full time step in place on copies; returns (JU, J, x, dt)."""
        JU, J, x = _arr(JU).copy(), _arr(J).copy(), _arr(x).copy()
        dt = self.L.orc_step(self._cp(), _p(JU), _p(J), _p(x), int(bool(moving)))
        return JU, J, x, dt

    def total_entropy(self, JU, J):
        return self.L.orc_total_entropy(self._cp(), _p(_arr(JU)), _p(_arr(J)))


def alpha():
    out = np.zeros(3)
    lib().orc_alpha(_p(out))
    return out
