"""Host-side checks of the C ABI: the library loads and exports every entry point that
include/esvdw.h declares, and the binding's parameter struct matches the header's layout.
No compute call is made here (no GPU)."""
import os
import re

from paper_2407_05568_amd import esvdw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "esvdw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+char\s*\*|int\s|long\s|void\s)\s*\*?(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_and_binding_agree():
    assert sorted(esvdw.SYMBOLS) == _declared()


def test_library_exports_every_declared_symbol():
    L = esvdw.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_params_struct_layout():
    # dim, n[3], lo[3], hi[3], bc[3], R, cv, a, b, dissipation, weno_lin[3], weno_eps, cfl, dt_fixed,
    # monitor_kind, kappa, mon_var[2], alpha[3], n_filter, mu, mesh_tol, fixed_mu, walls, step[2],
    # inflow, inflow_prim[4] (natural alignment)
    import ctypes
    P = esvdw.Params
    assert P.n.offset == 4 and P.lo.offset == 16 and P.bc.offset == 64
    assert P.R.offset == 80 and P.dissipation.offset == 112 and P.weno_lin.offset == 120
    assert P.fixed_mu.offset == 224 and P.walls.offset == 228 and P.step.offset == 232
    assert P.inflow.offset == 240 and P.inflow_prim.offset == 248 and ctypes.sizeof(P) == 280
