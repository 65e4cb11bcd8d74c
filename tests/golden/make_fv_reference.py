"""Writes the stored reference solutions fv_*.txt with the second-order finite-volume solver of
oracle/fv_reference.py at 10 000 cells (reduced units, delta = 0.0125), as the paper computes
its references (Example 5.2; Example 5.7 in 1D spherical coordinates):

- fv_rp1.txt, fv_rp2.txt, fv_rp3.txt: Table 5.1's shock tubes on [0, 1] split at 0.5, at
  t = 0.15, 0.45 and 0.2 (the paper's t Z_c^{-1/2} is t in reduced units);
- fv_sphere.txt: Example 5.7's sphere (RP1 inside r < 0.5) on r in [0, 2], at t = 0.2 in the
  paper's unit = 0.2 sqrt(3/8) in reduced units.

Columns: x (or r), rho, v, p at every 10th cell centre.  Run from the repository root:
    python tests/golden/make_fv_reference.py
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fv_reference as fv  # noqa: E402
from paper_2407_05568_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
T_END = {"rp1": 0.15, "rp2": 0.45, "rp3": 0.2}


def save(name, x, rho, v, p, note):
    a = np.stack([x, rho, v, p], axis=1)[5::10]
    np.savetxt(os.path.join(HERE, "fv_%s.txt" % name), a, fmt="%.17g",
               header="%s; columns x rho v p at every 10th of 10000 cells" % note)


def main(which):
    u = synth.units("reduced")
    eos = fv.VdW(u["R"], u["cv"], u["a"], u["b"])
    for name in which:
        if name == "sphere":
            t = 0.2 * math.sqrt(3.0 / 8.0)
            rp = synth.TABLE_5_1["RP1"]
            x, rho, v, p = fv.riemann(eos, rp[0], rp[1], t, n=10000, lo=0.0, hi=2.0, x0=0.5, geometry="spherical")
            save(name, x, rho, v, p, "Example 5.7 sphere, 1D spherical FV, t = %.17g (reduced)" % t)
        else:
            rp = synth.TABLE_5_1[name.upper()]
            x, rho, v, p = fv.riemann(eos, rp[0], rp[1], T_END[name], n=10000)
            save(name, x, rho, v, p, "Table 5.1 %s, planar FV, t = %g (reduced)" % (name.upper(), T_END[name]))
        print("wrote fv_%s.txt" % name, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["rp1", "rp2", "rp3", "sphere"])
