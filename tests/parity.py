"""Per-node parity bar shared by the GPU tests.

The scheme is not equally well conditioned everywhere: the nonlinear MR-WENO weights and the
sign test of the dissipation amplify rounding differences at some nodes by orders of
magnitude more than at others.  A single global allowance derived from the worst node would
let a local kernel error of that size pass anywhere, so the bar is set node by node:

  * the oracle is run again on inputs perturbed by one unit in the last place (random signs,
    several seeds); s[v, i] = max over seeds of |perturbed - reference| / max |reference[v]| is
    the oracle's own sensitivity at node i of field v;
  * the GPU must satisfy |gpu - reference| / max |reference[v]| <= max(bar, 8 s[v, i]) at every
    node;
  * the literal bar therefore binds at every node where 8 s <= bar; the others ("excluded"
    nodes) are bounded by their own sensitivity, and their share is reported.

`record()` prints one line per check and, if the environment names a file in PARITY_LOG,
appends the same numbers to it as JSON (the per-case table of the design notes is made from
that log)."""
import json
import os

import numpy as np

ULP = 2.0 ** -52
FACTOR = 8.0


def perturb(a, seed):
    """a with every element moved by one unit in the last place (relative), random signs."""
    rng = np.random.default_rng(seed)
    return a * (1.0 + ULP * rng.choice([-1.0, 1.0], size=np.shape(a)))


def _fields(a):
    a = np.asarray(a, dtype=np.float64)
    return a.reshape(a.shape[0], -1) if a.ndim > 1 else a.reshape(1, -1)


def sensitivity(ref, perturbed):
    """Per field and node: max over the perturbed runs of |p - ref| / max |ref[field]|."""
    r = _fields(ref)
    sc = np.abs(r).max(axis=1, keepdims=True)
    sc[sc == 0] = 1.0
    s = np.zeros_like(r)
    for p in perturbed:
        s = np.maximum(s, np.abs(_fields(p) - r) / sc)
    return s


def check(name, gpu, ref, perturbed, bar, per_field=False):
    """Assert the per-node bar; returns the numbers it records.  per_field=True: each node of a
    field is allowed 8 times that field's largest sensitivity (for runs whose switches spread
    over the whole grid within the run, see the spherical shock test)."""
    r = _fields(ref)
    g = _fields(gpu).reshape(r.shape)
    sc = np.abs(r).max(axis=1, keepdims=True)
    sc[sc == 0] = 1.0
    e = np.abs(g - r) / sc
    s = sensitivity(ref, perturbed)
    if per_field:
        s = np.broadcast_to(s.max(axis=1, keepdims=True), s.shape)
    tol = np.maximum(bar, FACTOR * s)
    excl = FACTOR * s > bar
    rec = dict(case=name, bar=bar, per_field=per_field, err_max=float(e.max()),
               err_max_bound=float(e[~excl].max()) if (~excl).any() else 0.0,
               excluded=float(excl.mean()), err_max_excluded=float(e[excl].max()) if excl.any() else 0.0,
               kappa=float(s.max()), worst_ratio=float((e / tol).max()), nodes=int(r.shape[1]),
               within_bar=float((e <= bar).mean()))
    print("parity %(case)s: err %(err_max).3e (bound nodes %(err_max_bound).3e <= %(bar).0e), excluded %(excluded).4f "
          "(their err %(err_max_excluded).3e), within the bar %(within_bar).4f, kappa %(kappa).3e, worst err/tol "
          "%(worst_ratio).3f" % rec, flush=True)
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")
    bad = np.argwhere(e > tol)
    assert bad.size == 0, ("%s: %d node-fields beyond the per-node bar, e.g. (field, node) %s: err %.3e tol %.3e"
                           % (name, len(bad), bad[0].tolist(), e[tuple(bad[0])], tol[tuple(bad[0])]))
    return rec
