"""Pins of the FP64 reference of the learned warm start (oracle/mlp_oracle.py)."""
import numpy as np

from oracle import mlp_oracle as mo


def test_bf16_rounding():
    """Round to nearest even at 8 significand bits: exact values stay, halfway cases go to even."""
    assert mo.bf16(1.0) == 1.0
    assert mo.bf16(1.0 + 2 ** -8) == 1.0          # halfway, even neighbour is 1.0
    assert mo.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # halfway, even neighbour is up
    assert mo.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    x = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(mo.bf16(x) - x) <= 2 ** -8 * np.abs(x))


def test_gradient_matches_finite_differences():
    """Backward pass (unquantised) against central differences of the loss."""
    rng = np.random.default_rng(1)
    P = mo.init_params(3)
    P[mo.SLICES["b1"][0]:mo.SLICES["b1"][1]] = rng.normal(scale=0.1, size=64)
    X = rng.normal(size=(7, mo.N_IN))
    T = rng.normal(size=(7, 2))
    loss, g = mo.loss_and_grad(P, X, T, 0.25, quantize=False)
    idx = np.concatenate([rng.choice(np.arange(a, b), 12, replace=False) for (a, b, s) in mo.SLICES.values()])
    for i in idx:
        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mo.loss_and_grad(Pp, X, T, 0.25, quantize=False)[0] - mo.loss_and_grad(Pm, X, T, 0.25, quantize=False)[0]) / (2 * h)
        # padded rows/columns are outside the model: their analytic gradient is defined as 0
        a, b, s = mo.SLICES["W1"]
        if a <= i < b and (i - a) // 64 >= mo.N_IN:
            continue
        a, b, s = mo.SLICES["W3"]
        if a <= i < b and (i - a) % 16 >= 2:
            continue
        a, b, s = mo.SLICES["b3"]
        if a <= i < b and (i - a) >= 2:
            continue
        assert abs(fd - g[i]) < 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_adam_first_step_moves_by_lr():
    """At step 1 the bias-corrected Adam update is lr * sign(g) (for |g| >> eps)."""
    P = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.1])
    P1, m, v = mo.adam(P, g, np.zeros(5), np.zeros(5), 1, 0.01)
    assert np.allclose(P1, -0.01 * np.sign(g), atol=1e-9)


def test_stencil_layout_and_boundary():
    f1 = np.arange(30.0).reshape(5, 6)
    f2 = -f1
    s = mo.stencil(f1, f2, 0, 0, ("outflow", "outflow"))
    assert s[0] == f1[0, 0] and s[1] == f2[0, 0]          # (dy, dx) = (-2, -2) clamps to (0, 0)
    assert s[24] == f1[0, 0] and s[25] == f2[0, 0]        # centre
    assert s[26] == f1[0, 1]                               # (0, +1)
    s = mo.stencil(f1, f2, 5, 4, ("periodic", "periodic"))
    assert s[48] == f1[(4 + 2) % 5, (5 + 2) % 6]
