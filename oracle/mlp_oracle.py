"""FP64 reference of the learned mesh warm start (TEST INFRASTRUCTURE: only tests, the smoke
check and the CPU-baseline leg of the benchmark use this module).

The network is a 50 -> 64 -> 64 -> 2 ReLU MLP on the 5 x 5 stencil of two node features:
f1 = |grad_xi rho|^2 / max |grad_xi rho|^2 (second-order central differences, boundary values
replicated or wrapped, as in the monitor of Section 4 of the paper) and f2 = tanh G (the
fundamental derivative, eq. fundamental).  The GPU path computes matrix products on BF16
operands with FP32 accumulation; this reference rounds the same operands to BF16 (round to
nearest even) and accumulates in FP64, so the two agree up to the accumulation order and the
rare BF16 rounding decision that falls on the other side.

Parameters are one flat FP64 vector in the library's packing: W1[64][64] (inputs 50..63 zero),
b1[64], W2[64][64], b2[64], W3[64][16] (outputs 2..15 zero), b3[16]; W[k][j] maps input k to
output j.
"""
import numpy as np

N_IN, N_H, N_OUT = 50, 64, 2
SLICES = {}
_o = 0
for _name, _shape in (("W1", (64, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 16)),
                      ("b3", (16,))):
    _n = int(np.prod(_shape))
    SLICES[_name] = (_o, _o + _n, _shape)
    _o += _n
NPARAM = _o  # 9360


def unpack(P):
    return {k: np.asarray(P[a:b], dtype=np.float64).reshape(s) for k, (a, b, s) in SLICES.items()}


def pack(d):
    P = np.zeros(NPARAM)
    for k, (a, b, s) in SLICES.items():
        P[a:b] = np.asarray(d[k], dtype=np.float64).reshape(-1)
    return P


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(seed):
    """He-style random initialisation (weights ~ N(0, 2/fan_in)), zero biases, zero paddings."""
    rng = np.random.default_rng(seed)
    d = {"W1": np.zeros((64, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, 16)), "b3": np.zeros(16)}
    d["W1"][:N_IN] = rng.normal(scale=np.sqrt(2.0 / N_IN), size=(N_IN, 64))
    d["W2"][:] = rng.normal(scale=np.sqrt(2.0 / 64), size=(64, 64))
    d["W3"][:, :N_OUT] = rng.normal(scale=np.sqrt(1.0 / 64), size=(64, N_OUT))
    return pack(d)


def features_from_fields(rho, G, dxi, bc):
    """f1 = |grad_xi rho|^2 / max, f2 = tanh G for fields of shape (ny, nx)."""
    def ext(f, axis, mode):
        if mode == "periodic":
            return np.roll(f, -1, axis), np.roll(f, 1, axis)
        p = np.concatenate([np.take(f, range(1, f.shape[axis]), axis), np.take(f, [-1], axis)], axis)
        m = np.concatenate([np.take(f, [0], axis), np.take(f, range(0, f.shape[axis] - 1), axis)], axis)
        return p, m
    gx_p, gx_m = ext(rho, 1, bc[0])
    gy_p, gy_m = ext(rho, 0, bc[1])
    gx = (gx_p - gx_m) / (2 * dxi[0])
    gy = (gy_p - gy_m) / (2 * dxi[1])
    t = gx * gx + gy * gy
    m = t.max()
    f1 = t / m if m > 0 else np.zeros_like(t)
    return f1, np.tanh(G)


def stencil(f1, f2, i0, i1, bc):
    """The 50 inputs of node (i0, i1): for dy, dx in -2..2 the pair (f1, f2) of the neighbour,
    indices replicated (outflow) or wrapped (periodic) at the boundary."""
    ny, nx = f1.shape
    out = np.zeros(N_IN)
    k = 0
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            a, b = i0 + dx, i1 + dy
            a = a % nx if bc[0] == "periodic" else min(max(a, 0), nx - 1)
            b = b % ny if bc[1] == "periodic" else min(max(b, 0), ny - 1)
            out[k], out[k + 1] = f1[b, a], f2[b, a]
            k += 2
    return out


def forward(P, X, quantize=True):
    """X: (B, 50).  Returns y (B, 2) and the intermediate values for the backward pass."""
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    p = unpack(P)
    Xq = q(np.pad(X, ((0, 0), (0, 64 - N_IN))))
    W1, W2, W3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    a1 = Xq @ W1 + p["b1"]
    h1 = q(np.maximum(a1, 0.0))
    a2 = h1 @ W2 + p["b2"]
    h2 = q(np.maximum(a2, 0.0))
    y = h2 @ W3 + p["b3"]
    return y[:, :N_OUT], (Xq, h1, h2, W1, W2, W3, y)


def loss_and_grad(P, X, T, scale, quantize=True):
    """loss = scale * sum |y - t|^2 and its gradient with respect to P (same packing)."""
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    y, (Xq, h1, h2, W1, W2, W3, yfull) = forward(P, X, quantize)
    e = y - T
    loss = scale * float((e * e).sum())
    dY = np.zeros((X.shape[0], 16))
    dY[:, :N_OUT] = 2.0 * scale * e
    dY = q(dY)
    g = {"W3": h2.T @ dY, "b3": dY.sum(0)}
    dH2 = q((dY @ W3.T) * (h2 > 0))
    g["W2"], g["b2"] = h1.T @ dH2, dH2.sum(0)
    dH1 = q((dH2 @ W2.T) * (h1 > 0))
    g["W1"], g["b1"] = Xq.T @ dH1, dH1.sum(0)
    g["W1"][N_IN:] = 0.0
    g["W3"][:, N_OUT:] = 0.0
    g["b3"][N_OUT:] = 0.0
    return loss, pack(g)


def adam(P, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), returns new (P, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v
