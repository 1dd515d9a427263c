"""FP64 reference of the surrogate network and its loss (test infrastructure).

Network: hidden layers h = silu(h W^T + b), silu(z) = z / (1 + exp(-z)); a
linear output layer with two heads, mu (log of the weight ratio) and s (log
of the error of mu).  Loss over n rows with targets y:

  L = 1/n sum_r [ 1/2 (y_r - mu_r)^2 + lambda (1/2 r_r^2 exp(-2 s_r) + s_r) ]

with r_r = y_r - mu_r held fixed in the second term (its gradient reaches s
only) and s clamped below at -15 (zero gradient there).  Parameters are a list
of (W [out][in], b [out]).

Pinned by central finite differences of L (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

S_MIN = -15.0


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """Returns the heads [n][n_out] and the per-layer (input, pre-activation)."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for i, (w, b) in enumerate(params):
        z = h @ w.T + b
        cache.append((h, z))
        h = silu(z) if i + 1 < len(params) else z
    return h, cache


def loss(params, x, y, lam):
    heads, _ = forward(params, x)
    mu, s_raw = heads[:, 0], heads[:, 1]
    s = np.maximum(s_raw, S_MIN)
    r = y - mu
    return float(np.mean(0.5 * r * r + lam * (0.5 * r * r * np.exp(-2 * s) + s)))


def gradients(params, x, y, lam):
    """d loss / d (W, b) for every layer (the r held fixed in the error term)."""
    heads, cache = forward(params, x)
    n = heads.shape[0]
    mu, s_raw = heads[:, 0], heads[:, 1]
    s = np.maximum(s_raw, S_MIN)
    r = y - mu
    g = np.zeros_like(heads)
    g[:, 0] = -r / n
    g[:, 1] = np.where(s_raw > S_MIN, lam * (1.0 - r * r * np.exp(-2 * s)) / n, 0.0)
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        h, z = cache[i]
        w, _ = params[i]
        grads[i] = (g.T @ h, g.sum(axis=0))
        if i > 0:
            g = (g @ w) * silu_grad(cache[i - 1][1])
    return grads


def pack(params):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params])


def unpack(flat, shapes):
    out, off = [], 0
    for n_out, n_in in shapes:
        w = flat[off:off + n_out * n_in].reshape(n_out, n_in)
        off += n_out * n_in
        b = flat[off:off + n_out]
        off += n_out
        out.append((w, b))
    return out
