"""FP64 reference of the surrogate network and its loss (test infrastructure).

Network: hidden layers h = silu(h W^T + b), silu(z) = z / (1 + exp(-z)); a
linear output layer with two heads, mu (log of the weight ratio) and s (log
of the error of mu).  Loss over n rows with targets y:

  L = 1/n sum_r [ 1/2 (y_r - mu_r)^2 + lambda (1/2 r_r^2 exp(-2 s_r) + s_r) ]

with r_r = y_r - mu_r held fixed in the second term (its gradient reaches s
only) and s clamped below at -15 (zero gradient there).  Targets may be
standardised first, y -> (y - y_mean) / y_std (``scale``); the heads are then
in standardised units.  Parameters are a list of (W [out][in], b [out]).

Input features of one (event, card) pair (``phys_features``): with the
momenta p_0..p_{n-1} (two incoming first, all massless), s_hat = 2 p_0.p_1
and s_ij = 2 p_i.p_j,
  [log s_hat, log(s_ij / s_hat) for i < j (row-major), M_Z, Gamma_Z,
   sin^2 theta_W, asinh Re chi, asinh Im chi, asinh Re chi_0, asinh Im chi_0]
where chi = s / (s - M_Z^2 + i M_Z Gamma_Z) is the Z propagator relative to
the photon's at the invariant mass s = s_ab of the resonant pair (a, b),
under the card (chi) and under the original card (chi_0).  ``raw_features``
is the plain [momenta (n*4), M_Z, Gamma_Z, sin^2 theta_W] row.

Training updates every parameter by Adam (Kingma and Ba, ICLR 2015, their
Algorithm 1): with gradient g at step t = 1, 2, ...
  m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
  theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
(``adam_step``).  The calibration factor k of the error head is the
``coverage`` quantile of |y - mu| / exp(s) over held-out pairs, the quantile
taken with linear interpolation between order statistics (Hyndman and Fan's
definition 7: position (n - 1) q of the sorted values) (``calibration_k``).

A BF16 network (the surrogate's precision: BF16 weights, FP32 sums) is
evaluated by ``forward_bf16``: its width x width layers take BF16-rounded
weights and BF16-rounded input activations (the operands of a BF16 product);
the first layer, the head and every sum stay in full precision.

Pinned (tests/test_oracle_mlp.py) by central finite differences of L,
hand-computed two-layer networks (forward values and loss at activations
where SiLU has closed forms), closed forms of Adam under constant and
alternating gradients, order statistics of small samples, BF16
rounding by hand-rounded values, the BF16 network by a hand-computed
three-layer case, and the features by momentum conservation, a direct (p_i + p_j)^2 and the propagator's pole
and high-energy limits.
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


def bf16(x):
    """Nearest bfloat16 value (8 significant bits, ties to even) of each
    element, returned as float64: x = m 2^e with 1/2 <= |m| < 1, the
    significand m 2^8 rounded to the nearest integer (half to even)."""
    m, e = np.frexp(np.asarray(x, dtype=np.float64))
    return np.ldexp(np.rint(m * 256.0), e - 8)


def forward_bf16(params, x):
    """Heads of the network with BF16 hidden layers: every width x width layer
    (all but the first and the head) multiplies BF16-rounded weights by
    BF16-rounded input activations; the first layer and the head keep their
    weights and inputs as given; every sum, bias and activation is exact
    (FP64 here)."""
    h = np.asarray(x, dtype=np.float64)
    last = len(params) - 1
    for i, (w, b) in enumerate(params):
        if 0 < i < last:
            w, h = bf16(w), bf16(h)
        z = h @ np.asarray(w, np.float64).T + b
        h = silu(z) if i < last else z
    return h


def raw_features(p, cards):
    """[n][npart*4 + 3] rows from momenta p [n][npart][4] and cards [n][3]."""
    p = np.asarray(p, dtype=np.float64)
    return np.concatenate([p.reshape(p.shape[0], -1), np.asarray(cards, dtype=np.float64)], axis=1)


def _mdot(a, b):
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def phys_features(p, cards, res, orig):
    """Physics features (module docstring) of momenta p [n][npart][4] with
    cards [n][3] = (M_Z, Gamma_Z, sin^2 theta_W); res = (a, b) the resonant
    pair; orig = (M_Z, Gamma_Z) of the original card."""
    p = np.asarray(p, dtype=np.float64)
    cards = np.asarray(cards, dtype=np.float64)
    npart = p.shape[1]
    s_hat = 2.0 * _mdot(p[:, 0], p[:, 1])
    cols = [np.log(s_hat)]
    for i in range(npart):
        for j in range(i + 1, npart):
            cols.append(np.log(np.maximum(np.abs(2.0 * _mdot(p[:, i], p[:, j])) / s_hat, 1e-300)))
    cols += [cards[:, 0], cards[:, 1], cards[:, 2]]
    s = 2.0 * _mdot(p[:, res[0]], p[:, res[1]])
    for mz, wz in ((cards[:, 0], cards[:, 1]), (orig[0], orig[1])):
        chi = s / (s - mz * mz + 1j * mz * wz)
        cols += [np.arcsinh(chi.real), np.arcsinh(chi.imag)]
    return np.stack(cols, axis=1)


def n_phys_features(npart):
    return 1 + npart * (npart - 1) // 2 + 3 + 4


def loss(params, x, y, lam, scale=(0.0, 1.0)):
    y = (np.asarray(y, dtype=np.float64) - scale[0]) / scale[1]
    heads, _ = forward(params, x)
    mu, s_raw = heads[:, 0], heads[:, 1]
    s = np.maximum(s_raw, S_MIN)
    r = y - mu
    return float(np.mean(0.5 * r * r + lam * (0.5 * r * r * np.exp(-2 * s) + s)))


def gradients(params, x, y, lam, scale=(0.0, 1.0)):
    """d loss / d (W, b) for every layer (the r held fixed in the error term)."""
    y = (np.asarray(y, dtype=np.float64) - scale[0]) / scale[1]
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


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam step number t (t >= 1) on flat arrays; returns (theta, m, v)."""
    theta, g = np.asarray(theta, np.float64), np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def quantile_linear(values, q):
    """Order-statistic quantile: sort, then interpolate linearly at position
    (n - 1) q between the two neighbouring order statistics."""
    x = np.sort(np.asarray(values, np.float64).ravel())
    h = (x.size - 1) * q
    lo = int(np.floor(h))
    hi = min(lo + 1, x.size - 1)
    return float(x[lo] + (h - lo) * (x[hi] - x[lo]))


def calibration_k(y, mu, s, coverage):
    """Calibration factor k: the coverage quantile of |y - mu| / exp(s)."""
    z = np.abs(np.asarray(y, np.float64) - np.asarray(mu, np.float64)) / np.exp(np.asarray(s, np.float64))
    return quantile_linear(z, coverage)


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
