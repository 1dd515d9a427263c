"""Pin of the FP64 reference network: analytic gradients of the loss against
central finite differences (including the error-head term with its held-fixed
residual, which the finite difference reproduces by holding r fixed)."""
import numpy as np

from oracle import mlp


def _net(seed=0, n_in=7, width=6, depth=2):
    rng = np.random.default_rng(seed)
    shapes = [(width, n_in)] + [(width, width)] * (depth - 1) + [(2, width)]
    params = [(rng.normal(size=s) / np.sqrt(s[1]), rng.normal(size=s[0]) * 0.1) for s in shapes]
    return params, shapes, rng


def _loss_fixed_r(params, x, y, lam, r_fixed):
    heads, _ = mlp.forward(params, x)
    mu, s = heads[:, 0], np.maximum(heads[:, 1], mlp.S_MIN)
    r = y - mu
    return float(np.mean(0.5 * r * r + lam * (0.5 * r_fixed * r_fixed * np.exp(-2 * s) + s)))


def test_gradients_match_finite_differences():
    params, shapes, rng = _net()
    x = rng.normal(size=(9, 7))
    y = rng.normal(size=9) * 0.3
    lam = 0.25
    heads, _ = mlp.forward(params, x)
    r_fixed = y - heads[:, 0]
    flat = mlp.pack(params)
    grads = mlp.pack(mlp.gradients(params, x, y, lam))
    eps = 1e-6
    fd = np.zeros_like(flat)
    for i in range(flat.size):
        up, dn = flat.copy(), flat.copy()
        up[i] += eps
        dn[i] -= eps
        fd[i] = (_loss_fixed_r(mlp.unpack(up, shapes), x, y, lam, r_fixed)
                 - _loss_fixed_r(mlp.unpack(dn, shapes), x, y, lam, r_fixed)) / (2 * eps)
    np.testing.assert_allclose(grads, fd, rtol=1e-6, atol=1e-9)


def test_silu_derivative_and_loss_value():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), rtol=1e-8, atol=1e-10)
    params, shapes, rng = _net(1)
    x = rng.normal(size=(5, 7))
    y = rng.normal(size=5)
    heads, _ = mlp.forward(params, x)
    mu, s = heads[:, 0], heads[:, 1]
    want = np.mean(0.5 * (y - mu) ** 2 + 0.5 * (0.5 * (y - mu) ** 2 * np.exp(-2 * s) + s))
    assert abs(mlp.loss(params, x, y, 0.5) - want) < 1e-14


def test_error_head_clamp_stops_gradient():
    params, shapes, rng = _net(2)
    w, b = params[-1]
    params[-1] = (w * 0, np.array([0.0, -20.0]))      # s = -20 < -15 everywhere
    x = rng.normal(size=(4, 7))
    g = mlp.gradients(params, x, np.ones(4), 1.0)
    assert np.all(g[-1][1][1] == 0.0) and np.all(g[-1][0][1] == 0.0)
