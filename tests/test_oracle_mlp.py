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


def _two_to_two(e, cos_t, phi=0.3):
    """Massless 2 -> 2 in the centre-of-mass frame, beam energy e."""
    sin_t = np.sqrt(1 - cos_t * cos_t)
    n = np.array([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t])
    return np.array([[[e, 0, 0, e], [e, 0, 0, -e], [e, *(e * n)], [e, *(-e * n)]]])


def test_phys_features_closed_form_two_to_two():
    """s = 4E^2, -t = 2E^2 (1 - cos), -u = 2E^2 (1 + cos), in row-major pair
    order (01, 02, 03, 12, 13, 23), then the card, then chi at s_23 = s."""
    e, c = 45.0, 0.35
    card = np.array([[91.0, 2.5, 0.23]])
    f = mlp.phys_features(_two_to_two(e, c), card, (2, 3), (91.0, 2.5))[0]
    assert f.size == mlp.n_phys_features(4) == 14
    want_pairs = np.log([1.0, (1 - c) / 2, (1 + c) / 2, (1 + c) / 2, (1 - c) / 2, 1.0])
    np.testing.assert_allclose(f[0], np.log(4 * e * e), rtol=1e-14)
    np.testing.assert_allclose(f[1:7], want_pairs, rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(f[7:10], card[0])


def test_phys_features_propagator_limits():
    mz, wz = 91.1876, 2.4952
    # on the pole (s_23 = M_Z^2): chi = -i M / Gamma
    f = mlp.phys_features(_two_to_two(mz / 2, -0.2), [[mz, wz, 0.22]], (2, 3), (mz, wz))[0]
    np.testing.assert_allclose(f[10], 0.0, atol=1e-12)
    np.testing.assert_allclose(f[11], np.arcsinh(-mz / wz), rtol=1e-12)
    np.testing.assert_allclose(f[12:14], f[10:12], rtol=1e-14, atol=1e-14)
    # far above the pole chi -> 1, and a different original card moves only chi_0
    g = mlp.phys_features(_two_to_two(1e6, 0.5), [[mz, wz, 0.22]], (2, 3), (90.0, 3.0))[0]
    np.testing.assert_allclose(g[10], np.arcsinh(1.0), rtol=1e-6)
    assert abs(g[11]) < 1e-6 and abs(g[13]) < 1e-6


def test_phys_features_momentum_conservation():
    """Outgoing i: s_0i + s_1i = sum_{j out, j != i} s_ij; sum of outgoing
    pairs = s_hat; every s_ij equals (p_i + p_j)^2 of the summed vector."""
    import synth
    p = synth.events("uu_eeg", 50)
    card = np.tile([91.5, 2.6, 0.2312], (50, 1))
    f = mlp.phys_features(p, card, (2, 3), (91.188, 2.441))
    s_hat = np.exp(f[:, 0])
    pairs = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    s = {pr: np.exp(f[:, 1 + k]) * s_hat for k, pr in enumerate(pairs)}
    for i in range(2, 5):
        rhs = sum(s[tuple(sorted((i, j)))] for j in range(2, 5) if j != i)
        np.testing.assert_allclose(s[(0, i)] + s[(1, i)], rhs, rtol=1e-10)
    np.testing.assert_allclose(sum(s[(i, j)] for i, j in pairs if i >= 2), s_hat, rtol=1e-10)
    for (i, j), v in s.items():
        q = p[:, i] + p[:, j]
        np.testing.assert_allclose(v, q[:, 0] ** 2 - (q[:, 1:] ** 2).sum(axis=1), rtol=1e-8)


def test_target_scale_is_a_change_of_units():
    """Standardising the targets equals training on (y - m) / s directly."""
    params, shapes, rng = _net(3)
    x = rng.normal(size=(6, 7))
    y = rng.normal(size=6) * 0.05 + 0.01
    a = mlp.gradients(params, x, y, 0.2, scale=(0.01, 0.05))
    b = mlp.gradients(params, x, (y - 0.01) / 0.05, 0.2)
    for (wa, ba), (wb, bb) in zip(a, b):
        np.testing.assert_allclose(wa, wb, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(ba, bb, rtol=1e-13, atol=1e-15)
