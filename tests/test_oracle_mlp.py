"""Pins of the FP64 reference network and its training arithmetic: analytic
gradients of the loss against central finite differences (including the
error-head term with its held-fixed residual, which the finite difference
reproduces by holding r fixed); forward values and losses of hand-computed
two-layer networks; Adam against its closed forms under constant and
alternating gradients and its scale invariance; the calibration quantile
against order statistics."""
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


def _hand_net():
    """A 3 -> 2 -> 2 network with integer weights: W1 [2][3], W2 [2][2]
    (not symmetric, so a transposed operand changes the result)."""
    w1 = np.array([[1.0, 0.0, 2.0], [0.0, 1.0, -1.0]])
    w2 = np.array([[2.0, 4.0], [1.0, 0.0]])
    return [(w1, np.zeros(2)), (w2, np.array([0.5, -1.0]))]


def test_forward_hand_computed_two_layers():
    """Rows chosen so that every hidden pre-activation is +-ln 3, ln 2 or
    -ln 2 / 2, where SiLU has closed forms: silu(ln 3) = (3/4) ln 3,
    silu(-ln 3) = -(1/4) ln 3, silu(ln 2) = (2/3) ln 2,
    silu(-ln 2 / 2) = -(ln 2 / 2)(sqrt 2 - 1)."""
    l2, l3, r2 = np.log(2.0), np.log(3.0), np.sqrt(2.0)
    x = np.array([[l3, -l3, 0.0], [0.0, 0.0, l2 / 2]])
    heads, cache = mlp.forward(_hand_net(), x)
    # row 0: h = (3/4 ln 3, -1/4 ln 3); row 1: h = (2/3 ln 2, -(ln 2/2)(sqrt 2 - 1))
    want = np.array([[0.5 * l3 + 0.5, 0.75 * l3 - 1.0],
                     [l2 * (10.0 / 3.0 - 2.0 * r2) + 0.5, (2.0 / 3.0) * l2 - 1.0]])
    np.testing.assert_allclose(heads, want, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(cache[1][0], [[0.75 * l3, -0.25 * l3], [2 * l2 / 3, -(l2 / 2) * (r2 - 1)]],
                               rtol=1e-15, atol=1e-15)


def test_loss_hand_computed():
    """Constant heads (zero last-layer weights, biases (mu, s)): with
    y = (1, 0), mu = 0.5, s = ln 2 every row has r^2 = 1/4 and
    exp(-2 s) = 1/4, so L = 1/8 + lambda (1/32 + ln 2); s = -20 is clamped
    to -15; standardised targets (y - 0.5) / 2 = (1/4, -1/4) with mu = s = 0
    give L = 1/32 (1 + lambda)."""
    net = _hand_net()
    x = np.array([[0.3, -0.2, 0.1], [1.0, 2.0, -3.0]])
    const = lambda mu, s: [net[0], (np.zeros((2, 2)), np.array([mu, s]))]   # noqa: E731
    lam = 0.1
    assert abs(mlp.loss(const(0.5, np.log(2.0)), x, [1.0, 0.0], lam) - (0.125 + lam * (1 / 32 + np.log(2.0)))) < 1e-15
    want = 0.125 + lam * (0.125 * np.exp(30.0) - 15.0)
    assert abs(mlp.loss(const(0.5, -20.0), x, [1.0, 0.0], lam) / want - 1.0) < 1e-15
    # y' = (0.25, -0.25) with mu = 0, s = 0: 1/2 * 1/16 + lam (1/2 * 1/16)
    assert abs(mlp.loss(const(0.0, 0.0), x, [1.0, 0.0], lam, scale=(0.5, 2.0)) - (1 / 32) * (1 + lam)) < 1e-15


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves theta by -lr g / (|g| + eps):
    after T steps theta_0 - T lr g / (|g| + eps).  A missing bias correction
    or swapped beta1 / beta2 breaks this."""
    g = np.array([3.0, -0.02, 0.0, 1e-5, -7.5e3])
    theta = np.array([0.1, -0.2, 0.3, 0.0, 1.0])
    m = v = np.zeros(5)
    lr, eps = 1e-3, 1e-8
    th = theta
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, g, m, v, t, lr, eps=eps)
    np.testing.assert_allclose(th, theta - 5 * lr * g / (np.abs(g) + eps), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(m, (1 - 0.9 ** 5) * g, rtol=1e-14)
    np.testing.assert_allclose(v, (1 - 0.999 ** 5) * g * g, rtol=1e-12)


def test_adam_alternating_gradient_closed_form():
    """Gradients g then -g: m_2 = -(1 - b1)^2 g, so the bias-corrected
    m_2 / (1 - b1^2) = -(1 - b1)/(1 + b1) g, while v_2 / (1 - b2^2) = g^2:
    the second step moves theta by +lr (1 - b1)/(1 + b1) g/(|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    b1, b2, lr, eps = 0.8, 0.95, 0.01, 1e-7
    th1, m, v = mlp.adam_step(np.zeros(3), g, 0.0, 0.0, 1, lr, b1, b2, eps)
    th2, m, v = mlp.adam_step(th1, -g, m, v, 2, lr, b1, b2, eps)
    np.testing.assert_allclose(th1, -lr * g / (np.abs(g) + eps), rtol=1e-14)
    np.testing.assert_allclose(th2 - th1, lr * (1 - b1) / (1 + b1) * g / (np.abs(g) + eps), rtol=1e-12)
    np.testing.assert_allclose(m, -(1 - b1) ** 2 * g, rtol=1e-14)


def test_adam_scale_invariance_without_eps():
    """eps = 0: the update does not change when every gradient is scaled by c > 0."""
    rng = np.random.default_rng(5)
    gs = rng.normal(size=(4, 6))
    a = b = np.zeros(6)
    ma = va = mb = vb = np.zeros(6)
    for t, g in enumerate(gs, 1):
        a, ma, va = mlp.adam_step(a, g, ma, va, t, 0.05, eps=0.0)
        b, mb, vb = mlp.adam_step(b, 1234.5 * g, mb, vb, t, 0.05, eps=0.0)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_quantile_and_calibration_order_statistics():
    """Position (n - 1) q between the sorted values: the median of 1..5 is
    3, q = 0.9 gives 4 + 0.6 = 4.6, q = 0 and 1 the extremes; it equals
    numpy's default ('linear') quantile.  calibration_k of |y - mu| = (1, 4,
    9, 16) with s = (0, ln 2, ln 3, ln 4) takes z = (1, 2, 3, 4)."""
    v = np.array([3.0, 1.0, 2.0, 5.0, 4.0])
    assert mlp.quantile_linear(v, 0.5) == 3.0
    assert abs(mlp.quantile_linear(v, 0.9) - 4.6) < 1e-15
    assert mlp.quantile_linear(v, 0.0) == 1.0 and mlp.quantile_linear(v, 1.0) == 5.0
    rng = np.random.default_rng(2)
    big = rng.exponential(size=1001)
    for q in (0.1, 0.5, 0.999):
        assert mlp.quantile_linear(big, q) == np.quantile(big, q)
    s = np.log([1.0, 2.0, 3.0, 4.0])
    y = np.array([1.0, -4.0, 9.0, 16.0])
    assert abs(mlp.calibration_k(y, 0.0, s, 1.0) - 4.0) < 1e-14
    assert abs(mlp.calibration_k(y, 0.0, s, 0.5) - 2.5) < 1e-14


def test_bf16_rounding_hand_values():
    """bfloat16 keeps 8 significant bits: between 1 and 2 its spacing is 2^-7,
    so 1 + 2^-8 is a tie that rounds to the even 1, 1 + 3 2^-8 a tie that
    rounds to the even 1 + 2^-6, 1 + 2^-8 + 2^-20 rounds up; 0.3 = 153.6 2^-9
    -> 154 2^-9; 0.7 = 179.2 2^-8 -> 179 2^-8; pi -> 3.140625 (402 2^-7);
    signs are kept and zero stays zero."""
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, 0.3, 0.7, np.pi, -0.7, 0.0])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, 154 * 2.0 ** -9, 179 * 2.0 ** -8, 3.140625,
                     -179 * 2.0 ** -8, 0.0])
    np.testing.assert_array_equal(mlp.bf16(x), want)


def test_forward_bf16_hand_computed_three_layers():
    """1 -> 2 -> 2 -> 2: the first layer's weight 2.01 is not a bfloat16 value
    and stays as it is; its activations silu(2.01) = 1.77250... (226.88 2^-7)
    and silu(-1) = -0.268941... (-137.70 2^-9) enter the hidden layer as
    227 2^-7 and -138 2^-9, its weights 0.3 and 0.7 as 154 2^-9 and
    179 2^-8; the head takes the hidden activations unrounded."""
    w0, w1, w2 = np.array([[2.01], [-1.0]]), np.array([[0.3, 0.7], [1.0, 0.5]]), np.array([[1.0, -1.0], [0.25, 0.5]])
    b1 = np.array([0.1, -0.2])
    params = [(w0, np.zeros(2)), (w1, b1), (w2, np.zeros(2))]
    h0 = np.array([227 / 128, -138 / 512])
    z1 = np.array([154 / 512 * h0[0] + 179 / 256 * h0[1], h0[0] + 0.5 * h0[1]]) + b1
    h1 = z1 / (1.0 + np.exp(-z1))
    want = np.array([[h1[0] - h1[1], 0.25 * h1[0] + 0.5 * h1[1]]])
    np.testing.assert_allclose(mlp.forward_bf16(params, np.array([[1.0]])), want, rtol=1e-15, atol=1e-16)
    # and the plain network differs at the level of the roundings
    plain, _ = mlp.forward(params, np.array([[1.0]]))
    assert np.max(np.abs(plain - want)) > 1e-4
