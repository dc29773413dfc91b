"""Pins of the oracle's U-Net reference: the backward pass against central
finite differences of the forward pass, convolution against a direct
per-voxel loop, and the pooling/upsampling adjoint identities."""
import numpy as np
import pytest

from oracle import unet as U


def test_conv3_matches_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 4, 4, 3))
    W = rng.standard_normal((27, 3, 5))
    b = rng.standard_normal(5)
    y = U.conv3(x, W, b)
    for v in [(0, 0, 0), (3, 1, 2), (1, 3, 3)]:
        ref = b.copy()
        for t, (di, dj, dk) in enumerate(U.TAPS):
            ref += x[(v[0] + di) % 4, (v[1] + dj) % 4, (v[2] + dk) % 4] @ W[t]
        np.testing.assert_allclose(y[v], ref, rtol=1e-13)


def test_pool_up_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((8, 8, 8, 2))
    y = rng.standard_normal((4, 4, 4, 2))
    assert np.sum(U.pool(x) * y) == pytest.approx(np.sum(x * U.pool_backward(y)), rel=1e-12)
    assert np.sum(U.up(y) * x) == pytest.approx(np.sum(y * U.up_backward(x)), rel=1e-12)


def test_conv3_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 4, 4, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((4, 4, 4, 2))
    dx, dW, db = U.conv3_backward(x, W, dy)
    f = lambda x_, W_, b_: np.sum(U.conv3(x_, W_, b_) * dy)  # noqa: E731
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 3, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert dx[idx] == pytest.approx((f(xp, W, b) - f(xm, W, b)) / (2 * eps), rel=1e-7, abs=1e-8)
    for idx in [(0, 0, 0), (13, 2, 1), (26, 1, 0)]:
        Wp, Wm = W.copy(), W.copy()
        Wp[idx] += eps
        Wm[idx] -= eps
        assert dW[idx] == pytest.approx((f(x, Wp, b) - f(x, Wm, b)) / (2 * eps), rel=1e-7, abs=1e-8)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)), rtol=1e-13)


def test_unet_backward_finite_differences():
    """The full network's parameter gradients of L = sum(yhat * g) against
    central differences (8^3 grid, every layer touched)."""
    rng = np.random.default_rng(3)
    p = U.init_params(seed=4)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x0 = rng.standard_normal((8, 8, 8, 4))
    gout = rng.standard_normal((8, 8, 8))
    y, cache = U.forward(p, x0)
    grads = U.backward(p, cache, gout)
    eps = 1e-6
    for name in ("l1a.w", "l2b.w", "l3b.w", "l4a.w", "l5a.b", "head.w", "head.b"):
        flat = p[name].reshape(-1)
        for j in rng.choice(flat.size, size=min(2, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + eps
            fp = np.sum(U.forward(p, x0)[0] * gout)
            flat[j] = old - eps
            fm = np.sum(U.forward(p, x0)[0] * gout)
            flat[j] = old
            fd = (fp - fm) / (2 * eps)
            assert grads[name].reshape(-1)[j] == pytest.approx(fd, rel=1e-6, abs=1e-7), name


def test_source_target_vanishes_for_the_linear_field():
    """t = lap chi / (s mu_chi) - delta is zero for the screening-off field
    (exact FFT solve of eq. linearised) and equals the mean-free source shift
    when the field solves lap chi = s mu_chi (delta + u)."""
    import oracle
    from workloads import lognormal_density

    n = 16
    rho = lognormal_density(n, 31.25, seed=4)
    delta = oracle.density_contrast(rho)
    c = oracle.eft_coefficients(0.3071, -0.3, 0.05, 0.7)
    chi = oracle.solve_chi_linear(delta, c, 1.0 / n)
    t = U.source_target(chi, rho, c["s"] * c["mu_chi"])
    assert np.abs(t).max() < 1e-10 * np.abs(delta).max()
    u = np.random.default_rng(2).standard_normal((n, n, n))
    u -= u.mean()
    chi_u = oracle.poisson_fft(c["s"] * c["mu_chi"] * (delta + u), 1.0 / n)
    np.testing.assert_allclose(U.source_target(chi_u, rho, c["s"] * c["mu_chi"]), u, atol=1e-10)


def test_input_features_standardised():
    from workloads import lognormal_density

    rho = lognormal_density(16, 31.25, seed=4)
    x = U.input_features(rho, -0.3, 0.1, 0.5)
    assert abs(x[..., 0].mean()) < 1e-12 and x[..., 0].std() == pytest.approx(1.0, rel=1e-12)
    assert np.all(x[..., 1] == -0.3) and np.all(x[..., 2] == 0.1) and np.all(x[..., 3] == 0.5)
    # lognormal densities have mean 1, so the feature is ln(rho + 1e-3) standardised
    lr = np.log(rho + 1e-3)
    np.testing.assert_allclose(x[..., 0], (lr - lr.mean()) / lr.std(), atol=1e-9)


def test_adam_first_step_moves_each_weight_by_lr_against_its_gradient_sign():
    """From m = v = 0 the bias-corrected moments of the first step are g and
    g^2 exactly, so the update is lr g / (|g| + eps): lr sign(g) for
    |g| >> eps, and nothing where g = 0."""
    rng = np.random.default_rng(3)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-3, 3, 50)
    g[7] = 0.0
    lr, eps = 1e-2, 1e-8
    w1, m1, v1, gn = U.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    np.testing.assert_allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert w1[7] == w[7]
    big = np.abs(g) > 1e-2
    np.testing.assert_allclose((w - w1)[big], lr * np.sign(g[big]), rtol=0, atol=lr * 1e-6)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-13)
    assert gn == pytest.approx(np.sqrt(np.sum(g * g)), rel=1e-14)


def test_adam_constant_gradient_sequence_is_exactly_bias_corrected():
    """A constant gradient g for T steps gives m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so after bias correction every step moves
    lr g / (|g| + eps): a missing or off-by-one correction fails."""
    g = np.array([3.0, -0.25, 1e-4, -7.0])
    w0 = np.array([0.5, -1.0, 2.0, 0.0])
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    lr, b1, b2, eps = 3e-3, 0.8, 0.99, 1e-8
    T = 25
    for t in range(1, T + 1):
        w, m, v, _ = U.adam_step(w, g, m, v, t, lr, beta1=b1, beta2=b2, eps=eps)
        np.testing.assert_allclose(m, (1 - b1**t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - b2**t) * g * g, rtol=1e-13)
    np.testing.assert_allclose(w, w0 - T * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_global_norm_clipping():
    """With grad_clip below ||g||, the moments see g grad_clip / ||g|| (a
    vector of norm grad_clip); above it, g unchanged."""
    g = np.array([3.0, 4.0])  # norm 5
    _, m, v, gn = U.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 1e-3, grad_clip=1.0)
    assert gn == 5.0
    np.testing.assert_allclose(m, 0.1 * np.array([0.6, 0.8]), rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * np.array([0.36, 0.64]), rtol=1e-13)
    _, m2, _, _ = U.adam_step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1, 1e-3, grad_clip=10.0)
    np.testing.assert_allclose(m2, 0.1 * g, rtol=1e-15)


def test_backward_rounding_hook_is_applied_to_activation_gradients_only():
    """With a rounding hook that is the identity the gradients are unchanged;
    with a hook that zeroes every activation gradient only the head's own
    parameters keep a gradient."""
    rng = np.random.default_rng(4)
    p = U.init_params(1)
    x0 = rng.standard_normal((8, 8, 8, 4))
    y, cache = U.forward(p, x0)
    dy = rng.standard_normal((8, 8, 8))
    g0 = U.backward(p, cache, dy)
    g1 = U.backward(p, cache, dy, rnd=lambda a: a.copy())
    for k in g0:
        np.testing.assert_array_equal(g0[k], g1[k])
    gz = U.backward(p, cache, dy, rnd=np.zeros_like)
    assert np.any(gz["head.w"] != 0)
    for name, _, _ in U.LAYERS:
        assert not np.any(gz[name + ".w"])
