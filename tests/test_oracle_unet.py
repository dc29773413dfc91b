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
