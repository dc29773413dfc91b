"""Pins of the oracle's grid/particle operations (deposit, FFT Poisson,
5-point gradient, interpolation, power spectrum)."""
import numpy as np
import pytest

import oracle
from oracle import fields as F


def _brute_force_deposit(pos, ng):
    """Per-particle, per-cell loop over the CIC tent W = prod max(0, 1-|dx|/h)
    with minimum-image distances (small inputs only)."""
    h = 1.0 / ng
    rho = np.zeros((ng, ng, ng))
    centres = (np.arange(ng) + 0.5) * h
    for p in range(pos.shape[1]):
        w = []
        for d in range(3):
            dx = pos[d, p] - centres
            dx -= np.round(dx)
            w.append(np.maximum(0.0, 1.0 - np.abs(dx) / h))
        rho += w[0][:, None, None] * w[1][None, :, None] * w[2][None, None, :]
    return rho * ng**3 / pos.shape[1]


def test_deposit_matches_brute_force_tent_sum():
    rng = np.random.default_rng(3)
    pos = rng.random((3, 40))
    pos[:, :4] = [[0.0, 0.999999, 0.5, 1 / 16], [0.0, 0.0, 0.031, 0.5], [0.9999, 0.5, 0.0, 0.25]]
    np.testing.assert_allclose(F.cic_deposit(pos, 8), _brute_force_deposit(pos, 8), rtol=1e-12, atol=1e-12)


def test_deposit_mass_conservation_and_lattice():
    rng = np.random.default_rng(1)
    pos = rng.random((3, 5000))
    rho = F.cic_deposit(pos, 16)
    assert rho.sum() == pytest.approx(16**3, rel=1e-13)
    q = (np.arange(16) + 0.5) / 16
    lat = np.stack([g.ravel() for g in np.meshgrid(q, q, q, indexing="ij")])
    np.testing.assert_allclose(F.cic_deposit(lat, 16), 1.0, atol=1e-13)


def test_deposit_integer_cell_shift_rolls_density():
    rng = np.random.default_rng(2)
    pos = rng.random((3, 300))
    shifted = np.mod(pos + np.array([[2 / 16], [0.0], [-3 / 16]]), 1.0)
    np.testing.assert_allclose(F.cic_deposit(shifted, 16), np.roll(F.cic_deposit(pos, 16), (2, 0, -3), axis=(0, 1, 2)),
                               rtol=1e-10, atol=1e-10)


def test_fft_poisson_inverts_7_point_laplacian():
    rng = np.random.default_rng(4)
    src = rng.standard_normal((16, 16, 16))
    src -= src.mean()
    u = F.poisson_fft(src, 1.0 / 16)
    np.testing.assert_allclose(F.laplacian7(u, 1.0 / 16), src, atol=1e-10)
    assert abs(u.mean()) < 1e-14


def test_fft_poisson_single_mode_closed_form():
    """lap_7 of cos(2 pi m x) has eigenvalue -(4/h^2) sin^2(pi m h)."""
    ng, m = 16, 3
    h = 1.0 / ng
    x = (np.arange(ng) + 0.5) * h
    src = np.cos(2 * np.pi * m * x)[:, None, None] * np.ones((1, ng, ng))
    u = F.poisson_fft(src, h)
    lam = -(4 / h**2) * np.sin(np.pi * m * h) ** 2
    np.testing.assert_allclose(u, src / lam, atol=1e-14)


def test_gradient_fourier_symbol():
    """D5 sin(kx) = [(8 sin kh - sin 2kh)/(6h)] cos(kx) for the 5-point stencil."""
    ng, m = 32, 5
    h = 1.0 / ng
    k = 2 * np.pi * m
    x = (np.arange(ng) + 0.5) * h
    f = np.sin(k * x)[None, :, None] * np.ones((ng, 1, ng))
    g = F.gradient5(f, h)
    expect = -((8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)) * np.cos(k * x)
    np.testing.assert_allclose(g[1], expect[None, :, None] * np.ones((ng, 1, ng)), atol=1e-10)
    np.testing.assert_allclose(g[0], 0.0, atol=1e-12)
    np.testing.assert_allclose(g[2], 0.0, atol=1e-12)


def test_interpolation_exact_for_linear_fields_away_from_wrap():
    ng = 16
    h = 1.0 / ng
    x = (np.arange(ng) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    field = np.stack([2 * X - Y, 3 * Z + 1, X + Y + Z])
    rng = np.random.default_rng(5)
    pos = 0.1 + 0.8 * rng.random((3, 100))
    got = F.cic_interpolate(field, pos)
    want = np.stack([2 * pos[0] - pos[1], 3 * pos[2] + 1, pos.sum(0)])
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_power_spectrum_single_mode():
    ng, box, m = 32, 100.0, 4
    x = (np.arange(ng) + 0.5) / ng
    f = 0.2 * np.cos(2 * np.pi * m * x)[:, None, None] * np.ones((1, ng, ng))
    k, p, cnt = F.power_spectrum(f, box)
    i = int(np.argmax(p))
    assert abs(k[i] - 2 * np.pi * m / box) < 0.5 * 2 * np.pi / box
    # two modes (+m, -m) each with |f_k|^2 = 0.01, averaged over the shell
    assert p[i] * cnt[i] == pytest.approx(2 * 0.01 * box**3, rel=1e-10)


def test_lone_particle_at_cell_centre_feels_no_self_force():
    ng = 16
    pos = np.array([[8.5 / 16], [4.5 / 16], [11.5 / 16]])
    for params in (dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=0.5),
                   dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=0.5, screening=False)):
        out = oracle.pm_step(pos, np.zeros((3, 1)), ng, params, dt_kick=1.0)
        np.testing.assert_allclose(out["acc"], 0.0, atol=1e-9)


def test_smoothed_ratio_is_a_normalised_symmetric_filter():
    """A constant boost stays constant; a boost linear in k stays linear more
    than 8 sigma from the ends of uniformly spaced bins (symmetric kernel);
    sigma = 0 gives the plain ratio."""
    k = 0.01 * np.arange(1, 201)
    den = 1.0 + k**2
    out = F.smoothed_ratio(k, 1.03 * den, den, 0.028)
    np.testing.assert_allclose(out, 1.03, rtol=1e-14)
    lin = 1.0 + 0.5 * k
    out = F.smoothed_ratio(k, lin * den, den, 0.028)
    inner = (k > k[0] + 8 * 0.028) & (k < k[-1] - 8 * 0.028)
    np.testing.assert_allclose(out[inner], lin[inner], rtol=1e-12)
    raw = F.smoothed_ratio(k, lin * den, den, 0.0)
    np.testing.assert_allclose(raw, lin, rtol=1e-15)
