"""Pins of the oracle's coefficient, growth and spherical closed-form code
against relations the paper fixes independently of the formulas used."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import coeffs as C

PARAMS = [
    (0.3071, -0.4, 0.0, 0.5),
    (0.3071, -0.2, 0.1, 0.33),
    (0.3071, -0.6, 0.1, 1.0),
    (0.257, -0.24, 0.0, 1.0),
    (0.3071, -0.24, -0.2, 0.8),
    (0.3071, -1.0, 0.2, 0.2),
]


@pytest.mark.parametrize("om0,ab0,am0,a", PARAMS)
def test_mu_factors_are_entries_of_inverse_action_matrix(om0, ab0, am0, a):
    """mu_Psi, mu_Phi, mu_chi are the first column of A^{-1} (eq. linearised),
    with A_ab the quadratic-action matrix of Sec. 2.2 at alpha_T = 0.  This
    fixes nu and xi (and the sign conventions of C2) without using the
    closed forms."""
    c = C.eft_coefficients(om0, ab0, am0, a)
    ab, am, C2 = c["alpha_b"], c["alpha_m"], c["C2"]
    A = np.array([[0.0, 1.0, -ab], [1.0, -1.0, am], [-ab, am, -C2]])
    inv = np.linalg.inv(A)
    assert inv[0, 0] == pytest.approx(c["mu_psi"], rel=1e-12)
    assert inv[0, 2] == pytest.approx(c["mu_chi"], rel=1e-12)
    assert inv[0, 1] == pytest.approx(1.0 + c["xi"] * ab / c["nu"], rel=1e-12)


@pytest.mark.parametrize("om0,ab0,am0,a", PARAMS)
def test_geff_closed_form_matches_planck_mass_integral(om0, ab0, am0, a):
    """Geff/G = exp(-int_0^a alpha_M(a')/a' da') (Sec. 2.4) by quadrature."""
    f = lambda x: C.alpha_of_a(am0, x, om0) / x  # noqa: E731
    val, _ = integrate.quad(f, 0.0, a, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert C.geff_over_g(a, om0, am0) == pytest.approx(math.exp(-val), rel=1e-10)


@pytest.mark.parametrize("om0,ab0,am0,a", PARAMS)
def test_time_derivatives_in_c2_by_finite_differences(om0, ab0, am0, a):
    """alphadot_B/H = d alpha_B / d ln a and Hdot/H^2 = d ln H / d ln a, the
    two derivative terms of C2 (Sec. 2.2), checked by central differences."""
    eps = 1e-5
    lp, lm = math.log(a) + eps, math.log(a) - eps
    dab = (C.alpha_of_a(ab0, math.exp(lp), om0) - C.alpha_of_a(ab0, math.exp(lm), om0)) / (2 * eps)
    dlnh = 0.5 * (math.log(C.e2(math.exp(lp), om0)) - math.log(C.e2(math.exp(lm), om0))) / (2 * eps)
    c = C.eft_coefficients(om0, ab0, am0, a)
    c_static = C.eft_coefficients(om0, ab0, am0, a, alpha_b_dot=False)
    assert c["C2"] - c_static["C2"] == pytest.approx(dab, rel=1e-8, abs=1e-12)
    om = c["omega_m_a"]
    rebuilt = (-c["alpha_m"] + c["alpha_b"] * (1 + c["alpha_m"]) + (1 + c["alpha_b"]) * dlnh + dab
               + 1.5 * om * c["geff"])
    assert c["C2"] == pytest.approx(rebuilt, rel=1e-8, abs=1e-10)


def test_lcdm_limit():
    """alpha_B0 = alpha_M0 = 0: no modification (Sec. 2.5: mu_Psi = 1, mu_chi = 0)."""
    c = C.eft_coefficients(0.3071, 0.0, 0.0, 0.7)
    assert c["xi"] == 0.0 and c["K"] == 0.0 and c["geff"] == 1.0
    assert abs(c["nu"]) < 1e-15 and abs(c["C2"]) < 1e-15


def test_geff_trend_with_alpha_m():
    """Geff/G stays 1 for alpha_M0 = 0, exceeds 1 today for alpha_M0 < 0 and
    is below 1 for alpha_M0 > 0 (Sec. 2.4, Fig. geff)."""
    assert C.geff_over_g(1.0, 0.3, 0.0) == 1.0
    assert C.geff_over_g(1.0, 0.3, -0.2) > 1.0
    assert C.geff_over_g(1.0, 0.3, 0.2) < 1.0


def test_ecosmog_coefficients_identity():
    """The Method II coefficients printed in Sec. 3.5.2,
    A = -C4/(4 E^2 a^4 nu) and B rho_bar delta = -(alpha_M - alpha_B) 3/2 Geff a Om delta / nu,
    equal -K/nu and xi s delta / nu of the code-unit equation."""
    c = C.eft_coefficients(0.3071, -0.36, 0.2, 0.7)
    a = 0.7
    A_eco = -c["C4"] / (4 * c["E2"] * a**4 * c["nu"])
    B_eco = -(c["alpha_m"] - c["alpha_b"]) * 1.5 * c["geff"] * a * 0.3071 / c["nu"]
    assert A_eco == pytest.approx(-c["K"] / c["nu"], rel=1e-14)
    assert B_eco == pytest.approx(c["xi"] * c["s"] / c["nu"], rel=1e-14)


@pytest.mark.parametrize("om0", [0.257, 0.3071])
def test_lcdm_growth_matches_heath_integral(om0):
    """With mu_Psi = 1 and Geff = G the growth ODE (eq. delta_mod_a) reduces to
    the standard one, whose growing mode is D = 5/2 Om0 E(a) int_0^a da/(a E)^3."""
    val, _ = integrate.quad(lambda x: 1.0 / (x * math.sqrt(C.e2(x, om0))) ** 3, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
    heath = 2.5 * om0 * math.sqrt(C.e2(1.0, om0)) * val
    assert C.growth_factor(1.0, om0) == pytest.approx(heath, rel=2e-8)


def test_eft_growth_enhanced_for_braiding():
    """Growth is enhanced when mu_Psi Geff/G > 1 (Sec. 2.6, Fig. dplus): the
    ratio increases with |alpha_B0| at alpha_M0 = 0."""
    d0 = C.growth_factor(1.0, 0.3071)
    r = [C.growth_factor(1.0, 0.3071, ab, 0.0) / d0 for ab in (-0.12, -0.24, -0.36)]
    assert 1.0 < r[0] < r[1] < r[2]


def test_spherical_root_solves_quadratic_and_limits():
    """x of eq. analytical solves (C4/2) x^2 - nu x + xi A = 0 (the cubic
    action's spherical equation), reduces to mu_chi A for A << 1 (linearised
    limit) and y = A for xi = 0 (GR)."""
    c = C.eft_coefficients(0.3, -0.5, 0.0, 1.0, alpha_b_dot=False)
    A = np.logspace(-6, 2, 50)
    x = C.spherical_x(A, c["nu"], c["C4"], c["xi"])
    printed = (c["nu"] - np.sqrt(c["nu"] ** 2 - 2 * A * c["C4"] * c["xi"])) / c["C4"]
    np.testing.assert_allclose(x, printed, rtol=1e-6)
    resid = 0.5 * c["C4"] * x**2 - c["nu"] * x + c["xi"] * A
    assert np.all(np.abs(resid) <= 1e-10 * np.maximum(A, 1.0))
    assert x[0] == pytest.approx(c["mu_chi"] * A[0], rel=1e-3)
    y, z = C.spherical_yz(A, x, c["alpha_b"], c["alpha_m"])
    np.testing.assert_allclose(C.spherical_yz(A, 0 * x, 0.0, 0.0)[0], A)


def test_point_mass_force_ratio_screened_near_and_enhanced_far():
    """Psi'/Psi'_GR = y/A tends to 1 close to a point mass (Vainshtein
    screening) and to mu_Psi far away (Sec. 2.7, Fig. spher-ana)."""
    c = C.eft_coefficients(0.3, -0.5, 0.0, 1.0)
    A = np.array([1e8, 1e-8])
    x = C.spherical_x(A, c["nu"], c["C4"], c["xi"])
    y, _ = C.spherical_yz(A, x, c["alpha_b"], c["alpha_m"])
    assert y[0] / A[0] == pytest.approx(1.0, abs=2e-4)
    assert y[1] / A[1] == pytest.approx(c["mu_psi"], rel=1e-6)


@pytest.mark.parametrize("mu", [1.0, 1.3, 0.7])
def test_growth_integrator_matches_eds_closed_form_with_constant_mu(mu):
    """Einstein-de Sitter background (Omega_m = 1, dlnH/dlna = -3/2) with a
    constant coupling mu: eq. delta_mod_a becomes D'' + D'/2 - (3/2) mu D = 0
    in ln a, solved by a^p with p = (-1 +- sqrt(1 + 24 mu))/4.  The start
    D = D' = a_start (slope 1) mixes both modes; the exact solution is that
    mix.  A dropped mu, a wrong friction term or a wrong Omega_m factor moves
    the result by percents."""
    a0, a1 = 1e-2, 1.0
    pp = (-1.0 + math.sqrt(1.0 + 24.0 * mu)) / 4.0
    pm = (-1.0 - math.sqrt(1.0 + 24.0 * mu)) / 4.0
    A = a0 * (1.0 - pm) / (pp - pm)
    B = a0 * (pp - 1.0) / (pp - pm)
    x = math.log(a1 / a0)
    exact = A * math.exp(pp * x) + B * math.exp(pm * x)
    rate = pp * A * math.exp(pp * x) + pm * B * math.exp(pm * x)
    d, dd = C.growth_factor(a1, 1.0, a_start=a0, n_steps=4000, mu_of_a=lambda a: mu, with_rate=True)
    assert d == pytest.approx(exact, rel=1e-10)
    assert dd == pytest.approx(rate, rel=1e-10)
