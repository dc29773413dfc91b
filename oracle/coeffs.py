"""Background and EFT coefficients, linear growth and the static spherical
closed form, in float64 (oracle; test infrastructure only).

Notation (code units, tildes dropped as in Sec. 3.1):

* Omega_m(a), E^2(a): flat LCDM background (eq. alpha-a; the background is
  reset to LCDM, Sec. 3.5.2).
* alpha_I(a) = alpha_I0 (1 - Omega_m(a)) / (1 - Omega_m0), I = B, M (eq. alpha-a).
* Geff/G = Omega_m(a)^(alpha_M0 / (3 (1 - Omega_m0)))  (Sec. 2.4, closed form).
* C2 with alpha_T = 0 (Sec. 2.2): -alpha_M + alpha_B (1 + alpha_M)
  + (1 + alpha_B) Hdot/H^2 + alphadot_B/H + rho_m/(2 H^2 M^2), where
  Hdot/H^2 = -3/2 Omega_m(a), alphadot_B/H = d alpha_B / d ln a
  = 3 Omega_m(a) alpha_B(a) and rho_m/(2 H^2 M^2) = 3/2 Omega_m(a) Geff/G.
* C4 = -4 alpha_B + 2 alpha_M (Sec. 2.2).
* nu = 2 alpha_B alpha_M - alpha_B^2 - C2, xi = alpha_B - alpha_M,
  mu_chi = xi/nu, mu_Psi = 1 + xi^2/nu (eq. linearised).
* s = 3/2 (Geff/G) a Omega_m0: source prefactor of eqs. phipsi_mod and
  chi_scm (the Omega_m printed there is the present-day value, because the
  density unit rho_* = Omega_m rho_c / a^3 of Sec. 3.1 is comoving).
* K = C4 / (4 E^2 a^4): prefactor of the screening bracket in eq. chi_scm.

With these, eq. chi_scm reads  nu lap(chi) - xi s delta - K N(chi) = 0 with
N = (lap chi)^2 - d_i d_j chi d_i d_j chi, and eq. phipsi_mod reads
lap(Psi) = s delta + xi lap(chi).
"""
from __future__ import annotations

import math

import numpy as np


def omega_m(a, om0):
    """Omega_m(a) of a flat LCDM background (eq. alpha-a)."""
    return om0 / (om0 + (1.0 - om0) * a**3)


def e2(a, om0):
    """E^2 = H^2/H0^2 = Omega_m0 a^-3 + 1 - Omega_m0."""
    return om0 / a**3 + 1.0 - om0


def alpha_of_a(alpha0, a, om0):
    """alpha_I(a) = alpha_I0 (1 - Omega_m(a)) / (1 - Omega_m0) (eq. alpha-a)."""
    return alpha0 * (1.0 - omega_m(a, om0)) / (1.0 - om0)


def geff_over_g(a, om0, alpha_m0):
    """Closed form Geff/G = Omega_m(a)^(alpha_M0 / (3 (1 - Omega_m0))) (Sec. 2.4)."""
    return omega_m(a, om0) ** (alpha_m0 / (3.0 * (1.0 - om0)))


def eft_coefficients(omega_m0, alpha_b0, alpha_m0, a, screening=True, alpha_b_dot=True):
    """All scalar coefficients of the code-unit equations at scale factor ``a``.

    ``screening=False`` is the linearised option (Sec. 3.5.1): C4 := 0, so
    K = 0.  ``alpha_b_dot=False`` drops alphadot_B/H from C2, as for the
    static test of Sec. 3.6.1.
    """
    om = omega_m(a, omega_m0)
    E2 = e2(a, omega_m0)
    ab = alpha_of_a(alpha_b0, a, omega_m0)
    am = alpha_of_a(alpha_m0, a, omega_m0)
    geff = geff_over_g(a, omega_m0, alpha_m0)
    hdot_h2 = -1.5 * om
    abdot_h = 3.0 * om * ab if alpha_b_dot else 0.0
    C2 = -am + ab * (1.0 + am) + (1.0 + ab) * hdot_h2 + abdot_h + 1.5 * om * geff
    C4 = (-4.0 * ab + 2.0 * am) if screening else 0.0
    nu = 2.0 * ab * am - ab * ab - C2
    xi = ab - am
    s = 1.5 * geff * a * omega_m0
    K = C4 / (4.0 * E2 * a**4)
    mu_chi = xi / nu if nu != 0.0 else 0.0
    mu_psi = 1.0 + xi * xi / nu if nu != 0.0 else 1.0
    lam = K * s * xi / nu**2 if nu != 0.0 else 0.0
    return dict(
        omega_m_a=om, E2=E2, alpha_b=ab, alpha_m=am, geff=geff, C2=C2, C4=C4,
        nu=nu, xi=xi, mu_chi=mu_chi, mu_psi=mu_psi, s=s, K=K, lam=lam,
    )


# ---------------------------------------------------------------- growth
def growth_factor(a_end, omega_m0, alpha_b0=0.0, alpha_m0=0.0, a_start=1e-3, n_steps=20000, mu_of_a=None,
                  with_rate=False, screening=True):
    """Growing mode D+(a_end) of eq. delta_mod_a, normalised to D = a at a_start.

    delta'' + (3/a + dlnH/da) delta' - 3/(2a^2) Omega_m(a) mu(a) delta = 0 with
    mu = (Geff/G) mu_Psi (Sec. 2.6), integrated in ln a with classical
    4th-order Runge-Kutta on a uniform grid.  ``mu_of_a`` replaces mu(a) by
    a given function (used to pin the integrator on closed forms).  With
    ``with_rate`` the result is (D, dD/dln a).
    """
    def mu_eff(a):
        if mu_of_a is not None:
            return mu_of_a(a)
        if alpha_b0 == 0.0 and alpha_m0 == 0.0:
            return 1.0
        c = eft_coefficients(omega_m0, alpha_b0, alpha_m0, a, screening=screening)
        return c["geff"] * c["mu_psi"]

    # variables y = (D, dD/dlna); with x = ln a:
    # D'' in a -> d2D/dx2 = a^2 D'' + a D'  and  dD/dx = a D'.
    def rhs(x, y):
        a = math.exp(x)
        om = omega_m(a, omega_m0)
        dlnh_dlna = -1.5 * om  # d ln H / d ln a for flat LCDM
        d, dd = y
        # a^2 D'' = -(3 + dlnH/dlna) a D' + 3/2 Om mu D ;  d2D/dx2 = a^2 D'' + a D'
        d2 = -(2.0 + dlnh_dlna) * dd + 1.5 * om * mu_eff(a) * d
        return np.array([dd, d2])

    x0, x1 = math.log(a_start), math.log(a_end)
    hstep = (x1 - x0) / n_steps
    y = np.array([a_start, a_start])
    x = x0
    for _ in range(n_steps):
        k1 = rhs(x, y)
        k2 = rhs(x + 0.5 * hstep, y + 0.5 * hstep * k1)
        k3 = rhs(x + 0.5 * hstep, y + 0.5 * hstep * k2)
        k4 = rhs(x + hstep, y + hstep * k3)
        y = y + hstep / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        x += hstep
    if with_rate:
        return float(y[0]), float(y[1])
    return float(y[0])


# ---------------------------------------------------------------- sphere
def spherical_x(A, nu, C4, xi):
    """x = (nu - sqrt(nu^2 - 2 A C4 xi)) / C4  (eq. analytical); linear limit for C4 = 0.

    Written in the cancellation-free form -2 A xi / (nu + sqrt(nu^2 - 2 A C4 xi))
    which is algebraically identical to the printed root.
    """
    A = np.asarray(A, dtype=np.float64)
    disc = nu * nu - 2.0 * A * C4 * xi
    disc = np.maximum(disc, 0.0)
    return 2.0 * A * xi / (nu + np.sqrt(disc))


def spherical_yz(A, x, alpha_b, alpha_m):
    """y = A + (alpha_B - alpha_M) x and z = A + alpha_B x (eq. analytical)."""
    return A + (alpha_b - alpha_m) * x, A + alpha_b * x
