"""Pins of the oracle's nonlinear scalar-field solve against what the paper
fixes: its printed Method I formulas, the bracket form of the screening term,
the spherical closed form, the exact linear (screening-off) solution, a
brute-force Newton solve on 8^3 grids and the scaling symmetry of the
equation.  All comparisons use operators written here from the paper's
printed stencils, not the oracle's C code."""
import math

import numpy as np
import pytest

import oracle
from oracle import coeffs as C
from workloads import gaussian_field, lognormal_density

R = np.roll


def _d2(u, h):
    """Printed second-derivative stencils (Sec. 3.2.1): dict of Dxx..Dyz."""
    out = {}
    for name, ax in (("xx", 0), ("yy", 1), ("zz", 2)):
        out[name] = (R(u, -1, ax) - 2 * u + R(u, 1, ax)) / h**2
    for name, (a0, a1) in (("xy", (0, 1)), ("xz", (0, 2)), ("yz", (1, 2))):
        pp = R(R(u, -1, a0), -1, a1)
        pm = R(R(u, -1, a0), 1, a1)
        mp = R(R(u, 1, a0), -1, a1)
        mm = R(R(u, 1, a0), 1, a1)
        out[name] = (pp - pm - mp + mm) / (4 * h**2)
    return out


def _bracket(u, h):
    """N_h = 2(Dxx Dyy + Dyy Dzz + Dzz Dxx) - 2(Dxy^2 + Dxz^2 + Dyz^2): the
    screening bracket as printed in Sec. 3.2.1."""
    d = _d2(u, h)
    return (2 * (d["xx"] * d["yy"] + d["yy"] * d["zz"] + d["zz"] * d["xx"])
            - 2 * (d["xy"] ** 2 + d["xz"] ** 2 + d["yz"] ** 2))


def _lap(u, h):
    d = _d2(u, h)
    return d["xx"] + d["yy"] + d["zz"]


def _smooth_field(ng, seed, amp):
    g = gaussian_field(ng, 100.0, lambda k: k**-3.0, seed=seed)
    return amp * g / np.abs(g).max()


# ------------------------------------------------------------- operator
def test_operator_pieces_match_printed_stencils():
    """The oracle's Laplacian and Lq satisfy the per-cell quadratic
    nu L - b - K [(2/3) L^2 - T] = 0 written with the printed bracket:
    with N_h = (2/3) lap^2 - T (Sec. 3.2.2, w = 1/3), Lq solves
    -(2/3) K Lq^2 + nu Lq + K T - b = 0."""
    ng, h = 16, 1 / 16
    chi = _smooth_field(ng, 7, 1e-3)
    delta = _smooth_field(ng, 8, 1.0)
    c = C.eft_coefficients(0.3071, -0.4, 0.05, 0.7)
    b = c["xi"] * c["s"] * delta
    op = oracle.chi_operator(chi, b, h, c["nu"], c["K"])
    np.testing.assert_allclose(op["lap"], _lap(chi, h), rtol=1e-10, atol=1e-10 * np.abs(_lap(chi, h)).max())
    T = (2.0 / 3.0) * _lap(chi, h) ** 2 - _bracket(chi, h)
    np.testing.assert_allclose(op["T"], T, rtol=1e-8, atol=1e-9 * np.abs(T).max())
    lq = op["lq"]
    resid = -(2 / 3) * c["K"] * lq**2 + c["nu"] * lq + c["K"] * T - b
    assert np.abs(resid).max() <= 1e-10 * np.abs(b).max()
    assert op["clamped"] == 0


def test_method_i_root_equals_laplacian_form_update():
    """Sec. 3.2.1's per-cell quadratic P chi^2 + Q chi + R = 0 with the minus
    root gives the same chi as the Laplacian-form update (S - h^2 Lq)/6 of
    Sec. 3.2.2.  Readings used: b carries the a Omega_m0 factor of eq.
    chi_scm, and q^(2) is evaluated with the centre value set to zero (its
    centre terms are already in P and Q)."""
    ng, h = 16, 1 / 16
    chi = _smooth_field(ng, 11, 2e-3)
    delta = _smooth_field(ng, 12, 1.0)
    a = 0.8
    c = C.eft_coefficients(0.3071, -0.36, 0.1, a)
    assert (c["nu"] ** 2 - (8 / 3) * c["K"] * c["xi"] * c["s"] * delta).min() > 0  # no void cells
    ab, am, C2, C4, E2 = c["alpha_b"], c["alpha_m"], c["C2"], c["C4"], c["E2"]
    nu_p = 2 * ab * am - ab**2 - C2
    S = sum(R(chi, s, ax) for ax in range(3) for s in (1, -1))
    zero_centre = chi.copy()
    # q2 evaluated with chi_ijk := 0, cell by cell via the bracket at that cell
    q2 = np.empty_like(chi)
    for i in range(ng):
        for j in range(ng):
            for k in range(ng):
                zero_centre[i, j, k] = 0.0
                loc = np.roll(np.roll(np.roll(zero_centre, -i + 2, 0), -j + 2, 1), -k + 2, 2)[:5, :5, :5]
                q2[i, j, k] = _bracket(loc, h)[2, 2, 2]
                zero_centre[i, j, k] = chi[i, j, k]
    bcell = 1.5 * c["geff"] * a * 0.3071 * delta
    P = -6 * C4 / (h**4 * a**4 * E2)
    Q = -6 * nu_p / h**2 + 2 * C4 * S / (h**4 * a**4 * E2)
    Rr = (am - ab) * bcell + nu_p * S / h**2 - C4 / (4 * a**4 * E2) * q2
    chi_m1 = (-Q - np.sqrt(Q**2 - 4 * P * Rr)) / (2 * P)
    op = oracle.chi_operator(chi, c["xi"] * c["s"] * delta, h, c["nu"], c["K"])
    chi_m2 = (S - h**2 * op["lq"]) / 6.0
    np.testing.assert_allclose(chi_m1, chi_m2, rtol=1e-7, atol=1e-9 * np.abs(chi_m2).max())


def test_discrete_root_matches_spherical_closed_form():
    """For chi = u0 r^2/2 the discrete stencils give lap = 3 u0 and T = 0
    exactly, so inside a uniform top-hat the local root must equal the
    spherical solution of eq. analytical: u0 = a^4 E^2 x(A) with
    A = s (delta0/3) / (a^4 E^2) (mean enclosed overdensity delta0)."""
    for (ab0, am0, a, d0) in ((-0.4, 0.0, 0.5, 3.0), (-0.6, 0.1, 1.0, 10.0), (-0.2, 0.0, 1.0, 50.0)):
        c = C.eft_coefficients(0.3071, ab0, am0, a)
        ng, h = 16, 1 / 16
        u0 = a**4 * c["E2"] * C.spherical_x(c["s"] * d0 / 3 / (a**4 * c["E2"]), c["nu"], c["C4"], c["xi"])
        x = (np.arange(ng) + 0.5) * h - 0.5
        r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
        chi = 0.5 * u0 * r2
        b = np.full((ng, ng, ng), c["xi"] * c["s"] * d0)
        op = oracle.chi_operator(chi, b, h, c["nu"], c["K"])
        sl = slice(2, ng - 2)
        np.testing.assert_allclose(op["lap"][sl, sl, sl], 3 * u0, rtol=1e-9)
        np.testing.assert_allclose(op["T"][sl, sl, sl], 0.0, atol=1e-9 * u0**2)
        np.testing.assert_allclose(op["lq"][sl, sl, sl], 3 * u0, rtol=1e-9)


# ------------------------------------------------------------- solves
def test_screening_off_mg_equals_fft_solution():
    """K = 0 (linearised option): the multigrid solution equals the exact
    discrete solution lap_7 chi = mu_chi s delta (eq. linearised)."""
    ng = 32
    delta = _smooth_field(ng, 3, 2.0)
    delta -= delta.mean()
    c = C.eft_coefficients(0.3071, -0.4, 0.0, 0.5, screening=False)
    chi, rep = oracle.solve_chi(delta, c, 1 / ng, tol=1e-13)
    ref = oracle.solve_chi_linear(delta, c, 1 / ng)
    assert rep["status"] == 0
    assert np.linalg.norm(chi - ref) / np.linalg.norm(ref) < 1e-11


def _newton_brute_force(delta, nu, K, xi_s, h, x0):
    """Newton on the 8^3 system with unknowns (chi, c):
    nu (lap + c) - b - K [N_h + (2/3)(2 lap c + c^2)] = 0 per cell (the
    per-cell quadratic written with the printed bracket, with Lq = lap + c),
    and sum chi = 0.  Dense Jacobian by complex-step differentiation."""
    n = delta.size
    b = xi_s * delta

    def F(z):
        chi = z[:n].reshape(delta.shape)
        c = z[n]
        lap = _lap(chi, h)
        eq = nu * (lap + c) - b - K * (_bracket(chi, h) + (2 / 3) * (2 * lap * c + c * c))
        return np.concatenate([eq.ravel(), [chi.sum()]])

    z = np.concatenate([x0.ravel(), [0.0]]).astype(np.complex128)
    for _ in range(30):
        f = F(z.real.astype(np.complex128)).real
        J = np.empty((n + 1, n + 1))
        for j in range(n + 1):
            zz = z.real.astype(np.complex128)
            zz[j] += 1e-30j
            J[:, j] = F(zz).imag / 1e-30
        dz = np.linalg.solve(J, -f)
        z = z.real + dz
        if np.abs(dz).max() < 1e-15 * np.abs(z).max():
            break
    return z[:n].real.reshape(delta.shape), z[n].real


@pytest.mark.parametrize("amp,params", [
    (1.5, (0.3071, -0.4, 0.0, 0.5)),
    (3.0, (0.3071, -0.6, 0.1, 1.0)),
    (2.0, (0.3071, -1.0, 0.2, 0.6)),
])
def test_fas_matches_brute_force_newton_8cubed(amp, params):
    ng, h = 8, 1 / 8
    rng = np.random.default_rng(int(amp * 10))
    delta = rng.standard_normal((ng, ng, ng))
    delta = (delta - delta.mean()) / np.abs(delta).max()
    c = C.eft_coefficients(*params)
    # largest underdensity at 80% of the void threshold, overdensity up to amp x that
    d_void = 3 * c["nu"] ** 2 / (8 * c["K"] * c["xi"] * c["s"])
    delta = np.where(delta < 0, delta * 0.8 * abs(d_void) / abs(delta.min()), delta * amp * 0.8 * abs(d_void))
    delta -= delta.mean()
    dsph = c["nu"] ** 2 - (8 / 3) * c["K"] * c["xi"] * c["s"] * delta
    assert dsph.min() > 0  # no void cells: both readings of the clamp agree
    chi_lin = oracle.solve_chi_linear(delta, c, h)
    chi_n, cmean = _newton_brute_force(delta, c["nu"], c["K"], c["xi"] * c["s"], h, chi_lin)
    chi_o, rep = oracle.solve_chi(delta, c, h, tol=1e-14, max_cycles=300)
    assert rep["status"] == 0
    assert np.linalg.norm(chi_o - chi_n) / np.linalg.norm(chi_n) < 1e-10
    # the solution is genuinely nonlinear: it differs from the linear one
    assert np.linalg.norm(chi_n - chi_lin) / np.linalg.norm(chi_lin) > 1e-3


def test_lambda_invariance():
    """With chi = (beta/nu) y and b = beta delta the equation becomes
    lap y - delta - lambda N_h(y) = 0 with lambda = K beta / nu^2 (the void
    condition is nu^2 (1 - (8/3) lambda delta) >= 0), so parameter sets with
    equal lambda give the same y."""
    ng, h = 32, 1 / 32
    delta = lognormal_density(ng, 500.0 * ng / 256, seed=5) - 1.0
    delta -= delta.mean()
    nu1, K1, beta1 = 0.26, 0.65, -0.03
    nu2, beta2 = 2.0 * nu1, 3.0 * beta1
    K2 = K1 * beta1 / nu1**2 * nu2**2 / beta2
    y = []
    for nu, K, beta in ((nu1, K1, beta1), (nu2, K2, beta2)):
        chi, rep = oracle.fas_solve(beta * delta, h, nu, K, tol=1e-12)
        assert rep["status"] == 0
        y.append(chi / (beta / nu))
    assert np.linalg.norm(y[0] - y[1]) / np.linalg.norm(y[0]) < 1e-10


def test_void_cells_sit_at_the_vertex():
    """In void cells the converged field satisfies lap chi = 3 nu/(4K) - c
    (discriminant set to zero, Sec. 3.3), with c the mean of Lq, and every
    other cell satisfies lap chi = Lq - c."""
    ng, h = 32, 1 / 32
    delta = lognormal_density(ng, 500.0 * ng / 256, seed=2) - 1.0
    delta -= delta.mean()
    c = C.eft_coefficients(0.3071, -0.6, 0.0, 1.0)
    chi, rep = oracle.solve_chi(delta, c, h, tol=1e-12)
    assert rep["status"] == 0 and rep["clamped"] > 1000
    b = c["xi"] * c["s"] * delta
    void = c["nu"] ** 2 - (8 / 3) * c["K"] * b < 0
    op = oracle.chi_operator(chi, b, h, c["nu"], c["K"])
    lap = _lap(chi, h)
    cmean = op["lq"].mean()
    scale = np.linalg.norm(b / c["nu"]) / math.sqrt(b.size)
    assert void.sum() == rep["clamped"]
    assert np.abs(lap[void] - (3 * c["nu"] / (4 * c["K"]) - cmean)).max() < 1e-8 * scale
    assert np.abs(lap[~void] - (op["lq"][~void] - cmean)).max() < 1e-8 * scale


def test_chi_vanishes_linearly_with_xi():
    """xi -> 0: chi -> mu_chi-scaled linear solution, chi = O(xi)."""
    ng, h = 16, 1 / 16
    delta = _smooth_field(ng, 21, 2.0)
    delta -= delta.mean()
    nu, K = 0.3, 0.6
    sols = []
    for beta in (1e-3, 2e-3):
        chi, _ = oracle.fas_solve(beta * delta, h, nu, K, tol=1e-13)
        sols.append(chi)
    lin = oracle.poisson_fft(1e-3 * delta / nu, h)
    assert np.linalg.norm(sols[1] - 2 * sols[0]) / np.linalg.norm(sols[1]) < 1e-2
    assert np.linalg.norm(sols[0] - lin) / np.linalg.norm(lin) < 1e-2
