"""The paper's static spherical test (Secs. 3.6.1 and 4.1) reproduced with
the oracle in Dirichlet mode: a truncated isothermal halo on a fixed grid,
faces held at the analytic solution of eq. analytical, compared with that
solution at the accuracy the paper prints."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import coeffs as C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "static_sphere.json")))


def _setup():
    g = GOLD
    c = C.eft_coefficients(g["omega_m0"], g["alpha_b0"], g["alpha_m0"], g["a"], alpha_b_dot=False)
    return g, c


def _analytic(r, g, c):
    """chi(r), Psi(r) with zero at infinity from x, y of eq. analytical:
    chi'/r = H0^2 x, Psi'/r = H0^2 y, A = G M(<r) / (H0^2 r^3) at a = 1."""
    H2 = g["H0_km_s_Mpc"] ** 2
    G, M, rt = g["G_mpc_kms2_per_msun"], g["mass_msun"], g["r_trunc_mpc"]

    def dchi(s):
        A = G * M * min(s, rt) / rt / (H2 * s**3)
        return H2 * s * C.spherical_x(A, c["nu"], c["C4"], c["xi"])

    def dpsi(s):
        A = G * M * min(s, rt) / rt / (H2 * s**3)
        x = C.spherical_x(A, c["nu"], c["C4"], c["xi"])
        return H2 * s * (A + c["xi"] * x)

    out = []
    for f in (dchi, dpsi):
        v = []
        for rr in np.atleast_1d(r):
            a1 = integrate.quad(f, rr, max(rr, rt), limit=200, epsabs=0, epsrel=1e-12)[0] if rr < rt else 0.0
            a2 = integrate.quad(f, max(rr, rt), np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
            v.append(-(a1 + a2))
        out.append(np.array(v))
    return out


def _solve(ng):
    g, c = _setup()
    L = g["box_mpc"]
    h = L / ng
    G, M, rt = g["G_mpc_kms2_per_msun"], g["mass_msun"], g["r_trunc_mpc"]
    # cell-averaged isothermal density, 8^3 sub-samples per cell, centre at the box-centre vertex
    sub = (np.arange(8) + 0.5) / 8
    x1 = (np.arange(ng)[:, None] + sub[None, :]).ravel() * h - L / 2
    rho = np.zeros((ng, ng, ng))
    X2 = (x1**2).reshape(ng, 8)
    for a in range(8):
        for b in range(8):
            r2 = X2[:, a][:, None, None, None] + X2[:, b][None, :, None, None] + X2[None, None, :, :]
            r = np.sqrt(r2)
            rho += np.where(r < rt, M / (4 * math.pi * rt * r2), 0.0).sum(axis=3)
    rho /= 8**3
    assert rho.sum() * h**3 == pytest.approx(M, rel=2e-2)  # truncated isothermal halo mass
    xc = (np.arange(-1, ng + 1) + 0.5) * h - L / 2
    rg = np.sqrt(xc[:, None, None] ** 2 + xc[None, :, None] ** 2 + xc[None, None, :] ** 2)
    ghost_mask = np.zeros(rg.shape, bool)
    ghost_mask[[0, -1], :, :] = True
    ghost_mask[:, [0, -1], :] = True
    ghost_mask[:, :, [0, -1]] = True
    rr = np.unique(np.round(rg[ghost_mask], 12))
    chi_a, psi_a = _analytic(rr, g, c)
    lut_chi = dict(zip(rr, chi_a))
    lut_psi = dict(zip(rr, psi_a))
    gchi = np.zeros(rg.shape)
    gpsi = np.zeros(rg.shape)
    keys = np.round(rg[ghost_mask], 12)
    gchi[ghost_mask] = [lut_chi[k] for k in keys]
    gpsi[ghost_mask] = [lut_psi[k] for k in keys]
    H2 = g["H0_km_s_Mpc"] ** 2
    K = c["C4"] / (4 * H2)  # physical units at a = 1: C4 / (4 H^2 a^2)
    src = 4 * math.pi * G * rho  # rho_m delta / (2 M^2) = 4 pi G delta rho
    chi, rep = oracle.fas_solve(c["xi"] * src, h, c["nu"], K, tol=1e-11, max_cycles=200, ghosts=gchi)
    assert rep["status"] == 0
    lapchi = oracle.chi_operator(chi, c["xi"] * src, h, c["nu"], K, ghosts=gchi)["lap"]
    psi, rep2 = oracle.fas_solve(src + c["xi"] * lapchi, h, 1.0, 0.0, tol=1e-11, max_cycles=200, ghosts=gpsi)
    assert rep2["status"] == 0
    rc = rg[1:-1, 1:-1, 1:-1]
    return g, c, chi, psi, rc, h


@pytest.mark.slow
@pytest.mark.parametrize("ng", [32, 64])
def test_static_sphere_matches_printed_accuracy(ng):
    g, c, chi, psi, rc, h = _solve(ng)
    # chi: mean in bins of the x coordinate (one bin per cell plane), Sec. 4.1
    rr = np.unique(np.round(rc, 12))
    chi_a, psi_a = _analytic(rr, g, c)
    lut_c = dict(zip(rr, chi_a))
    lut_p = dict(zip(rr, psi_a))
    keys = np.round(rc, 12)
    chi_exact = np.vectorize(lut_c.get)(keys)
    ratio = chi.mean(axis=(1, 2)) / chi_exact.mean(axis=(1, 2))
    assert np.abs(ratio - 1).max() < g["chi_binned_rel_tol"]
    if ng == 64:
        psi_exact = np.vectorize(lut_p.get)(keys)
        edges = np.arange(0, rc.max() + h, h)
        which = np.digitize(rc.ravel(), edges)
        num = np.bincount(which, psi.ravel()) / np.maximum(np.bincount(which), 1)
        ana = np.bincount(which, psi_exact.ravel()) / np.maximum(np.bincount(which), 1)
        good = np.bincount(which) > 0
        rel = np.abs(num[good] / ana[good] - 1)
        rmid = (edges[np.minimum(np.nonzero(good)[0], len(edges) - 1)] - 0.5 * h)
        assert rel.max() < g["psi_rel_tol"]
        assert rel[rmid >= 0.2].max() < g["psi_rel_tol_beyond_4_cells"]


def _tophat_closed_form(c, delta_in, radius):
    """u(r) = chi'(r)/r of eq. analytical in code units for an isolated top-hat
    of contrast delta_in and radius `radius`: 2K u^2 - nu u + xi s m(r)/r^3
    = 0 with m(r) = delta_in min(r, radius)^3 / 3, on the root that is
    continuous to the linear solution; chi(r) = -int_r^inf s u(s) ds."""
    nu, K, xs = c["nu"], c["K"], c["xi"] * c["s"]

    def u(r):
        m = delta_in * min(r, radius) ** 3 / 3.0
        return 2.0 * xs * m / r**3 / (nu + math.sqrt(nu * nu - 8.0 * K * xs * m / r**3))

    def chi(r):
        lo = integrate.quad(lambda s: s * u(s), r, max(r, radius), epsabs=0, epsrel=1e-12)[0] if r < radius else 0.0
        hi = integrate.quad(lambda s: s * u(s), max(r, radius), np.inf, epsabs=0, epsrel=1e-12, limit=400)[0]
        return -(lo + hi)

    return u, chi


def test_tophat_interior_is_exact_for_the_discrete_operator():
    """Inside a top-hat the closed form is chi = u0 r^2 / 2 + const, for which
    the second differences are exact and the cross differences vanish
    (T = 0): the discrete operator's residual vanishes to rounding at every
    cell whose stencil lies inside (Sec. 2.7 against Sec. 3.2)."""
    from workloads import tophat_density

    ng, R, d_in = 32, 10.0, 8.0
    c = C.eft_coefficients(0.3071, -0.6, 0.0, 1.0)
    h = 1.0 / ng
    delta = np.where(tophat_density(ng, R, d_in) > 1.0, d_in, 0.0)
    u, _ = _tophat_closed_form(c, d_in, R * h)
    u0 = u(0.5 * R * h)
    x = (np.arange(ng) + 0.5 - ng / 2) * h
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    chi = 0.5 * u0 * r2
    xg = (np.arange(-1, ng + 1) + 0.5 - ng / 2) * h
    ghosts = 0.5 * u0 * (xg[:, None, None] ** 2 + xg[None, :, None] ** 2 + xg[None, None, :] ** 2)
    op = oracle.chi_operator(chi, c["xi"] * c["s"] * delta, h, c["nu"], c["K"], ghosts=ghosts)
    inner = np.sqrt(r2) < (R - 2.0) * h
    assert inner.sum() > 500
    assert np.abs(op["T"][inner]).max() < 1e-9 * u0**2
    assert np.abs(op["r"][inner]).max() < 1e-11 * abs(3.0 * u0)
    assert op["lq"][inner] == pytest.approx(3.0 * u0, rel=1e-12)


@pytest.mark.slow
def test_tophat_full_solve_matches_closed_form_gradient():
    """Full nonlinear solve of a strongly screened top-hat (delta 10, radius 8
    cells of a 64^3 grid, alpha_B0 = -0.6, a = 1; (8/3)|lambda| delta = 16.6),
    faces held at the closed form (whose mass is that of the cells the
    top-hat covers): the radial gradient chi'(r) matches the closed form
    within 1 % more than 2 cells inside the edge, where the closed form is
    a quadratic the discrete operator treats exactly.  Outside, the
    screening term's discretisation at the staircase edge costs a first-order
    error (measured -2.0 % at radius 8 cells and -1.2 % at 12 cells on a 96^3
    grid, while the linearised field is within 1e-4): bound 3 %.  The same
    solve with screening off matches its closed form within 1 % everywhere."""
    from workloads import tophat_density

    ng, R, d_in = 64, 8.0, 10.0
    h = 1.0 / ng
    inside = tophat_density(ng, R, d_in) > 1.0
    delta = np.where(inside, d_in, 0.0)
    r_eff = (3.0 * inside.sum() / (4.0 * math.pi)) ** (1.0 / 3.0) * h
    xg = (np.arange(-1, ng + 1) + 0.5 - ng / 2) * h
    rg = np.sqrt(xg[:, None, None] ** 2 + xg[None, :, None] ** 2 + xg[None, None, :] ** 2)
    face = np.zeros(rg.shape, bool)
    face[[0, -1]] = True
    face[:, [0, -1]] = True
    face[:, :, [0, -1]] = True
    x = xg[1:-1]
    X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
    for screening, ext_tol in ((True, 3e-2), (False, 1e-2)):
        c = C.eft_coefficients(0.3071, -0.6, 0.0, 1.0, screening=screening)
        if screening:
            u, chi_of_r = _tophat_closed_form(c, d_in, r_eff)
        else:  # K = 0: u = mu_chi s m / r^3
            def u(rv):
                return c["mu_chi"] * c["s"] * d_in * min(rv, r_eff) ** 3 / 3.0 / rv**3

            def chi_of_r(rv):
                lo = integrate.quad(lambda q: q * u(q), rv, max(rv, r_eff))[0] if rv < r_eff else 0.0
                return -(lo + integrate.quad(lambda q: q * u(q), max(rv, r_eff), np.inf, limit=400)[0])
        rr = np.unique(np.round(rg[face], 12))
        lut = {k: chi_of_r(k) for k in rr}
        ghosts = np.zeros(rg.shape)
        ghosts[face] = [lut[k] for k in np.round(rg[face], 12)]
        chi, rep = oracle.fas_solve(c["xi"] * c["s"] * delta, h, c["nu"], c["K"], tol=1e-11, max_cycles=200,
                                    ghosts=ghosts)
        assert rep["status"] == 0
        full = ghosts.copy()
        full[1:-1, 1:-1, 1:-1] = chi
        g = [(np.roll(full, -1, ax) - np.roll(full, 1, ax))[1:-1, 1:-1, 1:-1] / (2 * h) for ax in range(3)]
        radial = (g[0] * X[0] + g[1] * X[1] + g[2] * X[2]) / r
        for lo, hi, tol in ((1.0, R - 2.0, 1e-2), (R + 2.0, 2.5 * R, ext_tol)):
            sel = (r > lo * h) & (r < hi * h)
            exact = np.array([rv * u(rv) for rv in r[sel]])
            worst = np.abs(radial[sel] / exact - 1.0).max()
            assert worst < tol, (screening, lo, hi, worst)
