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
