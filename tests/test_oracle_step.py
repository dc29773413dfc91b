"""Pins of the oracle's full PM step."""
import numpy as np
import pytest

import oracle
from workloads import lattice_displacement_ics, zeldovich_ics


def test_screening_off_force_ratio_is_geff_mu_psi():
    """Linearised option: Psi_tot satisfies lap Psi = mu_Psi s delta with s
    carrying Geff/G (eqs. linearised, phipsi_mod), so per particle
    g_EFT / g_LCDM = (Geff/G) mu_Psi exactly for the same positions."""
    ng = 16
    pos = lattice_displacement_ics(ng, 100.0, seed=3, rms_cells=0.5)
    vel = np.zeros_like(pos)
    p = dict(omega_m0=0.3071, alpha_b0=-0.3, alpha_m0=0.15, a=0.7)
    eft = oracle.pm_step(pos, vel, ng, dict(p, screening=False), dt_kick=1.0)
    lcdm = oracle.pm_step(pos, vel, ng, dict(p, alpha_b0=0.0, alpha_m0=0.0), dt_kick=1.0)
    c = eft["coeffs"]
    np.testing.assert_allclose(eft["acc"], c["geff"] * c["mu_psi"] * lcdm["acc"], rtol=1e-9,
                               atol=1e-12 * np.abs(lcdm["acc"]).max())


def test_momentum_conservation_linear_parts():
    """The 5-point gradient of a periodic potential sums to zero over the
    grid; with CIC deposit and interpolation by the same kernel, the total
    force on all particles vanishes for the linear (screening-off) step."""
    ng = 16
    pos = zeldovich_ics(ng, 250.0, seed=1)
    out = oracle.pm_step(pos, np.zeros_like(pos), ng, dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=1.0,
                                                          screening=False), dt_kick=1.0)
    tot = out["acc"].sum(axis=1)
    assert np.abs(tot).max() < 1e-10 * np.abs(out["acc"]).sum()


def test_uniform_lattice_gives_zero_force_and_exact_kick():
    ng = 16
    q = (np.arange(ng) + 0.5) / ng
    pos = np.stack([g.ravel() for g in np.meshgrid(q, q, q, indexing="ij")])
    vel = np.random.default_rng(0).standard_normal(pos.shape)
    out = oracle.pm_step(pos, vel, ng, dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=0.5), dt_kick=0.3,
                         dt_drift=0.1)
    np.testing.assert_allclose(out["acc"], 0.0, atol=1e-12)
    np.testing.assert_allclose(out["vel"], vel, atol=1e-12)
    np.testing.assert_allclose(out["pos"], np.mod(pos + 0.1 * vel, 1.0), atol=1e-12)


def test_fifth_force_enhances_gravity_when_unscreened():
    """mu_Psi > 1 (Sec. 4.2): with screening the fifth force is weaker than
    in the linearised step, but still adds to Newtonian gravity."""
    ng = 32
    pos = lattice_displacement_ics(ng, 100.0, seed=0)
    p = dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=0.5)
    full = oracle.pm_step(pos, np.zeros_like(pos), ng, p, dt_kick=1.0)
    lin = oracle.pm_step(pos, np.zeros_like(pos), ng, dict(p, screening=False), dt_kick=1.0)
    newton = oracle.pm_step(pos, np.zeros_like(pos), ng, dict(p, alpha_b0=0.0), dt_kick=1.0)
    nf, nl, nn = (np.linalg.norm(o["acc"]) for o in (full, lin, newton))
    assert nn < nf < nl
    assert full["report"]["status"] == 0
