"""Multi-step particle-mesh evolution and the Bardeen potentials in float64
(oracle; test infrastructure only).

* code_time: the code-unit time of Sec. 3.1, t~ = t H0 / a^2, so that
  dt~ = da / (a^3 E(a)); the particle equations are dx/dt~ = v and
  dv/dt~ = -grad Psi (Psi = Psi_N + xi chi, eq. phipsi_mod).
* potentials: Psi = Psi_N + (alpha_B - alpha_M) chi and
  Phi = Psi_N + alpha_B chi (eqs. phipsi_mod), and Psi + Phi.
* evolve: kick-drift-kick leapfrog in t~ between scale factors a_k, one
  force evaluation per a_k (the coefficients taken at a_k), kicks over
  [a_{k-1/2}, a_{k+1/2}] and drifts over [a_k, a_{k+1}], the previous step's
  scalar field as the next solve's guess (Sec. 3.5.1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from .coeffs import e2, eft_coefficients
from .solver import pm_step


def code_time(a0, a1, omega_m0):
    """int_{a0}^{a1} da / (a^3 E(a)) by adaptive quadrature."""
    val, _ = integrate.quad(lambda a: 1.0 / (a**3 * math.sqrt(e2(a, omega_m0))), a0, a1, epsabs=0.0, epsrel=1e-13,
                            limit=200)
    return val


def potentials(psi_n, chi, params):
    """(Psi, Phi, Psi + Phi) from Psi_N and chi at params["a"]."""
    c = eft_coefficients(params["omega_m0"], params["alpha_b0"], params["alpha_m0"], params["a"],
                         screening=params.get("screening", True), alpha_b_dot=params.get("alpha_b_dot", True))
    psi = psi_n + c["xi"] * chi
    phi = psi_n + c["alpha_b"] * chi
    return psi, phi, psi + phi


def scale_factors(a_start, a_end, nsteps, log_spacing=False):
    """a_k for k = 0 .. 2 nsteps in half steps (index 2k is a_k)."""
    t = np.arange(2 * nsteps + 1) / (2.0 * nsteps)
    if log_spacing:
        return a_start * (a_end / a_start) ** t
    return a_start + (a_end - a_start) * t


def evolve(pos, vel, ng, params, a_start, a_end, nsteps, tol=1e-12, log_spacing=False, linear_chi=False):
    """KDK from a_start to a_end; returns dict(pos, vel, psi, chi, reports)."""
    a = scale_factors(a_start, a_end, nsteps, log_spacing)
    om0 = params["omega_m0"]
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    chi = None
    reports = []
    out = None
    for k in range(nsteps + 1):
        lo = a[2 * k - 1] if k > 0 else a[0]
        hi = a[2 * k + 1] if k < nsteps else a[2 * nsteps]
        dk = code_time(lo, hi, om0)
        dd = code_time(a[2 * k], a[2 * k + 2], om0) if k < nsteps else 0.0
        prm = dict(params, a=float(a[2 * k]))
        out = pm_step(pos, vel, ng, prm, dt_kick=dk, dt_drift=dd, tol=tol, chi_guess=chi, linear_chi=linear_chi)
        pos, vel, chi = out["pos"], out["vel"], out["chi"]
        reports.append(out["report"])
    return dict(pos=pos, vel=vel, psi=out["psi"], chi=chi, reports=reports)
