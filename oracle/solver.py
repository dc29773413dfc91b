"""Scalar-field and Poisson solves and the full PM gravity step in float64
(oracle; test infrastructure only).

The nonlinear scalar-field solve calls the plain-C FAS multigrid in
``oracle/csrc/chi_fas.c`` (damped Jacobi, Laplacian-form Newton update with
mean subtraction, void clamp).  Linear problems are solved exactly with the
FFT eigen-decomposition of the periodic 7-point Laplacian.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build
from .coeffs import eft_coefficients
from .fields import (
    cic_deposit,
    cic_interpolate,
    density_contrast,
    gradient5,
    poisson_fft,
)

_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.ensure_built())
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.orc_chi_solve.argtypes = [
            ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp,
        ]
        _lib.orc_chi_solve.restype = ctypes.c_int
        _lib.orc_chi_operator.argtypes = [
            ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, dp,
        ]
        _lib.orc_chi_operator.restype = ctypes.c_longlong
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fas_solve(b, h, nu, K, tol=1e-12, max_cycles=200, npre=6, npost=6, omega=0.6, guess=None, ghosts=None):
    """Solve lap chi = Lq(K T(chi) - b) - <.> (periodic) or with the Dirichlet
    ghost values ``ghosts`` ((n+2)^3) by FAS V-cycles.

    Returns (chi, report) with report = dict(rel_residual, vcycles, clamped, status).
    """
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = b.shape[0]
    chi = np.zeros_like(b) if guess is None else np.array(guess, dtype=np.float64, order="C", copy=True)
    gh = None if ghosts is None else np.ascontiguousarray(ghosts, dtype=np.float64)
    rep = np.zeros(4)
    lib.orc_chi_solve(n, float(h), _ptr(b), _ptr(gh), float(nu), float(K), float(tol), int(max_cycles),
                      int(npre), int(npost), float(omega), _ptr(chi), _ptr(rep))
    return chi, dict(rel_residual=float(rep[0]), vcycles=int(rep[1]), clamped=int(rep[2]), status=int(rep[3]))


def chi_operator(chi, b, h, nu, K, ghosts=None):
    """Discrete operator pieces at ``chi``: dict(lap, lq, T, r, clamped)."""
    lib = _load()
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = chi.shape[0]
    out = {k: np.empty_like(chi) for k in ("lap", "lq", "T", "r")}
    gh = None if ghosts is None else np.ascontiguousarray(ghosts, dtype=np.float64)
    ncl = lib.orc_chi_operator(n, float(h), _ptr(b), _ptr(gh), float(nu), float(K), _ptr(chi),
                               _ptr(out["lap"]), _ptr(out["lq"]), _ptr(out["T"]), _ptr(out["r"]))
    out["clamped"] = int(ncl)
    return out


def relative_residual(chi, delta, coeffs, h):
    """||r||_2 / ||xi s delta / nu||_2 of the discrete scalar-field system."""
    b = coeffs["xi"] * coeffs["s"] * delta
    op = chi_operator(chi, b, h, coeffs["nu"], coeffs["K"])
    return float(np.linalg.norm(op["r"]) / np.linalg.norm(b / coeffs["nu"]))


def solve_poisson(delta, coeffs, h):
    """Newtonian potential: lap_7 Psi_N = s delta, <Psi_N> = 0 (eq. phipsi_mod,
    with Geff/G inside s)."""
    return poisson_fft(coeffs["s"] * delta, h)


def solve_chi_linear(delta, coeffs, h):
    """Screening-off scalar field: lap_7 chi = mu_chi s delta, exact (eq. linearised)."""
    return poisson_fft(coeffs["mu_chi"] * coeffs["s"] * delta, h)


def solve_chi(delta, coeffs, h, tol=1e-12, max_cycles=200, guess=None, **kw):
    """Nonlinear scalar field of eq. chi_scm on the periodic grid."""
    nu, xi = coeffs["nu"], coeffs["xi"]
    if xi == 0.0:
        return np.zeros_like(delta), dict(rel_residual=0.0, vcycles=0, clamped=0, status=0)
    b = xi * coeffs["s"] * delta
    return fas_solve(b, h, nu, coeffs["K"], tol=tol, max_cycles=max_cycles, guess=guess, **kw)


def pm_step(pos, vel, ng, params, dt_kick, dt_drift=0.0, tol=1e-12, chi_guess=None, linear_chi=False):
    """One PM gravity step: CIC deposit, Poisson, scalar field, combined 5-point
    gradient of Psi_N + xi chi, CIC interpolation, kick (and optional drift).

    ``params``: dict(omega_m0, alpha_b0, alpha_m0, a[, screening, alpha_b_dot]).
    Returns a dict with rho, delta, psi, chi, g_grid, acc (per particle),
    vel, pos and the solve report.
    """
    h = 1.0 / ng
    c = eft_coefficients(params["omega_m0"], params["alpha_b0"], params["alpha_m0"], params["a"],
                         screening=params.get("screening", True), alpha_b_dot=params.get("alpha_b_dot", True))
    rho = cic_deposit(pos, ng)
    delta = density_contrast(rho)
    psi = solve_poisson(delta, c, h)
    if linear_chi or c["K"] == 0.0:
        chi = solve_chi_linear(delta, c, h) if c["xi"] != 0.0 else np.zeros_like(delta)
        rep = dict(rel_residual=0.0, vcycles=0, clamped=0, status=0)
    else:
        chi, rep = solve_chi(delta, c, h, tol=tol, guess=chi_guess)
    g = gradient5(psi + c["xi"] * chi, h)
    acc = cic_interpolate(g, pos)
    vel_new = np.asarray(vel, dtype=np.float64) + acc * dt_kick
    pos_new = np.mod(np.asarray(pos, dtype=np.float64) + vel_new * dt_drift, 1.0) if dt_drift else np.array(pos, dtype=np.float64)
    return dict(coeffs=c, rho=rho, delta=delta, psi=psi, chi=chi, g_grid=g, acc=acc, vel=vel_new, pos=pos_new, report=rep)
