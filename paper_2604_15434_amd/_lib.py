"""ctypes binding of libpmeft.so (the C ABI in include/pmeft.h).

Argument marshalling only: tensors are passed as device pointers with the
caller's current HIP stream; every step of the computation runs in the
library's HIP kernels.  The first call fails with an ImportError if the
library has not been built (``python -m paper_2604_15434_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmeft.so")

PM_OK, PM_EINVAL, PM_EUNSTABLE, PM_ENOCONV, PM_ENONFINITE, PM_EHIP, PM_ENOMEM = 0, -1, -2, -3, -4, -5, -6
PM_F32, PM_F64 = 0, 1
PM_PREC_F64, PM_PREC_MIXED, PM_PREC_ANY = 0, 1, 2
PM_GUESS_ZERO, PM_GUESS_GIVEN, PM_GUESS_LINEAR, PM_GUESS_LEARNED = 0, 1, 2, 3


class EftParams(ctypes.Structure):
    _fields_ = [("omega_m0", ctypes.c_double), ("alpha_b0", ctypes.c_double), ("alpha_m0", ctypes.c_double),
                ("a", ctypes.c_double), ("screening", ctypes.c_int), ("alpha_b_dot", ctypes.c_int)]


class EftCoeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("omega_m_a", "E2", "alpha_b", "alpha_m", "geff", "C2", "C4", "nu",
                                                "xi", "mu_chi", "mu_psi", "s", "K", "lambda_")]


class MgOpts(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_vcycles", ctypes.c_int), ("n_pre", ctypes.c_int),
                ("n_post", ctypes.c_int), ("precision", ctypes.c_int), ("guess", ctypes.c_int),
                ("learned_params", ctypes.c_void_p), ("learned_ws", ctypes.c_void_p),
                ("learned_ws_bytes", ctypes.c_size_t), ("smoother", ctypes.c_int), ("jacobi_weight", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("chi", ctypes.c_void_p), ("ng", ctypes.c_int), ("dtype", ctypes.c_int),
                ("p", EftParams)]


class MgReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("vcycles", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("residual_hist", ctypes.c_double * 64), ("mean_shift", ctypes.c_double),
                ("clamped_cells", ctypes.c_longlong), ("ms", ctypes.c_float)]


class StepReport(ctypes.Structure):
    _fields_ = [("poisson", MgReport), ("scalar", MgReport), ("ms_deposit", ctypes.c_float),
                ("ms_force", ctypes.c_float), ("ms_total", ctypes.c_float)]


class EvolveReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int), ("force_evaluations", ctypes.c_int),
                ("max_scalar_vcycles", ctypes.c_int), ("poisson_vcycles", ctypes.c_longlong),
                ("scalar_vcycles", ctypes.c_longlong), ("clamped_cells_last", ctypes.c_longlong),
                ("max_rel_residual", ctypes.c_double), ("a_end", ctypes.c_double), ("ms_total", ctypes.c_float)]


EXPORTS = ("pm_eft_coefficients", "pm_grid_levels", "pm_workspace_bytes", "pm_deposit", "mg_poisson_solve",
           "mg_scalar_solve", "pm_force_interp", "pm_step", "pm_kernel_timing_enable", "pm_kernel_timing_read",
           "pm_strerror", "pm_sort_workspace_bytes", "pm_sort_particles", "mg_batched_workspace_bytes", "mg_scalar_solve_batched", "pm_autotune_workspace_bytes",
           "pm_autotune", "pm_get_launch_shape", "pm_set_launch_shape", "pm_tune_save", "pm_tune_load", "ws_unet_param_count", "ws_unet_workspace_bytes", "ws_unet_forward", "ws_unet_train_step",
           "ws_unet_forward_train", "ws_unet_backward", "ws_adam_workspace_bytes", "ws_adam_step",
           "ws_unet_tensor", "ws_conv3", "ws_conv3_first", "pm_potentials", "pm_evolve", "pm_code_time",
           "pm_plan_check", "pm_set_step_concurrency", "pm_deposit_noalloc", "pm_deposit_noalloc_max_bytes", "ws_unet_guess", "pm_power_workspace_bytes", "pm_field_power", "pm_particle_power", "pm_boost")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_15434_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, ll, i, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_longlong, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    lib.pm_eft_coefficients.argtypes = [P(EftParams), P(EftCoeffs)]
    lib.pm_grid_levels.argtypes = [i]
    lib.pm_workspace_bytes.argtypes = [i, ll, i, i]
    lib.pm_workspace_bytes.restype = sz
    lib.pm_deposit.argtypes = [vp, ll, i, i, vp, vp, sz, vp]
    lib.mg_poisson_solve.argtypes = [vp, i, i, P(EftParams), P(MgOpts), vp, P(MgReport), vp, sz, vp]
    lib.mg_scalar_solve.argtypes = [vp, i, i, P(EftParams), P(MgOpts), vp, P(MgReport), vp, sz, vp]
    lib.pm_force_interp.argtypes = [vp, vp, i, i, P(EftParams), vp, ll, vp, d, vp, vp, sz, vp]
    lib.pm_step.argtypes = [vp, vp, ll, i, i, P(EftParams), P(MgOpts), P(MgOpts), d, d, vp, vp, P(StepReport),
                            vp, sz, vp]
    lib.pm_kernel_timing_enable.argtypes = [i]
    lib.pm_kernel_timing_read.argtypes = [P(d), P(ll)]
    lib.pm_sort_workspace_bytes.argtypes = [ll, i]
    lib.pm_sort_workspace_bytes.restype = sz
    lib.pm_sort_particles.argtypes = [vp, vp, vp, ll, i, i, vp, sz, vp]
    lib.pm_sort_particles.restype = i
    lib.pm_autotune_workspace_bytes.argtypes = [i, i]
    lib.pm_autotune_workspace_bytes.restype = sz
    lib.pm_autotune.argtypes = [i, i, vp, sz, vp]
    lib.pm_get_launch_shape.argtypes = [i, i, P(i), P(i)]
    lib.pm_set_launch_shape.argtypes = [i, i, i, i]
    lib.pm_tune_save.argtypes = [ctypes.c_char_p]
    lib.pm_tune_load.argtypes = [ctypes.c_char_p]
    for name in ("pm_autotune", "pm_get_launch_shape", "pm_set_launch_shape", "pm_tune_save", "pm_tune_load"):
        getattr(lib, name).restype = i
    lib.mg_batched_workspace_bytes.argtypes = [P(Problem), i, i]
    lib.mg_batched_workspace_bytes.restype = sz
    lib.mg_scalar_solve_batched.argtypes = [P(Problem), i, P(MgOpts), P(MgReport), vp, sz, vp]
    lib.mg_scalar_solve_batched.restype = i
    lib.ws_unet_param_count.restype = ll
    lib.ws_unet_workspace_bytes.argtypes = [i, i]
    lib.ws_unet_workspace_bytes.restype = sz
    lib.ws_unet_forward.argtypes = [vp, vp, i, P(EftParams), vp, vp, sz, vp]
    lib.ws_unet_train_step.argtypes = [vp, vp, vp, ll, d, d, vp, vp, i, P(EftParams), vp, P(d), P(d), vp, sz, vp]
    lib.ws_unet_forward_train.argtypes = [vp, vp, i, P(EftParams), vp, vp, sz, vp]
    lib.ws_unet_backward.argtypes = [vp, vp, i, vp, vp, sz, vp]
    lib.ws_adam_workspace_bytes.argtypes = [ll]
    lib.ws_adam_workspace_bytes.restype = sz
    lib.ws_adam_step.argtypes = [vp, vp, vp, vp, ll, ll, d, d, d, d, d, P(d), vp, sz, vp]
    lib.ws_unet_tensor.argtypes = [vp, i, i, i, vp, vp]
    lib.ws_conv3.argtypes = [i, i, i, i, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.ws_conv3_first.argtypes = [i, vp, vp, vp, P(ctypes.c_float), vp, vp]
    for name in ("ws_unet_forward", "ws_unet_train_step", "ws_conv3", "ws_conv3_first", "ws_unet_forward_train",
                 "ws_unet_backward", "ws_adam_step", "ws_unet_tensor"):
        getattr(lib, name).restype = i
    lib.pm_potentials.argtypes = [vp, vp, i, i, P(EftParams), vp, vp, vp, vp]
    lib.pm_potentials.restype = i
    lib.pm_evolve.argtypes = [vp, vp, ll, i, i, P(EftParams), d, d, i, i, P(MgOpts), P(MgOpts), vp, vp,
                              P(EvolveReport), vp, sz, vp]
    lib.pm_evolve.restype = i
    lib.pm_code_time.argtypes = [d, d, d]
    lib.pm_code_time.restype = d
    lib.pm_power_workspace_bytes.argtypes = [i, i]
    lib.pm_power_workspace_bytes.restype = sz
    lib.pm_field_power.argtypes = [vp, i, i, d, i, P(d), P(d), P(d), vp, sz, vp]
    lib.pm_field_power.restype = i
    lib.pm_particle_power.argtypes = [vp, ll, i, i, d, i, P(d), P(d), P(d), vp, sz, vp]
    lib.pm_particle_power.restype = i
    lib.pm_boost.argtypes = [P(d), P(d), P(d), i, d, P(d)]
    lib.pm_boost.restype = i
    lib.pm_deposit_noalloc.argtypes = [vp, ll, i, i, vp, vp]
    lib.pm_deposit_noalloc.restype = i
    lib.pm_deposit_noalloc_max_bytes.restype = sz
    lib.pm_set_step_concurrency.argtypes = [i]
    lib.pm_set_step_concurrency.restype = i
    lib.ws_unet_guess.argtypes = [vp, vp, i, i, P(EftParams), vp, vp, sz, vp, sz, vp]
    lib.ws_unet_guess.restype = i
    lib.pm_plan_check.argtypes = [i, ll, i, i]
    lib.pm_plan_check.restype = i
    lib.pm_strerror.argtypes = [i]
    lib.pm_strerror.restype = ctypes.c_char_p
    for name in ("pm_eft_coefficients", "pm_grid_levels", "pm_deposit", "mg_poisson_solve", "mg_scalar_solve",
                 "pm_force_interp", "pm_step", "pm_kernel_timing_enable", "pm_kernel_timing_read"):
        getattr(lib, name).restype = i
    return lib


_LIB = None


def lib():
    """The loaded library; raises ImportError if libpmeft.so was not built."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB
