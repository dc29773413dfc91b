"""MI355X-native particle-mesh gravity step of the cubic-screening EFT of
dark energy (HIP kernels behind the C ABI of include/pmeft.h).

The Python functions below have the names of the C entry points and only
marshal arguments: torch tensors on the GPU go in as device pointers with the
current HIP stream, parameters and options as C structs.  Fields are
``(ng, ng, ng)`` tensors in C order, particles ``(3, np)`` tensors (structure
of arrays), float32 or float64.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib as L

__all__ = [
    "MgOpts", "PmError", "Workspace", "mg_batched_workspace_bytes", "mg_poisson_solve", "mg_scalar_solve",
    "mg_scalar_solve_batched", "pm_autotune", "pm_deposit", "pm_eft_coefficients", "pm_get_launch_shape",
    "pm_set_launch_shape", "pm_sort_particles", "pm_tune_load", "pm_tune_save",
    "pm_force_interp", "pm_grid_levels", "pm_kernel_timing_enable", "pm_kernel_timing_read", "pm_step",
    "pm_strerror", "pm_workspace_bytes", "pm_potentials", "pm_evolve", "pm_code_time", "pm_field_power",
    "pm_particle_power", "pm_boost", "pm_set_step_concurrency",
]


class PmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {pm_strerror(code)} (code {code})")


@dataclass
class MgOpts:
    rel_tol: float = 1e-7
    max_vcycles: int = 50
    n_pre: int = 1
    n_post: int = 2
    precision: str = "f64"  # "f64" | "mixed"
    guess: str = "zero"     # "zero" | "given" | "linear" | "learned"
    learned: object = None  # warmstart.WarmStart, for guess "learned"
    smoother: str = "rbgs"  # "rbgs" | "jacobi"
    jacobi_weight: float = 0.6

    def c(self, ng=None):
        prec = {"f64": L.PM_PREC_F64, "mixed": L.PM_PREC_MIXED}[self.precision]
        guess = {"zero": L.PM_GUESS_ZERO, "given": L.PM_GUESS_GIVEN, "linear": L.PM_GUESS_LINEAR,
                 "learned": L.PM_GUESS_LEARNED}[self.guess]
        o = L.MgOpts(self.rel_tol, self.max_vcycles, self.n_pre, self.n_post, prec, guess)
        o.smoother = {"rbgs": 0, "jacobi": 1}[self.smoother]
        o.jacobi_weight = float(self.jacobi_weight)
        if self.guess == "learned":
            if self.learned is None or ng is None:
                raise ValueError("guess 'learned' needs MgOpts.learned (a WarmStart) and the grid size")
            ws = self.learned.inference_workspace(ng)
            o.learned_params = self.learned.params.data_ptr()
            o.learned_ws = ws.data_ptr()
            o.learned_ws_bytes = ws.numel()
        return o


def _params(p):
    return L.EftParams(float(p["omega_m0"]), float(p["alpha_b0"]), float(p["alpha_m0"]), float(p["a"]),
                       int(p.get("screening", 1)), int(p.get("alpha_b_dot", 1)))


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return L.PM_F64
    if t.dtype == torch.float32:
        return L.PM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _check(t, shape, dt, name):
    if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape) or _dtype_code(t) != dt:
        raise ValueError(f"{name}: need a contiguous device tensor of shape {tuple(shape)} and matching dtype")


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _report(r):
    return dict(status=r.status, vcycles=r.vcycles, rel_residual=r.rel_residual,
                residual_hist=list(r.residual_hist[: min(max(r.vcycles + 1, 1), 64)]), mean_shift=r.mean_shift,
                clamped_cells=r.clamped_cells, ms=r.ms)


def pm_kernel_timing_enable(on=True):
    rc = L.lib().pm_kernel_timing_enable(int(bool(on)))
    if rc:
        raise PmError(rc, "pm_kernel_timing_enable")


def pm_kernel_timing_read():
    """{slot: (total_ms, launches)} for the finest-level smoother launches
    timed since the last read (slots: scalar_f64, scalar_f32, poisson_f64,
    poisson_f32 for half-sweeps, the same with _fused for fused sweeps)."""
    ms = (ctypes.c_double * 8)()
    n = (ctypes.c_longlong * 8)()
    rc = L.lib().pm_kernel_timing_read(ms, n)
    if rc:
        raise PmError(rc, "pm_kernel_timing_read")
    names = ("scalar_f64", "scalar_f32", "poisson_f64", "poisson_f32", "scalar_f64_fused", "scalar_f32_fused",
             "poisson_f64_fused", "poisson_f32_fused")
    return {k: (ms[q], n[q]) for q, k in enumerate(names)}


def pm_strerror(code):
    return L.lib().pm_strerror(int(code)).decode()


def pm_eft_coefficients(params):
    c = L.EftCoeffs()
    rc = L.lib().pm_eft_coefficients(ctypes.byref(_params(params)), ctypes.byref(c))
    out = {n: getattr(c, n) for n, _ in L.EftCoeffs._fields_}
    out["lambda"] = out.pop("lambda_")
    out["status"] = rc
    return out


def pm_grid_levels(ng):
    return L.lib().pm_grid_levels(int(ng))


def pm_workspace_bytes(ng, np_, dtype, precision="any"):
    prec = {"f64": L.PM_PREC_F64, "mixed": L.PM_PREC_MIXED, "any": L.PM_PREC_ANY}[precision]
    return int(L.lib().pm_workspace_bytes(int(ng), int(np_), int(dtype), prec))


class Workspace:
    """Caller-owned scratch for the library (a uint8 device tensor)."""

    def __init__(self, ng, np_=0, dtype=L.PM_F64, precision="any", device="cuda"):
        import torch

        self.nbytes = pm_workspace_bytes(ng, np_, dtype, precision)
        if self.nbytes == 0:
            raise PmError(L.PM_EINVAL, f"workspace for ng={ng}")
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        if self.buf.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def _ws(ws, ng, np_, dt):
    return ws if ws is not None else Workspace(ng, np_, dt)


def pm_deposit(pos, ng, rho, ws=None, stream=None):
    dt = _dtype_code(pos)
    npart = pos.shape[1]
    _check(pos, (3, npart), dt, "pos")
    _check(rho, (ng, ng, ng), dt, "rho")
    ws = _ws(ws, ng, npart, dt)
    rc = L.lib().pm_deposit(ctypes.c_void_p(pos.data_ptr()), npart, dt, int(ng), ctypes.c_void_p(rho.data_ptr()),
                          ws.ptr, ws.nbytes, _stream(stream))
    if rc:
        raise PmError(rc, "pm_deposit")


def _grid_solve(fn, name, rho, params, opts, out, ws, stream):
    dt = _dtype_code(rho)
    ng = rho.shape[0]
    _check(rho, (ng, ng, ng), dt, "rho")
    _check(out, (ng, ng, ng), dt, "out")
    ws = _ws(ws, ng, 0, dt)
    rep = L.MgReport()
    rc = fn(ctypes.c_void_p(rho.data_ptr()), int(ng), dt, ctypes.byref(_params(params)), ctypes.byref(opts.c(ng)),
            ctypes.c_void_p(out.data_ptr()), ctypes.byref(rep), ws.ptr, ws.nbytes, _stream(stream))
    if rc not in (L.PM_OK, L.PM_ENOCONV):
        raise PmError(rc, name)
    return _report(rep)


def mg_poisson_solve(rho, params, opts, psi, ws=None, stream=None):
    return _grid_solve(L.lib().mg_poisson_solve, "mg_poisson_solve", rho, params, opts, psi, ws, stream)


def mg_scalar_solve(rho, params, opts, chi, ws=None, stream=None):
    return _grid_solve(L.lib().mg_scalar_solve, "mg_scalar_solve", rho, params, opts, chi, ws, stream)


def mg_batched_workspace_bytes(problems, precision="f64"):
    arr = _problems(problems)
    prec = {"f64": L.PM_PREC_F64, "mixed": L.PM_PREC_MIXED}[precision]
    return int(L.lib().mg_batched_workspace_bytes(arr, len(problems), prec))


def _problems(problems):
    arr = (L.Problem * len(problems))()
    for k, pr in enumerate(problems):
        rho, chi = pr["rho"], pr["chi"]
        dt = _dtype_code(rho)
        ng = rho.shape[0]
        _check(rho, (ng, ng, ng), dt, "rho")
        _check(chi, (ng, ng, ng), dt, "chi")
        arr[k] = L.Problem(rho.data_ptr(), chi.data_ptr(), ng, dt, _params(pr["params"]))
    return arr


def mg_scalar_solve_batched(problems, opts, ws=None, stream=None):
    """Solve many scalar-field problems in one call.  problems: list of dicts
    with device tensors ``rho`` and ``chi`` (ng^3, either dtype, ng may
    differ) and ``params``; returns the list of per-problem reports."""
    import torch

    arr = _problems(problems)
    n = len(problems)
    need = mg_batched_workspace_bytes(problems, opts.precision)
    if need == 0:
        raise PmError(L.PM_EINVAL, "mg_scalar_solve_batched")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=problems[0]["rho"].device)
    reps = (L.MgReport * n)()
    rc = L.lib().mg_scalar_solve_batched(arr, n, ctypes.byref(opts.c()), reps, ctypes.c_void_p(ws.data_ptr()),
                                         ws.numel(), _stream(stream))
    if rc not in (L.PM_OK, L.PM_ENOCONV):
        raise PmError(rc, "mg_scalar_solve_batched")
    return [_report(r) for r in reps]


def pm_sort_particles(pos, ng, vel=None, ids=None, ws=None, stream=None):
    """Reorder particles (and vel, int64 ids) by the cell of their CIC base
    corner, stably and deterministically (in place)."""
    import torch

    dt = _dtype_code(pos)
    npart = pos.shape[1]
    _check(pos, (3, npart), dt, "pos")
    if vel is not None:
        _check(vel, (3, npart), dt, "vel")
    if ids is not None and (ids.dtype != torch.int64 or not ids.is_contiguous() or ids.numel() != npart
                            or not ids.is_cuda):
        raise ValueError("ids: need a contiguous int64 device tensor of np entries")
    need = int(L.lib().pm_sort_workspace_bytes(npart, dt))
    if need == 0:
        raise PmError(L.PM_EINVAL, "pm_sort_particles")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=pos.device)
    rc = L.lib().pm_sort_particles(ctypes.c_void_p(pos.data_ptr()),
                                   ctypes.c_void_p(vel.data_ptr() if vel is not None else 0),
                                   ctypes.c_void_p(ids.data_ptr() if ids is not None else 0), npart, int(ng), dt,
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    if rc:
        raise PmError(rc, "pm_sort_particles")


def pm_autotune(ng, precision="f64", ws=None, stream=None):
    """Time the launch-shape candidates for (ng, precision) and keep the fastest."""
    import torch

    prec = {"f64": L.PM_PREC_F64, "mixed": L.PM_PREC_MIXED}[precision]
    need = int(L.lib().pm_autotune_workspace_bytes(int(ng), prec))
    if need == 0:
        raise PmError(L.PM_EINVAL, "pm_autotune")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rc = L.lib().pm_autotune(int(ng), prec, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    if rc:
        raise PmError(rc, "pm_autotune")
    return pm_get_launch_shape(ng, 4 if precision == "mixed" else 8)


def pm_get_launch_shape(ng, word_bytes):
    """(block_cycle_grid, tiled_smoother) for (ng, word size)."""
    b, t = ctypes.c_int(0), ctypes.c_int(0)
    rc = L.lib().pm_get_launch_shape(int(ng), int(word_bytes), ctypes.byref(b), ctypes.byref(t))
    if rc:
        raise PmError(rc, "pm_get_launch_shape")
    return b.value, t.value


def pm_set_launch_shape(ng, word_bytes, block_cycle_grid, tiled_smoother=1):
    rc = L.lib().pm_set_launch_shape(int(ng), int(word_bytes), int(block_cycle_grid), int(tiled_smoother))
    if rc:
        raise PmError(rc, "pm_set_launch_shape")


def pm_tune_save(path):
    rc = L.lib().pm_tune_save(str(path).encode())
    if rc:
        raise PmError(rc, "pm_tune_save")


def pm_tune_load(path):
    rc = L.lib().pm_tune_load(str(path).encode())
    if rc:
        raise PmError(rc, "pm_tune_load")


def pm_force_interp(psi, chi, params, pos, vel, dt_kick, acc_out=None, ws=None, stream=None):
    dt = _dtype_code(pos)
    ng = psi.shape[0]
    npart = pos.shape[1]
    _check(psi, (ng, ng, ng), dt, "psi")
    if chi is not None:
        _check(chi, (ng, ng, ng), dt, "chi")
    _check(pos, (3, npart), dt, "pos")
    _check(vel, (3, npart), dt, "vel")
    if acc_out is not None:
        _check(acc_out, (3, npart), dt, "acc_out")
    ws = _ws(ws, ng, npart, dt)
    rc = L.lib().pm_force_interp(ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(chi.data_ptr() if chi is not None else 0),
                               int(ng), dt, ctypes.byref(_params(params)), ctypes.c_void_p(pos.data_ptr()), npart,
                               ctypes.c_void_p(vel.data_ptr()), float(dt_kick),
                               ctypes.c_void_p(acc_out.data_ptr() if acc_out is not None else 0), ws.ptr, ws.nbytes,
                               _stream(stream))
    if rc:
        raise PmError(rc, "pm_force_interp")


def pm_step(pos, vel, ng, params, poisson_opts, scalar_opts, dt_kick, dt_drift, psi, chi, ws=None, stream=None):
    dt = _dtype_code(pos)
    npart = pos.shape[1]
    _check(pos, (3, npart), dt, "pos")
    _check(vel, (3, npart), dt, "vel")
    _check(psi, (ng, ng, ng), dt, "psi")
    _check(chi, (ng, ng, ng), dt, "chi")
    ws = _ws(ws, ng, npart, dt)
    rep = L.StepReport()
    rc = L.lib().pm_step(ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()), npart, int(ng), dt,
                       ctypes.byref(_params(params)), ctypes.byref(poisson_opts.c(ng)), ctypes.byref(scalar_opts.c(ng)),
                       float(dt_kick), float(dt_drift), ctypes.c_void_p(psi.data_ptr()),
                       ctypes.c_void_p(chi.data_ptr()), ctypes.byref(rep), ws.ptr, ws.nbytes, _stream(stream))
    if rc not in (L.PM_OK, L.PM_ENOCONV):
        raise PmError(rc, "pm_step")
    return dict(poisson=_report(rep.poisson), scalar=_report(rep.scalar), ms_deposit=rep.ms_deposit,
                ms_force=rep.ms_force, ms_total=rep.ms_total, status=rc)


def pm_potentials(psi_n, chi, params, psi_out=None, phi_out=None, lens_out=None, stream=None):
    """Psi = Psi_N + xi chi, Phi = Psi_N + alpha_B chi and Psi + Phi (each
    output optional) from Psi_N and chi."""
    dt = _dtype_code(psi_n)
    ng = psi_n.shape[0]
    _check(psi_n, (ng, ng, ng), dt, "psi_n")
    _check(chi, (ng, ng, ng), dt, "chi")
    for t, nm in ((psi_out, "psi_out"), (phi_out, "phi_out"), (lens_out, "lens_out")):
        if t is not None:
            _check(t, (ng, ng, ng), dt, nm)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)  # noqa: E731
    rc = L.lib().pm_potentials(ptr(psi_n), ptr(chi), int(ng), dt, ctypes.byref(_params(params)), ptr(psi_out),
                               ptr(phi_out), ptr(lens_out), _stream(stream))
    if rc:
        raise PmError(rc, "pm_potentials")


def pm_code_time(a0, a1, omega_m0):
    """int_{a0}^{a1} da / (a^3 E(a)) (the code time of a kick or drift)."""
    return float(L.lib().pm_code_time(float(a0), float(a1), float(omega_m0)))


def pm_evolve(pos, vel, ng, params, a_start, a_end, nsteps, poisson_opts, scalar_opts, psi, chi, log_spacing=False,
              ws=None, stream=None):
    """Kick-drift-kick evolution from a_start to a_end (see pmeft.h)."""
    dt = _dtype_code(pos)
    npart = pos.shape[1]
    _check(pos, (3, npart), dt, "pos")
    _check(vel, (3, npart), dt, "vel")
    _check(psi, (ng, ng, ng), dt, "psi")
    _check(chi, (ng, ng, ng), dt, "chi")
    ws = _ws(ws, ng, npart, dt)
    rep = L.EvolveReport()
    rc = L.lib().pm_evolve(ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vel.data_ptr()), npart, int(ng), dt,
                           ctypes.byref(_params(params)), float(a_start), float(a_end), int(nsteps),
                           int(bool(log_spacing)), ctypes.byref(poisson_opts.c(ng)), ctypes.byref(scalar_opts.c(ng)),
                           ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(chi.data_ptr()), ctypes.byref(rep),
                           ws.ptr, ws.nbytes, _stream(stream))
    if rc not in (L.PM_OK, L.PM_ENOCONV):
        raise PmError(rc, "pm_evolve")
    return {n: getattr(rep, n) for n, _ in L.EvolveReport._fields_}


def _power_out(nbins):
    return [(ctypes.c_double * nbins)() for _ in range(3)]


def _power_ws(n, particles, ws):
    import torch

    need = int(L.lib().pm_power_workspace_bytes(int(n), int(particles)))
    if need == 0:
        raise PmError(L.PM_EINVAL, f"power spectrum workspace for n={n}")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    return ws


def pm_field_power(field, box, nbins=None, ws=None, stream=None):
    """(k, P, counts) of a periodic (n, n, n) device field (see pmeft.h)."""
    import numpy as np

    dt = _dtype_code(field)
    n = field.shape[0]
    _check(field, (n, n, n), dt, "field")
    nb = n // 4 if nbins is None else int(nbins)
    ws = _power_ws(n, 0, ws)
    k, p, c = _power_out(nb)
    rc = L.lib().pm_field_power(ctypes.c_void_p(field.data_ptr()), int(n), dt, float(box), nb, k, p, c,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    if rc:
        raise PmError(rc, "pm_field_power")
    return np.array(k), np.array(p), np.array(c)


def pm_particle_power(pos, n, box, nbins=None, ws=None, stream=None):
    """(k, P, counts) of the CIC density of the particles on an n^3 grid."""
    import numpy as np

    dt = _dtype_code(pos)
    npart = pos.shape[1]
    _check(pos, (3, npart), dt, "pos")
    nb = n // 4 if nbins is None else int(nbins)
    ws = _power_ws(n, 1, ws)
    k, p, c = _power_out(nb)
    rc = L.lib().pm_particle_power(ctypes.c_void_p(pos.data_ptr()), npart, dt, int(n), float(box), nb, k, p, c,
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
    if rc:
        raise PmError(rc, "pm_particle_power")
    return np.array(k), np.array(p), np.array(c)


def pm_boost(k, pk_num, pk_den, sigma_k=0.0):
    """Gaussian-smoothed P_num / P_den over the bins (host)."""
    import numpy as np

    nb = len(k)
    arr = lambda a: (ctypes.c_double * nb)(*[float(x) for x in a])  # noqa: E731
    out = (ctypes.c_double * nb)()
    rc = L.lib().pm_boost(arr(k), arr(pk_num), arr(pk_den), nb, float(sigma_k), out)
    if rc:
        raise PmError(rc, "pm_boost")
    return np.array(out)


def pm_set_step_concurrency(side_by_side=True):
    """pm_step's solves side by side (True, default) or both on the caller's
    stream from the calling thread (False); returns the previous setting."""
    return bool(L.lib().pm_set_step_concurrency(int(bool(side_by_side))))
