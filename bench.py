#!/usr/bin/env python3
"""Benchmark of the EFTofDE particle-mesh gravity step on one MI355X.

Workload: 256^3 grid and 256^3 particles in a 500 Mpc/h box, drawn from a
lognormal density (log-sigma 1.5, power-law-break spectrum, seed 2), with
alpha_B0 = -0.2, alpha_M0 = 0, a = 1 (Omega_m0 = 0.3071).  One step is the
whole hot path: CIC deposit, Poisson multigrid, screened scalar-field
multigrid to relative residual 1e-7 (both from a zero guess, every step
solving the same input from scratch), 5-point gradient, CIC interpolation
and kick.  Inputs are resident in device memory before the timed region;
the particles are put in CIC base-cell order once before timing (the order
a PM code keeps them in, re-sorting every few steps), which lets the
deposit gather instead of scatter.

Modes
  plain   : FP64 everywhere (particles, fields, V-cycles), zero guess.
  fp32    : FP32 particles and fields; mixed-precision solves (FP32 V-cycles
            on the FP64 defect, FP64 residual/test/coarsest solve), zero guess.
  learned : as fp32, with the learned warm start of the scalar field (the
            trained weights of paper_2604_15434_amd/weights; the network's
            forward pass and the linear pass on its source are inside the
            timed step).
The headline value is the learned mode when the weights exist, else fp32.
Launch shapes are autotuned for the grid before timing (--no-tune: defaults).

Prints one JSON line (rank 0).  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--ng 256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PARAMS = dict(omega_m0=0.3071, alpha_b0=-0.2, alpha_m0=0.0, a=1.0)


def smoother_bytes_per_launch(ng, itemsize, fused=False):
    """Algorithmic bytes of one finest-level smoother launch, counted as a
    smoother sweep is counted for the roofline: a full sweep (both colours)
    reads the iterate and the right-hand side and writes the iterate, 3 words
    per cell.  A half-sweep launch (one colour) is half of that; a fused
    launch is a full sweep."""
    return 3 * itemsize * ng**3 // (1 if fused else 2)


def smoother_operand_bytes_per_launch(ng, itemsize, with_tau, fused=False):
    """Bytes one launch must move with its operands as they are stored.
    Half-sweep, per cell of its colour: read own colour (edges), other colour
    (faces), delta (and the FAS source tau on the FP32 level), write own
    colour.  Fused sweep, per cell: read the old iterate, delta (and tau),
    write the new iterate."""
    if fused:
        return itemsize * (3 + (1 if with_tau else 0)) * ng**3
    per_cell = itemsize * (4 + (1 if with_tau else 0))
    return per_cell * ng**3 // 2


def run_mode(P, torch, mode, pos_np, ng, steps, warmup, net=None, presort=False):
    dt = torch.float64 if mode == "plain" else torch.float32
    prec = "f64" if mode == "plain" else "mixed"
    pos0 = torch.from_numpy(pos_np).to(device="cuda", dtype=dt).contiguous()
    if presort:  # once, before timing: the CIC base-cell order a PM code keeps its particles in
        P.pm_sort_particles(pos0, ng)
        torch.cuda.synchronize()
    pos = pos0.clone()
    vel = torch.zeros_like(pos)
    psi = torch.zeros((ng, ng, ng), dtype=dt, device="cuda")
    chi = torch.zeros_like(psi)
    ws = P.Workspace(ng, pos.shape[1], 1 if dt == torch.float64 else 0, "any")
    # smoothing schedules measured fastest inside the step: scalar field (1, 2)
    # everywhere; Poisson (1, 2) in FP64, (1, 3) in mixed precision
    opts = P.MgOpts(rel_tol=1e-7, max_vcycles=60, n_pre=1, n_post=2, precision=prec, guess="zero")
    popts = P.MgOpts(rel_tol=1e-7, max_vcycles=60, n_pre=1, n_post=3 if prec == "mixed" else 2, precision=prec,
                     guess="zero")
    sopts = opts
    if mode == "learned":
        sopts = P.MgOpts(rel_tol=1e-7, max_vcycles=60, n_pre=1, n_post=2, precision=prec, guess="learned",
                         learned=net)
    for k in range(warmup):
        # the last warm-up step runs with the launch timing on too: its events
        # (the pool the timed step reuses) have then been recorded once
        if k == warmup - 1:
            P.pm_kernel_timing_enable(True)
        P.pm_step(pos, vel, ng, PARAMS, popts, sopts, 1e-3, 0.0, psi, chi, ws=ws)
    torch.cuda.synchronize()
    P.pm_kernel_timing_enable(True)  # (creates the event pool if no warm-up step did)
    P.pm_kernel_timing_enable(False)
    P.pm_kernel_timing_read()  # clear
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        # the smoother's launch timing (two events around each finest-level
        # launch, about 0.5 ms per step on the two streams) runs in the last
        # timed step only
        if k == steps - 1:
            P.pm_kernel_timing_enable(True)
        reps.append(P.pm_step(pos, vel, ng, PARAMS, popts, sopts, 1e-3, 0.0, psi, chi, ws=ws))
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    P.pm_kernel_timing_enable(False)
    kt = P.pm_kernel_timing_read()
    # outside the timed region: the same finest-level smoother with nothing
    # running beside it, from one standalone scalar solve on this step's
    # density (zero guess, the mode's precision)
    rho = torch.zeros((ng, ng, ng), dtype=dt, device="cuda")
    P.pm_deposit(pos, ng, rho)
    solo = torch.zeros_like(rho)
    torch.cuda.synchronize()
    P.pm_kernel_timing_enable(True)
    P.mg_scalar_solve(rho, PARAMS, opts, solo)
    torch.cuda.synchronize()
    P.pm_kernel_timing_enable(False)
    kt_alone = P.pm_kernel_timing_read()
    del rho, solo
    last = reps[-1]
    ok = all(r["status"] == 0 and r["scalar"]["rel_residual"] <= 1e-7 for r in reps)
    return dict(ms_per_step=wall, converged=ok, sweeps={"scalar": [opts.n_pre, opts.n_post],
                                                       "poisson": [popts.n_pre, popts.n_post]},
                scalar_vcycles=last["scalar"]["vcycles"],
                scalar_residual_hist=[float(f"{x:.3g}") for x in last["scalar"]["residual_hist"][:last["scalar"]["vcycles"] + 1]],
                poisson_vcycles=last["poisson"]["vcycles"], scalar_rel_residual=last["scalar"]["rel_residual"],
                ms_deposit=last["ms_deposit"], ms_poisson=last["poisson"]["ms"], ms_scalar=last["scalar"]["ms"],
                ms_force=last["ms_force"], kernel_timing=kt, kernel_timing_alone=kt_alone,
                itemsize=8 if dt == torch.float64 else 4)


def smoother_sources(kernel):
    """Source files that define a smoother kernel: the half-sweep kernels, or
    the fused two-colour sweep."""
    last = "sweep2_kernels.hip" if kernel.startswith("k_sweep2_tile") else "smooth_kernels.hip"
    return [os.path.join(ROOT, "paper_2604_15434_amd", "csrc", f) for f in ("mg_stencil.h", "tile_window.h", last)]


def smoother_source_hash(kernel):
    import hashlib

    h = hashlib.sha256()
    for f in smoother_sources(kernel):
        h.update(open(f, "rb").read())
    return h.hexdigest()


def smoother_kernel(itemsize, tiled, ng):
    """Name of the finest-level scalar-field smoother the launch shape selects
    (the tile configuration rule of smooth_kernels.hip)."""
    r = "double" if itemsize == 8 else "float"
    nh = ng // 2
    tj, tk = 8, (32 if itemsize == 8 else 64)
    # the fused sweep: tiles of tj rows by tk packed elements, chunks of at
    # least 8 planes, at least 256 tiles (sweep2_kernels.hip)
    if tiled == 4 and ng >= 64 and nh % tk == 0 and ng % tj == 0 and (ng // tj) * (nh // tk) * (ng // 8) >= 256:
        return f"k_sweep2_tile<{r}, true, {tk}, {tj}>"
    if tiled and ng >= 64:
        if tiled == 3 and nh % 64 == 0 and ng % 16 == 0 and (ng // 16) * (nh // 64) * (ng // 16) >= 512:
            return f"k_smooth_tile<{r}, true, 64, 4, 16>"
        if tiled >= 2 and nh % 64 == 0 and ng % 16 == 0 and (ng // 8) * (nh // 64) * (ng // 16) >= 512:
            return f"k_smooth_tile<{r}, true, 64, 2, {8 if itemsize == 8 else 16}>"
        # small tiles only where they still give 256 tiles
        if nh % 64 == 0 and ng % 8 == 0 and (ng // 4) * (nh // 64) * (ng // 8) >= 256:
            return f"k_smooth_tile<{r}, true, 64, 1, 8>"
        if nh % 32 == 0 and ng % 8 == 0 and (ng // 8) * (nh // 32) * (ng // 8) >= 256:
            return f"k_smooth_tile<{r}, true, 32, 1, 8>"
    return f"k_smooth<{r}, true>"


def measured_traffic(kernel, ng):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken on the current smoother source at this grid."""
    path = os.path.join(ROOT, "profiles", f"pm_step_{ng}_smoother_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for k in rec.get("kernels", {}).values():
        if k.get("kernel") == kernel and k.get("source_sha256") == smoother_source_hash(kernel):
            return round(k["traffic_bytes"])
    return None


def roofline(res, ng, tiled):
    """Dominant kernel: the finest-level scalar-field smoother of the mode.
    The step runs its Poisson solve beside the scalar solve, so the timed
    launches share the GPU with the other solve's kernels; the figure is what
    the kernel achieves inside the step, not alone."""
    slot = "scalar_f64" if res["itemsize"] == 8 else "scalar_f32"
    fused = res["kernel_timing"].get(slot + "_fused", (0.0, 0))[1] > 0
    if fused:
        slot += "_fused"
    ms, n = res["kernel_timing"][slot]
    if n == 0:
        return None
    bytes_launch = smoother_bytes_per_launch(ng, res["itemsize"], fused)
    operand_bytes = smoother_operand_bytes_per_launch(ng, res["itemsize"], with_tau=res["itemsize"] == 4, fused=fused)
    achieved = bytes_launch / (ms / n * 1e-3) / 1e9
    kernel = smoother_kernel(res["itemsize"], tiled, ng)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, ng),
           "kernel": f"{kernel} (finest level, {'both colours' if fused else 'one colour'})",
           "bytes_per_launch": bytes_launch,
           "bytes_rule": "3 words per cell per full sweep (iterate + right-hand side read, iterate written)",
           "operand_bytes_per_launch": operand_bytes,
           "operand_GBps": round(operand_bytes / (ms / n * 1e-3) / 1e9, 1),
           "avg_launch_us": round(ms / n * 1e3, 2), "launches": n,
           "note": "launch times from the last timed step, where the Poisson solve runs concurrently on a second stream"}
    ms_a, n_a = res.get("kernel_timing_alone", {}).get(slot, (0.0, 0))
    if n_a:
        ach_a = bytes_launch / (ms_a / n_a * 1e-3) / 1e9
        out["alone"] = {"achieved": round(ach_a, 1), "frac": round(ach_a / HBM_PEAK_GBS, 4),
                        "avg_launch_us": round(ms_a / n_a * 1e3, 2), "launches": n_a,
                        "note": "the same launches in one standalone scalar solve on the step's density, "
                                "outside the timed region, nothing running beside it"}
    return out


def cpu_baseline(pos_np, ng):
    """The oracle on a bounded sample of the same workload, extrapolated to
    ms per step: deposit and interpolation on 1/8 of the particles (x8),
    exact FFT Poisson, one FAS V-cycle of the scalar field at full size times
    the number of oracle V-cycles to 1e-7 on a 64^3 grid of the same
    statistics, 5-point gradient."""
    import numpy as np

    import oracle
    from workloads import lognormal_density

    c = oracle.eft_coefficients(**PARAMS)
    h = 1.0 / ng
    sub = pos_np[:, ::8]
    t0 = time.perf_counter()
    rho_s = oracle.cic_deposit(sub, ng)
    t_dep = (time.perf_counter() - t0) * 8
    delta = oracle.density_contrast(rho_s)
    t0 = time.perf_counter()
    psi = oracle.solve_poisson(delta, c, h)
    t_pois = time.perf_counter() - t0
    b = c["xi"] * c["s"] * delta
    t0 = time.perf_counter()
    oracle.fas_solve(b, h, c["nu"], c["K"], tol=1e-30, max_cycles=1)
    t_cyc = time.perf_counter() - t0
    rho64 = lognormal_density(64, 500.0 * 64 / 256, seed=2)
    _, rep64 = oracle.solve_chi(oracle.density_contrast(rho64), c, 1.0 / 64, tol=1e-7, max_cycles=200)
    t0 = time.perf_counter()
    g = oracle.gradient5(psi, h)
    t_grad = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.cic_interpolate(g, sub)
    t_interp = (time.perf_counter() - t0) * 8
    ms = (t_dep + t_pois + rep64["vcycles"] * t_cyc + t_grad + t_interp) * 1e3
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(ms, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": (f"oracle on the {ng}^3 workload: deposit+interpolation on 1/8 of the particles (x8), "
                       f"FFT Poisson, 1 FAS V-cycle at {ng}^3 ({t_cyc:.2f} s) x {rep64['vcycles']} V-cycles "
                       f"(oracle count to 1e-7 at 64^3, same statistics), gradient; OpenMP threads {threads}"),
            "cpu_model": cpu_model()}


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def one_thread_baseline(ng, ics):
    """The same bounded sample with one OpenMP thread, in a child process (the
    oracle's thread count is fixed when its library loads).  The child runs
    only the oracle: it imports no GPU code."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--ng", str(ng),
                          "--ics", ics], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        return None
    return json.loads(out.stdout.strip().splitlines()[-1])


def run_scan(P, torch, per_size=16, sizes=(64, 128, 192, 256), tol=1e-7):
    """The batched parameter scan: per_size lognormal densities at each grid
    size (cell 500/256 Mpc/h, seeds 4000+), alpha_B0 ~ U[-1, 0], alpha_M0 ~
    U[0, 0.2], a = 1 (seed 4), FP32 arrays with mixed-precision solves to tol;
    one mg_scalar_solve_batched call against the same problems solved one
    after another."""
    from workloads import lognormal_density, scan_params

    probs = []
    prms = scan_params(per_size * len(sizes), seed=4, a=1.0)
    for s_i, ng in enumerate(sizes):
        for k in range(per_size):
            idx = s_i * per_size + k
            rho = torch.from_numpy(lognormal_density(ng, 500.0 * ng / 256, seed=4000 + idx)).to("cuda", torch.float32)
            probs.append(dict(rho=rho, chi=torch.zeros_like(rho), params=prms[idx]))
    opts = P.MgOpts(rel_tol=tol, max_vcycles=60, precision="mixed")
    ws = torch.empty(P.mg_batched_workspace_bytes(probs, "mixed"), dtype=torch.uint8, device="cuda")
    P.mg_scalar_solve_batched(probs, opts, ws=ws)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = P.mg_scalar_solve_batched(probs, opts, ws=ws)
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) * 1e3
    pws = {}
    t0 = time.perf_counter()
    for pr in probs:
        ng = pr["rho"].shape[0]
        if ng not in pws:
            pws[ng] = P.Workspace(ng, 0, 0, "mixed")
        P.mg_scalar_solve(pr["rho"], pr["params"], opts, torch.zeros_like(pr["chi"]), ws=pws[ng])
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) * 1e3
    cells = sum(pr["rho"].numel() for pr in probs)
    cyc = sum(r["vcycles"] * pr["rho"].numel() for r, pr in zip(reps, probs))
    return {"problems": len(probs), "sizes": list(sizes), "per_size": per_size, "tol": tol,
            "ms_batched": round(batched, 2), "ms_sequential": round(seq, 2),
            "speedup": round(seq / batched, 3), "all_converged": all(r["status"] == 0 for r in reps),
            "vcycles_min_max": [min(r["vcycles"] for r in reps), max(r["vcycles"] for r in reps)],
            "cells": cells, "cells_vcycles_per_s": round(cyc / (batched * 1e-3), 1)}


def make_particles(ng, ics):
    """Particle positions of the workload (host, [3, ng^3]) and the box size."""
    if ics == "lognormal":
        from workloads import lognormal_particles

        box = 500.0 * ng / 256
        return lognormal_particles(ng, box, seed=2)[0], box
    from workloads import zeldovich_ics

    box = 1000.0 * ng / 512
    return zeldovich_ics(ng, box, seed=5), box


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ng", type=int, default=256)
    ap.add_argument("--modes", default="plain,fp32,learned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-save", default=None, help="write the autotuned launch shapes to this file")
    ap.add_argument("--tune-load", default=None, help="use the launch shapes of this file (implies --no-tune)")
    ap.add_argument("--ics", default="lognormal", choices=("lognormal", "zeldovich"),
                    help="lognormal: ng^3 particles from the log-sigma 1.5 lognormal density (seed 2, 500 ng/256 "
                         "Mpc/h); zeldovich: Zel'dovich load of the sigma8 = 0.8 spectrum (seed 5, 1000 ng/512 Mpc/h)")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the batched parameter scan (16 problems each at 64^3..256^3), timed by default "
                         "after the steps at 256^3")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2604_15434_amd", "weights", "unet_warmstart.f32"))
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="print only the oracle's bounded-sample figure for the workload (no GPU)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(make_particles(args.ng, args.ics)[0], args.ng)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2604_15434_amd as P

    ng = args.ng
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] generating {ng}^3 {args.ics} particles", file=sys.stderr, flush=True)
    pos_np, box = make_particles(ng, args.ics)
    modes = args.modes.split(",")
    net = None
    if "learned" in modes:
        if os.path.exists(args.weights) and ng % 64 == 0:
            from paper_2604_15434_amd.warmstart import WarmStart

            net = WarmStart.load(args.weights)
        else:
            print(f"[bench] no learned mode (weights {args.weights} missing or ng % 64 != 0)", file=sys.stderr,
                  flush=True)
            modes.remove("learned")
    shapes = {}
    if args.tune_load:
        P.pm_tune_load(args.tune_load)
    elif not args.no_tune:
        for prec in ("f64", "mixed"):
            P.pm_autotune(ng, prec)
    if args.tune_save:
        P.pm_tune_save(args.tune_save)
    for prec, word in (("f64", 8), ("mixed", 4)):
        shapes[prec] = dict(zip(("block_cycle_grid", "tiled_smoother"), P.pm_get_launch_shape(ng, word)))
    print(f"[bench] launch shapes: {shapes}", file=sys.stderr, flush=True)
    results = {}
    for mode in modes:
        print(f"[bench] mode {mode}: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
        results[mode] = run_mode(P, torch, mode, pos_np, ng, args.steps, args.warmup, net, presort=True)
        print(f"[bench] mode {mode}: {results[mode]['ms_per_step']:.3f} ms/step, "
              f"V-cycles chi {results[mode]['scalar_vcycles']} psi {results[mode]['poisson_vcycles']}",
              file=sys.stderr, flush=True)
    head = next((m for m in ("learned", "fp32") if m in results and results[m]["converged"]), next(iter(results)))

    def tiled_of(mode):
        return shapes["f64" if mode == "plain" else "mixed"]["tiled_smoother"]
    r = results[head]
    line = {
        "metric": f"ms per {ng}^3 PM step (scalar MG to rel. residual 1e-7), plain vs learned+FP32",
        "value": round(r["ms_per_step"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "plain" else ("f32+f64+bf16" if head == "learned" else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": (f"PM step, {ng}^3 grid, {ng}^3 lognormal particles (log-sigma 1.5, seed 2), "
                                f"{box:g} Mpc/h, alpha_B0=-0.2 alpha_M0=0 a=1, tol 1e-7; particles in CIC base-cell order" if args.ics == "lognormal"
                                else f"PM step, {ng}^3 grid, {ng}^3 Zel'dovich particles (sigma8 0.8, seed 5; "
                                f"sorted by CIC cell once before timing), "
                                f"{box:g} Mpc/h, alpha_B0=-0.2 alpha_M0=0 a=1, tol 1e-7"),
                   "mode": head, "launch_shapes": shapes},
        "plain_ms_per_step": round(results["plain"]["ms_per_step"], 3) if "plain" in results else None,
        "speedup_vs_plain": round(results["plain"]["ms_per_step"] / r["ms_per_step"], 3) if "plain" in results
        else None,
        "modes": {m: {k: v for k, v in res.items() if k not in ("kernel_timing", "kernel_timing_alone", "itemsize")}
                  for m, res in results.items()},
        "cells_vcycles_per_s": round(ng**3 * r["scalar_vcycles"] / (r["ms_scalar"] * 1e-3), 1)
        if r["ms_scalar"] > 0 else None,
        "roofline": roofline(r, ng, tiled_of(head)),
        "roofline_modes": {m: roofline(res, ng, tiled_of(m)) for m, res in results.items()},
    }
    if not args.no_scan and ng == 256:
        print("[bench] batched parameter scan", file=sys.stderr, flush=True)
        line["scan"] = run_scan(P, torch)
        print(f"[bench] scan: {line['scan']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(pos_np, ng)
        one = one_thread_baseline(ng, args.ics)
        if one:
            line["cpu_baseline"]["one_thread"] = {"value": one["value"], "unit": "ms", "cores": 1}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
