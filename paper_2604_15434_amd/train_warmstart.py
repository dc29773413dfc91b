"""Training driver of the learned warm start (runs on the GPU).

Samples are ng^3 particles drawn from lognormal density fields (log-sigma
1.5, power-law-break spectrum) and deposited by the library's CIC kernel, as
the PM step sees them (shot noise included), on 64^3 and 128^3 grids whose
cell matches the 256^3 / 500 Mpc/h workload (box = 500 ng / 256 Mpc/h), each
with its own (alpha_B0 ~ U[-1, 0], alpha_M0 ~ U[0, 0.2], a ~ U[0.2, 1]).  Labels are the scalar fields solved by
this library in FP64 to relative residual 1e-8; the network learns the
nonlinear part t of the normalised source (see include/pmeft.h).  Every
forward, backward and Adam step runs in the library's kernels.

  python -m paper_2604_15434_amd.train_warmstart --n64 1000 --n128 1000 \\
      --minutes 12 --out paper_2604_15434_amd/weights/unet_warmstart.f32
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

CELL_MPC = 500.0 / 256


def _particles(args):
    from workloads import lognormal_particles

    ng, seed = args
    pos, _ = lognormal_particles(ng, CELL_MPC * ng, seed=seed)
    return pos


def iter_samples(n64, n128, seed0=1000, workers=12):
    """(ng, seed, params, pos) of each sample: ng^3 particles drawn from a
    lognormal density, as the PM step deposits them (shot noise included)."""
    from workloads import scan_params

    specs = [(64, seed0 + i) for i in range(n64)] + [(128, seed0 + n64 + i) for i in range(n128)]
    params = scan_params(len(specs), seed=seed0)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for (ng, sd), p, pos in zip(specs, params, ex.map(_particles, specs, chunksize=4)):
            yield ng, sd, p, pos


def label(P, torch, rho_d, prm, tol=1e-8):
    chi = torch.zeros_like(rho_d)
    rep = P.mg_scalar_solve(rho_d, prm, P.MgOpts(rel_tol=tol, max_vcycles=80, precision="f64"), chi)
    return chi, rep


def rel_source_error(net, torch, rho_d, chi_d, prm):
    """sqrt(mean (yhat - t)^2) / rms(delta) on one sample (no update)."""
    loss = net.train_step(rho_d, chi_d, prm, 0.0)
    return math.sqrt(loss) / float(rho_d.std())


def solve_cost(P, torch, rho_d, prm, guess, net=None, tol=1e-7, reps=2):
    opts = P.MgOpts(rel_tol=tol, max_vcycles=60, precision="mixed", guess=guess, learned=net)
    best = None
    for _ in range(reps):
        chi = torch.zeros_like(rho_d)
        rep = P.mg_scalar_solve(rho_d, prm, opts, chi)
        if best is None or rep["ms"] < best["ms"]:
            best = rep
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n64", type=int, default=1000)
    ap.add_argument("--n128", type=int, default=1000)
    ap.add_argument("--holdout", type=float, default=0.05)
    ap.add_argument("--minutes", type=float, default=10.0)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--init", default=None, help="start from these weights")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    import torch

    import paper_2604_15434_amd as P
    from paper_2604_15434_amd.warmstart import WarmStart

    t0 = time.time()
    data = []
    n_all = args.n64 + args.n128
    for idx, (ng, sd, prm, pos) in enumerate(iter_samples(args.n64, args.n128)):
        c = P.pm_eft_coefficients(prm)
        if not (c["nu"] > 0):
            continue
        rho_d = torch.empty((ng, ng, ng), dtype=torch.float64, device="cuda")
        P.pm_deposit(torch.from_numpy(pos).cuda(), ng, rho_d)
        chi_d, rep = label(P, torch, rho_d, prm)
        if rep["status"] != 0:
            print(f"[train] sample {idx} (ng {ng}, seed {sd}) label not converged: {rep['rel_residual']:.2e}",
                  flush=True)
            continue
        data.append((ng, sd, prm, rho_d, chi_d))
        if idx % 200 == 0:
            print(f"[train] samples {idx}/{n_all} ({time.time() - t0:.1f} s)", flush=True)
    rng = np.random.default_rng(args.seed)
    order = rng.permutation(len(data))
    n_hold = max(4, int(args.holdout * len(data)))
    hold = [data[i] for i in order[:n_hold]]
    train = [data[i] for i in order[n_hold:]]
    print(f"[train] {len(train)} training / {len(hold)} held-out samples; data {time.time() - t0:.1f} s", flush=True)

    net = WarmStart.load(args.init) if args.init else WarmStart(seed=args.seed)

    def holdout_error():
        return float(np.mean([rel_source_error(net, torch, r, c, p) for (_, _, p, r, c) in hold]))

    herr0 = holdout_error()
    print(f"[train] initial held-out relative source error {herr0:.4f}", flush=True)
    best = (herr0, net.params.clone(), net.step)
    budget = args.minutes * 60.0
    t2 = time.time()
    step, epoch = 0, 0
    est_total = None
    errs, norms = [], []
    clip = 0.0
    next_eval = 90.0
    warm = 1000
    # learning rate: linear warmup, then cosine decay to 1e-5 over the time budget;
    # global-norm clipping at twice the median of the recently sampled norms
    while time.time() - t2 < budget:
        perm = rng.permutation(len(train))
        for k in perm:
            ng, sd, prm, rho_d, chi_d = train[k]
            el = time.time() - t2
            if el >= budget:
                break
            if est_total is None and step == 200:
                est_total = int(budget / (el / 200))
            frac = min(step / est_total, 1.0) if est_total else 0.0
            lr = 1e-5 + 0.5 * (args.lr - 1e-5) * (1 + math.cos(math.pi * frac))
            lr *= min(1.0, (step + 1) / warm)
            sample = step % 10 == 0
            out = net.train_step(rho_d, chi_d, prm, lr, grad_clip=clip, want_norm=sample, want_loss=sample)
            step += 1
            if sample:
                loss, gn = out
                errs.append(math.sqrt(loss) / float(rho_d.std()))
                norms.append(gn)
                if len(norms) >= 20 and len(norms) % 20 == 0:
                    clip = 2.0 * float(np.median(norms[-200:]))
            if step % 1000 == 0:
                print(f"[train] step {step} epoch {epoch} lr {lr:.2e} clip {clip:.3g} recent rel err "
                      f"{np.mean(errs[-50:]):.4f} ({time.time() - t2:.0f} s)", flush=True)
            if time.time() - t2 >= next_eval:
                next_eval += 90.0
                herr = holdout_error()
                print(f"[train] held-out relative source error {herr:.4f} at step {step}", flush=True)
                if herr < best[0]:
                    best = (herr, net.params.clone(), net.step)
        epoch += 1
    torch.cuda.synchronize()
    herr = holdout_error()
    if herr < best[0]:
        best = (herr, net.params.clone(), net.step)
    net.params.copy_(best[1])
    herr = best[0]
    print(f"[train] done: {step} steps, {epoch} epochs, {time.time() - t2:.0f} s; best held-out relative source "
          f"error {herr:.4f}", flush=True)

    # cost of the solve from the zero, linearised and learned guesses on held-out 128^3 samples
    rows = []
    for (ng, sd, prm, rho_d, chi_d) in [h for h in hold if h[0] == 128][:6]:
        r = {g: solve_cost(P, torch, rho_d, prm, g, net) for g in ("zero", "linear", "learned")}
        rows.append((sd, prm, r))
        print(f"[eval] ng {ng} seed {sd} aB0 {prm['alpha_b0']:+.3f} aM0 {prm['alpha_m0']:.3f} a {prm['a']:.3f}: " +
              "  ".join(f"{g} {x['vcycles']} cyc {x['ms']:.2f} ms" for g, x in r.items()), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    meta = dict(samples=dict(n64=args.n64, n128=args.n128, seed0=1000, holdout=len(hold), train=len(train),
                             cell_mpc=CELL_MPC, sigma_g=1.5, label_tol=1e-8,
                             density="CIC deposit of ng^3 lognormal particles"),
                training=dict(steps=step, epochs=epoch, seconds=round(time.time() - t2, 1), lr=args.lr,
                              schedule="linear warmup over 1000 steps, cosine to 1e-5 over the time budget",
                              clipping="global norm, twice the median of the last 200 sampled norms", batch=1,
                              kept="best held-out error of the evaluations every 90 s"),
                heldout_rel_source_error=round(herr, 5),
                eval_128=[dict(seed=sd, params=prm, **{g: dict(vcycles=x["vcycles"], ms=round(x["ms"], 3))
                                                      for g, x in r.items()}) for sd, prm, r in rows])
    net.save(args.out, meta=meta)
    print(f"[train] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
