"""Writes unet_forward_<n>.txt: the FP64 oracle network's output at sampled
voxels of an n^3 seeded lognormal density, for fixed seeded parameters (the
recipe below; the GPU test rebuilds the same parameters and input).

    python tests/golden/make_unet_forward.py 128 256

The network is the warm start's 3-level U-Net (16/32/64 channels, 3x3x3
convolutions, periodic padding); its inputs are the standardised log-density
and the broadcast (alpha_B0, alpha_M0, a).  Only oracle/ and the seeded input
generators are called."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import unet as U  # noqa: E402
from workloads import lognormal_density  # noqa: E402

PARAMS = dict(alpha_b0=-0.35, alpha_m0=0.12, a=0.7)
SAMPLES = 2048


def flat_params(seed=21):
    """He-normal weights, biases ~ N(0, 0.05^2), head ~ N(0, 1/16) and 0.02,
    flattened in the network's layer order (weights W[27][cin][cout], then
    biases, per layer; then the head), as FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in U.LAYERS:
        parts.append(rng.standard_normal(27 * ci * co) * np.sqrt(2.0 / (27 * ci)))
        parts.append(rng.standard_normal(co) * 0.05)
    parts.append(rng.standard_normal(16) * 0.25)
    parts.append(np.array([0.02]))
    return np.concatenate(parts).astype(np.float32)


def oracle_params(flat):
    p, o = {}, 0
    flat = flat.astype(np.float64)
    for name, ci, co in U.LAYERS:
        p[name + ".w"] = flat[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        p[name + ".b"] = flat[o:o + co]
        o += co
    p["head.w"] = flat[o:o + 16]
    p["head.b"] = flat[o + 16:o + 17]
    return p


def density(n):
    return lognormal_density(n, 500.0 * n / 256, seed=40 + n)


def sample_index(n):
    return np.random.default_rng(n).choice(n**3, SAMPLES, replace=False)


def main(sizes):
    for n in sizes:
        x0 = U.input_features(density(n), PARAMS["alpha_b0"], PARAMS["alpha_m0"], PARAMS["a"])
        y, _ = U.forward(oracle_params(flat_params()), x0, keep=False)
        idx = sample_index(n)
        vals = y.reshape(-1)[idx]
        with open(os.path.join(HERE, f"unet_forward_{n}.txt"), "w") as f:
            f.write(f"# oracle network output at {SAMPLES} sampled voxels of a {n}^3 lognormal density\n")
            f.write(f"# written by make_unet_forward.py (parameters flat_params(21), input density({n}), "
                    f"alpha_B0 {PARAMS['alpha_b0']}, alpha_M0 {PARAMS['alpha_m0']}, a {PARAMS['a']})\n")
            f.write(f"# rms over the grid {float(np.sqrt(np.mean(y**2))):.9e}\n")
            for i, v in zip(idx, vals):
                f.write(f"{int(i)} {float(v):.9e}\n")
        print(n, "done", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [128])
