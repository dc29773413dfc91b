"""Build libpmeft.so (HIP, gfx950) in-tree with hipcc.

``python -m paper_2604_15434_amd.build`` or ``build()``.  The library is
written next to this file as ``libpmeft.so``.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmeft.so")
SOURCES = ["mg_kernels.hip", "smooth_kernels.hip", "tile_kernels.hip", "pm_kernels.hip", "pmeft_api.hip", "unet_kernels.hip",
           "unet_api.hip", "spectrum_kernels.hip", "sweep2_kernels.hip", "noalloc_api.hip"]
ARCH = os.environ.get("PMEFT_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpmeft.so")


def _wait(procs, verbose):
    for p in procs:
        err = p.communicate()[1]
        lines = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
        if verbose and lines:
            print("\n".join(lines))


def build(verbose: bool = False, jobs: int = 3) -> str:
    objs = []
    procs = []
    common = [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        # packed FP32 math is disabled: hipcc would otherwise fuse float pairs
        # into v_pk_* instructions, which this project avoids.
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
    ]
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = common + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs, verbose)
            procs = []
    _wait(procs, verbose)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
