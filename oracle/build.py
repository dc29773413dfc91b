"""Build the oracle's plain-C solver (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` compiles
``oracle/csrc/chi_fas.c`` with gcc into ``oracle/_liboracle.so``.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "chi_fas.c")
LIB = os.path.join(HERE, "_liboracle.so")


def build(verbose=False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
