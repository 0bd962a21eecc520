"""Build libsedg.so in-tree for gfx950.

    python -m paper_2011_03338_amd.build

The HIP sources are compiled with hipcc for gfx950 only; the host table
builder is plain C++ (quad precision through libquadmath).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsedg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tab_o = os.path.join(BUILD, "sedg_tables.o")
    ker_o = os.path.join(BUILD, "sedg_kernels.o")
    _run(["g++", "-O2", "-fPIC", "-std=gnu++17", "-Wall", "-c", os.path.join(CSRC, "sedg_tables.cpp"), "-o", tab_o])
    _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "sedg_kernels.hip"), "-o", ker_o])
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, ker_o, tab_o, "-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
