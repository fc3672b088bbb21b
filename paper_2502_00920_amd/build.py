"""Build the HIP library libmclbm.so for gfx950 with hipcc (in-tree).

Usage: python -m paper_2502_00920_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmclbm.so")
SOURCES = ["mclbm_kernels.hip", "mclbm_api.cpp", "mclbm_serve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-fvisibility=hidden", "-fno-gpu-rdc",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


DEMO = os.path.join(PKG, "mclbm_demo")
PATTERN = os.path.join(PKG, "march_pattern")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-x", "hip", *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_demo(verbose)
    build_pattern(verbose)
    return LIB


def build_demo(verbose: bool = False) -> str:
    """The stand-alone C++ user of the ABI (host code only, linked to libmclbm.so)."""
    tmp = DEMO + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "mclbm_demo.cpp"),
           "-L", PKG, "-lmclbm", "-Wl,-rpath,$ORIGIN", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, DEMO)
    return DEMO


def build_pattern(verbose: bool = False) -> str:
    """The march-pattern bandwidth probe (a stand-alone HIP program)."""
    tmp = PATTERN + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(CSRC, "march_pattern.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PATTERN)
    return PATTERN


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
