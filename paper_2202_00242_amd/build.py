"""Builds libvgicp.so (the HIP library behind include/vgicp.h) for gfx950 with hipcc.

Usage: python -m paper_2202_00242_amd.build [--force]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvgicp.so")
SOURCES = ["capi.hip", "imu.hip", "kernels.hip", "lm.hip", "preprocess.hip", "voxelmap.hip"]
HEADERS = ["common.h", "device_math.h", "internal.h"]
ARCH = os.environ.get("VGICP_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for the device code (the compiler would otherwise
# form them from plain float code).
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
         f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
         "-Wno-unknown-pragmas"]


def _inputs():
    inc = os.path.join(os.path.dirname(HERE), "include", "vgicp.h")
    return [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [inc]


def build(force: bool = False, verbose: bool = False) -> str:
    """Compiles the library in-tree; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(p) <= t for p in _inputs()):
            return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc] + FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
