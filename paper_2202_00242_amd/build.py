"""Builds libvgicp.so (the HIP library behind include/vgicp.h) for gfx950 with hipcc.

Every source is compiled to an object of its own (in parallel) and the objects are linked into
the shared library; no device symbol crosses translation units, so no relocatable device code
is needed.

Usage: python -m paper_2202_00242_amd.build [--force]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvgicp.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["capi.hip", "imu.hip", "kernels.hip", "lm.hip", "preprocess.hip",
           "voxelmap.hip"]
HEADERS = ["common.h", "device_math.h", "internal.h"]
ARCH = os.environ.get("VGICP_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for the device code (the compiler would otherwise
# form them from plain float code).
CFLAGS = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
          "-Wno-unknown-pragmas"]
LDFLAGS = ["-shared", "-fPIC", f"--offload-arch={ARCH}"]


def _inputs():
    inc = os.path.join(os.path.dirname(HERE), "include", "vgicp.h")
    return [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [inc]


def _compile(hipcc: str, src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    tmp = obj + f".tmp{os.getpid()}"
    cmd = [hipcc] + CFLAGS + ["-c", "-o", tmp, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, obj)
    return obj


def build(force: bool = False, verbose: bool = False, jobs: int = 0) -> str:
    """Compiles the library in-tree; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(p) <= t for p in _inputs()):
            return LIB
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, verbose), SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc] + LDFLAGS + ["-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
