"""VGICP oracle: the plain FP64 CPU reference that the GPU path is checked against.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import this package. The product library never imports it, and this package imports
nothing from the product.

Two independent implementations live here:

* ``oracle.cpp`` (loaded through ctypes, wrapped below): the definition of the VGICP matching
  cost of Sec. III-A, Eqs. (2)-(3), with its Gauss-Newton linearization, in FP64 with a fixed
  evaluation order and compensated sums;
* ``ref.py``: a NumPy brute-force twin for tiny inputs (voxels found by scanning every target
  point, 3x3 inverses by ``numpy.linalg.inv``) used to cross-check the C++ oracle.

Array conventions (same as the product's): clouds are SoA, ``xyz`` of shape (3, n) and ``cov``
of shape (6, n) holding xx, xy, xz, yy, yz, zz; poses are row-major 3x4 ``[R | t]``
world-from-local, 12 float64 values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID_ARG, E_NONFINITE, E_KEY_RANGE = 0, 1, 2, 3
_STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_NONFINITE", 3: "E_KEY_RANGE"}


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS_NAMES.get(status, status)}")
        self.status = status


def build(force: bool = False) -> str:
    """Compiles oracle.cpp with g++ (FP64, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P, D, I64, I32, I = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int32,
                             ctypes.c_int)
        L.oracle_voxel_coord.argtypes = [D, D, ctypes.POINTER(I64)]
        L.oracle_pack_key.argtypes = [I64, I64, I64]
        L.oracle_pack_key.restype = I64
        L.oracle_unpack_key.argtypes = [I64, P, P, P]
        L.oracle_map_build.argtypes = [P, P, I64, D, ctypes.POINTER(P)]
        L.oracle_map_size.argtypes = [P]
        L.oracle_map_size.restype = I64
        L.oracle_map_export.argtypes = [P, P, P, P, P]
        L.oracle_map_free.argtypes = [P]
        L.oracle_relative_pose.argtypes = [P, P, P]
        L.oracle_linearize.argtypes = [P, P, P, I64, P, P, I, P, P, P, P, P]
        L.oracle_evaluate.argtypes = [P, P, P, I64, P, P, P, P, P]
        L.oracle_cost_fixed.argtypes = [P, P, P, I64, P, P, P, P, P]
        L.oracle_point_omega.argtypes = [P, P, P, I64, P, P, P, P]
        L.oracle_gradient.argtypes = [P, P, P, I64, P, P, I, P, P, P, P]
        L.oracle_linearize_factors.argtypes = [P, I32, P, P, P, I32, P, I32, P, I32, I, P, P, P, P]
        L.oracle_max_threads.restype = I
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _pose(T):
    T = np.asarray(T, dtype=np.float64)
    if T.shape == (4, 4):
        T = T[:3, :]
    return _f64(T.reshape(12))


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


def voxel_coord(v: float, res: float) -> int:
    k = ctypes.c_int64()
    _check(lib().oracle_voxel_coord(float(v), float(res), ctypes.byref(k)), "voxel_coord")
    return k.value


def pack_key(kx: int, ky: int, kz: int) -> int:
    return lib().oracle_pack_key(kx, ky, kz)


def unpack_key(key: int):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib().oracle_unpack_key(key, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def relative_pose(T_target, T_source) -> np.ndarray:
    out = np.empty(12)
    lib().oracle_relative_pose(_p(_pose(T_target)), _p(_pose(T_source)), _p(out))
    return out


@dataclass
class Cloud:
    """A cloud promoted exactly to FP64 (the oracle's own copy)."""

    xyz: np.ndarray  # (3, n) float64
    cov: np.ndarray  # (6, n) float64

    @staticmethod
    def of(xyz, cov) -> "Cloud":
        xyz = _f64(xyz)
        cov = _f64(cov)
        if xyz.ndim != 2 or xyz.shape[0] != 3 or cov.shape != (6, xyz.shape[1]):
            raise ValueError("cloud must be xyz (3, n) and cov (6, n)")
        return Cloud(xyz, cov)

    @property
    def n(self) -> int:
        return self.xyz.shape[1]


class VoxelMap:
    """Voxel map of one target cloud (Sec. III-A)."""

    def __init__(self, xyz, cov, res: float):
        self.cloud = Cloud.of(xyz, cov)
        self.res = float(res)
        h = ctypes.c_void_p()
        _check(lib().oracle_map_build(_p(self.cloud.xyz), _p(self.cloud.cov), self.cloud.n,
                                      self.res, ctypes.byref(h)), "map_build")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_map_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def __len__(self) -> int:
        return lib().oracle_map_size(self._h)

    def export(self):
        V = len(self)
        keys = np.empty(V, np.int64)
        mean = np.empty((V, 3))
        cov = np.empty((V, 6))
        count = np.empty(V, np.int32)
        lib().oracle_map_export(self._h, _p(keys), _p(mean), _p(cov), _p(count))
        return {"keys": keys, "mean": mean, "cov": cov, "count": count}


def linearize(vmap: VoxelMap, xyz, cov, T_target, T_source, binary: bool):
    """Gauss-Newton factor of Eq. (2): returns dict(H, b, e, inliers, corr)."""
    c = Cloud.of(xyz, cov)
    dim = 12 if binary else 6
    H = np.empty(dim * dim)
    b = np.empty(dim)
    e = ctypes.c_double()
    nin = ctypes.c_int64()
    corr = np.empty(c.n, np.int32)
    _check(lib().oracle_linearize(vmap.handle, _p(c.xyz), _p(c.cov), c.n, _p(_pose(T_target)),
                                  _p(_pose(T_source)), int(bool(binary)), _p(H), _p(b),
                                  ctypes.byref(e), ctypes.byref(nin), _p(corr)), "linearize")
    return {"H": H.reshape(dim, dim), "b": b, "e": e.value, "inliers": nin.value, "corr": corr}


def evaluate(vmap: VoxelMap, xyz, cov, T_target, T_source):
    c = Cloud.of(xyz, cov)
    e = ctypes.c_double()
    nin = ctypes.c_int64()
    corr = np.empty(c.n, np.int32)
    _check(lib().oracle_evaluate(vmap.handle, _p(c.xyz), _p(c.cov), c.n, _p(_pose(T_target)),
                                 _p(_pose(T_source)), ctypes.byref(e), ctypes.byref(nin),
                                 _p(corr)), "evaluate")
    return {"e": e.value, "inliers": nin.value, "corr": corr}


def cost_fixed(vmap: VoxelMap, xyz, cov, T_target, T_source, corr, omega=None) -> float:
    c = Cloud.of(xyz, cov)
    corr = np.ascontiguousarray(corr, dtype=np.int32)
    om = None if omega is None else _f64(omega, (c.n, 9))
    e = ctypes.c_double()
    _check(lib().oracle_cost_fixed(vmap.handle, _p(c.xyz), _p(c.cov), c.n, _p(_pose(T_target)),
                                   _p(_pose(T_source)), _p(corr), _p(om), ctypes.byref(e)),
           "cost_fixed")
    return e.value


def point_omega(vmap: VoxelMap, xyz, cov, T_target, T_source, corr) -> np.ndarray:
    c = Cloud.of(xyz, cov)
    corr = np.ascontiguousarray(corr, dtype=np.int32)
    om = np.empty((c.n, 9))
    _check(lib().oracle_point_omega(vmap.handle, _p(c.xyz), _p(c.cov), c.n, _p(_pose(T_target)),
                                    _p(_pose(T_source)), _p(corr), _p(om)), "point_omega")
    return om


def gradient(vmap: VoxelMap, xyz, cov, T_target, T_source, binary: bool, corr):
    """Exact gradient of Eq. (2), correspondences frozen: dict(g_xi, g_points (3, n), e)."""
    c = Cloud.of(xyz, cov)
    corr = np.ascontiguousarray(corr, dtype=np.int32)
    g = np.empty(12 if binary else 6)
    gp = np.empty((3, c.n))
    e = ctypes.c_double()
    _check(lib().oracle_gradient(vmap.handle, _p(c.xyz), _p(c.cov), c.n, _p(_pose(T_target)),
                                 _p(_pose(T_source)), int(bool(binary)), _p(corr), _p(g), _p(gp),
                                 ctypes.byref(e)), "gradient")
    return {"g_xi": g, "g_points": gp, "e": e.value}


def linearize_factors(maps, clouds, poses, factors, nthreads: int = 0):
    """OpenMP over factors. maps: list[VoxelMap]; clouds: list[(xyz, cov)] or list[Cloud];
    poses: (P, 12) or (P, 3, 4); factors: (F, 5) int32 rows (map, cloud, target pose,
    source pose, binary). Returns H (F, 12, 12), b (F, 12), e (F,), inliers (F,)."""
    cl = [c if isinstance(c, Cloud) else Cloud.of(*c) for c in clouds]
    poses = _f64(np.asarray(poses, dtype=np.float64).reshape(-1, 12))
    factors = np.ascontiguousarray(factors, dtype=np.int32).reshape(-1, 5)
    F = factors.shape[0]
    mh = (ctypes.c_void_p * len(maps))(*[m.handle.value for m in maps])
    xp = (ctypes.c_void_p * len(cl))(*[c.xyz.ctypes.data for c in cl])
    cp = (ctypes.c_void_p * len(cl))(*[c.cov.ctypes.data for c in cl])
    npts = np.array([c.n for c in cl], np.int64)
    H = np.empty((F, 12, 12))
    b = np.empty((F, 12))
    e = np.empty(F)
    nin = np.empty(F, np.int64)
    _check(lib().oracle_linearize_factors(
        ctypes.cast(mh, ctypes.c_void_p), len(maps), ctypes.cast(xp, ctypes.c_void_p),
        ctypes.cast(cp, ctypes.c_void_p), _p(npts), len(cl), _p(poses), poses.shape[0],
        _p(factors), F, int(nthreads), _p(H), _p(b), _p(e), _p(nin)), "linearize_factors")
    return {"H": H, "b": b, "e": e, "inliers": nin}


def max_threads() -> int:
    return lib().oracle_max_threads()
