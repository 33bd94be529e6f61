"""Python binding of libvgicp (include/vgicp.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor shapes, dtypes and
devices, passes raw pointers and the current HIP stream, and wraps the opaque handles. Device
memory and streams come from PyTorch. Importing it without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# VGICP_LIB selects another build of the same library (for side-by-side measurements)
LIB_PATH = os.environ.get("VGICP_LIB") or os.path.join(_HERE, "libvgicp.so")

VGICP_OK, VGICP_E_INVALID_ARG, VGICP_E_NONFINITE, VGICP_E_KEY_RANGE = 0, 1, 2, 3
VGICP_E_CAPACITY, VGICP_E_OOM, VGICP_E_HIP = 4, 5, 6
STATUS_NAMES = {0: "VGICP_OK", 1: "VGICP_E_INVALID_ARG", 2: "VGICP_E_NONFINITE",
                3: "VGICP_E_KEY_RANGE", 4: "VGICP_E_CAPACITY", 5: "VGICP_E_OOM",
                6: "VGICP_E_HIP"}

VGICP_ACC_FP64, VGICP_ACC_KAHAN_FP32, VGICP_NAIVE_WORLD_FP32, VGICP_MATH_FP64 = 0, 1, 2, 3
VGICP_LAYOUT_AUTO, VGICP_LAYOUT_HASH, VGICP_LAYOUT_GRID = 0, 1, 2
PRECISIONS = {"acc_fp64": 0, "kahan_fp32": 1, "naive_world_fp32": 2, "math_fp64": 3}


class VGICPError(RuntimeError):
    def __init__(self, status: int, what: str, message: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Cloud(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("cov", ctypes.c_void_p), ("n", ctypes.c_int64)]


class Factor(ctypes.Structure):
    _fields_ = [("target_map", ctypes.c_int32), ("source_cloud", ctypes.c_int32),
                ("target_pose", ctypes.c_int32), ("source_pose", ctypes.c_int32),
                ("binary", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("lookahead", ctypes.c_int32)]

    def as_tuple(self):
        return (self.block, self.tile, self.blocks_per_cu, self.lookahead)


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2202_00242_amd.build`")
    L = ctypes.CDLL(path)
    P, I32, I64, D, S = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                         ctypes.c_int)
    sig = {
        "vgicp_build_voxelmap": [P, P, I64, D, P, P],
        "vgicp_build_voxelmap_layout": [P, P, I64, D, I32, P, P],
        "vgicp_voxelmap_size": [P, P, P],
        "vgicp_voxelmap_layout": [P, P],
        "vgicp_voxelmap_export": [P, P, P, P, P, P],
        "vgicp_destroy_voxelmap": [P],
        "vgicp_linearize": [P, P, P, I64, P, P, I32, S, P, P, P, P, P, P],
        "vgicp_linearize_noalloc": [P, P, P, I64, P, P, I32, S, P, P, P, P, P, P],
        "vgicp_evaluate": [P, P, P, I64, P, P, S, P, P, P, P],
        "vgicp_backward": [P, P, P, I64, P, P, I32, P, P, S, P, P, P],
        "vgicp_backward_tangent": [P, P, P, I64, P, P, P, P, I32, P, P, S, P, P, P],
        "vgicp_batch_create": [P, I32, P, I32, P, I32, I32, P],
        "vgicp_batch_set_schedule": [P, P],
        "vgicp_batch_refresh": [P, P],
        "vgicp_batch_overlap": [P, P, P, P, P],
        "vgicp_batch_lm_step": [P, P, S, D, I32, P, P, P, P],
        "vgicp_batch_lm_iterate": [P, P, S, P, I32, I32, P, P],
        "vgicp_batch_lm_solver": [P, I32],
        "vgicp_batch_lm_info": [P, P, P],
        "vgicp_batch_get_schedule": [P, P],
        "vgicp_batch_autotune": [P, P, S, ctypes.c_char_p, P, P],
        "vgicp_batch_linearize": [P, P, S, P, P, P, P, P],
        "vgicp_batch_evaluate": [P, P, S, P, P, P],
        "vgicp_batch_backward": [P, P, S, P, P, P, P, P],
        "vgicp_batch_destroy": [P],
        "vgicp_linearize_batched": [P, I32, P, I32, P, I32, P, I32, S, P, P, P, P, P],
        "vgicp_sync_status": [P],
        "vgicp_downsample": [P, P, I64, D, D, P, P, I64, P, P],
        "vgicp_knn": [P, I64, I32, D, P, P],
        "vgicp_point_covariances": [P, I64, P, I32, D, D, P, P],
        "vgicp_imu_preintegrate": [P, I64, P, I32, P, D, D, P, P, P],
        "vgicp_imu_linearize": [P, P, P, I32, P, P, I32, P, P, P, P, P],
        "vgicp_imu_preintegrate_bias": [P, I64, P, I32, P, D, D, P, P, P, P],
        "vgicp_imu_linearize_bias": [P, P, P, P, P, I32, P, P, P, I32, P, D, D, P, P, P, P],
        "vgicp_relative_pose": [P, P, P],
        "vgicp_se3_retract": [P, P, P],
        "vgicp_se3_right_jacobian": [P, P],
        "vgicp_pose_order": [I32, P, I32, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = S
    L.vgicp_last_error.restype = ctypes.c_char_p
    L.vgicp_last_error.argtypes = []
    L.vgicp_version.restype = ctypes.c_char_p
    L.vgicp_version.argtypes = []
    return L


_lib = load_library()


def _check(st: int, what: str):
    if st != VGICP_OK:
        raise VGICPError(st, what, _lib.vgicp_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if isinstance(stream, torch.cuda.Stream) else int(stream)


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _cloud(xyz: torch.Tensor, cov: torch.Tensor):
    _dev(xyz, torch.float32, name="xyz")
    n = xyz.shape[1] if xyz.dim() == 2 else -1
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape (3, n)")
    _dev(cov, torch.float32, (6, n), name="cov")
    return n


def _pose(T) -> np.ndarray:
    a = T.detach().cpu().numpy() if isinstance(T, torch.Tensor) else np.asarray(T)
    a = np.asarray(a, dtype=np.float64)
    if a.shape == (4, 4):
        a = a[:3]
    a = np.ascontiguousarray(a.reshape(12))
    return a


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return _lib.vgicp_version().decode()


class VoxelMap:
    """Owning handle of a library voxel map (freed with the object)."""

    def __init__(self, handle: ctypes.c_void_p, resolution: float):
        self._h = handle
        self.resolution = resolution

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.vgicp_destroy_voxelmap(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self):
        return vgicp_voxelmap_size(self)

    @property
    def layout(self) -> int:
        return vgicp_voxelmap_layout(self)

    def __len__(self):
        return self.size()[0]


def vgicp_downsample(xyz: torch.Tensor, resolution: float, t: Optional[torch.Tensor] = None,
                     scan_duration: float = 0.0, stream=None):
    """Voxel-grid filter: returns (xyz_out (3, m) float32, t_out (m,) float32 or None)."""
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape (3, n)")
    n = xyz.shape[1]
    _dev(xyz, torch.float32, (3, n), "xyz")
    if t is not None:
        _dev(t, torch.float32, (n,), "t")
    out = torch.empty((3, max(n, 1)), dtype=torch.float32, device=xyz.device)
    tout = torch.empty(max(n, 1), dtype=torch.float32, device=xyz.device) if t is not None else None
    m = ctypes.c_int64()
    _check(_lib.vgicp_downsample(_ptr(xyz), _ptr(t), n, float(resolution), float(scan_duration),
                                 _ptr(out), _ptr(tout), n, ctypes.byref(m), _stream(stream)),
           "vgicp_downsample")
    m = m.value
    xo = out.view(-1)[:3 * m].view(3, m)
    return xo, (tout[:m] if tout is not None else None)


def vgicp_knn(xyz: torch.Tensor, k: int, cell: float = 0.0, stream=None) -> torch.Tensor:
    """k nearest neighbours: int32 (k, n), column i nearest first (itself included)."""
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape (3, n)")
    n = xyz.shape[1]
    _dev(xyz, torch.float32, (3, n), "xyz")
    nbr = torch.empty((int(k), n), dtype=torch.int32, device=xyz.device)
    _check(_lib.vgicp_knn(_ptr(xyz), n, int(k), float(cell), _ptr(nbr), _stream(stream)),
           "vgicp_knn")
    return nbr


def vgicp_point_covariances(xyz: torch.Tensor, neighbors: torch.Tensor, scale: float = 0.01,
                            eps: float = 1e-3, stream=None) -> torch.Tensor:
    """(6, n) float32 covariances from neighbour lists ((k, n) int32, -1 = none)."""
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape (3, n)")
    n = xyz.shape[1]
    _dev(xyz, torch.float32, (3, n), "xyz")
    if neighbors.dim() != 2 or neighbors.shape[1] != n:
        raise ValueError("neighbors must have shape (k, n)")
    _dev(neighbors, torch.int32, None, "neighbors")
    cov = torch.empty((6, n), dtype=torch.float32, device=xyz.device)
    _check(_lib.vgicp_point_covariances(_ptr(xyz), n, _ptr(neighbors), neighbors.shape[0],
                                        float(scale), float(eps), _ptr(cov), _stream(stream)),
           "vgicp_point_covariances")
    return cov


def vgicp_imu_preintegrate(imu: torch.Tensor, seg: torch.Tensor, bias: torch.Tensor,
                           gyro_sigma: float, acc_sigma: float, stream=None):
    """imu (m, 7) f64 rows [w, a, dt]; seg (F + 1,) i64; bias (F, 6) f64 [b_a, b_w].
    Returns (preint (F, 16) f64, cov (F, 9, 9) f64)."""
    F = seg.shape[0] - 1
    _dev(imu, torch.float64, None, "imu")
    if imu.dim() != 2 or imu.shape[1] != 7:
        raise ValueError("imu must have shape (m, 7)")
    _dev(seg, torch.int64, (F + 1,), "seg")
    _dev(bias, torch.float64, (F, 6), "bias")
    pre = torch.empty((F, 16), dtype=torch.float64, device=imu.device)
    cov = torch.empty((F, 9, 9), dtype=torch.float64, device=imu.device)
    _check(_lib.vgicp_imu_preintegrate(_ptr(imu), imu.shape[0], _ptr(seg), F, _ptr(bias),
                                       float(gyro_sigma),
                                       float(acc_sigma), _ptr(pre), _ptr(cov), _stream(stream)),
           "vgicp_imu_preintegrate")
    return pre, cov


def vgicp_imu_linearize(preint: torch.Tensor, cov: torch.Tensor, states: torch.Tensor,
                        poses: torch.Tensor, velocities: torch.Tensor, gravity, stream=None):
    """Returns dict(H (F, 18, 18), b (F, 18), err (F,)) as device f64 tensors."""
    F = preint.shape[0]
    P = poses.shape[0]
    _dev(preint, torch.float64, (F, 16), "preint")
    _dev(cov, torch.float64, (F, 9, 9), "cov")
    _dev(states, torch.int32, (F, 2), "states")
    _dev(poses, torch.float64, (P, 12), "poses")
    _dev(velocities, torch.float64, (P, 3), "velocities")
    g = np.ascontiguousarray(np.asarray(gravity, np.float64).reshape(3))
    out = {"H": torch.empty((F, 18, 18), dtype=torch.float64, device=preint.device),
           "b": torch.empty((F, 18), dtype=torch.float64, device=preint.device),
           "err": torch.empty(F, dtype=torch.float64, device=preint.device)}
    _check(_lib.vgicp_imu_linearize(_ptr(preint), _ptr(cov), _ptr(states), F, _ptr(poses),
                                    _ptr(velocities), P, _np_ptr(g), _ptr(out["H"]),
                                    _ptr(out["b"]), _ptr(out["err"]), _stream(stream)),
           "vgicp_imu_linearize")
    return out


def vgicp_imu_preintegrate_bias(imu: torch.Tensor, seg: torch.Tensor, bias: torch.Tensor,
                                gyro_sigma: float, acc_sigma: float, stream=None):
    """vgicp_imu_preintegrate plus the bias derivatives. Returns (preint (F, 16), cov (F, 9, 9),
    bias_jac (F, 9, 6)) f64 device tensors."""
    F = seg.shape[0] - 1
    _dev(imu, torch.float64, None, "imu")
    if imu.dim() != 2 or imu.shape[1] != 7:
        raise ValueError("imu must have shape (m, 7)")
    _dev(seg, torch.int64, (F + 1,), "seg")
    _dev(bias, torch.float64, (F, 6), "bias")
    pre = torch.empty((F, 16), dtype=torch.float64, device=imu.device)
    cov = torch.empty((F, 9, 9), dtype=torch.float64, device=imu.device)
    jac = torch.empty((F, 9, 6), dtype=torch.float64, device=imu.device)
    _check(_lib.vgicp_imu_preintegrate_bias(_ptr(imu), imu.shape[0], _ptr(seg), F, _ptr(bias),
                                            float(gyro_sigma), float(acc_sigma), _ptr(pre),
                                            _ptr(cov), _ptr(jac), _stream(stream)),
           "vgicp_imu_preintegrate_bias")
    return pre, cov, jac


def vgicp_imu_linearize_bias(preint: torch.Tensor, cov: torch.Tensor, bias_jac: torch.Tensor,
                             preint_bias: torch.Tensor, states: torch.Tensor,
                             poses: torch.Tensor, velocities: torch.Tensor,
                             biases: torch.Tensor, gravity, bias_walk_acc: float,
                             bias_walk_gyro: float, stream=None):
    """The 30-unknown IMU factor with bias states. Returns dict(H (F, 30, 30), b (F, 30),
    err (F,)) as device f64 tensors."""
    F = preint.shape[0]
    P = poses.shape[0]
    _dev(preint, torch.float64, (F, 16), "preint")
    _dev(cov, torch.float64, (F, 9, 9), "cov")
    _dev(bias_jac, torch.float64, (F, 9, 6), "bias_jac")
    _dev(preint_bias, torch.float64, (F, 6), "preint_bias")
    _dev(states, torch.int32, (F, 2), "states")
    _dev(poses, torch.float64, (P, 12), "poses")
    _dev(velocities, torch.float64, (P, 3), "velocities")
    _dev(biases, torch.float64, (P, 6), "biases")
    g = np.ascontiguousarray(np.asarray(gravity, np.float64).reshape(3))
    out = {"H": torch.empty((F, 30, 30), dtype=torch.float64, device=preint.device),
           "b": torch.empty((F, 30), dtype=torch.float64, device=preint.device),
           "err": torch.empty(F, dtype=torch.float64, device=preint.device)}
    _check(_lib.vgicp_imu_linearize_bias(_ptr(preint), _ptr(cov), _ptr(bias_jac),
                                         _ptr(preint_bias), _ptr(states), F, _ptr(poses),
                                         _ptr(velocities), _ptr(biases), P, _np_ptr(g),
                                         float(bias_walk_acc), float(bias_walk_gyro),
                                         _ptr(out["H"]), _ptr(out["b"]), _ptr(out["err"]),
                                         _stream(stream)), "vgicp_imu_linearize_bias")
    return out


def vgicp_build_voxelmap(xyz: torch.Tensor, cov: torch.Tensor, resolution: float,
                         stream=None, layout: int = VGICP_LAYOUT_AUTO) -> VoxelMap:
    n = _cloud(xyz, cov)
    h = ctypes.c_void_p()
    if layout != VGICP_LAYOUT_AUTO:
        return vgicp_build_voxelmap_layout(xyz, cov, resolution, layout, stream)
    _check(_lib.vgicp_build_voxelmap(_ptr(xyz), _ptr(cov), n, float(resolution),
                                     _stream(stream), ctypes.byref(h)), "vgicp_build_voxelmap")
    return VoxelMap(h, float(resolution))


def vgicp_build_voxelmap_layout(xyz: torch.Tensor, cov: torch.Tensor, resolution: float,
                                layout: int, stream=None) -> VoxelMap:
    n = _cloud(xyz, cov)
    h = ctypes.c_void_p()
    _check(_lib.vgicp_build_voxelmap_layout(_ptr(xyz), _ptr(cov), n, float(resolution),
                                            int(layout), _stream(stream), ctypes.byref(h)),
           "vgicp_build_voxelmap_layout")
    return VoxelMap(h, float(resolution))


def vgicp_voxelmap_layout(m: VoxelMap) -> int:
    v = ctypes.c_int32()
    _check(_lib.vgicp_voxelmap_layout(m.handle, ctypes.byref(v)), "vgicp_voxelmap_layout")
    return v.value


def vgicp_voxelmap_size(m: VoxelMap):
    V, cap = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.vgicp_voxelmap_size(m.handle, ctypes.byref(V), ctypes.byref(cap)),
           "vgicp_voxelmap_size")
    return V.value, cap.value


def vgicp_voxelmap_export(m: VoxelMap, stream=None):
    V, _ = vgicp_voxelmap_size(m)
    dev = torch.device("cuda", torch.cuda.current_device())
    keys = torch.empty(V, dtype=torch.int64, device=dev)
    mean = torch.empty((3, V), dtype=torch.float64, device=dev)
    cov = torch.empty((6, V), dtype=torch.float64, device=dev)
    count = torch.empty(V, dtype=torch.int32, device=dev)
    _check(_lib.vgicp_voxelmap_export(m.handle, _ptr(keys), _ptr(mean), _ptr(cov), _ptr(count),
                                      _stream(stream)), "vgicp_voxelmap_export")
    return {"keys": keys, "mean": mean, "cov": cov, "count": count}


def vgicp_linearize(m: VoxelMap, xyz, cov, T_target, T_source, binary: bool,
                    precision: int = VGICP_ACC_FP64, want_corr: bool = False, stream=None,
                    out=None):
    """Returns dict(H (d, d) f64, b (d,) f64, err (1,) f64, inliers (1,) i64, corr (n,) i32|None)
    as device tensors; d = 12 if binary else 6."""
    return _linearize(_lib.vgicp_linearize, "vgicp_linearize", m, xyz, cov, T_target, T_source,
                      binary, precision, want_corr, stream, out)


def vgicp_linearize_noalloc(m: VoxelMap, xyz, cov, T_target, T_source, binary: bool,
                            precision: int = VGICP_ACC_FP64, want_corr: bool = False,
                            stream=None, out=None):
    """vgicp_linearize through the library's allocation-free entry point (static device scratch;
    pass `out` to allocate nothing on this side either)."""
    return _linearize(_lib.vgicp_linearize_noalloc, "vgicp_linearize_noalloc", m, xyz, cov,
                      T_target, T_source, binary, precision, want_corr, stream, out)


def _linearize(fn, name, m, xyz, cov, T_target, T_source, binary, precision, want_corr, stream,
               out):
    n = _cloud(xyz, cov)
    d = 12 if binary else 6
    dev = xyz.device
    if out is None:
        out = {"H": torch.empty((d, d), dtype=torch.float64, device=dev),
               "b": torch.empty(d, dtype=torch.float64, device=dev),
               "err": torch.empty(1, dtype=torch.float64, device=dev),
               "inliers": torch.empty(1, dtype=torch.int64, device=dev),
               "corr": torch.empty(n, dtype=torch.int32, device=dev) if want_corr else None}
    Tt, Ts = _pose(T_target), _pose(T_source)
    _check(fn(m.handle, _ptr(xyz), _ptr(cov), n, _np_ptr(Tt), _np_ptr(Ts), int(bool(binary)),
              int(precision), _ptr(out["H"]), _ptr(out["b"]), _ptr(out["err"]),
              _ptr(out["inliers"]), _ptr(out.get("corr")), _stream(stream)), name)
    return out


def vgicp_evaluate(m: VoxelMap, xyz, cov, T_target, T_source, precision: int = VGICP_ACC_FP64,
                   want_corr: bool = False, stream=None):
    n = _cloud(xyz, cov)
    dev = xyz.device
    out = {"err": torch.empty(1, dtype=torch.float64, device=dev),
           "inliers": torch.empty(1, dtype=torch.int64, device=dev),
           "corr": torch.empty(n, dtype=torch.int32, device=dev) if want_corr else None}
    Tt, Ts = _pose(T_target), _pose(T_source)
    _check(_lib.vgicp_evaluate(m.handle, _ptr(xyz), _ptr(cov), n, _np_ptr(Tt), _np_ptr(Ts),
                               int(precision), _ptr(out["err"]), _ptr(out["inliers"]),
                               _ptr(out["corr"]), _stream(stream)), "vgicp_evaluate")
    return out


def vgicp_backward(m: VoxelMap, xyz, cov, T_target, T_source, binary: bool, corr,
                   grad_err: torch.Tensor, precision: int = VGICP_ACC_FP64,
                   want_points: bool = True, stream=None):
    """Returns (grad_xi (6|12,) f64, grad_xyz (3, n) f32 or None) as device tensors."""
    n = _cloud(xyz, cov)
    _dev(corr, torch.int32, (n,), "corr")
    _dev(grad_err, torch.float64, (1,), "grad_err")
    dev = xyz.device
    gxi = torch.empty(12 if binary else 6, dtype=torch.float64, device=dev)
    gp = torch.empty((3, n), dtype=torch.float32, device=dev) if want_points else None
    Tt, Ts = _pose(T_target), _pose(T_source)
    _check(_lib.vgicp_backward(m.handle, _ptr(xyz), _ptr(cov), n, _np_ptr(Tt), _np_ptr(Ts),
                               int(bool(binary)), _ptr(corr), _ptr(grad_err), int(precision),
                               _ptr(gxi), _ptr(gp), _stream(stream)), "vgicp_backward")
    return gxi, gp


def vgicp_backward_tangent(m: VoxelMap, xyz, cov, T_target, T_source, xi_target, xi_source,
                           binary: bool, corr, grad_err: torch.Tensor,
                           precision: int = VGICP_ACC_FP64, want_points: bool = True,
                           stream=None):
    """vgicp_backward at T Exp(xi), the pose gradient in the tangent coordinates xi.
    xi_target / xi_source: 6 values or None. Returns (grad_xi (6|12,) f64, grad_xyz (3, n) f32
    or None) as device tensors."""
    n = _cloud(xyz, cov)
    _dev(corr, torch.int32, (n,), "corr")
    _dev(grad_err, torch.float64, (1,), "grad_err")
    dev = xyz.device
    gxi = torch.empty(12 if binary else 6, dtype=torch.float64, device=dev)
    gp = torch.empty((3, n), dtype=torch.float32, device=dev) if want_points else None
    Tt, Ts = _pose(T_target), _pose(T_source)
    xt = None if xi_target is None else np.ascontiguousarray(xi_target, np.float64).reshape(6)
    xs = None if xi_source is None else np.ascontiguousarray(xi_source, np.float64).reshape(6)
    _check(_lib.vgicp_backward_tangent(m.handle, _ptr(xyz), _ptr(cov), n, _np_ptr(Tt),
                                       _np_ptr(Ts), None if xt is None else _np_ptr(xt),
                                       None if xs is None else _np_ptr(xs), int(bool(binary)),
                                       _ptr(corr), _ptr(grad_err), int(precision), _ptr(gxi),
                                       _ptr(gp), _stream(stream)), "vgicp_backward_tangent")
    return gxi, gp


class Batch:
    """A prepared batch of factors (vgicp_batch_*). Keeps the clouds and maps alive."""

    def __init__(self, maps: Sequence[VoxelMap], clouds: Sequence[tuple], factors,
                 n_poses: int):
        self._maps = list(maps)
        self._clouds = [(x, c) for x, c in clouds]
        carr = (Cloud * max(1, len(clouds)))()
        for i, (x, c) in enumerate(self._clouds):
            n = _cloud(x, c)
            carr[i] = Cloud(x.data_ptr(), c.data_ptr(), n)
        f = np.ascontiguousarray(np.asarray(factors, dtype=np.int32).reshape(-1, 5))
        self.n_factors = f.shape[0]
        self.n_poses = int(n_poses)
        marr = (ctypes.c_void_p * max(1, len(maps)))(*[m.handle.value for m in maps])
        h = ctypes.c_void_p()
        _check(_lib.vgicp_batch_create(marr, len(maps), carr, len(clouds), _np_ptr(f),
                                       self.n_factors, self.n_poses, ctypes.byref(h)),
               "vgicp_batch_create")
        self._h = h
        self.factors = f

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.vgicp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def overlap(self, poses: torch.Tensor, stream=None):
        """Overlap rate (inliers / n) and inlier count of every factor at `poses`."""
        dev = self._device()
        rates = torch.empty(self.n_factors, dtype=torch.float64, device=dev)
        nin = torch.empty(self.n_factors, dtype=torch.int64, device=dev)
        _check(_lib.vgicp_batch_overlap(self._h, _ptr(self._poses(poses)), _ptr(rates),
                                        _ptr(nin), _stream(stream)), "vgicp_batch_overlap")
        return {"rates": rates, "inliers": nin}

    def lm_step(self, poses, precision=VGICP_ACC_FP64, lam: float = 1e-4,
                fixed_pose: int = -1, stream=None):
        """One Levenberg-Marquardt step of the factors' pose graph: new poses, the step
        [P, 6] and the costs before and after."""
        Pz = self._poses(poses)
        dev = self._device()
        out = {"poses": torch.empty((self.n_poses, 12), dtype=torch.float64, device=dev),
               "delta": torch.empty((self.n_poses, 6), dtype=torch.float64, device=dev),
               "cost": torch.empty(2, dtype=torch.float64, device=dev)}
        _check(_lib.vgicp_batch_lm_step(self._h, _ptr(Pz), int(precision), float(lam),
                                        int(fixed_pose), _ptr(out["poses"]), _ptr(out["delta"]),
                                        _ptr(out["cost"]), _stream(stream)),
               "vgicp_batch_lm_step")
        return out

    def lm_iterate(self, poses: torch.Tensor, lam: torch.Tensor, iterations: int,
                   precision=VGICP_ACC_FP64, fixed_pose: int = -1, stream=None):
        """`iterations` LM iterations decided on the device; poses ([P, 12] f64) and lam ([1]
        f64) are updated in place. Returns the costs [iterations + 1]."""
        Pz = self._poses(poses)
        lz = _dev(lam, torch.float64, (1,), "lambda")
        cost = torch.empty(int(iterations) + 1, dtype=torch.float64, device=self._device())
        _check(_lib.vgicp_batch_lm_iterate(self._h, _ptr(Pz), int(precision), _ptr(lz),
                                           int(fixed_pose), int(iterations), _ptr(cost),
                                           _stream(stream)), "vgicp_batch_lm_iterate")
        return cost

    def lm_solver(self, solver: int):
        """0: automatic (banded when possible, from both ends when long enough), 1: dense,
        2: banded in one sweep (when possible)."""
        _check(_lib.vgicp_batch_lm_solver(self._h, int(solver)), "vgicp_batch_lm_solver")

    def lm_info(self):
        """(banded, half-bandwidth of the ordered system): banded is 0 for the dense solver, 1 for
        the banded one in one sweep, 2 for the banded one from both ends."""
        b, w = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.vgicp_batch_lm_info(self._h, ctypes.byref(b), ctypes.byref(w)),
               "vgicp_batch_lm_info")
        return int(b.value), int(w.value)

    def refresh(self, stream=None):
        """Re-copies the clouds' covariances after the caller changed them."""
        _check(_lib.vgicp_batch_refresh(self._h, _stream(stream)), "vgicp_batch_refresh")

    def set_schedule(self, block: int, tile: int, blocks_per_cu: int, lookahead: int = 4):
        s = Schedule(block, tile, blocks_per_cu, lookahead)
        _check(_lib.vgicp_batch_set_schedule(self._h, ctypes.byref(s)),
               "vgicp_batch_set_schedule")

    def get_schedule(self):
        s = Schedule()
        _check(_lib.vgicp_batch_get_schedule(self._h, ctypes.byref(s)),
               "vgicp_batch_get_schedule")
        return s.as_tuple()

    def _poses(self, poses: torch.Tensor):
        return _dev(poses, torch.float64, (self.n_poses, 12), "poses")

    def autotune(self, poses, precision=VGICP_ACC_FP64, cache_path=None, stream=None):
        s = Schedule()
        cp = None if cache_path is None else str(cache_path).encode()
        _check(_lib.vgicp_batch_autotune(self._h, _ptr(self._poses(poses)), int(precision), cp,
                                         ctypes.byref(s), _stream(stream)),
               "vgicp_batch_autotune")
        return s.as_tuple()

    def _device(self):
        return self._clouds[0][0].device if self._clouds else torch.device("cuda")

    def alloc_outputs(self, device=None):
        dev = device if device is not None else self._device()
        F = self.n_factors
        return {"H": torch.empty((F, 12, 12), dtype=torch.float64, device=dev),
                "b": torch.empty((F, 12), dtype=torch.float64, device=dev),
                "err": torch.empty(F, dtype=torch.float64, device=dev),
                "inliers": torch.empty(F, dtype=torch.int64, device=dev)}

    def linearize(self, poses, precision=VGICP_ACC_FP64, out=None, stream=None):
        out = out or self.alloc_outputs()
        _check(_lib.vgicp_batch_linearize(self._h, _ptr(self._poses(poses)), int(precision),
                                          _ptr(out["H"]), _ptr(out["b"]), _ptr(out["err"]),
                                          _ptr(out["inliers"]), _stream(stream)),
               "vgicp_batch_linearize")
        return out

    def backward(self, poses, grad_err, precision=VGICP_ACC_FP64, want_points: bool = True,
                 want_factors: bool = False, stream=None):
        """Gradient of sum_f grad_err[f] e_f at `poses` (correspondences held): per pose
        [P, 6] (right perturbation, [omega; rho]), optionally per factor [F, 12] ([source |
        target]) and per source point ([3, n] per cloud, the clouds' own order)."""
        dev = self._device()
        g = _dev(grad_err, torch.float64, (self.n_factors,), "grad_err")
        out = {"grad_poses": torch.empty((self.n_poses, 6), dtype=torch.float64, device=dev),
               "grad_factors": (torch.empty((self.n_factors, 12), dtype=torch.float64,
                                            device=dev) if want_factors else None),
               "grad_points": ([torch.empty_like(x) for x, _ in self._clouds]
                               if want_points else None)}
        parr = None
        if want_points:
            parr = (ctypes.c_void_p * max(1, len(self._clouds)))(
                *[t.data_ptr() for t in out["grad_points"]])
        _check(_lib.vgicp_batch_backward(self._h, _ptr(self._poses(poses)), int(precision),
                                         _ptr(g), _ptr(out["grad_poses"]),
                                         _ptr(out["grad_factors"]), parr, _stream(stream)),
               "vgicp_batch_backward")
        return out

    def evaluate(self, poses, precision=VGICP_ACC_FP64, out=None, stream=None):
        F = self.n_factors
        dev = self._device()
        out = out or {"err": torch.empty(F, dtype=torch.float64, device=dev),
                      "inliers": torch.empty(F, dtype=torch.int64, device=dev)}
        _check(_lib.vgicp_batch_evaluate(self._h, _ptr(self._poses(poses)), int(precision),
                                         _ptr(out["err"]), _ptr(out["inliers"]),
                                         _stream(stream)), "vgicp_batch_evaluate")
        return out


def vgicp_batch_create(maps, clouds, factors, n_poses) -> Batch:
    return Batch(maps, clouds, factors, n_poses)


def vgicp_linearize_batched(maps, clouds, poses, factors, precision=VGICP_ACC_FP64,
                            stream=None):
    """One-shot batch (create, linearize, destroy); synchronises the stream."""
    carr = (Cloud * max(1, len(clouds)))()
    for i, (x, c) in enumerate(clouds):
        carr[i] = Cloud(x.data_ptr(), c.data_ptr(), _cloud(x, c))
    marr = (ctypes.c_void_p * max(1, len(maps)))(*[m.handle.value for m in maps])
    f = np.ascontiguousarray(np.asarray(factors, dtype=np.int32).reshape(-1, 5))
    F = f.shape[0]
    _dev(poses, torch.float64, (poses.shape[0], 12), "poses")
    dev = poses.device
    out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device=dev),
           "b": torch.empty((F, 12), dtype=torch.float64, device=dev),
           "err": torch.empty(F, dtype=torch.float64, device=dev),
           "inliers": torch.empty(F, dtype=torch.int64, device=dev)}
    _check(_lib.vgicp_linearize_batched(marr, len(maps), carr, len(clouds), _ptr(poses),
                                        poses.shape[0], _np_ptr(f), F, int(precision),
                                        _ptr(out["H"]), _ptr(out["b"]), _ptr(out["err"]),
                                        _ptr(out["inliers"]), _stream(stream)),
           "vgicp_linearize_batched")
    return out


def vgicp_sync_status(stream=None):
    _check(_lib.vgicp_sync_status(_stream(stream)), "vgicp_sync_status")


def vgicp_relative_pose(T_target, T_source) -> np.ndarray:
    out = np.empty(12)
    Tt, Ts = _pose(T_target), _pose(T_source)
    _check(_lib.vgicp_relative_pose(_np_ptr(Tt), _np_ptr(Ts), _np_ptr(out)),
           "vgicp_relative_pose")
    return out


def vgicp_se3_retract(T, xi) -> np.ndarray:
    out = np.empty(12)
    x = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(6))
    Tp = _pose(T)
    _check(_lib.vgicp_se3_retract(_np_ptr(Tp), _np_ptr(x), _np_ptr(out)), "vgicp_se3_retract")
    return out


def vgicp_pose_order(P: int, links):
    """The LM solver's pose order for P poses and links ((k, 2) pose indices): (pos, bandwidth),
    pos[p] = position of pose p. Host only."""
    lk = np.ascontiguousarray(np.asarray(links, dtype=np.int32).reshape(-1, 2))
    pos = np.empty(max(int(P), 1), np.int32)
    bw = ctypes.c_int32()
    _check(_lib.vgicp_pose_order(int(P), _np_ptr(lk), int(lk.shape[0]), _np_ptr(pos),
                                 ctypes.byref(bw)), "vgicp_pose_order")
    return pos[:int(P)], int(bw.value)


def vgicp_se3_right_jacobian(xi) -> np.ndarray:
    out = np.empty(36)
    x = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(6))
    _check(_lib.vgicp_se3_right_jacobian(_np_ptr(x), _np_ptr(out)), "vgicp_se3_right_jacobian")
    return out.reshape(6, 6)
