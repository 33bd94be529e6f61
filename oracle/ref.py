"""NumPy brute-force twin of the oracle, for tiny inputs only.

TEST INFRASTRUCTURE ONLY (see the package docstring). Shares no code with ``oracle.cpp``: the
voxel of a source point is found by scanning every target point's integer coordinates (no
sorting, no hashing), inverses come from ``numpy.linalg.inv`` and every matrix product is
written as the definition of Sec. III-A, Eqs. (2)-(3), with explicit Jacobians.
"""
from __future__ import annotations

import numpy as np


def skew(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def sym3(c6):
    xx, xy, xz, yy, yz, zz = c6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]], dtype=np.float64)


def as34(T):
    T = np.asarray(T, dtype=np.float64)
    return T[:3, :] if T.shape == (4, 4) else T.reshape(3, 4)


def relative(T_target, T_source):
    """T_t^-1 T_s as (R, t)."""
    Tt, Ts = as34(T_target), as34(T_source)
    Rt, tt, Rs, ts = Tt[:, :3], Tt[:, 3], Ts[:, :3], Ts[:, 3]
    return Rt.T @ Rs, Rt.T @ (ts - tt)


def brute_voxel(target_xyz, target_cov, res, q):
    """Members of the voxel containing q, found by scanning all target points.
    Returns (mean, cov (3x3), count, member index list) or None."""
    kq = np.floor(np.asarray(q, dtype=np.float64) / res)
    members = []
    for j in range(target_xyz.shape[1]):
        kj = np.floor(target_xyz[:, j].astype(np.float64) / res)
        if np.array_equal(kj, kq):
            members.append(j)
    if not members:
        return None
    mean = np.zeros(3)
    cov = np.zeros(6)
    for j in members:
        mean += target_xyz[:, j]
        cov += target_cov[:, j]
    n = len(members)
    return mean / n, sym3(cov / n), n, members


def linearize(target_xyz, target_cov, res, src_xyz, src_cov, T_target, T_source, binary):
    target_xyz = np.asarray(target_xyz, dtype=np.float64)
    target_cov = np.asarray(target_cov, dtype=np.float64)
    src_xyz = np.asarray(src_xyz, dtype=np.float64)
    src_cov = np.asarray(src_cov, dtype=np.float64)
    R, t = relative(T_target, T_source)
    dim = 12 if binary else 6
    H = np.zeros((dim, dim))
    b = np.zeros(dim)
    e = 0.0
    inliers = 0
    for k in range(src_xyz.shape[1]):
        mu = src_xyz[:, k]
        C = sym3(src_cov[:, k])
        q = R @ mu + t
        vox = brute_voxel(target_xyz, target_cov, res, q)
        if vox is None:
            continue
        mean, Cv, _, _ = vox
        d = mean - q
        Omega = np.linalg.inv(Cv + R @ C @ R.T)
        Js = np.hstack([R @ skew(mu), -R])
        J = np.hstack([Js, np.hstack([-skew(q), np.eye(3)])]) if binary else Js
        e += d @ Omega @ d
        H += J.T @ Omega @ J
        b += J.T @ Omega @ d
        inliers += 1
    return {"H": H, "b": b, "e": e, "inliers": inliers}


def cost(target_xyz, target_cov, res, src_xyz, src_cov, T_target, T_source):
    """Eq. (2) by brute force (fresh voxel lookup per point)."""
    R, t = relative(T_target, T_source)
    src_xyz = np.asarray(src_xyz, dtype=np.float64)
    e = 0.0
    for k in range(src_xyz.shape[1]):
        mu = src_xyz[:, k]
        q = R @ mu + t
        vox = brute_voxel(np.asarray(target_xyz, np.float64), np.asarray(target_cov, np.float64),
                          res, q)
        if vox is None:
            continue
        mean, Cv, _, _ = vox
        d = mean - q
        e += d @ np.linalg.inv(Cv + R @ sym3(src_cov[:, k]) @ R.T) @ d
    return e
