"""Oracle of the preprocessing of Sec. III-C: voxel-grid filter, k nearest neighbours, and point
covariances estimated from those neighbours (the covariances C_k of Sec. III-A).

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy in FP64; the loops over points
and voxels are Python loops on purpose, so that each step reads as its definition.

The section names the steps, not their arithmetic; the readings taken here:

* voxel-grid filter: a point belongs to the cell floor(p / res) per axis (FP64, the same key rule
  as the voxel map, |cell| < 2^20). Every output point is the FP64 mean of its members' positions
  (and timestamps), rounded to FP32. With timestamps, a cell's members are taken in ascending
  (t, index) order and a point whose timestamp differs from the running mean timestamp of the
  cell's current voxel by more than d_scan / 10 starts a new voxel in that cell (so the first and
  last points of a sweep do not fuse); without timestamps a cell is one voxel, summed in index
  order. Output order: ascending cell (x, then y, then z), then voxel creation order in the cell.
* k nearest neighbours: the k points with the smallest squared distance
  ((dx*dx + dy*dy) + dz*dz, FP64 from the FP32 coordinates), ties broken by the lower index; the
  point itself is included (distance 0). Fewer than k points: trailing entries are -1. Layout
  [k][n], the neighbours of point i in column i, nearest first.
* covariance: S = sum over the listed neighbours of (p - m)(p - m)^T about their mean m (FP64).
  Plane regularization (GICP): with n the unit eigenvector of the smallest eigenvalue of S,
  C = scale * (I - (1 - eps) n n^T), i.e. the eigenvalues replaced by scale * (1, 1, eps).
  scale <= 0 returns the raw covariance S / m (m = number of listed neighbours). FP32 output,
  6 planes xx, xy, xz, yy, yz, zz.
"""
from __future__ import annotations

import numpy as np

from . import E_KEY_RANGE, E_NONFINITE, OracleError

KEY_LIMIT = 1 << 20


def cells(xyz, res):
    """(3, n) int64 cells floor(p / res) in FP64, with the range and finiteness checks."""
    p = np.asarray(xyz, np.float32).reshape(3, -1).astype(np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        c = np.floor(p / float(res))
    if not np.all(np.isfinite(c)):
        raise OracleError(E_NONFINITE, "downsample")
    if np.any(np.abs(c) >= KEY_LIMIT):
        raise OracleError(E_KEY_RANGE, "downsample")
    return c.astype(np.int64)


def downsample(xyz, res, t=None, scan_duration=0.0):
    """Voxel-grid filter. Returns (xyz_out (3, m) float32, t_out (m,) float32 or None,
    count (m,) int64, cell (3, m) int64)."""
    p = np.asarray(xyz, np.float32).reshape(3, -1)
    n = p.shape[1]
    c = cells(p, res)
    idx = np.arange(n)
    tt = None
    if t is not None:
        tt = np.asarray(t, np.float32).reshape(-1).astype(np.float64)
        if not np.all(np.isfinite(tt)):
            raise OracleError(E_NONFINITE, "downsample")
        order = np.lexsort((idx, tt, c[2], c[1], c[0]))
    else:
        order = np.lexsort((idx, c[2], c[1], c[0]))
    thr = float(scan_duration) / 10.0
    p64 = p.astype(np.float64)
    out, out_t, counts, out_c = [], [], [], []

    def emit(s, st, cnt, cell):
        out.append([s[0] / cnt, s[1] / cnt, s[2] / cnt])
        out_t.append(st / cnt)
        counts.append(cnt)
        out_c.append(cell)

    i = 0
    while i < n:
        cell = tuple(int(v) for v in c[:, order[i]])
        j = i
        while j < n and tuple(int(v) for v in c[:, order[j]]) == cell:
            j += 1
        s, st, cnt = [0.0, 0.0, 0.0], 0.0, 0
        for q in order[i:j]:
            if tt is not None and cnt > 0 and abs(tt[q] - st / cnt) > thr:
                emit(s, st, cnt, cell)
                s, st, cnt = [0.0, 0.0, 0.0], 0.0, 0
            for a in range(3):
                s[a] = s[a] + p64[a, q]
            if tt is not None:
                st = st + tt[q]
            cnt += 1
        emit(s, st, cnt, cell)
        i = j
    m = len(out)
    xo = np.array(out, np.float64).reshape(m, 3).T.astype(np.float32)
    to = np.array(out_t, np.float64).astype(np.float32) if tt is not None else None
    return (np.ascontiguousarray(xo), to, np.array(counts, np.int64),
            np.array(out_c, np.int64).reshape(m, 3).T)


def sq_dist(P, Q):
    """Squared distances (len(Q), len(P)) in FP64: (dx*dx + dy*dy) + dz*dz, no contraction."""
    dx = P[None, :, 0] - Q[:, None, 0]
    dy = P[None, :, 1] - Q[:, None, 1]
    dz = P[None, :, 2] - Q[:, None, 2]
    return (dx * dx + dy * dy) + dz * dz


def knn(xyz, k, rows=None, chunk=512):
    """k nearest neighbours by (squared distance, index). Returns int32 (k, len(rows)), rows
    defaulting to every point."""
    P = np.asarray(xyz, np.float32).reshape(3, -1).T.astype(np.float64)
    n = P.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, np.int64)
    out = np.full((k, len(rows)), -1, np.int32)
    kk = min(k, n)
    if kk == 0:
        return out
    for c0 in range(0, len(rows), chunk):
        r = rows[c0:c0 + chunk]
        d2 = sq_dist(P, P[r])
        kth = np.partition(d2, kk - 1, axis=1)[:, kk - 1]
        for a in range(len(r)):
            cand = np.flatnonzero(d2[a] <= kth[a])
            sel = cand[np.lexsort((cand, d2[a, cand]))][:kk]
            out[:kk, c0 + a] = sel
    return out


def normals(xyz, nbr):
    """Per point: the scatter matrix S of its listed neighbours, its eigenvalues (ascending) and
    the unit eigenvector of the smallest one (numpy.linalg.eigh)."""
    P = np.asarray(xyz, np.float32).reshape(3, -1).T.astype(np.float64)
    nb = np.asarray(nbr).reshape(nbr.shape[0], -1)
    valid = nb >= 0
    pts = P[np.where(valid, nb, 0).T]                 # (n, k, 3)
    w = valid.T.astype(np.float64)[:, :, None]        # (n, k, 1)
    m = np.maximum(w.sum(axis=1), 1.0)                # (n, 1)
    mean = (pts * w).sum(axis=1) / m
    d = (pts - mean[:, None, :]) * w
    S = np.einsum("nki,nkj->nij", d, d)
    lam, U = np.linalg.eigh(S)
    return S, lam, U[:, :, 0], m[:, 0]


def covariances(xyz, nbr, scale=0.01, eps=1e-3):
    """(6, n) FP32 point covariances from the neighbour lists nbr ([k][n], -1 = none)."""
    S, _, nrm, m = normals(xyz, nbr)
    if scale > 0:
        C = scale * (np.eye(3)[None] - (1.0 - eps) * nrm[:, :, None] * nrm[:, None, :])
    else:
        C = S / m[:, None, None]
    six = np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]])
    return np.ascontiguousarray(six.astype(np.float32))
