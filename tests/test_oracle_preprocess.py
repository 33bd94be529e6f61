"""Pins of the preprocessing oracle (oracle/preprocess.py), on the CPU.

* voxel-grid filter: hand cases on exact cell faces (including -0.0 and -1e-30), the cell count
  against a brute-force set of Python floor() tuples, conservation of the point sum, invariance
  to the input order on dyadic coordinates (exact sums), the timestamp split on a hand-built
  sweep seam, and the no-split limit;
* k nearest neighbours: scipy's k-d tree on continuous random clouds (no ties), a hand-built
  lattice whose equal distances must come out in index order, fewer points than k, duplicates;
* covariances: points on a known plane give scale (I - (1 - eps) n n^T); eps = 1 gives scale I;
  rotating the cloud rotates the covariances; the raw form equals numpy.cov (bias=True).
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle
from oracle import preprocess as pp


def soa(pts):
    return np.ascontiguousarray(np.asarray(pts, np.float32).T)


# ------------------------------------------------------------------ voxel-grid filter

def test_downsample_hand_cases():
    pts = [(0.25, 0.25, 0.25), (0.75, 0.75, 0.75),   # cell (0, 0, 0): mean 0.5
           (1.0, 0.0, 0.0),                           # on a face: cell (1, 0, 0)
           (-0.0, 2.5, 0.0),                          # -0.0 -> cell 0
           (-1e-30, 0.0, 0.0)]                        # -> cell -1
    xo, to, cnt, cell = pp.downsample(soa(pts), 1.0)
    assert to is None
    assert cell.T.tolist() == [[-1, 0, 0], [0, 0, 0], [0, 2, 0], [1, 0, 0]]
    assert cnt.tolist() == [1, 2, 1, 1]
    np.testing.assert_array_equal(xo.T, np.array([[-1e-30, 0, 0], [0.5, 0.5, 0.5],
                                                  [0.0, 2.5, 0.0], [1.0, 0.0, 0.0]], np.float32))


def test_downsample_cell_count_and_conservation():
    rng = np.random.default_rng(5)
    pts = rng.normal(size=(3000, 3)) * np.array([4.0, 3.0, 0.5])
    for res in (0.25, 0.3, 1.0):
        p32 = pts.astype(np.float32)
        brute = {tuple(math.floor(float(v) / res) for v in p) for p in p32}
        xo, _, cnt, cell = pp.downsample(soa(p32), res)
        assert len(cnt) == len(brute)
        assert {tuple(c) for c in cell.T.tolist()} == brute
        assert cnt.sum() == len(p32)
        total = (xo.astype(np.float64) * cnt).sum(axis=1)
        np.testing.assert_allclose(total, p32.astype(np.float64).sum(axis=0), rtol=1e-6,
                                   atol=1e-3)
        # every output point lies in its cell
        assert np.all(np.floor(xo.astype(np.float64) / res) == cell)


def test_downsample_order_invariance_on_dyadic_points():
    rng = np.random.default_rng(6)
    pts = (rng.integers(-64, 64, size=(2000, 3)) / 8.0).astype(np.float32)
    a = pp.downsample(soa(pts), 0.5)
    b = pp.downsample(soa(pts[rng.permutation(len(pts))]), 0.5)
    for x, y in zip(a, b):
        if x is not None:
            np.testing.assert_array_equal(x, y)


def test_downsample_timestamp_split_at_the_seam():
    d = 0.1  # scan duration: split when |t - t_voxel| > 0.01
    pts = [(0.1, 0.1, 0.1), (0.2, 0.2, 0.2),          # start of the sweep
           (0.3, 0.3, 0.3), (0.4, 0.4, 0.4),          # end of the sweep, same cell
           (5.1, 0.1, 0.1), (5.2, 0.1, 0.1)]          # another cell, within 0.01 s
    t = [0.0, 0.002, 0.098, 0.1, 0.05, 0.055]
    xo, to, cnt, cell = pp.downsample(soa(pts), 1.0, t=np.array(t, np.float32), scan_duration=d)
    assert cnt.tolist() == [2, 2, 2]
    assert cell.T.tolist() == [[0, 0, 0], [0, 0, 0], [5, 0, 0]]
    f = lambda a, b: np.float32((np.float64(np.float32(a)) + np.float64(np.float32(b))) / 2)
    np.testing.assert_array_equal(xo[:, 0], [f(0.1, 0.2)] * 3)
    np.testing.assert_array_equal(xo[:, 1], [f(0.3, 0.4)] * 3)
    np.testing.assert_array_equal(to, [f(0.0, 0.002), f(0.098, 0.1), f(0.05, 0.055)])
    # a long scan duration never splits: same points as without timestamps
    xo2, _, cnt2, _ = pp.downsample(soa(pts), 1.0, t=np.array(t, np.float32), scan_duration=10.0)
    xo3, _, cnt3, _ = pp.downsample(soa(pts), 1.0)
    assert cnt2.tolist() == cnt3.tolist() == [4, 2]
    np.testing.assert_allclose(xo2, xo3, rtol=1e-7)


def test_downsample_split_follows_the_running_mean():
    # t = 0, 0.008, 0.016, 0.024: the third differs from the mean 0.004 by 0.012 > 0.01 and
    # starts a voxel; the fourth differs from that voxel's mean 0.016 by 0.008 and joins it.
    pts = [(0.5, 0.5, 0.5)] * 4
    t = np.array([0.016, 0.0, 0.024, 0.008], np.float32)  # input order is not time order
    _, to, cnt, _ = pp.downsample(soa(pts), 1.0, t=t, scan_duration=0.1)
    assert cnt.tolist() == [2, 2]
    assert to[0] == np.float32((np.float64(np.float32(0.0)) + np.float64(np.float32(0.008))) / 2)


def test_downsample_errors():
    with pytest.raises(oracle.OracleError):
        pp.downsample(soa([(np.nan, 0, 0)]), 1.0)
    with pytest.raises(oracle.OracleError):
        pp.downsample(soa([(2.0 ** 21, 0, 0)]), 1.0)
    xo, _, cnt, _ = pp.downsample(np.zeros((3, 0), np.float32), 1.0)
    assert xo.shape == (3, 0) and len(cnt) == 0


# ------------------------------------------------------------------ k nearest neighbours

def test_knn_matches_a_kd_tree():
    rng = np.random.default_rng(7)
    pts = (rng.normal(size=(1500, 3)) * np.array([5.0, 5.0, 1.0])).astype(np.float32)
    nbr = pp.knn(soa(pts), 10)
    d, idx = cKDTree(pts.astype(np.float64)).query(pts.astype(np.float64), k=10)
    np.testing.assert_array_equal(nbr, idx.T)
    assert np.all(nbr[0] == np.arange(len(pts)))  # the point itself comes first
    rows = np.array([3, 700, 1499])
    np.testing.assert_array_equal(pp.knn(soa(pts), 10, rows=rows), idx[rows].T)


def test_knn_equal_distances_in_index_order():
    g = np.array([(x, y, z) for x in range(3) for y in range(3) for z in range(3)], np.float32)
    nbr = pp.knn(soa(g), 7, rows=[13])  # centre (1, 1, 1): itself, then the 6 face neighbours
    assert nbr[:, 0].tolist() == [13, 4, 10, 12, 14, 16, 22]
    nbr = pp.knn(soa(g), 9, rows=[0])  # corner: itself, 3 at distance 1, then 3 at sqrt 2, ...
    assert nbr[:, 0].tolist() == [0, 1, 3, 9, 4, 10, 12, 13, 2]


def test_knn_small_and_duplicate_clouds():
    pts = np.array([(0, 0, 0), (1, 0, 0), (0, 0, 0)], np.float32)
    nbr = pp.knn(soa(pts), 5)
    assert nbr[:, 2].tolist() == [0, 2, 1, -1, -1]  # the duplicate with the lower index first
    assert nbr[:, 0].tolist() == [0, 2, 1, -1, -1]
    assert pp.knn(np.zeros((3, 0), np.float32), 4).shape == (4, 0)


# ------------------------------------------------------------------ covariances

def plane_cloud(rng, n, normal, spread=1.0):
    normal = normal / np.linalg.norm(normal)
    u = np.cross(normal, [1.0, 0.0, 0.0] if abs(normal[0]) < 0.9 else [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(normal, u)
    a, b = rng.uniform(-spread, spread, size=(2, n))
    return a[:, None] * u + b[:, None] * v, normal


def test_covariance_of_points_on_a_plane():
    rng = np.random.default_rng(8)
    for _ in range(5):
        pts, nrm = plane_cloud(rng, 400, rng.normal(size=3))
        pts32 = pts.astype(np.float32)
        nbr = pp.knn(soa(pts32), 10)
        c6 = pp.covariances(soa(pts32), nbr, scale=0.01, eps=1e-3)
        want = 0.01 * (np.eye(3) - 0.999 * np.outer(nrm, nrm))
        w6 = np.array([want[0, 0], want[0, 1], want[0, 2], want[1, 1], want[1, 2], want[2, 2]])
        # FP32 input points lie on the plane to ~6e-8 m: the normal is good to ~1e-6
        np.testing.assert_allclose(c6, np.repeat(w6[:, None], c6.shape[1], axis=1), atol=1e-7)


def test_covariance_isotropic_and_rotation():
    rng = np.random.default_rng(9)
    pts = (rng.normal(size=(300, 3)) * np.array([3.0, 2.0, 0.3])).astype(np.float32)
    nbr = pp.knn(soa(pts), 10)
    iso = pp.covariances(soa(pts), nbr, scale=0.02, eps=1.0)
    np.testing.assert_array_equal(iso, np.repeat(np.array([[0.02], [0], [0], [0.02], [0],
                                                           [0.02]], np.float32), 300, axis=1))
    R = Rotation.from_rotvec([0.3, -0.5, 0.8]).as_matrix()
    rp = (pts.astype(np.float64) @ R.T).astype(np.float32)
    _, lam, _, _ = pp.normals(soa(pts), nbr)
    ok = (lam[:, 1] - lam[:, 0]) > 1e-2 * lam[:, 2]  # well-separated smallest eigenvalue
    a = pp.covariances(soa(pts), nbr)
    b = pp.covariances(soa(rp), nbr)  # same neighbour lists: distances are rotation invariant
    for i in np.flatnonzero(ok):
        A = np.array([[a[0, i], a[1, i], a[2, i]], [a[1, i], a[3, i], a[4, i]],
                      [a[2, i], a[4, i], a[5, i]]], np.float64)
        B = np.array([[b[0, i], b[1, i], b[2, i]], [b[1, i], b[3, i], b[4, i]],
                      [b[2, i], b[4, i], b[5, i]]], np.float64)
        np.testing.assert_allclose(R @ A @ R.T, B, atol=2e-5)
    assert ok.sum() > 200


def test_raw_covariance_is_numpy_cov():
    rng = np.random.default_rng(10)
    pts = rng.normal(size=(200, 3)).astype(np.float32)
    nbr = pp.knn(soa(pts), 8)
    c6 = pp.covariances(soa(pts), nbr, scale=0.0)
    for i in (0, 57, 199):
        C = np.cov(pts[nbr[:, i]].astype(np.float64).T, bias=True)
        np.testing.assert_allclose(c6[:, i], [C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2],
                                              C[2, 2]], rtol=1e-6, atol=1e-7)
    # fewer listed neighbours (-1 entries) use the listed ones only
    nb = nbr.copy()
    nb[5:, 0] = -1
    C = np.cov(pts[nbr[:5, 0]].astype(np.float64).T, bias=True)
    np.testing.assert_allclose(pp.covariances(soa(pts), nb, scale=0.0)[:, 0],
                               [C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2]],
                               rtol=1e-6, atol=1e-7)
