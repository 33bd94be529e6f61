"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a hand derivation
(tests/golden), a closed form, an invariant, a brute-force search, a finite difference, or a
second implementation (oracle/ref.py) that shares no code with oracle.cpp.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import ref
from tests import se3, tiny
from tests.metrics import factor_errors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
I12 = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float64)


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def golden_inputs(g):
    return (np.array(g["target_xyz"]), np.array(g["target_cov"]), g["res"],
            np.array(g["source_xyz"]), np.array(g["source_cov"]),
            np.array(g["T_target"], float), np.array(g["T_source"], float))


# ---------------------------------------------------------------- hand-derived worked cases

@pytest.mark.parametrize("name", ["single_point_identity.json", "single_point_rotated.json"])
def test_hand_case_unary(name):
    g = load(name)
    txyz, tcov, res, sxyz, scov, Tt, Ts = golden_inputs(g)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary=False)
    ex = g["expected_unary"]
    assert r["inliers"] == ex["inliers"]
    assert list(r["corr"]) == ex["corr"]
    np.testing.assert_allclose(r["e"], ex["e"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["b"], ex["b"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["H"], np.array(ex["H"]), rtol=0, atol=1e-15)


def test_hand_case_binary_identity_blocks():
    g = load("single_point_identity.json")
    txyz, tcov, res, sxyz, scov, Tt, Ts = golden_inputs(g)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary=True)
    H6 = np.array(g["expected_unary"]["H"])
    b6 = np.array(g["expected_unary"]["b"])
    np.testing.assert_allclose(r["H"], np.block([[H6, -H6], [-H6, H6]]), atol=1e-15)
    np.testing.assert_allclose(r["b"], np.concatenate([b6, -b6]), atol=1e-15)


def test_hand_case_binary_rotated():
    g = load("single_point_rotated.json")
    txyz, tcov, res, sxyz, scov, Tt, Ts = golden_inputs(g)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary=True)
    ex = g["expected_binary_partial"]
    np.testing.assert_allclose(r["b"], ex["b"], atol=1e-15)
    np.testing.assert_allclose(r["H"][9:12, 9:12], ex["H_rho_t_rho_t"], atol=1e-15)
    np.testing.assert_allclose(r["H"][3:6, 9:12], ex["H_rho_s_rho_t"], atol=1e-15)
    np.testing.assert_allclose(r["H"][:6, :6], g["expected_unary"]["H"], atol=1e-15)


# ---------------------------------------------------------------- voxel keys

@pytest.mark.parametrize("v,res,k", [
    (1.0, 0.5, 2), (0.999999999, 0.5, 1), (-1e-30, 1.0, -1), (-0.0, 1.0, 0), (0.0, 1.0, 0),
    (-0.5, 0.5, -1), (-0.25, 0.5, -1), (2.75, 0.25, 11), (-2.75, 0.25, -11),
    (0.3, 0.1, 2),  # 0.3 / 0.1 = 2.9999999999999996 in FP64: the division decides, not 3
])
def test_voxel_coord_faces(v, res, k):
    assert oracle.voxel_coord(v, res) == k


def test_voxel_coord_range_and_nonfinite():
    lim = 2 ** 20
    assert oracle.voxel_coord((lim - 1) * 1.0 + 0.5, 1.0) == lim - 1
    assert oracle.voxel_coord(-(lim - 1) * 1.0, 1.0) == -(lim - 1)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.voxel_coord(lim * 1.0, 1.0)
    assert ei.value.status == oracle.E_KEY_RANGE
    with pytest.raises(oracle.OracleError) as ei:
        oracle.voxel_coord(-lim * 1.0, 1.0)
    assert ei.value.status == oracle.E_KEY_RANGE
    with pytest.raises(oracle.OracleError) as ei:
        oracle.voxel_coord(float("nan"), 1.0)
    assert ei.value.status == oracle.E_NONFINITE
    with pytest.raises(oracle.OracleError) as ei:
        oracle.voxel_coord(1.0, 0.0)
    assert ei.value.status == oracle.E_INVALID_ARG


def test_pack_roundtrip_and_order():
    rng = np.random.default_rng(1)
    ks = rng.integers(-(2 ** 20) + 1, 2 ** 20, size=(400, 3))
    packed = [oracle.pack_key(*map(int, k)) for k in ks]
    for k, p in zip(ks, packed):
        assert p >= 0
        assert oracle.unpack_key(p) == tuple(int(x) for x in k)
    lex = sorted(range(len(ks)), key=lambda i: tuple(ks[i]))
    byp = sorted(range(len(ks)), key=lambda i: packed[i])
    assert lex == byp


# ---------------------------------------------------------------- voxel statistics

def test_voxel_stats_closed_form():
    # one voxel with one point, one voxel with two points (res 1)
    xyz = np.array([[0.2, 3.1, 3.7], [0.3, 0.4, 0.6], [0.9, -0.5, -0.1]], dtype=np.float32)
    cov = np.zeros((6, 3), dtype=np.float32)
    cov[0] = [0.1, 0.2, 0.4]
    cov[3] = [0.3, 0.5, 0.7]
    cov[5] = [0.2, 0.1, 0.3]
    cov[1] = [0.01, 0.02, -0.02]
    m = oracle.VoxelMap(xyz, cov, 1.0)
    ex = m.export()
    assert len(m) == 2
    assert list(ex["count"]) == [1, 2]
    assert ex["keys"][0] == oracle.pack_key(0, 0, 0)
    assert ex["keys"][1] == oracle.pack_key(3, 0, -1)
    x64 = xyz.astype(np.float64)
    c64 = cov.astype(np.float64)
    np.testing.assert_array_equal(ex["mean"][0], x64[:, 0])
    np.testing.assert_array_equal(ex["cov"][0], c64[:, 0])
    np.testing.assert_array_equal(ex["mean"][1], (x64[:, 1] + x64[:, 2]) / 2)
    np.testing.assert_array_equal(ex["cov"][1], (c64[:, 1] + c64[:, 2]) / 2)


def brute_voxelize(xyz, cov, res):
    """Group by integer coordinates with a plain dict scan; ids by sorted key tuple."""
    groups = {}
    for j in range(xyz.shape[1]):
        k = tuple(int(np.floor(float(xyz[a, j]) / res)) for a in range(3))
        groups.setdefault(k, []).append(j)
    out = []
    for k in sorted(groups):
        js = groups[k]
        out.append((k, xyz[:, js].astype(np.float64).mean(axis=1),
                    cov[:, js].astype(np.float64).mean(axis=1), len(js)))
    return out


@pytest.mark.parametrize("seed,res", [(0, 1.0), (1, 0.5), (2, 0.25), (3, 0.3)])
def test_voxelize_brute_force(seed, res):
    rng = np.random.default_rng(seed)
    xyz, cov = tiny.cloud(rng, 300, extent=1.5)
    # put some points exactly on voxel faces
    xyz[0, :40] = (np.round(xyz[0, :40] / res) * res).astype(np.float32)
    m = oracle.VoxelMap(xyz, cov, res)
    ex = m.export()
    bf = brute_voxelize(xyz, cov, res)
    assert len(m) == len(bf)
    for v, (k, mean, c, n) in enumerate(bf):
        assert oracle.unpack_key(int(ex["keys"][v])) == k
        assert ex["count"][v] == n
        np.testing.assert_allclose(ex["mean"][v], mean, rtol=0, atol=1e-14)
        np.testing.assert_allclose(ex["cov"][v], c, rtol=0, atol=1e-15)


def test_voxel_ids_permutation_invariant():
    rng = np.random.default_rng(5)
    xyz, cov = tiny.cloud(rng, 500, extent=2.0)
    perm = rng.permutation(500)
    a = oracle.VoxelMap(xyz, cov, 0.5).export()
    b = oracle.VoxelMap(xyz[:, perm], cov[:, perm], 0.5).export()
    np.testing.assert_array_equal(a["keys"], b["keys"])
    np.testing.assert_array_equal(a["count"], b["count"])
    np.testing.assert_allclose(a["mean"], b["mean"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(a["cov"], b["cov"], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- brute-force twin

def tiny_case(seed, n_t=120, n_s=60, res=0.5, binary=False, pose_scale=(0.2, 0.3)):
    rng = np.random.default_rng(seed)
    txyz, tcov = tiny.cloud(rng, n_t, extent=1.2)
    sxyz = tiny.source_near(rng, txyz, n_s, noise=0.05)
    scov = tiny.plane_cov(rng, n_s).astype(np.float32)
    Tt = se3.random_pose(rng, *pose_scale)
    G = se3.random_pose(rng, 0.05, 0.05)
    # express the source in its own frame: T_s = T_t G, points p_s = (T_t G)^-1 (T_t p)
    Ts = Tt @ G
    Ginv = se3.inv(G)
    sxyz = (Ginv[:3, :3] @ sxyz.astype(np.float64) + Ginv[:3, 3:4]).astype(np.float32)
    return txyz, tcov, res, sxyz, scov, Tt, Ts


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("binary", [False, True])
def test_linearize_matches_numpy_brute_force(seed, binary):
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(seed, binary=binary)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    b = ref.linearize(txyz, tcov, res, sxyz, scov, Tt, Ts, binary)
    assert r["inliers"] == b["inliers"] and r["inliers"] > 10
    err = factor_errors(r["H"], r["b"], r["e"], b["H"], b["b"], b["e"])
    assert max(err["H"], err["b"], err["e"]) < 1e-12, err


# ---------------------------------------------------------------- derivatives

def fd_pose_gradient(fun, Tt, Ts, binary, h=1e-6):
    """Central differences of fun(Tt, Ts) wrt right perturbations [xi_s | xi_t]."""
    dim = 12 if binary else 6
    g = np.zeros(dim)
    for i in range(dim):
        xi = np.zeros(6)
        xi[i % 6] = h
        if i < 6:
            ep, em = fun(Tt, se3.retract(Ts, xi)), fun(Tt, se3.retract(Ts, -xi))
        else:
            ep, em = fun(se3.retract(Tt, xi), Ts), fun(se3.retract(Tt, -xi), Ts)
        g[i] = (ep - em) / (2 * h)
    return g


@pytest.mark.parametrize("binary", [False, True])
def test_fd_frozen_omega_equals_2b(binary):
    """With correspondences and Omega frozen, e(xi) is the Gauss-Newton quadratic's parent:
    its gradient at xi = 0 is 2 b."""
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(11, n_t=200, n_s=120)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    om = oracle.point_omega(m, sxyz, scov, Tt, Ts, r["corr"])
    fun = lambda A, B: oracle.cost_fixed(m, sxyz, scov, A, B, r["corr"], om)  # noqa: E731
    g = fd_pose_gradient(fun, Tt, Ts, binary)
    den = np.sqrt(np.diag(r["H"]) * r["e"])
    assert np.max(np.abs(g - 2 * r["b"]) / den) < 1e-6


@pytest.mark.parametrize("binary", [False, True])
def test_fd_hessian_at_zero_residual_equals_2H(binary):
    """Where every residual is zero the curvature term of e vanishes, so the FD Hessian of the
    cost (Omega and correspondences frozen) is exactly 2 H = 2 sum J^T Omega J."""
    rng = np.random.default_rng(12)
    cells = np.unique(rng.integers(-3, 3, size=(60, 3)), axis=0).T
    txyz = (cells + rng.uniform(0.2, 0.8, size=cells.shape)).astype(np.float32)
    tcov = tiny.plane_cov(rng, txyz.shape[1]).astype(np.float32)
    m = oracle.VoxelMap(txyz, tcov, 1.0)
    means = m.export()["mean"].T
    Tt = se3.random_pose(rng, 0.5, 2.0)
    Ts = Tt @ se3.random_pose(rng, 0.05, 0.05)
    Tst = se3.inv(se3.inv(Tt) @ Ts)
    sxyz = Tst[:3, :3] @ means + Tst[:3, 3:4]          # FP64 source points on the means
    scov = tiny.plane_cov(rng, sxyz.shape[1])
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    assert r["inliers"] == sxyz.shape[1] and r["e"] < 1e-20
    om = oracle.point_omega(m, sxyz, scov, Tt, Ts, r["corr"])
    dim = 12 if binary else 6
    h = 1e-4
    Hfd = np.zeros((dim, dim))
    for i in range(dim):
        for j in range(dim):
            vals = []
            for si, sj in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                xs = np.zeros(6)
                xt = np.zeros(6)
                (xs if i < 6 else xt)[i % 6] += si * h
                (xs if j < 6 else xt)[j % 6] += sj * h
                vals.append(oracle.cost_fixed(m, sxyz, scov, se3.retract(Tt, xt),
                                              se3.retract(Ts, xs), r["corr"], om))
            Hfd[i, j] = (vals[0] - vals[1] - vals[2] + vals[3]) / (4 * h * h)
    diag = np.sqrt(np.outer(np.diag(r["H"]), np.diag(r["H"])))
    assert np.max(np.abs(Hfd - 2 * r["H"]) / (2 * diag)) < 1e-5


@pytest.mark.parametrize("binary", [False, True])
def test_gradient_matches_fd_with_varying_omega(binary):
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(21, n_t=200, n_s=120)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    gr = oracle.gradient(m, sxyz, scov, Tt, Ts, binary, r["corr"])
    fun = lambda A, B: oracle.cost_fixed(m, sxyz, scov, A, B, r["corr"])  # noqa: E731
    g = fd_pose_gradient(fun, Tt, Ts, binary)
    scale = np.linalg.norm(g)
    assert np.max(np.abs(g - gr["g_xi"])) / scale < 1e-7
    # points: perturb each coordinate of a few points (FP64 copies)
    x64 = sxyz.astype(np.float64)
    h = 1e-6
    for k in list(np.flatnonzero(r["corr"] >= 0)[:8]):
        for a in range(3):
            xp = x64.copy()
            xm = x64.copy()
            xp[a, k] += h
            xm[a, k] -= h
            fd = (oracle.cost_fixed(m, xp, scov, Tt, Ts, r["corr"]) -
                  oracle.cost_fixed(m, xm, scov, Tt, Ts, r["corr"])) / (2 * h)
            assert abs(fd - gr["g_points"][a, k]) <= 1e-6 * max(1.0, abs(fd))
    # moving every source point by delta in its own frame is the translation rho = delta:
    # sum_k de/dmu_k equals de/drho_s
    np.testing.assert_allclose(gr["g_xi"][3:6], gr["g_points"].sum(axis=1), rtol=1e-12,
                               atol=1e-12 * np.abs(gr["g_xi"]).max())


def test_target_gradient_is_adjoint_of_source():
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(22, n_t=200, n_s=120)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, True)
    gr = oracle.gradient(m, sxyz, scov, Tt, Ts, True, r["corr"])
    Tst = se3.inv(se3.inv(Tt) @ Ts)
    np.testing.assert_allclose(gr["g_xi"][6:], -se3.adjoint(Tst).T @ gr["g_xi"][:6],
                               atol=1e-12 * np.abs(gr["g_xi"]).max())


# ---------------------------------------------------------------- structure and invariances

@pytest.mark.parametrize("binary", [False, True])
def test_H_symmetric_psd(binary):
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(31, n_t=300, n_s=200)
    m = oracle.VoxelMap(txyz, tcov, res)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    H = r["H"]
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-13 * np.abs(H).max())
    w = np.linalg.eigvalsh(H)
    assert w.min() > -1e-10 * w.max()


def test_binary_is_adjoint_expansion_of_unary():
    """J_t = -J_s Ad(T_st): the 12x12 factor equals A^T H_6 A with A = [I | -Ad(T_st)]."""
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(32, n_t=300, n_s=200)
    m = oracle.VoxelMap(txyz, tcov, res)
    u = oracle.linearize(m, sxyz, scov, Tt, Ts, False)
    bi = oracle.linearize(m, sxyz, scov, Tt, Ts, True)
    Tst = se3.inv(se3.inv(Tt) @ Ts)
    A = np.hstack([np.eye(6), -se3.adjoint(Tst)])
    err = factor_errors(bi["H"], bi["b"], bi["e"], A.T @ u["H"] @ A, A.T @ u["b"], u["e"])
    assert max(err["H"], err["b"], err["e"]) < 1e-12, err


@pytest.mark.parametrize("binary", [False, True])
def test_common_rigid_motion_invariance(binary):
    txyz, tcov, res, sxyz, scov, Tt, Ts = tiny_case(41, n_t=300, n_s=200)
    m = oracle.VoxelMap(txyz, tcov, res)
    r0 = oracle.linearize(m, sxyz, scov, Tt, Ts, binary)
    G = se3.random_pose(np.random.default_rng(7), 2.0, 50.0)
    r1 = oracle.linearize(m, sxyz, scov, G @ Tt, G @ Ts, binary)
    np.testing.assert_array_equal(r0["inliers"], r1["inliers"])
    err = factor_errors(r1["H"], r1["b"], r1["e"], r0["H"], r0["b"], r0["e"])
    assert max(err["H"], err["b"], err["e"]) < 1e-9, err


def test_integer_voxel_shift():
    """Shifting the target cloud by an integer number of voxels, with the target pose moved
    back by the same amount, shifts every key by that integer and leaves e unchanged."""
    res = 0.5
    txyz, tcov, _, sxyz, scov, Tt, Ts = tiny_case(42, n_t=300, n_s=200, res=res)
    txyz = (np.round(txyz.astype(np.float64) * 1024) / 1024).astype(np.float32)  # 2^-10 grid
    shift = np.array([3, -7, 11])
    m0 = oracle.VoxelMap(txyz, tcov, res)
    txyz1 = (txyz.astype(np.float64) + (shift * res)[:, None]).astype(np.float32)
    # keep the test exact: only shift when FP32 represents the moved points exactly
    assert np.array_equal(txyz1.astype(np.float64) - (shift * res)[:, None],
                          txyz.astype(np.float64))
    m1 = oracle.VoxelMap(txyz1, tcov, res)
    k0 = np.array([oracle.unpack_key(int(k)) for k in m0.export()["keys"]])
    k1 = np.array([oracle.unpack_key(int(k)) for k in m1.export()["keys"]])
    np.testing.assert_array_equal(k1 - k0, np.tile(shift, (len(k0), 1)))
    back = np.eye(4)
    back[:3, 3] = -shift * res
    r0 = oracle.evaluate(m0, sxyz, scov, Tt, Ts)
    r1 = oracle.evaluate(m1, sxyz, scov, Tt @ back, Ts)
    assert r0["inliers"] == r1["inliers"]
    np.testing.assert_array_equal(r0["corr"], r1["corr"])
    np.testing.assert_allclose(r1["e"], r0["e"], rtol=1e-10)


# ---------------------------------------------------------------- special cases

def test_isotropic_reduces_to_point_to_point():
    """C = C' = s^2/2 I gives Omega = I / s^2: the textbook point-to-point Gauss-Newton
    normal equations sum J^T J / s^2, sum J^T d / s^2, sum |d|^2 / s^2."""
    rng = np.random.default_rng(51)
    s2 = 0.0625  # s^2 / 2 = 2^-5 is exact in FP32
    txyz = rng.uniform(-1, 1, size=(3, 150)).astype(np.float32)
    tcov = np.zeros((6, 150), np.float32)
    tcov[[0, 3, 5]] = s2 / 2
    sxyz = tiny.source_near(rng, txyz, 80, 0.05)
    scov = np.zeros((6, 80), np.float32)
    scov[[0, 3, 5]] = s2 / 2
    Tt = np.eye(4)
    Ts = se3.random_pose(rng, 0.05, 0.05)
    m = oracle.VoxelMap(txyz, tcov, 0.5)
    r = oracle.linearize(m, sxyz, scov, Tt, Ts, False)
    ex = m.export()
    R, t = Ts[:3, :3], Ts[:3, 3]
    H = np.zeros((6, 6))
    b = np.zeros(6)
    e = 0.0
    for k in range(80):
        v = r["corr"][k]
        if v < 0:
            continue
        mu = sxyz[:, k].astype(np.float64)
        d = ex["mean"][v] - (R @ mu + t)
        J = np.hstack([R @ se3.hat(mu), -R])
        H += J.T @ J / s2
        b += J.T @ d / s2
        e += d @ d / s2
    err = factor_errors(r["H"], r["b"], r["e"], H, b, e)
    assert max(err["H"], err["b"], err["e"]) < 1e-10, err


def test_zero_residual():
    """Source points placed on the voxel means (one point per voxel): d = 0, so e = 0, b = 0
    and H stays positive semi-definite."""
    rng = np.random.default_rng(61)
    res = 1.0
    cells = rng.choice(np.arange(-4, 4), size=(3, 30))
    txyz = (cells + 0.5).astype(np.float32)
    tcov = tiny.plane_cov(rng, 30).astype(np.float32)
    m = oracle.VoxelMap(txyz, tcov, res)
    means = m.export()["mean"].T        # FP64 source points exactly on the voxel means
    scov = tiny.plane_cov(rng, means.shape[1])
    r = oracle.linearize(m, means, scov, np.eye(4), np.eye(4), True)
    assert r["inliers"] == means.shape[1]
    assert r["e"] == 0.0
    assert np.all(r["b"] == 0.0)
    w = np.linalg.eigvalsh(r["H"])
    assert w.min() > -1e-12 * w.max()
    # a binary factor cannot see a motion common to both poses: 6 null directions
    assert np.sum(w < 1e-12 * w.max()) == 6


def test_zero_inliers_and_empty():
    rng = np.random.default_rng(71)
    txyz, tcov = tiny.cloud(rng, 50, extent=1.0)
    m = oracle.VoxelMap(txyz, tcov, 0.5)
    far = (txyz + 100.0).astype(np.float32)
    r = oracle.linearize(m, far, tcov, np.eye(4), np.eye(4), True)
    assert r["inliers"] == 0 and r["e"] == 0.0
    assert np.all(r["H"] == 0) and np.all(r["b"] == 0)
    assert np.all(r["corr"] == -1)
    empty = np.zeros((3, 0), np.float32)
    r = oracle.linearize(m, empty, np.zeros((6, 0), np.float32), np.eye(4), np.eye(4), False)
    assert r["inliers"] == 0 and r["e"] == 0.0
    m0 = oracle.VoxelMap(empty, np.zeros((6, 0), np.float32), 1.0)
    assert len(m0) == 0
    r = oracle.evaluate(m0, txyz, tcov, np.eye(4), np.eye(4))
    assert r["inliers"] == 0 and r["e"] == 0.0


def test_error_contract():
    rng = np.random.default_rng(81)
    txyz, tcov = tiny.cloud(rng, 20)
    bad = txyz.copy()
    bad[1, 3] = np.nan
    with pytest.raises(oracle.OracleError) as ei:
        oracle.VoxelMap(bad, tcov, 1.0)
    assert ei.value.status == oracle.E_NONFINITE
    far = txyz.copy()
    far[0, 0] = 2.0 ** 21
    with pytest.raises(oracle.OracleError) as ei:
        oracle.VoxelMap(far, tcov, 1.0)
    assert ei.value.status == oracle.E_KEY_RANGE
    with pytest.raises(oracle.OracleError) as ei:
        oracle.VoxelMap(txyz, tcov, -1.0)
    assert ei.value.status == oracle.E_INVALID_ARG
    m = oracle.VoxelMap(txyz, tcov, 1.0)
    T = np.eye(4)
    T[0, 3] = np.inf
    with pytest.raises(oracle.OracleError) as ei:
        oracle.linearize(m, txyz, tcov, np.eye(4), T, False)
    assert ei.value.status == oracle.E_NONFINITE
    # a transformed source point far outside the key range cannot hold a voxel: a plain miss
    T = np.eye(4)
    T[0, 3] = 2.0 ** 22
    r = oracle.linearize(m, txyz, tcov, np.eye(4), T, False)
    assert r["inliers"] == 0


def test_linearize_factors_matches_single_calls():
    rng = np.random.default_rng(91)
    maps, clouds, poses = [], [], []
    for i in range(3):
        xyz, cov = tiny.cloud(rng, 200, extent=1.5)
        maps.append(oracle.VoxelMap(xyz, cov, 0.5))
        clouds.append((xyz, cov))
        poses.append(se3.to12(se3.random_pose(rng, 0.03, 0.05)))
    factors = np.array([[0, 1, 0, 1, 1], [1, 2, 1, 2, 0], [2, 0, 2, 0, 1], [0, 0, 0, 0, 0]],
                       np.int32)
    out = oracle.linearize_factors(maps, clouds, np.array(poses), factors, nthreads=2)
    for f, (mi, ci, ti, si, bi) in enumerate(factors):
        r = oracle.linearize(maps[mi], *clouds[ci], poses[ti], poses[si], bool(bi))
        dim = 12 if bi else 6
        np.testing.assert_array_equal(out["H"][f][:dim, :dim], r["H"])
        np.testing.assert_array_equal(out["b"][f][:dim], r["b"])
        assert out["e"][f] == r["e"] and out["inliers"][f] == r["inliers"]
        assert np.all(out["H"][f][dim:, :] == 0) and np.all(out["H"][f][:, dim:] == 0)


def test_relative_pose_fixed_order():
    """T_t^-1 T_s from the oracle equals the exact product up to FP64 rounding, and the
    fixed-order formula is what it evaluates (bitwise equal to a same-order NumPy loop)."""
    rng = np.random.default_rng(101)
    Tt = se3.random_pose(rng, 3.0, 500.0)
    Ts = se3.random_pose(rng, 3.0, 500.0)
    out = oracle.relative_pose(Tt, Ts).reshape(3, 4)
    np.testing.assert_allclose(out, (se3.inv(Tt) @ Ts)[:3], atol=1e-11)
    Rt, Rs, tt, ts = Tt[:3, :3], Ts[:3, :3], Tt[:3, 3], Ts[:3, 3]
    exp = np.empty((3, 4))
    for r in range(3):
        for c in range(3):
            exp[r, c] = (Rt[0, r] * Rs[0, c] + Rt[1, r] * Rs[1, c]) + Rt[2, r] * Rs[2, c]
        dt = ts - tt
        exp[r, 3] = (Rt[0, r] * dt[0] + Rt[1, r] * dt[1]) + Rt[2, r] * dt[2]
    np.testing.assert_array_equal(out, exp)
