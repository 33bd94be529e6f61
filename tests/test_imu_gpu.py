"""IMU preintegration factor on the GPU against the oracle (oracle/imu.py), through the C ABI.

Both sides compute in FP64 with the samples in the same order (the kernels contract multiply-adds
and use their own 3x3 products and Cholesky whitening): preintegrated values agree to 1e-12
relative, covariances to 1e-10 of their largest entry, and the Gauss-Newton blocks to 1e-8 on
the scale-free metric of the matching-cost factor (max |dH_ab| / sqrt(H_aa H_bb), b against
sqrt(H_aa e), e relative)."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import imu as oimu
from tests.gpu_util import dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

G = np.array([0.0, 0.0, -9.80665])
SG, SA = 1.7e-3, 2.0e-2


@pytest.fixture(scope="module")
def V():
    import paper_2202_00242_amd.vgicp as V
    return V


def make_factors(rng, F, max_len=300, min_len=1):
    lens = rng.integers(min_len, max_len, size=F)
    lens[0] = min_len  # the shortest segment
    seg = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    m = int(seg[-1])
    rows = np.zeros((m, 7))
    rows[:, :3] = rng.normal(size=(m, 3)) * 0.6
    rows[:, 3:6] = rng.normal(size=(m, 3)) * 1.5 + np.array([0.0, 0.0, 9.8])
    rows[:, 6] = rng.uniform(0.002, 0.01, size=m)
    bias = rng.normal(size=(F, 6)) * 0.02
    return rows, seg, bias


def world_integrate(R, t, v, rows, bias):
    ba, bw = bias[:3], bias[3:]
    for w, a, dt in zip(rows[:, :3], rows[:, 3:6], rows[:, 6]):
        acc = R @ (a - ba)
        t = t + v * dt + 0.5 * G * dt * dt + 0.5 * acc * dt * dt
        v = v + G * dt + acc * dt
        R = R @ Rotation.from_rotvec((w - bw) * dt).as_matrix()
    return R, t, v


def test_preintegration_matches_oracle(V):
    rng = np.random.default_rng(1)
    F = 257
    rows, seg, bias = make_factors(rng, F)
    pre, cov = V.vgicp_imu_preintegrate(dev(rows), dev(seg), dev(bias), SG, SA)
    V.vgicp_sync_status()
    pre, cov = pre.cpu().numpy(), cov.cpu().numpy()
    for f in range(F):
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], bias[f], SG, SA)
        np.testing.assert_allclose(pre[f, :9].reshape(3, 3), ref["dR"], atol=1e-12)
        sc = max(1.0, np.abs(ref["dp"]).max(), np.abs(ref["dv"]).max())
        np.testing.assert_allclose(pre[f, 9:12], ref["dv"], atol=1e-12 * sc)
        np.testing.assert_allclose(pre[f, 12:15], ref["dp"], atol=1e-12 * sc)
        assert abs(pre[f, 15] - ref["dt"]) <= 1e-14
        np.testing.assert_allclose(cov[f], ref["cov"], atol=1e-10 * np.abs(ref["cov"]).max())
        np.testing.assert_array_equal(cov[f], cov[f].T)


def test_linearization_matches_oracle(V):
    rng = np.random.default_rng(2)
    F = 96
    # at least two samples: one accelerometer sample moves dv and dp along one direction only,
    # which leaves the covariance singular
    rows, seg, bias = make_factors(rng, F, 200, min_len=2)
    # states: a chain; state f+1 integrated from state f, then perturbed
    P = F + 1
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t, v = rng.normal(size=3) * 5, rng.normal(size=3)
    poses, vels = [np.hstack([R, t[:, None]])], [v]
    for f in range(F):
        R, t, v = world_integrate(R, t, v, rows[seg[f]:seg[f + 1]], bias[f])
        poses.append(np.hstack([R, t[:, None]]))
        vels.append(v)
    poses, vels = np.array(poses), np.array(vels)
    truth = (poses.copy(), vels.copy())
    for p in range(1, P):
        poses[p, :, :3] = poses[p, :, :3] @ Rotation.from_rotvec(rng.normal(size=3) * 0.01).as_matrix()
        poses[p, :, 3] += rng.normal(size=3) * 0.05
        vels[p] += rng.normal(size=3) * 0.05
    states = np.stack([np.arange(F), np.arange(1, F + 1)], 1).astype(np.int32)
    pre, cov = V.vgicp_imu_preintegrate(dev(rows), dev(seg), dev(bias), SG, SA)
    out = V.vgicp_imu_linearize(pre, cov, dev(states), dev(poses.reshape(P, 12)), dev(vels), G)
    V.vgicp_sync_status()
    H, b, e = (out[k].cpu().numpy() for k in ("H", "b", "err"))
    worst = 0.0
    for f in range(F):
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], bias[f], SG, SA)
        lin = oimu.linearize(ref, poses[f], vels[f], poses[f + 1], vels[f + 1], G)
        d = np.sqrt(np.maximum(np.diag(lin["H"]), 1e-300))
        eH = np.max(np.abs(H[f] - lin["H"]) / np.outer(d, d))
        eb = np.max(np.abs(b[f] - lin["b"]) / (d * np.sqrt(lin["e"])))
        ee = abs(e[f] - lin["e"]) / lin["e"]
        worst = max(worst, eH, eb, ee)
    assert worst <= 1e-8, worst
    # at the integrated states the residual vanishes
    out = V.vgicp_imu_linearize(pre, cov, dev(states), dev(truth[0].reshape(P, 12)),
                                dev(truth[1]), G)
    assert out["err"].max().item() < 1e-12


def test_imu_edge_cases(V):
    rng = np.random.default_rng(3)
    rows, seg, bias = make_factors(rng, 4, 20, min_len=2)
    seg2 = np.array([0, 5, 5, seg[3], seg[4]], np.int64)  # factor 1 has no sample
    pre, cov = V.vgicp_imu_preintegrate(dev(rows), dev(seg2), dev(bias), SG, SA)
    V.vgicp_sync_status()
    p = pre.cpu().numpy()
    np.testing.assert_array_equal(p[1], np.r_[np.eye(3).ravel(), np.zeros(7)])
    assert np.all(cov.cpu().numpy()[1] == 0.0)
    empty = torch.empty((0, 7), dtype=torch.float64, device="cuda")
    pre0, _ = V.vgicp_imu_preintegrate(empty, dev(np.zeros(1, np.int64)),
                                       torch.empty((0, 6), dtype=torch.float64, device="cuda"),
                                       SG, SA)
    assert pre0.shape == (0, 16)
    bad = seg.copy()
    bad[2] = bad[1] - 1  # decreasing segment
    V.vgicp_imu_preintegrate(dev(rows), dev(bad), dev(bias), SG, SA)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    r2 = rows.copy()
    r2[3, 6] = 0.0  # a zero interval
    V.vgicp_imu_preintegrate(dev(r2), dev(seg), dev(bias), SG, SA)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_NONFINITE
    pre, cov = V.vgicp_imu_preintegrate(dev(rows), dev(seg), dev(bias), SG, SA)
    poses = np.tile(np.eye(3, 4).reshape(1, 12), (2, 1))
    st = np.array([[0, 1], [0, 2], [1, 0], [1, 1]], np.int32)  # state 2 does not exist
    V.vgicp_imu_linearize(pre, cov, dev(st), dev(poses), dev(np.zeros((2, 3))), G)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    V.vgicp_sync_status()
    # a single sample leaves the covariance singular: reported, not silently whitened
    one = np.array([0, 1], np.int64)
    pre1, cov1 = V.vgicp_imu_preintegrate(dev(rows[:1]), dev(one), dev(bias[:1]), SG, SA)
    V.vgicp_imu_linearize(pre1, cov1, dev(np.array([[0, 1]], np.int32)), dev(poses),
                          dev(np.zeros((2, 3))), G)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_NONFINITE
