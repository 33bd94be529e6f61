"""IMU preintegration factor on the GPU against the oracle (oracle/imu.py), through the C ABI.

Both sides compute in FP64 with the samples in the same order (the kernels contract multiply-adds
and use their own 3x3 products and Cholesky whitening): preintegrated values agree to 1e-12
relative, covariances to 1e-10 of their largest entry, and the Gauss-Newton blocks to 1e-8 on
the scale-free metric of the matching-cost factor (max |dH_ab| / sqrt(H_aa H_bb), b against
sqrt(H_aa e), e relative). The factor with bias states (first-order bias correction, bias random
walk, 30 unknowns) is held to the same bounds, its bias derivatives to 1e-12."""
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


SBA, SBW = 3.0e-3, 2.0e-4


def test_bias_jacobians_match_oracle(V):
    """The preintegration's bias derivatives against the oracle's, and the preintegrated values
    and covariance unchanged from the plain call."""
    rng = np.random.default_rng(11)
    F = 129
    rows, seg, bias = make_factors(rng, F)
    pre, cov, jac = V.vgicp_imu_preintegrate_bias(dev(rows), dev(seg), dev(bias), SG, SA)
    pre0, cov0 = V.vgicp_imu_preintegrate(dev(rows), dev(seg), dev(bias), SG, SA)
    V.vgicp_sync_status()
    assert torch.equal(pre, pre0) and torch.equal(cov, cov0)
    jac = jac.cpu().numpy()
    worst = 0.0
    for f in range(F):
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], bias[f], SG, SA)["J_bias"]
        worst = max(worst, np.abs(jac[f].reshape(9, 6) - ref).max() / max(1.0, np.abs(ref).max()))
    print(f"bias derivatives vs oracle: {worst:.2e}")
    assert worst <= 1e-12


def test_linearization_with_bias_states_matches_oracle(V):
    """The 30-unknown factor (first-order bias correction, bias random walk) against the oracle on
    a chain of states whose biases differ from the preintegration's; at the integrated states
    with the preintegration's own biases and a constant bias the residual vanishes."""
    rng = np.random.default_rng(12)
    F = 80
    rows, seg, bias = make_factors(rng, F, 200, min_len=2)
    P = F + 1
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t, v = rng.normal(size=3) * 5, rng.normal(size=3)
    b_true = rng.normal(size=6) * 0.02
    poses, vels = [np.hstack([R, t[:, None]])], [v]
    for f in range(F):
        R, t, v = world_integrate(R, t, v, rows[seg[f]:seg[f + 1]], b_true)
        poses.append(np.hstack([R, t[:, None]]))
        vels.append(v)
    poses, vels = np.array(poses), np.array(vels)
    pre_bias = b_true + rng.normal(size=(F, 6)) * 2e-3  # preintegrated with nearby biases
    states = np.stack([np.arange(F), np.arange(1, F + 1)], 1).astype(np.int32)
    pre, cov, jac = V.vgicp_imu_preintegrate_bias(dev(rows), dev(seg), dev(pre_bias), SG, SA)
    # perturbed states and state biases
    pp, vv = poses.copy(), vels.copy()
    for p in range(1, P):
        pp[p, :, :3] = pp[p, :, :3] @ Rotation.from_rotvec(rng.normal(size=3) * 0.01).as_matrix()
        pp[p, :, 3] += rng.normal(size=3) * 0.05
        vv[p] += rng.normal(size=3) * 0.05
    bb = b_true + rng.normal(size=(P, 6)) * 5e-3
    out = V.vgicp_imu_linearize_bias(pre, cov, jac, dev(pre_bias), dev(states),
                                     dev(pp.reshape(P, 12)), dev(vv), dev(bb), G, SBA, SBW)
    V.vgicp_sync_status()
    H, b, e = (out[k].cpu().numpy() for k in ("H", "b", "err"))
    worst = 0.0
    for f in range(F):
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], pre_bias[f], SG, SA)
        lin = oimu.linearize_bias(ref, pp[f], vv[f], bb[f], pp[f + 1], vv[f + 1], bb[f + 1], G,
                                  SBA, SBW)
        d = np.sqrt(np.maximum(np.diag(lin["H"]), 1e-300))
        eH = np.max(np.abs(H[f].reshape(30, 30) - lin["H"]) / np.outer(d, d))
        eb = np.max(np.abs(b[f] - lin["b"]) / (d * np.sqrt(lin["e"])))
        ee = abs(e[f] - lin["e"]) / lin["e"]
        worst = max(worst, eH, eb, ee)
    print(f"30-unknown IMU factor vs oracle: {worst:.2e}")
    assert worst <= 1e-8, worst
    # the integrated states with their constant true bias: only the second order of the bias
    # correction is left (the preintegration biases are 2e-3 away; without the correction the
    # median cost of these factors is ~1, with it below 2e-5)
    same = np.tile(b_true, (P, 1))
    out = V.vgicp_imu_linearize_bias(pre, cov, jac, dev(pre_bias), dev(states),
                                     dev(poses.reshape(P, 12)), dev(vels), dev(same), G, SBA,
                                     SBW)
    V.vgicp_sync_status()
    print(f"cost at the integrated states: {out['err'].max().item():.2e}")
    assert out["err"].max().item() < 1e-3


def test_bias_factor_errors(V):
    rng = np.random.default_rng(13)
    rows, seg, bias = make_factors(rng, 3, 20, min_len=2)
    pre, cov, jac = V.vgicp_imu_preintegrate_bias(dev(rows), dev(seg), dev(bias), SG, SA)
    poses = np.tile(np.eye(3, 4).reshape(1, 12), (3, 1))
    st = np.array([[0, 1], [1, 2], [2, 3]], np.int32)  # state 3 does not exist
    V.vgicp_imu_linearize_bias(pre, cov, jac, dev(bias), dev(st), dev(poses),
                               dev(np.zeros((3, 3))), dev(np.zeros((3, 6))), G, SBA, SBW)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    with pytest.raises(V.VGICPError) as ei:  # a zero random-walk density, refused on the host
        V.vgicp_imu_linearize_bias(pre, cov, jac, dev(bias), dev(st), dev(poses),
                                   dev(np.zeros((3, 3))), dev(np.zeros((3, 6))), G, 0.0, SBW)
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    V.vgicp_sync_status()
