"""Pins of the oracle's Levenberg-Marquardt step (oracle/lm.py), on the CPU.

* the SE(3) exponential against scipy's matrix exponential of the twist;
* the assembly against the quadratic form it must represent: for any step, the sum over factors
  of [d_s; d_t]^T H_f [d_s; d_t] and of b_f^T [d_s; d_t] (block placement, order, unary case);
* the damped solve: the step satisfies the damped normal equations, idle and fixed poses stay;
* the whole step on real VGICP factors: from perturbed poses of an odometry scene (8 keyframes
  and the newest scan), a few LM iterations lower the cost and bring the poses to the truth.
"""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import lm
from tests import se3


def test_se3_exp_matches_matrix_exponential():
    rng = np.random.default_rng(1)
    for scale in (1e-9, 1e-4, 0.3, 2.5):
        for _ in range(20):
            xi = rng.normal(size=6) * scale
            tw = np.zeros((4, 4))
            tw[:3, :3] = lm._hat(xi[:3])
            tw[:3, 3] = xi[3:]
            ref = scipy.linalg.expm(tw)
            np.testing.assert_allclose(lm.se3_exp(xi), ref, atol=1e-12, rtol=1e-12)
            np.testing.assert_allclose(lm.se3_exp(xi)[:3, :3],
                                       Rotation.from_rotvec(xi[:3]).as_matrix(), atol=1e-12)


def test_assembly_is_the_sum_of_factor_quadratic_forms():
    rng = np.random.default_rng(2)
    P = 5
    factors = np.array([[0, 0, 1, 0, 1], [0, 0, 2, 1, 1], [0, 0, 4, 3, 1], [0, 0, 0, 2, 0],
                        [0, 0, 3, 3, 1], [0, 0, 1, 4, 1]], np.int32)
    F = len(factors)
    Hf = np.zeros((F, 12, 12))
    bf = np.zeros((F, 12))
    for f in range(F):
        d = 12 if factors[f, 4] else 6
        M = rng.normal(size=(d, d))
        Hf[f, :d, :d] = M @ M.T
        bf[f, :d] = rng.normal(size=d)
    H, b = lm.assemble(factors, Hf, bf, P)
    for _ in range(5):
        x = rng.normal(size=6 * P)
        q = lin = 0.0
        for f, (_, _, tp, sp, bi) in enumerate(factors):
            v = np.concatenate([x[6 * sp:6 * sp + 6], x[6 * tp:6 * tp + 6]])
            q += v @ Hf[f] @ v
            lin += bf[f] @ v
        assert np.isclose(x @ H @ x, q, rtol=1e-12)
        assert np.isclose(b @ x, lin, rtol=1e-12)
    assert np.allclose(H, H.T)


def test_damped_solve_and_idle_poses():
    rng = np.random.default_rng(3)
    P = 4
    M = rng.normal(size=(18, 18))
    H = np.zeros((24, 24))
    H[:18, :18] = M @ M.T  # pose 3 idle
    b = np.zeros(24)
    b[:18] = rng.normal(size=18)
    for lam, fixed in ((0.0, -1), (1e-3, 0), (10.0, 1)):
        A, g = lm.damp(H, b, lam, fixed)
        x = np.linalg.solve(A, g)
        idle = np.zeros(24, bool)
        idle[18:] = True
        if fixed >= 0:
            idle[6 * fixed:6 * fixed + 6] = True
        assert np.all(x[idle] == 0.0)
        Hd = H + lam * np.diag(np.diag(H))
        act = ~idle
        np.testing.assert_allclose(Hd[np.ix_(act, act)] @ x[act], -b[act], rtol=1e-9,
                                   atol=1e-9 * np.abs(b).max())


def rot_err_deg(Ta, Tb):
    Ra = np.asarray(Ta).reshape(3, 4)[:, :3]
    Rb = np.asarray(Tb).reshape(3, 4)[:, :3]
    c = (np.trace(Ra.T @ Rb) - 1) / 2
    return np.degrees(np.arccos(np.clip(c, -1, 1)))


def trans_err(Ta, Tb):
    return np.linalg.norm(np.asarray(Ta).reshape(3, 4)[:, 3] - np.asarray(Tb).reshape(3, 4)[:, 3])


def odometry_graph(seed=0):
    """Poses [8 keyframes, newest scan]; binary factors scan <-> keyframe and keyframe chain,
    res 0.5 m; truth and a perturbed start (keyframe 0 is the gauge)."""
    u = synth.urban(seed)
    clouds = list(u["targets"]) + [u["source"]]
    maps = [oracle.VoxelMap(x, c, 0.5) for x, c in clouds]
    truth = np.concatenate([u["T_targets"], [u["T_source_truth"]]]).reshape(-1, 12)
    start = truth.copy()
    rng = np.random.default_rng(100 + seed)
    for i in range(1, 8):
        start[i] = se3.to12(se3.to44(truth[i]) @ se3.se3_exp(
            np.concatenate([rng.normal(size=3) * np.radians(0.5), rng.normal(size=3) * 0.05])))
    start[8] = np.asarray(u["T_source"]).reshape(12)
    S = 8
    fac = []
    for k in range(8):
        fac.append([k, S, k, S, 1])  # newest scan onto keyframe k
        fac.append([S, k, S, k, 1])  # keyframe k onto the newest scan
    for k in range(7):
        fac.append([k + 1, k, k + 1, k, 1])
        fac.append([k, k + 1, k, k + 1, 1])
    return {"maps": maps, "clouds": [oracle.Cloud.of(x, c) for x, c in clouds], "raw": clouds,
            "truth": truth, "start": start, "factors": np.array(fac, np.int32)}


def test_lm_iterations_reach_the_truth():
    g = odometry_graph()
    maps, clouds, truth, start, factors = g["maps"], g["clouds"], g["truth"], g["start"], g["factors"]
    poses, lam = start.copy(), 1e-4
    costs = []
    for _ in range(8):
        st = lm.lm_step(maps, clouds, poses, factors, lam, fixed_pose=0)
        costs.append(st["cost"][0])
        if st["cost"][1] < st["cost"][0]:
            poses, lam = st["poses"], lam / 10
        else:
            lam *= 10
    e0 = max(max(rot_err_deg(start[i], truth[i]), 10 * trans_err(start[i], truth[i]))
             for i in range(1, 9))
    e1 = max(max(rot_err_deg(poses[i], truth[i]), 10 * trans_err(poses[i], truth[i]))
             for i in range(1, 9))
    print(f"cost {costs[0]:.1f} -> {costs[-1]:.1f}; worst pose error {e0:.3f} -> {e1:.3f}")
    assert costs[-1] < 0.5 * costs[0]
    assert e1 < 0.25 * e0
    assert np.allclose(poses[0], truth[0])  # the gauge stays
