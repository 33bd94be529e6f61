"""Pins of the IMU preintegration oracle (oracle/imu.py), on the CPU.

* SO(3) exponential and logarithm against scipy's rotations, the right Jacobian and its inverse
  against finite differences;
* closed forms: a constant turn rate gives dR = Exp(w T) with no velocity or position change; a
  constant acceleration without rotation gives dv = a T, dp = a T^2 / 2; biases subtract;
* the states of a trajectory integrated forward in the world frame with gravity (Eqs. (4)-(6),
  written out separately below) make the residual vanish;
* the propagated covariance equals the sum over samples of J_k Q_k J_k^T with J_k the finite-
  difference Jacobian of the preintegrated measurement with respect to sample k's noise;
* the residual's Jacobian against finite differences of the residual under the retraction, and
  the gradient of the cost (W frozen) equal to 2 b;
* bias states: the bias derivatives of the preintegrated values against re-integrations with
  perturbed biases and against closed forms, the first-order correction (exact at the
  preintegration's own bias, second order away from it), the 15 x 30 Jacobian of the factor
  with bias unknowns and its random-walk rows, and its cost gradient equal to 2 b.
"""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import imu
from oracle.lm import se3_exp

G = np.array([0.0, 0.0, -9.80665])


def test_so3_maps():
    rng = np.random.default_rng(1)
    for scale in (1e-9, 1e-3, 0.5, 2.0):
        w = rng.normal(size=3) * scale
        np.testing.assert_allclose(imu.so3_exp(w), Rotation.from_rotvec(w).as_matrix(),
                                   atol=1e-13)
        np.testing.assert_allclose(imu.so3_log(imu.so3_exp(w)), w, atol=1e-12)
        Jr = imu.right_jacobian(w)
        for a in range(3):
            d = np.zeros(3)
            d[a] = 1e-6
            fd = (imu.so3_log(imu.so3_exp(w).T @ imu.so3_exp(w + d))
                  - imu.so3_log(imu.so3_exp(w).T @ imu.so3_exp(w - d))) / 2e-6
            np.testing.assert_allclose(fd, Jr[:, a], atol=1e-8)
        np.testing.assert_allclose(imu.right_jacobian_inv(w) @ Jr, np.eye(3), atol=1e-10)


def samples(w, a, dt, m):
    return np.array([np.concatenate([w, a, [dt]])] * m)


def test_closed_forms():
    w = np.array([0.1, -0.2, 0.3])
    ba, bw = np.array([0.01, 0.02, -0.03]), np.array([0.001, -0.002, 0.003])
    pre = imu.preintegrate(samples(w + bw, ba, 0.005, 200), np.concatenate([ba, bw]), 1e-3, 1e-2)
    np.testing.assert_allclose(pre["dR"], imu.so3_exp(w * 1.0), atol=1e-12)
    np.testing.assert_allclose(pre["dv"], 0.0, atol=1e-15)
    np.testing.assert_allclose(pre["dp"], 0.0, atol=1e-15)
    assert abs(pre["dt"] - 1.0) < 1e-12
    a = np.array([0.5, -1.0, 2.0])
    pre = imu.preintegrate(samples(bw, a + ba, 0.01, 50), np.concatenate([ba, bw]), 1e-3, 1e-2)
    np.testing.assert_allclose(pre["dR"], np.eye(3), atol=1e-15)
    np.testing.assert_allclose(pre["dv"], a * 0.5, rtol=1e-12)
    np.testing.assert_allclose(pre["dp"], a * 0.125, rtol=1e-12)


def world_integrate(R, t, v, imu_rows, bias):
    """Eqs. (4)-(6) in the world frame with gravity, one sample at a time."""
    ba, bw = bias[:3], bias[3:]
    for row in imu_rows:
        w, a, dt = row[:3], row[3:6], row[6]
        acc = R @ (a - ba)
        t = t + v * dt + 0.5 * G * dt * dt + 0.5 * acc * dt * dt
        v = v + G * dt + acc * dt
        R = R @ Rotation.from_rotvec((w - bw) * dt).as_matrix()
    return R, t, v


def random_imu(rng, m):
    rows = np.zeros((m, 7))
    rows[:, :3] = rng.normal(size=(m, 3)) * 0.5
    rows[:, 3:6] = rng.normal(size=(m, 3)) * 2.0 + np.array([0.0, 0.0, 9.8])
    rows[:, 6] = rng.uniform(0.004, 0.006, size=m)
    return rows


def test_residual_vanishes_on_the_integrated_trajectory():
    rng = np.random.default_rng(2)
    for _ in range(5):
        rows = random_imu(rng, 120)
        bias = rng.normal(size=6) * 0.01
        Ri = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
        ti, vi = rng.normal(size=3) * 10, rng.normal(size=3)
        Rj, tj, vj = world_integrate(Ri, ti, vi, rows, bias)
        pre = imu.preintegrate(rows, bias, 1e-3, 1e-2)
        Ti, Tj = np.hstack([Ri, ti[:, None]]), np.hstack([Rj, tj[:, None]])
        r = imu.residual(pre, Ti, vi, Tj, vj, G)
        assert np.abs(r).max() < 1e-11, r
        # a wrong state is seen
        r2 = imu.residual(pre, Ti, vi, Tj, vj + 0.01, G)
        assert np.abs(r2[3:6]).max() > 1e-3


def measurement(rows, bias):
    pre = imu.preintegrate(rows, bias, 1.0, 1.0)
    return pre["dR"], pre["dv"], pre["dp"]


def test_covariance_is_the_linearized_noise_propagation():
    rng = np.random.default_rng(3)
    rows = random_imu(rng, 25)
    bias = rng.normal(size=6) * 0.01
    sg, sa = 2e-3, 3e-2
    pre = imu.preintegrate(rows, bias, sg, sa)
    dR0, dv0, dp0 = measurement(rows, bias)
    S = np.zeros((9, 9))
    h = 1e-6
    for k in range(len(rows)):
        Jk = np.zeros((9, 6))
        for c in range(6):
            out = []
            for sgn in (1.0, -1.0):
                rr = rows.copy()
                rr[k, c] -= sgn * h  # the true rate / acceleration is the measured one minus noise
                dR, dv, dp = measurement(rr, bias)
                out.append(np.concatenate([imu.so3_log(dR0.T @ dR), dv - dv0, dp - dp0]))
            Jk[:, c] = (out[0] - out[1]) / (2 * h)
        Q = np.diag([sg ** 2 / rows[k, 6]] * 3 + [sa ** 2 / rows[k, 6]] * 3)
        S += Jk @ Q @ Jk.T
    np.testing.assert_allclose(pre["cov"], S, rtol=1e-6, atol=1e-6 * np.abs(S).max())


def retract(T, xi):
    M = np.eye(4)
    M[:3, :] = np.asarray(T).reshape(3, 4)
    return (M @ se3_exp(xi))[:3, :]


def test_jacobian_and_gradient():
    rng = np.random.default_rng(4)
    rows = random_imu(rng, 60)
    bias = rng.normal(size=6) * 0.01
    pre = imu.preintegrate(rows, bias, 1e-3, 1e-2)
    Ri = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    Ti = np.hstack([Ri, rng.normal(size=(3, 1))])
    Tj = np.hstack([Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(size=(3, 1))])
    vi, vj = rng.normal(size=3), rng.normal(size=3)

    def res(d):
        return imu.residual(pre, retract(Ti, d[0:6]), vi + d[6:9], retract(Tj, d[9:15]),
                            vj + d[15:18], G)

    J = imu.jacobian(pre, Ti, vi, Tj, vj, G)
    h = 1e-6
    for c in range(18):
        d = np.zeros(18)
        d[c] = h
        fd = (res(d) - res(-d)) / (2 * h)
        np.testing.assert_allclose(J[:, c], fd, atol=2e-7 * max(1.0, np.abs(fd).max()))
    lin = imu.linearize(pre, Ti, vi, Tj, vj, G)
    W = np.linalg.inv(pre["cov"])
    for c in range(18):
        d = np.zeros(18)
        d[c] = h
        fd = (res(d) @ W @ res(d) - res(-d) @ W @ res(-d)) / (2 * h)
        assert abs(fd - 2 * lin["b"][c]) <= 1e-6 * np.abs(2 * lin["b"]).max(), (c, fd)
    np.testing.assert_allclose(lin["H"], lin["H"].T, atol=1e-9 * np.abs(lin["H"]).max())


# ---------------------------------------------------------------------------- bias states


def test_bias_jacobians_match_finite_differences():
    """The derivatives of (dR, dv, dp) with respect to (b_a, b_w) carried by the preintegration
    against FP64 central differences of whole re-integrations with perturbed biases."""
    rng = np.random.default_rng(5)
    for m in (1, 7, 80):
        rows = random_imu(rng, m)
        b0 = rng.normal(size=6) * 0.02
        pre = imu.preintegrate(rows, b0, 1e-3, 1e-2)
        J = pre["J_bias"]
        assert np.all(J[0:3, 0:3] == 0.0)  # the rotation does not see the accelerometer bias
        h = 1e-6
        fd = np.zeros((9, 6))
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            p = imu.preintegrate(rows, b0 + d, 1e-3, 1e-2)
            q = imu.preintegrate(rows, b0 - d, 1e-3, 1e-2)
            fd[0:3, k] = imu.so3_log(q["dR"].T @ p["dR"]) / (2 * h)
            fd[3:6, k] = (p["dv"] - q["dv"]) / (2 * h)
            fd[6:9, k] = (p["dp"] - q["dp"]) / (2 * h)
        np.testing.assert_allclose(J, fd, atol=1e-7 * max(1.0, np.abs(fd).max()))


def test_bias_jacobian_closed_forms():
    """Constant samples: d(dv)/d(b_a) = -T I and d(dp)/d(b_a) = -T^2/2 I without rotation;
    d(dR)/d(b_w) = -J_r(w T) T for a constant turn rate."""
    a = np.array([0.3, -0.2, 9.7])
    pre = imu.preintegrate(samples(np.zeros(3), a, 0.01, 100), np.zeros(6), 1e-3, 1e-2)
    np.testing.assert_allclose(pre["J_bias"][3:6, 0:3], -1.0 * np.eye(3), atol=1e-12)
    np.testing.assert_allclose(pre["J_bias"][6:9, 0:3], -0.5 * np.eye(3), atol=1e-12)
    w = np.array([0.4, -0.1, 0.2])
    pre = imu.preintegrate(samples(w, np.zeros(3), 0.005, 200), np.zeros(6), 1e-3, 1e-2)
    np.testing.assert_allclose(pre["J_bias"][0:3, 3:6], -imu.right_jacobian(w * 1.0) * 1.0,
                               atol=1e-12)


def test_bias_correction_at_own_bias_and_to_first_order():
    """At the preintegration's own bias the corrected values are the preintegrated ones and the
    first nine residuals are the fixed-bias factor's; a preintegration at a bias 1e-3 off
    corrected to the true bias lands within second order (100x closer than uncorrected)."""
    rng = np.random.default_rng(6)
    rows = random_imu(rng, 100)
    b_true = rng.normal(size=6) * 0.02
    ref = imu.preintegrate(rows, b_true, 1e-3, 1e-2)
    dR, dv, dp = imu.corrected(ref, b_true)
    assert np.array_equal(dv, ref["dv"]) and np.array_equal(dp, ref["dp"])
    np.testing.assert_allclose(dR, ref["dR"], atol=1e-15)
    Ti = np.hstack([Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(size=(3, 1))])
    Tj = np.hstack([Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(size=(3, 1))])
    vi, vj, bj = rng.normal(size=3), rng.normal(size=3), rng.normal(size=6) * 0.02
    r = imu.residual_bias(ref, Ti, vi, b_true, Tj, vj, bj, G)
    np.testing.assert_allclose(r[:9], imu.residual(ref, Ti, vi, Tj, vj, G), atol=1e-14)
    np.testing.assert_allclose(r[9:], bj - b_true, atol=0)
    off = imu.preintegrate(rows, b_true + rng.normal(size=6) * 1e-3, 1e-3, 1e-2)
    cR, cv, cp = imu.corrected(off, b_true)
    err_c = max(np.abs(imu.so3_log(ref["dR"].T @ cR)).max(), np.abs(cv - ref["dv"]).max(),
                np.abs(cp - ref["dp"]).max())
    err_u = max(np.abs(imu.so3_log(ref["dR"].T @ off["dR"])).max(),
                np.abs(off["dv"] - ref["dv"]).max(), np.abs(off["dp"] - ref["dp"]).max())
    assert err_c < 1e-2 * err_u, (err_c, err_u)


def test_bias_residual_jacobian_and_gradient():
    """The 15 x 30 Jacobian over [xi_i, v_i, b_i, xi_j, v_j, b_j] against central differences
    (poses by the retraction, velocities and biases additively) at a bias away from the
    preintegration's, and the gradient of the weighted cost equal to 2 b."""
    rng = np.random.default_rng(7)
    rows = random_imu(rng, 60)
    b0 = rng.normal(size=6) * 0.01
    pre = imu.preintegrate(rows, b0, 1e-3, 1e-2)
    Ti = np.hstack([Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(size=(3, 1))])
    Tj = np.hstack([Rotation.from_rotvec(rng.normal(size=3)).as_matrix(), rng.normal(size=(3, 1))])
    vi, vj = rng.normal(size=3), rng.normal(size=3)
    bi, bj = b0 + rng.normal(size=6) * 0.05, rng.normal(size=6) * 0.01

    def res(d):
        return imu.residual_bias(pre, retract(Ti, d[0:6]), vi + d[6:9], bi + d[9:15],
                                 retract(Tj, d[15:21]), vj + d[21:24], bj + d[24:30], G)

    J = imu.jacobian_bias(pre, Ti, vi, bi, Tj, vj, bj, G)
    h = 1e-6
    for c in range(30):
        d = np.zeros(30)
        d[c] = h
        fd = (res(d) - res(-d)) / (2 * h)
        np.testing.assert_allclose(J[:, c], fd, atol=2e-7 * max(1.0, np.abs(fd).max()))
    sba, sbw = 3e-3, 4e-4
    lin = imu.linearize_bias(pre, Ti, vi, bi, Tj, vj, bj, G, sba, sbw)
    W = np.zeros((15, 15))
    W[:9, :9] = np.linalg.inv(pre["cov"])
    W[9:, 9:] = np.linalg.inv(imu.bias_walk_cov(sba, sbw, pre["dt"]))
    for c in range(30):
        d = np.zeros(30)
        d[c] = h
        fd = (res(d) @ W @ res(d) - res(-d) @ W @ res(-d)) / (2 * h)
        assert abs(fd - 2 * lin["b"][c]) <= 1e-6 * np.abs(2 * lin["b"]).max(), (c, fd)
    # the random walk alone: +-W_b blocks on the two bias states
    Wb = np.linalg.inv(imu.bias_walk_cov(sba, sbw, pre["dt"]))
    Jb = J[9:15]
    np.testing.assert_array_equal(Jb[:, 9:15], -np.eye(6))
    np.testing.assert_array_equal(Jb[:, 24:30], np.eye(6))
    np.testing.assert_allclose((Jb.T @ Wb @ Jb)[24:30, 9:15], -Wb, rtol=1e-15)
