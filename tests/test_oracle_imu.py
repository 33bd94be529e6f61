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
  the gradient of the cost (W frozen) equal to 2 b.
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
