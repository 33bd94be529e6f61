"""Oracle of the IMU preintegration factor of Sec. III-B (Eqs. (4)-(9)), after the on-manifold
preintegration the section cites (Forster et al.).

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy in FP64, one factor at a time,
samples in order.

Conventions (the same as the matching-cost factor): a state is a world-from-body pose
T = [R | t] (row-major 3x4) and a world-frame velocity v; the tangent of a pose is
xi = [omega; rho] with T <- T Exp(xi) (so R <- R Exp(omega), t <- t + R rho to first order) and
a velocity moves additively. The biases (b_a, b_w) of a factor are given and held fixed.

* Preintegration over samples k = 0..m-1 (gyro w_k, accelerometer a_k, interval dt_k), Eqs.
  (4)-(6) taken from the body frame at time i (R_i = I, v_i = 0, t_i = 0, no gravity):
      dR_{k+1} = dR_k Exp((w_k - b_w) dt_k)
      dv_{k+1} = dv_k + dR_k (a_k - b_a) dt_k
      dp_{k+1} = dp_k + dv_k dt_k + 1/2 dR_k (a_k - b_a) dt_k^2
  and the covariance of the preintegration noise (dphi, dv, dp) propagated with the white
  gyro / accelerometer noise of densities sigma_g, sigma_a (discrete variance sigma^2 / dt_k):
      S_{k+1} = A_k S_k A_k^T + B_k diag(sigma_g^2/dt_k I, sigma_a^2/dt_k I) B_k^T.
* Residual (Eqs. (7)-(9) read as constraints on the states i, j; the "v" of Eq. (9) is v_i):
      r_R = Log(dR^T R_i^T R_j)
      r_v = R_i^T (v_j - v_i - g dt) - dv
      r_p = R_i^T (t_j - t_i - v_i dt - 1/2 g dt^2) - dp
  cost e = r^T S^-1 r, and the Gauss-Newton blocks H = J^T S^-1 J, b = J^T S^-1 r over the 18
  unknowns [xi_i (6), v_i (3), xi_j (6), v_j (3)] (e(d) ~= e + 2 b^T d + d^T H d).
"""
from __future__ import annotations

import numpy as np


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def so3_exp(w):
    """Rodrigues' formula (second-order series near zero)."""
    w = np.asarray(w, float)
    th = np.linalg.norm(w)
    K = hat(w)
    if th < 1e-8:
        return np.eye(3) + K + K @ K / 2.0
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * K @ K


def so3_log(R):
    """Rotation vector of R (angle in [0, pi))."""
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return v / 2.0
    return th / (2.0 * np.sin(th)) * v


def right_jacobian(w):
    """J_r(w): Exp(w + d) ~= Exp(w) Exp(J_r(w) d)."""
    th = np.linalg.norm(w)
    K = hat(w)
    if th < 1e-8:
        return np.eye(3) - K / 2.0 + K @ K / 6.0
    return (np.eye(3) - (1.0 - np.cos(th)) / th ** 2 * K
            + (th - np.sin(th)) / th ** 3 * K @ K)


def right_jacobian_inv(w):
    th = np.linalg.norm(w)
    K = hat(w)
    if th < 1e-8:
        return np.eye(3) + K / 2.0 + K @ K / 12.0
    return (np.eye(3) + K / 2.0
            + (1.0 / th ** 2 - (1.0 + np.cos(th)) / (2.0 * th * np.sin(th))) * K @ K)


def preintegrate(imu, bias, sigma_g, sigma_a):
    """imu: (m, 7) rows [w (3), a (3), dt]; bias: [b_a (3), b_w (3)].
    Returns dR (3, 3), dv, dp, dt_total and the 9x9 covariance of (dphi, dv, dp)."""
    imu = np.asarray(imu, float).reshape(-1, 7)
    ba, bw = np.asarray(bias, float)[:3], np.asarray(bias, float)[3:]
    dR, dv, dp, T = np.eye(3), np.zeros(3), np.zeros(3), 0.0
    S = np.zeros((9, 9))
    for w, a, dt in zip(imu[:, :3], imu[:, 3:6], imu[:, 6]):
        wt, at = w - bw, a - ba
        E = so3_exp(wt * dt)
        A = np.eye(9)
        A[0:3, 0:3] = E.T
        A[3:6, 0:3] = -dR @ hat(at) * dt
        A[6:9, 0:3] = -0.5 * dR @ hat(at) * dt * dt
        A[6:9, 3:6] = np.eye(3) * dt
        B = np.zeros((9, 6))
        B[0:3, 0:3] = right_jacobian(wt * dt) * dt
        B[3:6, 3:6] = dR * dt
        B[6:9, 3:6] = 0.5 * dR * dt * dt
        Q = np.diag([sigma_g ** 2 / dt] * 3 + [sigma_a ** 2 / dt] * 3)
        S = A @ S @ A.T + B @ Q @ B.T
        dp = dp + dv * dt + 0.5 * dR @ at * dt * dt
        dv = dv + dR @ at * dt
        dR = dR @ E
        T += dt
    return {"dR": dR, "dv": dv, "dp": dp, "dt": T, "cov": S}


def residual(pre, Ti, vi, Tj, vj, g):
    Ti = np.asarray(Ti, float).reshape(3, 4)
    Tj = np.asarray(Tj, float).reshape(3, 4)
    Ri, ti, Rj, tj = Ti[:, :3], Ti[:, 3], Tj[:, :3], Tj[:, 3]
    dt = pre["dt"]
    g = np.asarray(g, float)
    rR = so3_log(pre["dR"].T @ Ri.T @ Rj)
    rv = Ri.T @ (vj - vi - g * dt) - pre["dv"]
    rp = Ri.T @ (tj - ti - vi * dt - 0.5 * g * dt * dt) - pre["dp"]
    return np.concatenate([rR, rv, rp])


def jacobian(pre, Ti, vi, Tj, vj, g):
    """9 x 18 Jacobian of the residual over [xi_i, v_i, xi_j, v_j]."""
    Ti = np.asarray(Ti, float).reshape(3, 4)
    Tj = np.asarray(Tj, float).reshape(3, 4)
    Ri, ti, Rj, tj = Ti[:, :3], Ti[:, 3], Tj[:, :3], Tj[:, 3]
    dt = pre["dt"]
    g = np.asarray(g, float)
    rR = so3_log(pre["dR"].T @ Ri.T @ Rj)
    Jinv = right_jacobian_inv(rR)
    J = np.zeros((9, 18))
    J[0:3, 0:3] = -Jinv @ Rj.T @ Ri
    J[0:3, 9:12] = Jinv
    J[3:6, 0:3] = hat(Ri.T @ (vj - vi - g * dt))
    J[3:6, 6:9] = -Ri.T
    J[3:6, 15:18] = Ri.T
    J[6:9, 0:3] = hat(Ri.T @ (tj - ti - vi * dt - 0.5 * g * dt * dt))
    J[6:9, 3:6] = -np.eye(3)
    J[6:9, 6:9] = -Ri.T * dt
    J[6:9, 12:15] = Ri.T @ Rj
    return J


def linearize(pre, Ti, vi, Tj, vj, g):
    r = residual(pre, Ti, vi, Tj, vj, g)
    J = jacobian(pre, Ti, vi, Tj, vj, g)
    W = np.linalg.inv(pre["cov"])
    return {"H": J.T @ W @ J, "b": J.T @ W @ r, "e": float(r @ W @ r), "r": r}
