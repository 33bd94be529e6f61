"""Oracle of the IMU preintegration factor of Sec. III-B (Eqs. (4)-(9)), after the on-manifold
preintegration the section cites (Forster et al.).

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy in FP64, one factor at a time,
samples in order.

Conventions (the same as the matching-cost factor): a state is a world-from-body pose
T = [R | t] (row-major 3x4), a world-frame velocity v and the IMU biases b = [b_a, b_w] (the
state of Eq. (1)); the tangent of a pose is xi = [omega; rho] with T <- T Exp(xi) (so
R <- R Exp(omega), t <- t + R rho to first order); velocities and biases move additively.

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
  unknowns [xi_i (6), v_i (3), xi_j (6), v_j (3)] (e(d) ~= e + 2 b^T d + d^T H d), the biases
  held at the preintegration's.
* Bias states (``linearize_bias``). The preintegration also carries the first-order
  derivatives of dR, dv, dp with respect to the biases it was computed with, b0, propagated
  sample by sample from the same recursions (perturbing b_w by d moves dR_{k+1} = dR_k E_k,
  E_k = Exp((w_k - b_w) dt_k), by dR_{k+1} Exp((E_k^T J_k - J_r((w_k - b_w) dt_k) dt_k) d);
  the velocity and position sums pick up -dR_k dt_k (b_a) and -dR_k [a_k - b_a]x J_k dt_k (b_w),
  and their half-dt^2 counterparts). With the bias of state i, db = b_i - b0, the preintegrated
  values are corrected to first order,
      dR(b_i) = dR Exp(J_R,w db_w),  dv(b_i) = dv + J_v db,  dp(b_i) = dp + J_p db,
  the residual above uses them, and a bias random-walk term r_b = b_j - b_i with covariance
  diag(sigma_ba^2, sigma_bw^2) dt joins it: 15 residuals over the 30 unknowns
  [xi_i, v_i, b_i, xi_j, v_j, b_j] (6, 3, 6, 6, 3, 6).
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
    # derivatives of (dR, dv, dp) with respect to (b_a, b_w) at the given biases
    JRw = np.zeros((3, 3))
    Jva, Jvw, Jpa, Jpw = (np.zeros((3, 3)) for _ in range(4))
    for w, a, dt in zip(imu[:, :3], imu[:, 3:6], imu[:, 6]):
        wt, at = w - bw, a - ba
        E = so3_exp(wt * dt)
        # the derivatives first: they use the values before this sample
        Jpa = Jpa + Jva * dt - 0.5 * dR * dt * dt
        Jpw = Jpw + Jvw * dt - 0.5 * dR @ hat(at) @ JRw * dt * dt
        Jva = Jva - dR * dt
        Jvw = Jvw - dR @ hat(at) @ JRw * dt
        JRw = E.T @ JRw - right_jacobian(wt * dt) * dt
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
    J = np.zeros((9, 6))   # rows (dR, dv, dp), columns (b_a, b_w)
    J[0:3, 3:6] = JRw
    J[3:6, 0:3], J[3:6, 3:6] = Jva, Jvw
    J[6:9, 0:3], J[6:9, 3:6] = Jpa, Jpw
    return {"dR": dR, "dv": dv, "dp": dp, "dt": T, "cov": S, "J_bias": J,
            "bias": np.asarray(bias, float).copy()}


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


def corrected(pre, b_i):
    """(dR, dv, dp) corrected to first order for the bias b_i (the preintegration's own bias
    gives them back unchanged)."""
    db = np.asarray(b_i, float) - pre["bias"]
    J = pre["J_bias"]
    dR = pre["dR"] @ so3_exp(J[0:3] @ db)
    return dR, pre["dv"] + J[3:6] @ db, pre["dp"] + J[6:9] @ db


def residual_bias(pre, Ti, vi, bi, Tj, vj, bj, g):
    """15 residuals: rotation, velocity, position with the bias-corrected preintegration, then
    the bias random walk b_j - b_i."""
    Ti = np.asarray(Ti, float).reshape(3, 4)
    Tj = np.asarray(Tj, float).reshape(3, 4)
    Ri, ti, Rj, tj = Ti[:, :3], Ti[:, 3], Tj[:, :3], Tj[:, 3]
    dt = pre["dt"]
    g = np.asarray(g, float)
    dR, dv, dp = corrected(pre, bi)
    rR = so3_log(dR.T @ Ri.T @ Rj)
    rv = Ri.T @ (vj - vi - g * dt) - dv
    rp = Ri.T @ (tj - ti - vi * dt - 0.5 * g * dt * dt) - dp
    return np.concatenate([rR, rv, rp, np.asarray(bj, float) - np.asarray(bi, float)])


def jacobian_bias(pre, Ti, vi, bi, Tj, vj, bj, g):
    """15 x 30 Jacobian over [xi_i, v_i, b_i, xi_j, v_j, b_j]."""
    Ti = np.asarray(Ti, float).reshape(3, 4)
    Tj = np.asarray(Tj, float).reshape(3, 4)
    Ri, ti, Rj, tj = Ti[:, :3], Ti[:, 3], Tj[:, :3], Tj[:, 3]
    dt = pre["dt"]
    g = np.asarray(g, float)
    db = np.asarray(bi, float) - pre["bias"]
    Jb = pre["J_bias"]
    dR, _, _ = corrected(pre, bi)
    rR = so3_log(dR.T @ Ri.T @ Rj)
    Jinv = right_jacobian_inv(rR)
    J = np.zeros((15, 30))
    # rotation: pose i, pose j, and the gyro bias through the correction Exp(J_R,w db_w)
    J[0:3, 0:3] = -Jinv @ Rj.T @ Ri
    J[0:3, 15:18] = Jinv
    phi = Jb[0:3, 3:6] @ db[3:6]
    J[0:3, 12:15] = -Jinv @ so3_exp(rR).T @ right_jacobian(phi) @ Jb[0:3, 3:6]
    # velocity
    J[3:6, 0:3] = hat(Ri.T @ (vj - vi - g * dt))
    J[3:6, 6:9] = -Ri.T
    J[3:6, 9:15] = -Jb[3:6]
    J[3:6, 21:24] = Ri.T
    # position
    J[6:9, 0:3] = hat(Ri.T @ (tj - ti - vi * dt - 0.5 * g * dt * dt))
    J[6:9, 3:6] = -np.eye(3)
    J[6:9, 6:9] = -Ri.T * dt
    J[6:9, 9:15] = -Jb[6:9]
    J[6:9, 18:21] = Ri.T @ Rj
    # bias random walk
    J[9:15, 9:15] = -np.eye(6)
    J[9:15, 24:30] = np.eye(6)
    return J


def bias_walk_cov(sigma_ba, sigma_bw, dt):
    """Covariance of b_j - b_i for white-noise bias rates of densities sigma_ba, sigma_bw."""
    return np.diag([sigma_ba ** 2 * dt] * 3 + [sigma_bw ** 2 * dt] * 3)


def linearize_bias(pre, Ti, vi, bi, Tj, vj, bj, g, sigma_ba, sigma_bw):
    """Gauss-Newton blocks of the 15-residual factor over the 30 unknowns: weight
    blockdiag(S^-1, (bias walk covariance)^-1)."""
    r = residual_bias(pre, Ti, vi, bi, Tj, vj, bj, g)
    J = jacobian_bias(pre, Ti, vi, bi, Tj, vj, bj, g)
    W = np.zeros((15, 15))
    W[0:9, 0:9] = np.linalg.inv(pre["cov"])
    W[9:15, 9:15] = np.linalg.inv(bias_walk_cov(sigma_ba, sigma_bw, pre["dt"]))
    return {"H": J.T @ W @ J, "b": J.T @ W @ r, "e": float(r @ W @ r), "r": r}
