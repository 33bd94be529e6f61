"""Oracle of one Levenberg-Marquardt step of the pose graph formed by VGICP factors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III-F optimizes the global mapping graph (submap poses linked by matching-cost factors,
Eq. (2)) with Levenberg-Marquardt. One step, written out plainly in FP64 with NumPy:

* every factor's Gauss-Newton blocks come from the C++ oracle (H_f 12x12 and b_f over the
  tangents [source | target], e = H_f, b_f, e_f as in ``linearize_factors``);
* the dense 6P x 6P system H, b is their sum at the factors' pose indices;
* damping (Marquardt): the diagonal entries are scaled by (1 + lambda); a row whose diagonal is
  zero (a pose no factor reaches) and the rows of an optional fixed pose are replaced by the
  identity with a zero right-hand side;
* the step solves (H + lambda diag H) delta = -b (``numpy.linalg.solve``);
* every pose moves by the right perturbation T_i Exp(delta_i), xi = [omega; rho], with the
  SE(3) exponential written out below (Rodrigues' formula and the left Jacobian of SO(3));
* the cost is the sum of the factors' costs, before and after.
"""
from __future__ import annotations

import numpy as np

from . import linearize_factors


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """4x4 Exp of xi = [omega; rho] (rotation first): R = exp([omega]x), t = V rho."""
    w, rho = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = np.linalg.norm(w)
    K = _hat(w)
    if th < 1e-8:
        R = np.eye(3) + K + K @ K / 2.0
        V = np.eye(3) + K / 2.0 + K @ K / 6.0
    else:
        R = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K
        V = (np.eye(3) + (1 - np.cos(th)) / th ** 2 * K
             + (th - np.sin(th)) / th ** 3 * K @ K)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def retract(T12, xi):
    """Row-major [R|t] (12) times Exp(xi)."""
    T = np.eye(4)
    T[:3, :] = np.asarray(T12, float).reshape(3, 4)
    return (T @ se3_exp(xi))[:3, :].reshape(12)


def assemble(factors, H_f, b_f, P):
    """Dense 6P x 6P H and 6P b from per-factor 12x12 blocks ([source | target])."""
    H = np.zeros((6 * P, 6 * P))
    b = np.zeros(6 * P)
    for f, (_, _, tp, sp, binary) in enumerate(np.asarray(factors)):
        s, t = 6 * int(sp), 6 * int(tp)
        H[s:s + 6, s:s + 6] += H_f[f, :6, :6]
        b[s:s + 6] += b_f[f, :6]
        if binary:
            H[s:s + 6, t:t + 6] += H_f[f, :6, 6:]
            H[t:t + 6, s:s + 6] += H_f[f, 6:, :6]
            H[t:t + 6, t:t + 6] += H_f[f, 6:, 6:]
            b[t:t + 6] += b_f[f, 6:]
    return H, b


def damp(H, b, lam, fixed_pose=-1):
    """(H + lam diag H, -b) with identity rows for zero diagonals and for the fixed pose."""
    A = H.copy()
    g = -b.copy()
    d = np.diag(H).copy()
    idle = ~(d > 0.0)
    if fixed_pose >= 0:
        idle[6 * fixed_pose:6 * fixed_pose + 6] = True
    A[np.arange(len(d)), np.arange(len(d))] = np.where(d > 0.0, d * (1.0 + lam), 1.0)
    A[idle, :] = 0.0
    A[:, idle] = 0.0
    A[idle, idle] = 1.0
    g[idle] = 0.0
    return A, g


def lm_step(maps, clouds, poses, factors, lam, fixed_pose=-1, nthreads=0):
    """One damped Gauss-Newton step from `poses` ((P, 12)): returns delta (P, 6), the new poses
    (P, 12), the costs before and after, and the assembled H, b."""
    poses = np.asarray(poses, float).reshape(-1, 12)
    P = poses.shape[0]
    r0 = linearize_factors(maps, clouds, poses, factors, nthreads)
    H, b = assemble(factors, r0["H"], r0["b"], P)
    A, g = damp(H, b, lam, fixed_pose)
    delta = np.linalg.solve(A, g).reshape(P, 6)
    new = np.stack([retract(poses[i], delta[i]) for i in range(P)])
    r1 = linearize_factors(maps, clouds, new, factors, nthreads)
    return {"delta": delta, "poses": new, "cost": np.array([r0["e"].sum(), r1["e"].sum()]),
            "H": H, "b": b}
