"""SE(3) helpers for the tests: exponential map and adjoint, tangent xi = [omega; rho].

Used only to perturb poses for finite differences and to build test poses; shared by nothing
outside the tests.
"""
import numpy as np


def hat(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def so3_exp(w):
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w)
    K = hat(w)
    if th < 1e-12:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th**2 * K @ K


def se3_exp(xi):
    """Exp([omega; rho]) as a 4x4 matrix: [Exp(omega) | V(omega) rho]."""
    xi = np.asarray(xi, dtype=np.float64)
    w, rho = xi[:3], xi[3:]
    th = np.linalg.norm(w)
    K = hat(w)
    if th < 1e-12:
        V = np.eye(3) + 0.5 * K + K @ K / 6.0
    else:
        V = np.eye(3) + (1 - np.cos(th)) / th**2 * K + (th - np.sin(th)) / th**3 * K @ K
    T = np.eye(4)
    T[:3, :3] = so3_exp(w)
    T[:3, 3] = V @ rho
    return T


def to44(T):
    T = np.asarray(T, dtype=np.float64)
    if T.shape == (4, 4):
        return T.copy()
    M = np.eye(4)
    M[:3, :] = T.reshape(3, 4)
    return M


def to12(T):
    return to44(T)[:3, :].reshape(12).copy()


def retract(T, xi):
    """Right perturbation T Exp(xi)."""
    return to44(T) @ se3_exp(xi)


def adjoint(T):
    """Ad(T) for xi = [omega; rho]: [[R, 0], [[t]x R, R]]."""
    T = to44(T)
    R, t = T[:3, :3], T[:3, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[3:, 3:] = R
    A[3:, :3] = hat(t) @ R
    return A


def inv(T):
    T = to44(T)
    R, t = T[:3, :3], T[:3, 3]
    M = np.eye(4)
    M[:3, :3] = R.T
    M[:3, 3] = -R.T @ t
    return M


def random_pose(rng, max_angle, max_trans):
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(0, max_angle)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    T = np.eye(4)
    T[:3, :3] = so3_exp(axis * ang)
    T[:3, 3] = d * rng.uniform(0, max_trans)
    return T
