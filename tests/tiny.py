"""Small seeded clouds for pin and property tests (sizes a pure-Python loop handles)."""
import numpy as np


def plane_cov(rng, n, scale=0.01, flat=1e-3):
    """Random plane-like SPD covariances scale * R diag(1, 1, flat) R^T, as (6, n)."""
    out = np.empty((6, n))
    for k in range(n):
        A = rng.normal(size=(3, 3))
        Q, _ = np.linalg.qr(A)
        C = scale * Q @ np.diag([1.0, 1.0, flat]) @ Q.T
        out[:, k] = [C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2]]
    return out


def random_spd_cov(rng, n, lo=0.01, hi=0.2):
    out = np.empty((6, n))
    for k in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        C = Q @ np.diag(rng.uniform(lo, hi, size=3)) @ Q.T
        out[:, k] = [C[0, 0], C[0, 1], C[0, 2], C[1, 1], C[1, 2], C[2, 2]]
    return out


def cloud(rng, n, extent=2.0, cov="plane"):
    """FP32 cloud: xyz (3, n) uniform in [-extent, extent]^3 and covariances (6, n)."""
    xyz = rng.uniform(-extent, extent, size=(3, n)).astype(np.float32)
    c = plane_cov(rng, n) if cov == "plane" else random_spd_cov(rng, n)
    return xyz, c.astype(np.float32)


def source_near(rng, target_xyz, n, noise=0.05):
    """Source points near random target points (mostly inliers)."""
    idx = rng.integers(0, target_xyz.shape[1], size=n)
    xyz = target_xyz[:, idx].astype(np.float64) + rng.normal(scale=noise, size=(3, n))
    return xyz.astype(np.float32)
