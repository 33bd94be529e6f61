"""Floating-point facts the kernels rely on, checked on the host in the same evaluation order.

* Power-of-two resolution: the kernels take the voxel coordinate of q = R mu + t from a
  transform with R and t pre-multiplied by 1/res. With res = 2^j every product and sum of that
  fixed order is the unscaled one times 2^-j exactly, so floor(q / res) is unchanged.
* The per-axis saturating conversion leaves out-of-range coordinates outside every map box
  when the box test is done in unsigned 32-bit arithmetic.
"""
import numpy as np

from tests import se3


def transform(R, t, p):
    # ((R0 x + R1 y) + R2 z) + t, no fused multiply-add (numpy float64 ops round each step)
    return ((R[:, 0:1] * p[0] + R[:, 1:2] * p[1]) + R[:, 2:3] * p[2]) + t[:, None]


def test_prescaled_transform_is_exact_for_power_of_two_resolution():
    rng = np.random.default_rng(5)
    for trial in range(40):
        T = se3.random_pose(rng, 3.1, 10.0 ** rng.uniform(-1, 3.7))
        R, t = T[:3, :3], T[:3, 3]
        p = (rng.normal(size=(3, 20000)) * 10.0 ** rng.uniform(-1, 2.5)).astype(np.float32)
        p = p.astype(np.float64)
        q = transform(R, t, p)
        for j in range(-4, 5):
            res = 2.0 ** j
            s = transform(R * (1.0 / res), t * (1.0 / res), p)
            assert np.array_equal(s, q / res), (trial, j)
            assert np.array_equal(np.floor(s), np.floor(q / res))


def test_prescaled_transform_differs_for_other_resolutions():
    """The shortcut is only taken for powers of two: for res = 0.3 it does change keys."""
    rng = np.random.default_rng(6)
    T = se3.random_pose(rng, 3.1, 300.0)
    R, t = T[:3, :3], T[:3, 3]
    p = (rng.normal(size=(3, 200000)) * 50.0).astype(np.float32).astype(np.float64)
    q = transform(R, t, p)
    s = transform(R * (1.0 / 0.3), t * (1.0 / 0.3), p)
    assert not np.array_equal(s, q / 0.3)


def test_saturated_coordinates_fail_every_box():
    lim = 2 ** 20
    rng = np.random.default_rng(7)
    for _ in range(2000):
        lo = int(rng.integers(-lim + 1, lim))
        ext = int(rng.integers(1, lim - lo + 1))  # lo + ext <= 2^20
        for k in (2 ** 31 - 1, -2 ** 31, lim, -lim, lim + 5, -lim - 5):
            if -lim < k < lim:
                continue
            d = ((k & 0xFFFFFFFF) - (lo & 0xFFFFFFFF)) & 0xFFFFFFFF  # uint32 wrap-around
            assert d >= ext, (lo, ext, k)
