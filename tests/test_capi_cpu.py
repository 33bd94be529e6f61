"""CPU-only checks of the C-ABI library: it loads, exports every symbol the header declares,
and its host-side helpers (relative pose, SE(3) retraction and right Jacobian, argument
validation that needs no device) are right. No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from tests import se3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vgicp.h")
LIB = os.path.join(ROOT, "paper_2202_00242_amd", "libvgicp.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"VGICP_API\s+[^;(]*?\b(vgicp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2202_00242_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ["vgicp_build_voxelmap", "vgicp_linearize", "vgicp_evaluate",
                 "vgicp_linearize_batched", "vgicp_backward", "vgicp_batch_create",
                 "vgicp_batch_linearize", "vgicp_batch_autotune", "vgicp_sync_status"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_library_hides_internal_symbols():
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported and all(s.startswith("vgicp_") for s in exported), sorted(exported)[:20]


def test_binding_names_match_header():
    import paper_2202_00242_amd.vgicp as V
    for s in declared_symbols():
        if s.startswith("vgicp_batch_") and s not in ("vgicp_batch_create",):
            continue  # batch calls are methods of vgicp.Batch
        if s in ("vgicp_last_error", "vgicp_destroy_voxelmap", "vgicp_version"):
            continue  # wrapped by VGICPError / VoxelMap.close / version()
        assert hasattr(V, s), s


def test_relative_pose_bit_exact_with_oracle():
    import paper_2202_00242_amd.vgicp as V
    rng = np.random.default_rng(3)
    for _ in range(200):
        Tt = se3.random_pose(rng, 3.1, 5000.0)
        Ts = se3.random_pose(rng, 3.1, 5000.0)
        np.testing.assert_array_equal(V.vgicp_relative_pose(Tt, Ts),
                                      oracle.relative_pose(Tt, Ts))


def test_se3_retract_and_right_jacobian():
    import paper_2202_00242_amd.vgicp as V
    rng = np.random.default_rng(4)
    for _ in range(20):
        T = se3.random_pose(rng, 3.0, 10.0)
        xi = rng.normal(size=6) * 0.7
        np.testing.assert_allclose(V.vgicp_se3_retract(T, xi).reshape(3, 4),
                                   se3.retract(T, xi)[:3], atol=1e-12)
        # Exp(xi + d) = Exp(xi) Exp(J d): compare numerically through the log of the
        # difference, small d
        J = V.vgicp_se3_right_jacobian(xi)
        h = 1e-6
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            A = se3.se3_exp(xi)
            B = se3.se3_exp(xi + d)
            D = se3.inv(A) @ B     # = Exp(J d) to first order
            w = np.array([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]]) / 2
            v = D[:3, 3]
            np.testing.assert_allclose(np.concatenate([w, v]) / h, J[:, k], atol=2e-6)
    np.testing.assert_array_equal(V.vgicp_se3_right_jacobian(np.zeros(6)), np.eye(6))
    with pytest.raises(V.VGICPError):
        V.vgicp_se3_right_jacobian([5, 0, 0, 0, 0, 0])


def test_argument_validation_without_device(lib):
    P = ctypes.c_void_p
    lib.vgicp_voxelmap_size.argtypes = [P, P, P]
    assert lib.vgicp_voxelmap_size(None, None, None) == 1  # E_INVALID_ARG
    lib.vgicp_build_voxelmap.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P, P]
    out = ctypes.c_void_p()
    assert lib.vgicp_build_voxelmap(None, None, 10, 1.0, None, ctypes.byref(out)) == 1
    assert lib.vgicp_build_voxelmap(None, None, 0, -1.0, None, ctypes.byref(out)) == 1
    assert lib.vgicp_build_voxelmap(None, None, -5, 1.0, None, ctypes.byref(out)) == 1
    lib.vgicp_last_error.restype = ctypes.c_char_p
    assert b"negative" in lib.vgicp_last_error()
    assert lib.vgicp_destroy_voxelmap(None) == 0
    lib.vgicp_batch_destroy.argtypes = [P]
    assert lib.vgicp_batch_destroy(None) == 0


def test_preprocessing_argument_validation_without_device(lib):
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.vgicp_last_error.restype = ctypes.c_char_p
    lib.vgicp_downsample.argtypes = [P, P, I64, D, D, P, P, I64, P, P]
    m = ctypes.c_int64(-1)
    assert lib.vgicp_downsample(None, None, 0, 1.0, 0.0, None, None, 0, None, None) == 1
    assert lib.vgicp_downsample(None, None, 10, 1.0, 0.0, None, None, 0, ctypes.byref(m),
                                None) == 1
    assert m.value == 0
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.vgicp_downsample(fake, None, 10, 0.0, 0.0, fake, None, 10, ctypes.byref(m),
                                None) == 1
    assert lib.vgicp_downsample(fake, fake, 10, 0.5, 0.0, fake, fake, 10, ctypes.byref(m),
                                None) == 1
    assert b"scan duration" in lib.vgicp_last_error()
    assert lib.vgicp_downsample(None, None, 0, 0.5, 0.0, None, None, 0, ctypes.byref(m),
                                None) == 0  # an empty cloud is valid
    lib.vgicp_knn.argtypes = [P, I64, I32, D, P, P]
    assert lib.vgicp_knn(fake, 10, 0, 0.0, fake, None) == 1
    assert lib.vgicp_knn(fake, 10, 33, 0.0, fake, None) == 1
    assert lib.vgicp_knn(fake, 10, 10, -1.0, fake, None) == 1
    assert lib.vgicp_knn(None, 0, 10, 0.0, None, None) == 0
    lib.vgicp_point_covariances.argtypes = [P, I64, P, I32, D, D, P, P]
    assert lib.vgicp_point_covariances(fake, 10, fake, 10, -1.0, 1e-3, fake, None) == 1
    assert lib.vgicp_point_covariances(fake, 10, fake, 10, 0.01, float("nan"), fake, None) == 1
    assert lib.vgicp_point_covariances(fake, 10, None, 10, 0.01, 1e-3, fake, None) == 1
    assert lib.vgicp_point_covariances(None, 0, None, 10, 0.01, 1e-3, None, None) == 0


def test_imu_argument_validation_without_device(lib):
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    I64 = ctypes.c_int64
    lib.vgicp_imu_preintegrate.argtypes = [P, I64, P, I32, P, D, D, P, P, P]
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.vgicp_imu_preintegrate(fake, 5, fake, -1, fake, 1e-3, 1e-2, fake, fake, None) == 1
    assert lib.vgicp_imu_preintegrate(fake, -5, fake, 3, fake, 1e-3, 1e-2, fake, fake, None) == 1
    assert lib.vgicp_imu_preintegrate(fake, 5, None, 3, fake, 1e-3, 1e-2, fake, fake, None) == 1
    assert lib.vgicp_imu_preintegrate(fake, 5, fake, 3, fake, 0.0, 1e-2, fake, fake, None) == 1
    assert lib.vgicp_imu_preintegrate(None, 0, None, 0, None, 1e-3, 1e-2, None, None, None) == 0
    lib.vgicp_imu_linearize.argtypes = [P, P, P, I32, P, P, I32, P, P, P, P, P]
    g = (ctypes.c_double * 3)(0.0, 0.0, -9.8)
    assert lib.vgicp_imu_linearize(fake, fake, fake, 2, fake, fake, 3, None, fake, fake, fake,
                                   None) == 1
    gn = (ctypes.c_double * 3)(0.0, float("nan"), -9.8)
    assert lib.vgicp_imu_linearize(fake, fake, fake, 2, fake, fake, 3, gn, fake, fake, fake,
                                   None) == 1
    assert lib.vgicp_imu_linearize(fake, fake, None, 2, fake, fake, 3, g, fake, fake, fake,
                                   None) == 1
    assert lib.vgicp_imu_linearize(None, None, None, 0, None, None, 0, g, None, None, None,
                                   None) == 0
