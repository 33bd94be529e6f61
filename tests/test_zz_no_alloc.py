"""The allocation-free single-factor entry point (vgicp_linearize_noalloc) against
vgicp_linearize: the same kernels on the library's static scratch must give bitwise the same
H, b, e, inliers and correspondences, on two calls in a row (the second on a smaller cloud, so
stale partial sums of the first would show) and in both orders of the two entry points; both
also meet the oracle's bound. Sizes beyond the static scratch are refused before any launch."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL_FP64_ACC, cloud_dev, compare_factor

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def V():
    import paper_2202_00242_amd.vgicp as V
    return V


def _same(a, b):
    for k in ("H", "b", "err", "inliers", "corr"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("binary", [False, True])
def test_noalloc_matches_linearize(V, binary):
    u = synth.urban(2)
    sxyz, scov = u["source"]
    txyz, tcov = u["targets"][3]
    Tt, Ts = u["T_targets"][3], u["T_source"]
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5)
    om = oracle.VoxelMap(txyz, tcov, 0.5)
    sx, sc = cloud_dev(sxyz, scov)
    n_small = 3001
    sxs, scs = sx[:, :n_small].contiguous(), sc[:, :n_small].contiguous()
    for prec in (0, 3):
        # large then small, the allocation-free call first each time
        a1 = V.vgicp_linearize_noalloc(m, sx, sc, Tt, Ts, binary, prec, want_corr=True)
        a2 = V.vgicp_linearize_noalloc(m, sxs, scs, Tt, Ts, binary, prec, want_corr=True)
        r1 = V.vgicp_linearize(m, sx, sc, Tt, Ts, binary, prec, want_corr=True)
        r2 = V.vgicp_linearize(m, sxs, scs, Tt, Ts, binary, prec, want_corr=True)
        torch.cuda.synchronize()
        V.vgicp_sync_status()
        _same(a1, r1)
        _same(a2, r2)
        ref1 = oracle.linearize(om, sxyz, scov, Tt, Ts, binary)
        ref2 = oracle.linearize(om, sxyz[:, :n_small], scov[:, :n_small], Tt, Ts, binary)
        np.testing.assert_array_equal(a1["corr"].cpu().numpy(), ref1["corr"])
        np.testing.assert_array_equal(a2["corr"].cpu().numpy(), ref2["corr"])
        compare_factor(a1, ref1, TOL_FP64_ACC, "noalloc large")
        compare_factor(a2, ref2, TOL_FP64_ACC, "noalloc small")


def test_noalloc_capacity(V):
    """33,554,432 points fill the 4,096 tiles of the static scratch (256-CU device); one more
    point is refused on the host (the cloud is real device memory of that size)."""
    props = torch.cuda.get_device_properties(0)
    if props.multi_processor_count != 256:
        pytest.skip("the point limit is stated for a 256-CU device")
    rng = np.random.default_rng(3)
    txyz = (rng.uniform(-2, 2, size=(3, 2000))).astype(np.float32)
    txyz[:, 0] = 0.25  # the voxel at the origin is occupied
    tcov = np.tile(np.array([[1e-2], [0], [0], [1e-2], [0], [1e-2]], np.float32), (1, 2000))
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5)
    n = 33_554_432 + 1
    xyz = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    cov = torch.zeros((6, n), dtype=torch.float32, device="cuda")
    cov[0] = cov[3] = cov[5] = 1e-2
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_linearize_noalloc(m, xyz, cov, np.eye(4)[:3].reshape(12),
                                  np.eye(4)[:3].reshape(12), False)
    assert ei.value.status == V.VGICP_E_CAPACITY
    xyz, cov = xyz[:, :n - 1].contiguous(), cov[:, :n - 1].contiguous()
    out = V.vgicp_linearize_noalloc(m, xyz, cov, np.eye(4)[:3].reshape(12),
                                    np.eye(4)[:3].reshape(12), False)
    ref = V.vgicp_linearize(m, xyz, cov, np.eye(4)[:3].reshape(12),
                            np.eye(4)[:3].reshape(12), False)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    assert torch.equal(out["H"], ref["H"]) and torch.equal(out["inliers"], ref["inliers"])
    assert out["inliers"].item() == n - 1  # every point at the origin voxel
