"""Full-size workloads on the GPU against the oracle.

* global batch (400 submaps, 7,960 binary factors; the benchmark workload) in the autotuned
  launch configuration, with the grid and with the hash lookup: every factor's inlier count,
  H, b and e; its LM step with the banded solver from both ends and in one sweep;
* the same loop 4.3-5.0 km from the world origin for each precision form (the FP64-key forms
  must keep correspondences bit-exact and meet their bounds; the world-FP32 form is reported);
* the differentiation set (32 urban scenes x 8 keyframes = 256 factors): correspondences equal
  to the oracle's own, autograd gradients against the oracle's exact gradient (pose tangents
  over the vector's norm, every source point on its own scale).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL_FP64_ACC, TOL_KAHAN, cloud_dev, dev, point_gradient_error
from tests.metrics import factor_errors

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def V():
    import paper_2202_00242_amd.vgicp as V
    return V


def setup_batch(V, data, layout=0):
    clouds = [cloud_dev(x, c) for x, c in data["clouds"]]
    maps = [V.vgicp_build_voxelmap(x, c, 0.5, layout=layout) for x, c in clouds]
    P = dev(np.ascontiguousarray(data["T"]))
    b = V.Batch(maps, clouds, data["factors"], P.shape[0])
    return clouds, maps, P, b


def oracle_inputs(data):
    maps = [oracle.VoxelMap(x, c, 0.5) for x, c in data["clouds"]]
    cl = [oracle.Cloud.of(x, c) for x, c in data["clouds"]]
    return maps, cl


def oracle_all(data):
    maps, cl = oracle_inputs(data)
    return oracle.linearize_factors(maps, cl, data["T"], data["factors"])


@pytest.fixture(scope="module")
def global_data():
    return synth.global_batch()


@pytest.fixture(scope="module")
def global_oracle(global_data):
    return oracle_inputs(global_data)


@pytest.fixture(scope="module")
def global_ref(global_data, global_oracle):
    maps, cl = global_oracle
    return oracle.linearize_factors(maps, cl, global_data["T"], global_data["factors"])


def errors_all(out, ref, idx):
    H = out["H"].cpu().numpy()
    b = out["b"].cpu().numpy()
    e = out["err"].cpu().numpy()
    return np.array([[v for k, v in factor_errors(H[f], b[f], e[f], ref["H"][f], ref["b"][f],
                                                    ref["e"][f]).items() if k != "H_fro"]
                     for f in idx])


@pytest.mark.parametrize("layout", [0, 1])  # automatic (the grid here), hash
def test_global_batch_all_factors(V, global_data, global_ref, layout):
    _, maps, P, b = setup_batch(V, global_data, layout)
    assert all(m.layout == (2 if layout == 0 else 1) for m in maps)
    sched = b.autotune(P, V.VGICP_ACC_FP64)
    out = b.linearize(P, V.VGICP_ACC_FP64)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    np.testing.assert_array_equal(out["inliers"].cpu().numpy(), global_ref["inliers"])
    err = errors_all(out, global_ref, range(len(global_data["factors"])))
    print(f"layout {layout} schedule {sched}: max factor error over {err.shape[0]} factors "
          f"{err.max():.3e}")
    assert err.max() <= TOL_FP64_ACC


def test_global_lm_step_both_ends(V, global_data, global_oracle):
    """The LM step of the global graph (400 poses, pose 0 fixed; half-bandwidth 131 unknowns
    after the pose ordering), FP64 math: the banded system solved from both ends (two 189-block
    ends around a 22-block separator) and in one sweep, against each other and against the
    oracle's dense NumPy step."""
    from oracle import lm
    _, _, P, b = setup_batch(V, global_data)
    banded, w = b.lm_info()
    assert banded == 2 and w == 131, (banded, w)
    a = b.lm_step(P, V.VGICP_MATH_FP64, 1e-4, fixed_pose=0)
    torch.cuda.synchronize()
    b.lm_solver(2)
    try:
        assert b.lm_info() == (1, w)
        o = b.lm_step(P, V.VGICP_MATH_FP64, 1e-4, fixed_pose=0)
        torch.cuda.synchronize()
    finally:
        b.lm_solver(0)
    V.vgicp_sync_status()
    maps, cl = global_oracle
    ref = lm.lm_step(maps, cl, global_data["T"], global_data["factors"], 1e-4, 0)

    def rel(x, y):
        return float(np.abs(x - y).max() / np.abs(y).max())
    da, d1 = a["delta"].cpu().numpy(), o["delta"].cpu().numpy()
    print(f"both ends vs one sweep {rel(da, d1):.2e}; vs oracle: both ends "
          f"{rel(da, ref['delta']):.2e}, one sweep {rel(d1, ref['delta']):.2e}")
    assert rel(da, d1) < 1e-9
    assert rel(da, ref["delta"]) < 1e-8 and rel(d1, ref["delta"]) < 1e-8
    c = a["cost"].cpu().numpy()
    np.testing.assert_allclose(c[0], ref["cost"][0], rtol=1e-10)
    # at the new poses a step difference of ~1e-8 may move a few of the 3.4e8 points across a
    # voxel boundary
    np.testing.assert_allclose(c[1], ref["cost"][1], rtol=1e-6)


@pytest.mark.parametrize("prec,tol", [(0, TOL_FP64_ACC), (1, TOL_KAHAN), (3, TOL_FP64_ACC)])
def test_precision_batch_forms(V, prec, tol):
    data = synth.precision_batch()
    F = len(data["factors"])
    idx = np.linspace(0, F - 1, 400).astype(int)
    sub = dict(data)
    sub["factors"] = data["factors"][idx]
    ref = oracle_all(sub)
    _, _, P, b = setup_batch(V, data)
    out = b.linearize(P, prec)
    torch.cuda.synchronize()
    nin = out["inliers"].cpu().numpy()[idx]
    np.testing.assert_array_equal(nin, ref["inliers"])
    err = errors_all({k: v[idx] for k, v in out.items()}, ref, range(len(idx)))
    print(f"precision {prec}: max {err.max():.3e} median {np.median(err.max(1)):.3e}")
    assert err.max() <= tol


def test_precision_batch_naive_world_is_reported(V):
    """World FP32 coordinates 4-5 km from the origin: keys may differ from the FP64 ones and the
    error is not bounded; this records it (no gate beyond sanity)."""
    data = synth.precision_batch()
    F = len(data["factors"])
    idx = np.linspace(0, F - 1, 200).astype(int)
    sub = dict(data)
    sub["factors"] = data["factors"][idx]
    ref = oracle_all(sub)
    _, _, P, b = setup_batch(V, data)
    out = b.linearize(P, V.VGICP_NAIVE_WORLD_FP32)
    torch.cuda.synchronize()
    nin = out["inliers"].cpu().numpy()[idx]
    mism = np.abs(nin - ref["inliers"]).sum()
    err = errors_all({k: v[idx] for k, v in out.items()}, ref, range(len(idx)))
    print(f"naive world FP32: inlier count difference {mism} of {ref['inliers'].sum()}, "
          f"max factor error {err.max():.3e}, median {np.median(err.max(1)):.3e}")
    assert np.all(np.isfinite(err))


def test_diff_set_gradients(V):
    from paper_2202_00242_amd.autograd import vgicp_cost
    scenes = synth.diff_set()
    worst = 0.0
    nf = 0
    for sc in scenes:
        sxyz, scov = sc["source"]
        sx, scd = cloud_dev(sxyz, scov)
        for ki, res in sc["factors"]:
            txyz, tcov = sc["targets"][ki]
            Tt = sc["T_targets"][ki]
            m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), res)
            xs = torch.zeros(6, dtype=torch.float64, requires_grad=True)
            xt = torch.zeros(6, dtype=torch.float64, requires_grad=True)
            pts = sx.clone().requires_grad_(True)
            e = vgicp_cost(xs, xt, pts, scd, m, Tt, sc["T_source"], True)
            e.backward()
            fw = V.vgicp_evaluate(m, sx, scd, Tt, sc["T_source"], want_corr=True)
            om = oracle.VoxelMap(txyz, tcov, res)
            corr = oracle.evaluate(om, sxyz, scov, Tt, sc["T_source"])["corr"]
            np.testing.assert_array_equal(fw["corr"].cpu().numpy(), corr)
            ref = oracle.gradient(om, sxyz, scov, Tt, sc["T_source"], True, corr)
            g = np.concatenate([xs.grad.numpy(), xt.grad.numpy()])
            e_xi = np.max(np.abs(g - ref["g_xi"])) / np.linalg.norm(ref["g_xi"])
            gp = pts.grad.cpu().numpy()
            e_pt = point_gradient_error(gp, ref["g_points"], om, sxyz, scov, Tt,
                                        sc["T_source"], corr)
            assert abs(e.item() - ref["e"]) <= 1e-4 * ref["e"]
            worst = max(worst, e_xi, e_pt)
            nf += 1
    print(f"{nf} factors: worst gradient error {worst:.3e}")
    assert nf == 256 and worst <= 1e-4


def diff_batch(V, scenes):
    """The differentiation set as one batch: 32 sources, 256 target maps, 9 poses per scene
    (8 keyframes, then the scan), 256 binary factors."""
    maps, omaps, clouds, sources, poses, factors = [], [], [], [], [], []
    for si, sc in enumerate(scenes):
        sources.append(sc["source"])
        clouds.append(cloud_dev(*sc["source"]))
        p0 = len(poses)
        poses.extend(np.asarray(T).reshape(12) for T in sc["T_targets"])
        poses.append(np.asarray(sc["T_source"]).reshape(12))
        for ki, res in sc["factors"]:
            txyz, tcov = sc["targets"][ki]
            factors.append([len(maps), si, p0 + ki, p0 + 8, 1])
            maps.append(V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), res))
            omaps.append(oracle.VoxelMap(txyz, tcov, res))
    factors = np.array(factors, np.int32)
    return maps, omaps, clouds, sources, np.stack(poses), factors


def test_diff_set_batched_backward(V):
    """All 256 factors of the differentiation set in one batch: costs from the batched evaluate
    and the batched backward's per-factor pose gradients and per-point gradients (each source
    point summed over its 8 factors) against the oracle's exact gradients."""
    from tests.gpu_util import point_scales, scaled_point_error
    scenes = synth.diff_set()
    maps, omaps, clouds, sources, poses, factors = diff_batch(V, scenes)
    b = V.Batch(maps, clouds, factors, poses.shape[0])
    Pd = dev(poses)
    fw = b.evaluate(Pd)
    g_err = np.random.default_rng(41).uniform(0.5, 1.5, size=len(factors))
    out = b.backward(Pd, dev(g_err), want_points=True, want_factors=True)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    e = fw["err"].cpu().numpy()
    gf = out["grad_factors"].cpu().numpy()
    worst_e = worst_f = worst_p = 0.0
    gsum = [np.zeros((3, x.shape[1])) for x, _ in sources]
    scale = [np.zeros(x.shape[1]) for x, _ in sources]
    for f, (mi, ci, ti, si, _) in enumerate(factors):
        xyz, cov = sources[ci]
        corr = oracle.evaluate(omaps[mi], xyz, cov, poses[ti], poses[si])["corr"]
        r = oracle.gradient(omaps[mi], xyz, cov, poses[ti], poses[si], True, corr)
        worst_e = max(worst_e, abs(e[f] - r["e"]) / r["e"])
        worst_f = max(worst_f, np.max(np.abs(gf[f] - g_err[f] * r["g_xi"]))
                      / np.linalg.norm(g_err[f] * r["g_xi"]))
        gsum[ci] += g_err[f] * r["g_points"]
        scale[ci] += g_err[f] * point_scales(omaps[mi], xyz, cov, poses[ti], poses[si], corr)
    for ci in range(len(sources)):
        worst_p = max(worst_p, scaled_point_error(out["grad_points"][ci].cpu().numpy(),
                                                  gsum[ci], scale[ci]))
    print(f"256 factors batched: cost {worst_e:.2e}, factor gradients {worst_f:.2e}, "
          f"point gradients {worst_p:.2e}")
    assert worst_e <= TOL_FP64_ACC and worst_f <= 1e-4 and worst_p <= 1e-4
