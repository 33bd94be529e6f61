"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar: voxel keys, counts, means (same FP64 summation order) and correspondences bit-exact;
H, b, e within the factor metric of tests/metrics.py: 1e-5 (FP32 math with FP64 accumulation,
FP64 math) and 1e-4 (Kahan-compensated FP32 accumulation).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests import se3, tiny
from tests.gpu_util import (TOL_FP64_ACC, TOL_KAHAN, cloud_dev, compare_factor, dev,
                            oracle_factor, tol_for)
from tests.metrics import factor_errors

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def V():
    import paper_2202_00242_amd.vgicp as V
    return V


PRECS = [0, 1, 3]  # ACC_FP64, KAHAN_FP32, MATH_FP64


# ----------------------------------------------------------------------------- voxel maps

def check_map_equal(V, xyz, cov, res, layout=0):
    m = V.vgicp_build_voxelmap(*cloud_dev(xyz, cov), res, layout=layout)
    ex = {k: v.cpu().numpy() for k, v in V.vgicp_voxelmap_export(m).items()}
    om = oracle.VoxelMap(xyz, cov, res).export()
    np.testing.assert_array_equal(ex["keys"], om["keys"])
    np.testing.assert_array_equal(ex["count"], om["count"])
    np.testing.assert_array_equal(ex["mean"].T, om["mean"])
    np.testing.assert_array_equal(ex["cov"].T, om["cov"])
    Vn, cap = m.size()
    assert Vn == len(om["keys"])
    if m.layout == V.VGICP_LAYOUT_HASH:
        assert cap >= 4 * Vn and cap & (cap - 1) == 0
    else:
        assert m.layout == V.VGICP_LAYOUT_GRID and cap * 32 >= Vn
    return m


def test_voxelmap_room(V):
    r = synth.room()
    check_map_equal(V, *r["target"], 1.0)


@pytest.mark.parametrize("res", [0.25, 0.5, 1.0])
def test_voxelmap_urban(V, res):
    u = synth.urban(0)
    check_map_equal(V, *u["targets"][0], res)


@pytest.mark.parametrize("layout", [1, 2])  # hash, grid
@pytest.mark.parametrize("n,res", [(1, 1.0), (2047, 0.5), (2048, 0.5), (2049, 0.3),
                                   (5000, 0.1), (70000, 0.7)])
def test_voxelmap_sizes_and_nonpow2(V, n, res, layout):
    rng = np.random.default_rng(n)
    xyz, cov = tiny.cloud(rng, n, extent=3.0, cov="spd")
    check_map_equal(V, xyz, cov, res, layout)


def wide_scene(rng):
    """Three clusters tens of km apart at 0.1 m: the voxel box needs 64-bit keys and its grid
    would exceed 2^24 bricks."""
    parts = []
    for c in ([-40e3, 1e3, 0.0], [0.0, 0.0, 0.0], [45e3, -2e3, 30.0]):
        x, _ = tiny.cloud(rng, 3000, extent=4.0)
        parts.append(x + np.array(c, np.float32)[:, None])
    xyz = np.concatenate(parts, 1).astype(np.float32)
    return xyz, tiny.plane_cov(rng, xyz.shape[1]).astype(np.float32)


def test_voxelmap_layout_choice(V, urban):
    txyz, tcov = urban["targets"][0]
    assert V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5).layout == V.VGICP_LAYOUT_GRID
    rng = np.random.default_rng(21)
    xyz, cov = wide_scene(rng)
    m = check_map_equal(V, xyz, cov, 0.1)
    assert m.layout == V.VGICP_LAYOUT_HASH
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_build_voxelmap(*cloud_dev(xyz, cov), 0.1, layout=V.VGICP_LAYOUT_GRID)
    assert ei.value.status == V.VGICP_E_CAPACITY
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_build_voxelmap(*cloud_dev(xyz, cov), 0.1, layout=7)
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    V.vgicp_sync_status()


@pytest.mark.parametrize("prec", PRECS)
def test_wide_scene_64bit_keys(V, prec):
    """Source near the three far clusters, each seen from a pose near the origin of its
    cluster's frame: the 64-bit-key table path against the oracle."""
    rng = np.random.default_rng(22)
    txyz, tcov = wide_scene(rng)
    sxyz = tiny.source_near(rng, txyz, 9000, noise=0.04)
    scov = tiny.plane_cov(rng, 9000).astype(np.float32)
    Tt = se3.random_pose(rng, 0.2, 1.0)
    Ts = Tt @ se3.random_pose(rng, 0.01, 0.02)
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.1)
    assert m.layout == V.VGICP_LAYOUT_HASH
    g = V.vgicp_linearize(m, *cloud_dev(sxyz, scov), Tt, Ts, True, prec, want_corr=True)
    om, ref = oracle_factor(txyz, tcov, 0.1, sxyz, scov, Tt, Ts, True)
    np.testing.assert_array_equal(g["corr"].cpu().numpy(), ref["corr"])
    assert ref["inliers"] > 500
    compare_factor(g, ref, tol_for(prec), f"wide p{prec}")


def test_voxelmap_empty_and_permutation(V):
    m = V.vgicp_build_voxelmap(*cloud_dev(np.zeros((3, 0)), np.zeros((6, 0))), 1.0)
    assert m.size()[0] == 0
    rng = np.random.default_rng(9)
    xyz, cov = tiny.cloud(rng, 3000, extent=2.0)
    perm = rng.permutation(3000)
    a = V.vgicp_voxelmap_export(V.vgicp_build_voxelmap(*cloud_dev(xyz, cov), 0.5))
    b = V.vgicp_voxelmap_export(V.vgicp_build_voxelmap(*cloud_dev(xyz[:, perm], cov[:, perm]),
                                                       0.5))
    assert torch.equal(a["keys"], b["keys"]) and torch.equal(a["count"], b["count"])


def test_voxelmap_errors(V):
    rng = np.random.default_rng(10)
    xyz, cov = tiny.cloud(rng, 100)
    bad = xyz.copy()
    bad[2, 50] = np.nan
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_build_voxelmap(*cloud_dev(bad, cov), 1.0)
    assert ei.value.status == V.VGICP_E_NONFINITE
    far = xyz.copy()
    far[0, 7] = 2.0 ** 21
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_build_voxelmap(*cloud_dev(far, cov), 1.0)
    assert ei.value.status == V.VGICP_E_KEY_RANGE
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_build_voxelmap(*cloud_dev(xyz, cov), 0.0)
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    V.vgicp_sync_status()  # nothing sticky left behind


# ----------------------------------------------------------------------------- one factor

@pytest.mark.parametrize("name", ["single_point_identity.json", "single_point_rotated.json"])
@pytest.mark.parametrize("prec", PRECS)
def test_hand_cases(V, name, prec):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    m = V.vgicp_build_voxelmap(*cloud_dev(np.array(g["target_xyz"]), np.array(g["target_cov"])),
                               g["res"])
    sx, sc = cloud_dev(np.array(g["source_xyz"]), np.array(g["source_cov"]))
    r = V.vgicp_linearize(m, sx, sc, g["T_target"], g["T_source"], False, prec, want_corr=True)
    ex = g["expected_unary"]
    np.testing.assert_allclose(r["H"].cpu().numpy(), ex["H"], atol=1e-6)
    np.testing.assert_allclose(r["b"].cpu().numpy(), ex["b"], atol=1e-6)
    np.testing.assert_allclose(r["err"].cpu().numpy()[0], ex["e"], rtol=1e-6)
    assert r["corr"].cpu().tolist() == ex["corr"]
    rb = V.vgicp_linearize(m, sx, sc, g["T_target"], g["T_source"], True, prec)
    txyz = np.array(g["target_xyz"])
    _, ref = oracle_factor(txyz, np.array(g["target_cov"]), g["res"], np.array(g["source_xyz"]),
                           np.array(g["source_cov"]), g["T_target"], g["T_source"], True)
    compare_factor(rb, ref, 1e-6, name)


@pytest.mark.parametrize("pose", ["identity", "truth", "perturbed"])
@pytest.mark.parametrize("prec", PRECS)
def test_room_unary(V, pose, prec):
    r = synth.room()
    (txyz, tcov), (sxyz, scov) = r["target"], r["source"]
    Ts = r["T_source"][pose]
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), r["res"])
    g = V.vgicp_linearize(m, *cloud_dev(sxyz, scov), r["T_target"], Ts, False, prec,
                          want_corr=True)
    om, ref = oracle_factor(txyz, tcov, r["res"], sxyz, scov, r["T_target"], Ts, False)
    np.testing.assert_array_equal(g["corr"].cpu().numpy(), ref["corr"])
    compare_factor(g, ref, tol_for(prec), f"room {pose} p{prec}")


@pytest.fixture(scope="module")
def urban():
    return synth.urban(0)


@pytest.mark.parametrize("layout", [1, 2])  # hash, grid
@pytest.mark.parametrize("prec", PRECS)
def test_urban_binary_all_factors(V, urban, prec, layout):
    sx, sc = cloud_dev(*urban["source"])
    worst = 0.0
    for ki, res in urban["factors"]:
        txyz, tcov = urban["targets"][ki]
        Tt = urban["T_targets"][ki]
        m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), res, layout=layout)
        assert m.layout == layout
        g = V.vgicp_linearize(m, sx, sc, Tt, urban["T_source"], True, prec, want_corr=True)
        om, ref = oracle_factor(txyz, tcov, res, *urban["source"], Tt, urban["T_source"], True)
        np.testing.assert_array_equal(g["corr"].cpu().numpy(), ref["corr"])
        err = compare_factor(g, ref, tol_for(prec), f"urban kf{ki} res{res} p{prec} l{layout}")
        worst = max(worst, err["H"], err["b"], err["e"])
    print(f"urban precision {prec} layout {layout}: worst factor error {worst:.3e}")


def test_layouts_bitwise_equal(V, urban):
    """Both lookup structures resolve the same ids, so every output is bitwise equal."""
    sx, sc = cloud_dev(*urban["source"])
    for ki, res in urban["factors"][:6]:
        txyz, tcov = urban["targets"][ki]
        Tt = urban["T_targets"][ki]
        out = []
        for layout in (V.VGICP_LAYOUT_HASH, V.VGICP_LAYOUT_GRID):
            m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), res, layout=layout)
            out.append(V.vgicp_linearize(m, sx, sc, Tt, urban["T_source"], True, 0,
                                         want_corr=True))
        for k in ("H", "b", "err", "inliers", "corr"):
            assert torch.equal(out[0][k], out[1][k]), (ki, res, k)


def test_evaluate_and_overlap(V, urban):
    sx, sc = cloud_dev(*urban["source"])
    txyz, tcov = urban["targets"][3]
    Tt = urban["T_targets"][3]
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5)
    g = V.vgicp_evaluate(m, sx, sc, Tt, urban["T_source"], want_corr=True)
    om = oracle.VoxelMap(txyz, tcov, 0.5)
    ref = oracle.evaluate(om, *urban["source"], Tt, urban["T_source"])
    np.testing.assert_array_equal(g["corr"].cpu().numpy(), ref["corr"])
    assert int(g["inliers"].item()) == ref["inliers"]
    assert abs(g["err"].item() - ref["e"]) <= TOL_FP64_ACC * ref["e"]


def test_deterministic(V, urban):
    sx, sc = cloud_dev(*urban["source"])
    m = V.vgicp_build_voxelmap(*cloud_dev(*urban["targets"][0]), 0.25)
    for prec in (0, 1):
        a = V.vgicp_linearize(m, sx, sc, urban["T_targets"][0], urban["T_source"], True, prec)
        b = V.vgicp_linearize(m, sx, sc, urban["T_targets"][0], urban["T_source"], True, prec)
        for k in ("H", "b", "err", "inliers"):
            assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 4097, 20001])
def test_ragged_and_edge_sizes(V, n):
    rng = np.random.default_rng(100 + n)
    txyz, tcov = tiny.cloud(rng, 4000, extent=2.0)
    sxyz = tiny.source_near(rng, txyz, n, noise=0.05) if n else np.zeros((3, 0), np.float32)
    scov = tiny.plane_cov(rng, n).astype(np.float32) if n else np.zeros((6, 0), np.float32)
    Tt = se3.random_pose(rng, 0.3, 2.0)
    Ts = Tt @ se3.random_pose(rng, 0.02, 0.03)
    for res, layout in ((0.5, 1), (0.5, 2), (0.3, 1), (0.3, 2)):
        m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), res, layout=layout)
        g = V.vgicp_linearize(m, *cloud_dev(sxyz, scov), Tt, Ts, True, 0, want_corr=True)
        om, ref = oracle_factor(txyz, tcov, res, sxyz, scov, Tt, Ts, True)
        np.testing.assert_array_equal(g["corr"].cpu().numpy(), ref["corr"])
        if ref["inliers"] == 0:
            assert g["err"].item() == 0.0 and not g["H"].any() and not g["b"].any()
        else:
            compare_factor(g, ref, TOL_FP64_ACC, f"n={n} res={res}")


def test_zero_inliers_and_sticky_error(V):
    rng = np.random.default_rng(200)
    txyz, tcov = tiny.cloud(rng, 500, extent=1.0)
    m = V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5)
    far = (txyz + 50).astype(np.float32)
    g = V.vgicp_linearize(m, *cloud_dev(far, tcov), np.eye(4), np.eye(4), True, 0)
    assert g["inliers"].item() == 0 and g["err"].item() == 0.0
    assert not g["H"].any() and not g["b"].any()
    V.vgicp_sync_status()
    bad = txyz.copy()
    bad[0, 3] = np.nan
    V.vgicp_linearize(m, *cloud_dev(bad, tcov), np.eye(4), np.eye(4), False, 0)
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_NONFINITE
    V.vgicp_sync_status()  # cleared
    with pytest.raises(V.VGICPError) as ei:
        T = np.eye(4)
        T[1, 3] = np.inf
        V.vgicp_linearize(m, *cloud_dev(txyz, tcov), np.eye(4), T, False, 0)
    assert ei.value.status == V.VGICP_E_NONFINITE


# ----------------------------------------------------------------------------- batches

def urban_batch(V, urban):
    maps, clouds, poses, factors = [], [cloud_dev(*urban["source"])], [urban["T_source"]], []
    for ki, res in urban["factors"]:
        maps.append(V.vgicp_build_voxelmap(*cloud_dev(*urban["targets"][ki]), res))
        poses.append(urban["T_targets"][ki])
        factors.append([len(maps) - 1, 0, len(poses) - 1, 0, 1])
    # a few unary factors too
    for ki in range(3):
        factors.append([3 * ki, 0, 1 + 3 * ki, 0, 0])
    return maps, clouds, np.array(poses), np.array(factors, np.int32)


def test_batched_matches_plain(V, urban):
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    b = V.Batch(maps, clouds, factors, P.shape[0])
    for prec in PRECS:
        out = b.linearize(P, prec)
        torch.cuda.synchronize()
        for f, (mi, ci, ti, si, bi) in enumerate(factors):
            g = V.vgicp_linearize(maps[mi], *clouds[ci], poses[ti], poses[si], bool(bi), prec)
            d = 12 if bi else 6
            Hb = out["H"][f].cpu().numpy()
            err = factor_errors(Hb[:d, :d], out["b"][f, :d].cpu().numpy(), out["err"][f].item(),
                                g["H"].cpu().numpy(), g["b"].cpu().numpy(), g["err"].item())
            # FP32 lane partials (forms 0-2) depend on how tiles split the points; FP64 math
            # differs only in the FP64 summation order
            tol = 1e-10 if prec == 3 else 1e-6
            assert max(err["H"], err["b"], err["e"]) < tol, (f, err)
            assert out["inliers"][f].item() == g["inliers"].item()
            if not bi:
                assert not np.any(Hb[6:, :]) and not np.any(Hb[:, 6:])
        V.vgicp_sync_status()


def test_batch_overlap_rates(V, urban):
    """Count-only mode: inlier counts equal the oracle's exactly, rates are inliers / n."""
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    b = V.Batch(maps, clouds, factors, P.shape[0])
    ov = b.overlap(P)
    ev = b.evaluate(P, 0)
    torch.cuda.synchronize()
    sxyz, scov = urban["source"]
    n = sxyz.shape[1]
    nin = ov["inliers"].cpu().numpy()
    assert np.array_equal(nin, ev["inliers"].cpu().numpy())
    for f, (mi, ci, ti, si, bi) in enumerate(factors):
        ki, res = urban["factors"][mi]
        om = oracle.VoxelMap(*urban["targets"][ki], res)
        ref = oracle.evaluate(om, sxyz, scov, poses[ti], poses[si])
        assert nin[f] == ref["inliers"], f
        assert ov["rates"][f].item() == ref["inliers"] / n
    V.vgicp_sync_status()


def test_batch_refresh_covariances(V, urban):
    """The batch reads its own (spatially ordered) copy of the clouds made at creation:
    changes are seen after refresh(), and then match a batch created from the changed
    clouds."""
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    b = V.Batch(maps, clouds, factors, P.shape[0])
    before = {k: v.clone() for k, v in b.linearize(P, 0).items()}
    for x, c in clouds:  # in place, on the caller's arrays
        c.mul_(1.5)
        x[0].add_(0.125)
    stale = b.linearize(P, 0)
    for k in before:
        assert torch.equal(stale[k], before[k]), k
    b.refresh()
    fresh = b.linearize(P, 0)
    ref = V.Batch(maps, clouds, factors, P.shape[0]).linearize(P, 0)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(fresh[k], ref[k]), k
    assert not torch.equal(fresh["H"], before["H"])
    for x, c in clouds:
        c.div_(1.5)
        x[0].sub_(0.125)


def test_batched_graph_replay_tracks_poses(V, urban):
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    b = V.Batch(maps, clouds, factors, P.shape[0])
    out = b.alloc_outputs()
    rng = np.random.default_rng(300)
    for it in range(3):
        b.linearize(P, 0, out=out)   # same pointers: graph replay after the first call
        torch.cuda.synchronize()
        host = P.cpu().numpy().reshape(-1, 12)
        for f in (0, 7, 23, 25):
            mi, ci, ti, si, bi = factors[f]
            ref = oracle.linearize(oracle.VoxelMap(*urban["targets"][urban["factors"][mi][0]],
                                                   urban["factors"][mi][1]),
                                   *urban["source"], host[ti], host[si], bool(bi))
            d = 12 if bi else 6
            err = factor_errors(out["H"][f].cpu().numpy()[:d, :d], out["b"][f, :d].cpu().numpy(),
                                out["err"][f].item(), ref["H"], ref["b"], ref["e"])
            assert max(err["H"], err["b"], err["e"]) <= TOL_FP64_ACC, (it, f, err)
            assert out["inliers"][f].item() == ref["inliers"]
        # move the source pose in place: the captured graph reads the new values
        Tn = se3.to12(se3.retract(host[0], rng.normal(size=6) * 0.01))
        P[0].copy_(dev(Tn))


def test_autotune_and_schedules(V, urban, tmp_path):
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    b = V.Batch(maps, clouds, factors, P.shape[0])
    ref = b.linearize(P, 0)
    ref = {k: v.clone() for k, v in ref.items()}
    cache = tmp_path / "tune.json"
    chosen = b.autotune(P, 0, cache_path=cache)
    assert chosen == b.get_schedule()
    assert json.loads(cache.read_text())
    for sched in [(256, 256, 1, 2), (512, 1024, 2, 8), (256, 8192, 8, 4), (512, 16384, 1, 4)]:
        b.set_schedule(*sched)
        out = b.linearize(P, 0)
        torch.cuda.synchronize()
        for f in range(len(factors)):
            d = 12 if factors[f][4] else 6
            err = factor_errors(out["H"][f].cpu().numpy()[:d, :d], out["b"][f, :d].cpu().numpy(),
                                out["err"][f].item(), ref["H"][f].cpu().numpy()[:d, :d],
                                ref["b"][f, :d].cpu().numpy(), ref["err"][f].item())
            assert max(err["H"], err["b"], err["e"]) < 1e-6  # FP32 lane partials regroup
        assert torch.equal(out["inliers"], ref["inliers"])
    b2 = V.Batch(maps, clouds, factors, P.shape[0])
    assert b2.autotune(P, 0, cache_path=cache) == chosen   # from the cache


def test_one_shot_batched_and_evaluate(V, urban):
    maps, clouds, poses, factors = urban_batch(V, urban)
    P = dev(poses.reshape(-1, 12))
    one = V.vgicp_linearize_batched(maps, clouds, P, factors, 0)
    b = V.Batch(maps, clouds, factors, P.shape[0])
    two = b.linearize(P, 0)
    ev = b.evaluate(P, 0)
    torch.cuda.synchronize()
    assert torch.equal(one["H"], two["H"]) and torch.equal(one["err"], two["err"])
    assert torch.equal(ev["inliers"], two["inliers"])
    assert torch.allclose(ev["err"], two["err"], rtol=1e-12, atol=0)


def test_batch_argument_errors(V, urban):
    maps, clouds, poses, factors = urban_batch(V, urban)
    bad = factors.copy()
    bad[0, 0] = 99
    with pytest.raises(V.VGICPError) as ei:
        V.Batch(maps, clouds, bad, len(poses))
    assert ei.value.status == V.VGICP_E_INVALID_ARG
    b = V.Batch(maps, clouds, factors, len(poses))
    for bad_sched in [(300, 1000, 2, 4), (256, 256 * 33, 2, 4), (256, 1024, 2, 3),
                      (256, 1024, 0, 4)]:
        with pytest.raises(V.VGICPError):
            b.set_schedule(*bad_sched)


def test_batch_empty_and_ragged_members(V):
    """A batch mixing empty, single-point and ragged source clouds (tile size + 1 included) with
    empty, single-voxel and ordinary maps in both layouts, unary and binary factors: every
    factor equal to the oracle, empty ones exactly zero."""
    rng = np.random.default_rng(300)
    txyz, tcov = tiny.cloud(rng, 6000, extent=3.0)
    one_xyz, one_cov = txyz[:, :1].copy(), tcov[:, :1].copy()
    e_xyz, e_cov = np.zeros((3, 0), np.float32), np.zeros((6, 0), np.float32)
    targets = [(txyz, tcov, 0.5, 2), (txyz, tcov, 0.5, 1), (e_xyz, e_cov, 0.5, 2),
               (e_xyz, e_cov, 0.5, 1), (one_xyz, one_cov, 0.25, 0)]
    sources = []
    for n in (0, 1, 257, 16385):
        sx = tiny.source_near(rng, txyz, n, noise=0.05) if n else e_xyz
        sc = tiny.plane_cov(rng, n).astype(np.float32) if n else e_cov
        sources.append((np.ascontiguousarray(sx, np.float32), np.ascontiguousarray(sc)))
    sources.append((one_xyz, one_cov))
    maps = [V.vgicp_build_voxelmap(*cloud_dev(x, c), res, layout=lay)
            for x, c, res, lay in targets]
    omaps = [oracle.VoxelMap(x, c, res) for x, c, res, _ in targets]
    clouds = [cloud_dev(x, c) for x, c in sources]
    poses = [se3.random_pose(rng, 0.2, 1.0)]
    poses.append(poses[0] @ se3.random_pose(rng, 0.02, 0.03))
    factors = []
    for mi in range(len(maps)):
        for ci in range(len(clouds)):
            factors.append([mi, ci, 0, 1, (mi + ci) % 2])
    factors = np.array(factors, np.int32)
    P = dev(np.array([se3.to12(T) for T in poses]))
    print(f"batch of {len(factors)} edge factors", flush=True)
    b = V.Batch(maps, clouds, factors, 2)
    for prec in (0, 3):
        out = b.linearize(P, prec)
        torch.cuda.synchronize()
        V.vgicp_sync_status()
        for f, (mi, ci, _, _, bi) in enumerate(factors):
            ref = oracle.linearize(omaps[mi], *sources[ci], poses[0], poses[1], bool(bi))
            assert out["inliers"][f].item() == ref["inliers"], (f, mi, ci)
            d = 12 if bi else 6
            H = out["H"][f].cpu().numpy()
            if ref["inliers"] == 0:
                assert out["err"][f].item() == 0.0 and not H.any() and not out["b"][f].any()
                continue
            err = factor_errors(H[:d, :d], out["b"][f, :d].cpu().numpy(), out["err"][f].item(),
                                ref["H"], ref["b"], ref["e"])
            assert max(err["H"], err["b"], err["e"]) <= TOL_FP64_ACC, (f, mi, ci, err)


def test_batch_skips_disjoint_pairs_exactly(V):
    """Factors whose source box, moved into the target frame, misses the target's voxels are
    skipped: their outputs are exact zeros, the others equal the oracle, and a source with a
    non-finite point is never skipped (its error is still reported)."""
    rng = np.random.default_rng(301)
    txyz, tcov = tiny.cloud(rng, 3000, extent=2.0)
    near = tiny.source_near(rng, txyz, 2000, noise=0.05).astype(np.float32)
    ncov = tiny.plane_cov(rng, 2000).astype(np.float32)
    maps = [V.vgicp_build_voxelmap(*cloud_dev(txyz, tcov), 0.5)]
    om = oracle.VoxelMap(txyz, tcov, 0.5)
    clouds = [cloud_dev(near, ncov)]
    T0 = np.eye(4)
    far = np.eye(4)
    far[0, 3] = 40.0   # the source 40 m away: disjoint
    edge = np.eye(4)
    edge[0, 3] = 2.9   # boxes touch within a voxel or so: must not be skipped wrongly
    poses = np.array([se3.to12(T) for T in (T0, far, edge)])
    factors = np.array([[0, 0, 0, 0, 1], [0, 0, 0, 1, 1], [0, 0, 0, 2, 0], [0, 0, 0, 1, 0]],
                       np.int32)
    b = V.Batch(maps, clouds, factors, 3)
    for count_only in (False, True):
        out = b.overlap(dev(poses)) if count_only else b.linearize(dev(poses))
        torch.cuda.synchronize()
        for f, (_, _, ti, si, bi) in enumerate(factors):
            Ts = [T0, far, edge][si]
            ref = oracle.linearize(om, near, ncov, T0, Ts, bool(bi))
            assert out["inliers"][f].item() == ref["inliers"], (f, count_only)
            if si == 1:
                assert ref["inliers"] == 0
                if not count_only:
                    assert out["err"][f].item() == 0.0 and not out["H"][f].any()
    assert out["inliers"][0].item() > 1000 and out["inliers"][2].item() > 0
    bad = near.copy()
    bad[0, 5] = np.nan
    b2 = V.Batch(maps, [cloud_dev(bad, ncov)], factors[1:2], 3)
    b2.linearize(dev(poses))
    with pytest.raises(V.VGICPError) as ei:
        V.vgicp_sync_status()
    assert ei.value.status == V.VGICP_E_NONFINITE


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_batch_nonpow2_resolution_and_wide_keys(V, prec):
    """Batched kernel on maps at a resolution that is not a power of two (0.3 m: the keys divide
    by res, and the pruning box uses 1/res), in the grid and the hash layout, next to a wide map
    whose keys need the 64-bit hash table: inlier counts exact and every factor within its bound
    against the oracle, in the linearization and the count-only mode; a factor 40 m away is
    skipped with exact zeros and one at the map's edge is not."""
    rng = np.random.default_rng(302)
    txyz, tcov = tiny.cloud(rng, 8000, extent=3.0)
    sxyz = tiny.source_near(rng, txyz, 5000, noise=0.05).astype(np.float32)
    scov = tiny.plane_cov(rng, 5000).astype(np.float32)
    wxyz, wcov = wide_scene(rng)
    wsx = tiny.source_near(rng, wxyz, 7000, noise=0.04).astype(np.float32)
    wsc = tiny.plane_cov(rng, 7000).astype(np.float32)
    targets = [(txyz, tcov, 0.3, V.VGICP_LAYOUT_GRID), (txyz, tcov, 0.3, V.VGICP_LAYOUT_HASH),
               (wxyz, wcov, 0.1, 0)]
    maps = [V.vgicp_build_voxelmap(*cloud_dev(x, c), res, layout=lay)
            for x, c, res, lay in targets]
    assert [m.layout for m in maps] == [V.VGICP_LAYOUT_GRID, V.VGICP_LAYOUT_HASH,
                                        V.VGICP_LAYOUT_HASH]
    omaps = [oracle.VoxelMap(x, c, res) for x, c, res, _ in targets]
    sources = [(sxyz, scov), (wsx, wsc)]
    clouds = [cloud_dev(x, c) for x, c in sources]
    T0 = se3.random_pose(rng, 0.2, 1.0)
    T1 = T0 @ se3.random_pose(rng, 0.01, 0.02)
    far = T1.copy()
    far[:3, 3] += T1[:3, :3] @ np.array([40.0, 0.0, 0.0])
    edge = T1.copy()
    edge[:3, 3] += T1[:3, :3] @ np.array([5.7, 0.0, 0.0])
    poses = [T0, T1, far, edge]
    factors = np.array([[0, 0, 0, 1, 1], [1, 0, 0, 1, 1], [0, 0, 0, 1, 0], [1, 0, 0, 1, 0],
                        [2, 1, 0, 1, 1], [2, 1, 0, 1, 0], [0, 0, 0, 2, 1], [1, 0, 0, 2, 0],
                        [0, 0, 0, 3, 1], [1, 0, 0, 3, 1]], np.int32)
    P = dev(np.array([se3.to12(T) for T in poses]))
    b = V.Batch(maps, clouds, factors, len(poses))
    out = b.linearize(P, prec)
    ov = b.overlap(P)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    for f, (mi, ci, ti, si, bi) in enumerate(factors):
        ref = oracle.linearize(omaps[mi], *sources[ci], poses[ti], poses[si], bool(bi))
        assert out["inliers"][f].item() == ref["inliers"], f
        assert ov["inliers"][f].item() == ref["inliers"], f
        if si == 2:
            assert ref["inliers"] == 0
            assert out["err"][f].item() == 0.0 and not out["H"][f].any()
            continue
        assert ref["inliers"] > (0 if si == 3 else 500), (f, ref["inliers"])
        d = 12 if bi else 6
        err = factor_errors(out["H"][f].cpu().numpy()[:d, :d], out["b"][f, :d].cpu().numpy(),
                            out["err"][f].item(), ref["H"], ref["b"], ref["e"])
        assert max(err["H"], err["b"], err["e"]) <= tol_for(prec), (f, err)
