"""GPU Levenberg-Marquardt step of a batch's pose graph against the oracle (oracle/lm.py).

* FP64-math form: the step, the new poses and both costs match the oracle's dense NumPy step;
* default form: the step within the error its FP32 Gauss-Newton terms allow;
* an idle pose (no factor) and the fixed pose do not move; two calls are bitwise equal;
* iterated with the usual lambda schedule, the GPU steps reach the truth like the oracle's;
* a 41-pose graph (40 submaps of the global loop, 690 binary factors, plus an idle pose): 246
  unknowns; FP64-math step against the oracle's dense solve with the banded solver (the default
  for this graph) and with the dense blocked Cholesky (four 64 x 64 blocks, so its panel
  products, trailing updates and multi-block triangular solves run), the two against each other;
* iterations decided on the device equal the same damping schedule run from the host.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import lm
from tests import se3
from tests.gpu_util import cloud_dev, dev
from tests.test_oracle_lm import odometry_graph, rot_err_deg, trans_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def V():
    import paper_2202_00242_amd.vgicp as V
    return V


@pytest.fixture(scope="module")
def graph():
    return odometry_graph()


def gpu_batch(V, g, extra_poses=0):
    clouds = [cloud_dev(x, c) for x, c in g["raw"]]
    maps = [V.vgicp_build_voxelmap(x, c, 0.5) for x, c in clouds]
    P = g["start"].shape[0] + extra_poses
    return V.Batch(maps, clouds, g["factors"], P)


def rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("lam", [1e-4, 1e-1])
def test_lm_step_fp64_matches_oracle(V, graph, lam):
    b = gpu_batch(V, graph)
    out = b.lm_step(dev(graph["start"]), V.VGICP_MATH_FP64, lam, fixed_pose=0)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    ref = lm.lm_step(graph["maps"], graph["clouds"], graph["start"], graph["factors"], lam, 0)
    d = out["delta"].cpu().numpy()
    c = out["cost"].cpu().numpy()
    print(f"lambda {lam}: delta rel err {rel(d, ref['delta']):.2e}, "
          f"cost {c} vs {ref['cost']}")
    assert rel(d, ref["delta"]) < 1e-8
    np.testing.assert_allclose(c, ref["cost"], rtol=1e-10)
    np.testing.assert_allclose(out["poses"].cpu().numpy(), ref["poses"], atol=1e-9)
    assert np.all(d[0] == 0.0)


def test_lm_step_default_form(V, graph):
    """FP32 terms perturb H and b by ~1e-6 (relative, the factor metric); the step moves by
    at most the conditioning of the damped system times that."""
    b = gpu_batch(V, graph)
    out = b.lm_step(dev(graph["start"]), V.VGICP_ACC_FP64, 1e-4, fixed_pose=0)
    torch.cuda.synchronize()
    ref = lm.lm_step(graph["maps"], graph["clouds"], graph["start"], graph["factors"], 1e-4, 0)
    A, _ = lm.damp(ref["H"], ref["b"], 1e-4, 0)
    Dh = np.sqrt(np.diag(A))
    cond = np.linalg.cond(A / Dh[:, None] / Dh[None, :])
    err = rel(out["delta"].cpu().numpy(), ref["delta"])
    print(f"default form: delta rel err {err:.2e}, scaled condition number {cond:.2e}")
    assert err < max(1e-4, 10 * cond * 2.3e-6)
    np.testing.assert_allclose(out["cost"].cpu().numpy(), ref["cost"], rtol=1e-5)


def test_lm_step_idle_pose_and_determinism(V, graph):
    b = gpu_batch(V, graph, extra_poses=1)
    P0 = np.concatenate([graph["start"], graph["start"][:1]])
    a = b.lm_step(dev(P0), V.VGICP_ACC_FP64, 1e-3, fixed_pose=2)
    c = b.lm_step(dev(P0), V.VGICP_ACC_FP64, 1e-3, fixed_pose=2)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], c[k]), k
    d = a["delta"].cpu().numpy()
    assert np.all(d[2] == 0.0) and np.all(d[-1] == 0.0)
    assert np.array_equal(a["poses"].cpu().numpy()[-1], P0[-1])
    assert np.array_equal(a["poses"].cpu().numpy()[2], P0[2])


def test_lm_iterations_reach_the_truth(V, graph):
    b = gpu_batch(V, graph)
    poses, lam = dev(graph["start"]), 1e-4
    first = None
    for _ in range(8):
        out = b.lm_step(poses, V.VGICP_ACC_FP64, lam, fixed_pose=0)
        c = out["cost"].cpu().numpy()
        first = c[0] if first is None else first
        if c[1] < c[0]:
            poses, lam = out["poses"].clone(), lam / 10
        else:
            lam *= 10
    V.vgicp_sync_status()
    p = poses.cpu().numpy()
    truth, start = graph["truth"], graph["start"]
    e0 = max(max(rot_err_deg(start[i], truth[i]), 10 * trans_err(start[i], truth[i]))
             for i in range(1, 9))
    e1 = max(max(rot_err_deg(p[i], truth[i]), 10 * trans_err(p[i], truth[i])) for i in range(1, 9))
    print(f"GPU LM: cost {first:.1f} -> {c[0]:.1f}; worst pose error {e0:.3f} -> {e1:.3f}")
    assert e1 < 0.25 * e0


@pytest.fixture(scope="module")
def band_graph():
    """40 submaps along the first straight of the global loop (~200 m): every pair within 50 m
    is a binary factor, so the system is block-banded (each pose linked to its ~20 nearest);
    pose 40 is idle (no factor) and pose 7 is held fixed."""
    data = synth.global_batch(n_submaps=40)
    poses = np.concatenate([data["T"], data["T"][:1]])
    maps = [oracle.VoxelMap(x, c, 0.5) for x, c in data["clouds"]]
    clouds = [oracle.Cloud.of(x, c) for x, c in data["clouds"]]
    return {"data": data, "poses": poses, "maps": maps, "clouds": clouds, "fixed": 7}


@pytest.fixture(scope="module")
def band_batch(V, band_graph):
    data = band_graph["data"]
    clouds = [cloud_dev(x, c) for x, c in data["clouds"]]
    maps = [V.vgicp_build_voxelmap(x, c, 0.5) for x, c in clouds]
    return V.Batch(maps, clouds, data["factors"], band_graph["poses"].shape[0])


@pytest.mark.parametrize("lam", [1e-4, 1e-1])
def test_lm_step_multiblock_fp64_matches_oracle(V, band_graph, band_batch, lam):
    g = band_graph
    P = g["poses"].shape[0]
    n = 6 * P
    assert P == 41 and -(-n // 64) >= 4  # four Cholesky blocks at least
    out = band_batch.lm_step(dev(g["poses"]), V.VGICP_MATH_FP64, lam, fixed_pose=g["fixed"])
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    ref = lm.lm_step(g["maps"], g["clouds"], g["poses"], g["data"]["factors"], lam, g["fixed"])
    d = out["delta"].cpu().numpy()
    c = out["cost"].cpu().numpy()
    print(f"lambda {lam}: {n} unknowns, delta rel err {rel(d, ref['delta']):.2e}, "
          f"cost {c} vs {ref['cost']}")
    assert rel(d, ref["delta"]) < 1e-8
    np.testing.assert_allclose(c, ref["cost"], rtol=1e-10)
    np.testing.assert_allclose(out["poses"].cpu().numpy(), ref["poses"], atol=1e-9)
    assert np.all(d[g["fixed"]] == 0.0) and np.all(d[-1] == 0.0)
    assert np.array_equal(out["poses"].cpu().numpy()[-1], g["poses"][-1])


def test_lm_step_multiblock_default_form(V, band_graph, band_batch):
    g = band_graph
    out = band_batch.lm_step(dev(g["poses"]), V.VGICP_ACC_FP64, 1e-4, fixed_pose=g["fixed"])
    torch.cuda.synchronize()
    ref = lm.lm_step(g["maps"], g["clouds"], g["poses"], g["data"]["factors"], 1e-4, g["fixed"])
    A, _ = lm.damp(ref["H"], ref["b"], 1e-4, g["fixed"])
    Dh = np.sqrt(np.diag(A))
    cond = np.linalg.cond(A / Dh[:, None] / Dh[None, :])
    err = rel(out["delta"].cpu().numpy(), ref["delta"])
    print(f"default form, 41 poses: delta rel err {err:.2e}, scaled condition {cond:.2e}")
    assert err < max(1e-4, 10 * cond * 2.3e-6)
    np.testing.assert_allclose(out["cost"].cpu().numpy(), ref["cost"], rtol=1e-5)


def test_lm_banded_and_dense_solvers_agree(V, band_graph, band_batch):
    """The banded solver (the 41-pose graph orders to a half-bandwidth of 65 unknowns), from
    both ends (15 blocks each, around an 11-block separator) and in one sweep, and the dense
    blocked Cholesky give the same step, all within the bound of the oracle's."""
    g = band_graph
    banded, w = band_batch.lm_info()
    assert banded == 2 and w == 6 * 10 + 5, (banded, w)
    P0 = dev(g["poses"])
    a = band_batch.lm_step(P0, V.VGICP_MATH_FP64, 1e-3, fixed_pose=g["fixed"])
    torch.cuda.synchronize()
    other = {}
    try:
        for solver, kind in ((2, 1), (1, 0)):
            band_batch.lm_solver(solver)
            assert band_batch.lm_info() == (kind, w)
            other[solver] = band_batch.lm_step(P0, V.VGICP_MATH_FP64, 1e-3, fixed_pose=g["fixed"])
            torch.cuda.synchronize()
    finally:
        band_batch.lm_solver(0)
    V.vgicp_sync_status()
    ref = lm.lm_step(g["maps"], g["clouds"], g["poses"], g["data"]["factors"], 1e-3, g["fixed"])
    da = a["delta"].cpu().numpy()
    d1, dd = other[2]["delta"].cpu().numpy(), other[1]["delta"].cpu().numpy()
    print(f"both ends vs one sweep {rel(da, d1):.2e}, vs dense {rel(da, dd):.2e}, vs oracle "
          f"{rel(da, ref['delta']):.2e}; one sweep vs oracle {rel(d1, ref['delta']):.2e}, "
          f"dense vs oracle {rel(dd, ref['delta']):.2e}")
    assert rel(da, d1) < 1e-9 and rel(da, dd) < 1e-9 and rel(d1, dd) < 1e-9
    for x in (da, d1, dd):
        assert rel(x, ref["delta"]) < 1e-8
    for o in other.values():  # the same linearization
        assert a["cost"][0].item() == o["cost"][0].item()


@pytest.mark.parametrize("fixed", [0, 20, 39])
def test_lm_step_fixed_pose_anywhere_in_the_split(V, band_graph, band_batch, fixed):
    """The fixed pose's unit diagonal lands in the top end, the separator or the reversed bottom
    end depending on its position in the pose order: the step from both ends equals the
    oracle's for fixed poses spread over the graph (the idle pose 40 stays put)."""
    g = band_graph
    assert band_batch.lm_info()[0] == 2
    out = band_batch.lm_step(dev(g["poses"]), V.VGICP_MATH_FP64, 1e-3, fixed_pose=fixed)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    ref = lm.lm_step(g["maps"], g["clouds"], g["poses"], g["data"]["factors"], 1e-3, fixed)
    d = out["delta"].cpu().numpy()
    print(f"fixed pose {fixed}: delta rel err {rel(d, ref['delta']):.2e}")
    assert rel(d, ref["delta"]) < 1e-8
    assert np.all(d[fixed] == 0.0) and np.all(d[-1] == 0.0)


@pytest.mark.parametrize("n_submaps", [24, 28, 32])
def test_lm_split_at_small_ends(V, n_submaps):
    """Short graphs along the first straight: ends of a few blocks around the separator (or one
    sweep below the threshold of 8 blocks per end). The automatic solver, one sweep and the
    dense solver give the oracle's step."""
    data = synth.global_batch(n_submaps=n_submaps)
    maps_o = [oracle.VoxelMap(x, c, 0.5) for x, c in data["clouds"]]
    clouds_o = [oracle.Cloud.of(x, c) for x, c in data["clouds"]]
    clouds = [cloud_dev(x, c) for x, c in data["clouds"]]
    maps = [V.vgicp_build_voxelmap(x, c, 0.5) for x, c in clouds]
    b = V.Batch(maps, clouds, data["factors"], n_submaps)
    P0 = dev(data["T"])
    kind, w = b.lm_info()
    steps = {}
    try:
        for solver in (0, 2, 1):
            b.lm_solver(solver)
            steps[solver] = b.lm_step(P0, V.VGICP_MATH_FP64, 1e-3, fixed_pose=0)["delta"]
            torch.cuda.synchronize()
    finally:
        b.lm_solver(0)
    V.vgicp_sync_status()
    ref = lm.lm_step(maps_o, clouds_o, data["T"], data["factors"], 1e-3, 0)
    ns = (w + 1) // 6
    print(f"{n_submaps} poses, half-bandwidth {w}: solver form {kind}, "
          f"{n_submaps - ns} blocks outside the separator; errors "
          + ", ".join(f"{k}: {rel(v.cpu().numpy(), ref['delta']):.2e}" for k, v in steps.items()))
    assert kind == (2 if n_submaps - ns >= 16 else 1)
    for v in steps.values():
        assert rel(v.cpu().numpy(), ref["delta"]) < 1e-8


def sparse_damped_system(factors, H_f, b_f, P, lam, fixed):
    """oracle/lm.py's assemble and damp, in sparse form (for systems too large for dense
    NumPy): per-factor [source | target] blocks summed, H + lam diag H, identity rows and
    columns for the fixed pose and zero diagonals, right-hand side -b."""
    import scipy.sparse as sp
    n = 6 * P
    rows, cols, vals = [], [], []
    b = np.zeros(n)
    r6 = np.repeat(np.arange(6), 6)
    c6 = np.tile(np.arange(6), 6)
    for f, (_, _, tp, spose, binary) in enumerate(np.asarray(factors)):
        s, t = 6 * int(spose), 6 * int(tp)
        pairs = [(s, s, H_f[f, :6, :6])]
        b[s:s + 6] += b_f[f, :6]
        if binary:
            pairs += [(s, t, H_f[f, :6, 6:]), (t, s, H_f[f, 6:, :6]), (t, t, H_f[f, 6:, 6:])]
            b[t:t + 6] += b_f[f, 6:]
        for r0, c0, blk in pairs:
            rows.append(r0 + r6)
            cols.append(c0 + c6)
            vals.append(blk.reshape(-1))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    d = H.diagonal()
    idle = ~(d > 0.0)
    if fixed >= 0:
        idle[6 * fixed:6 * fixed + 6] = True
    keep = sp.diags((~idle).astype(float))
    A = keep @ H @ keep + sp.diags(np.where(idle, 1.0, lam * d))
    g = np.where(idle, 0.0, -b)
    return A.tocsr(), g


def test_lm_long_chain_beyond_one_sweep(V):
    """4,000 poses in a chain, each linked to its 4 successors (half-bandwidth 29 unknowns): one
    sweep would need 6P + 18 (w + 1) <= 18,221 values of LDS, so only the solve from both ends
    (two ends of ~2,000 poses) keeps the system banded. The step solves the damped system that
    the batch's own linearization gives (residual, with the system assembled in sparse form as
    the oracle does), and equals the dense solver's step. Every factor matches a 3,000-point
    cloud against the voxel map of the full cloud it was taken from, at poses near identity."""
    data = synth.global_batch(n_submaps=24)
    x, c = data["clouds"][0]
    sub = slice(0, None, max(1, x.shape[1] // 3000))
    xs, cs = np.ascontiguousarray(x[:, sub]), np.ascontiguousarray(c[:, sub])
    P, k, lam = 4000, 4, 1e-3
    factors = np.array([(0, 0, a, a + d, 1) for a in range(P) for d in range(1, k + 1)
                        if a + d < P], dtype=np.int32)
    rng = np.random.default_rng(11)
    poses = np.stack([se3.random_pose(rng, 0.01, 0.05)[:3].reshape(12) for _ in range(P)])
    mx, mc = cloud_dev(x, c)
    m = V.vgicp_build_voxelmap(mx, mc, 0.5)
    b = V.Batch([m], [cloud_dev(xs, cs)], factors, P)
    kind, w = b.lm_info()
    assert kind == 2 and w == 6 * k + 5, (kind, w)
    assert 6 * P + 18 * (w + 1) > 18221  # beyond one sweep
    P0 = dev(poses)
    step = b.lm_step(P0, V.VGICP_MATH_FP64, lam, fixed_pose=0)
    lin = b.linearize(P0, V.VGICP_MATH_FP64)
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    A, g = sparse_damped_system(factors, lin["H"].cpu().numpy(), lin["b"].cpu().numpy(), P,
                                lam, 0)
    delta = step["delta"].cpu().numpy().reshape(-1)
    res = np.abs(A @ delta - g).max() / np.abs(g).max()
    b.lm_solver(1)
    try:
        assert b.lm_info()[0] == 0
        dense = b.lm_step(P0, V.VGICP_MATH_FP64, lam, fixed_pose=0)["delta"].cpu().numpy()
        b.lm_solver(2)  # one sweep does not fit: dense again
        assert b.lm_info()[0] == 0
    finally:
        b.lm_solver(0)
    V.vgicp_sync_status()
    print(f"{P} poses, w {w}: residual {res:.2e}, both ends vs dense "
          f"{rel(delta.reshape(P, 6), dense):.2e}, inliers per factor "
          f"{lin['inliers'].float().mean().item():.0f}")
    assert res < 1e-10
    assert rel(delta.reshape(P, 6), dense) < 1e-9
    assert np.all(delta[:6] == 0.0)


def test_lm_iterate_equals_host_schedule(V, band_graph, band_batch):
    """Iterations decided on the device (one linearization per iteration, the current poses'
    linearization reused) give bitwise the poses, damping and costs of the same schedule run from
    the host with one full step per iteration."""
    g = band_graph
    iters = 5
    poses = dev(g["poses"])
    lam = 1e-4
    costs = []
    for _ in range(iters):
        out = band_batch.lm_step(poses, V.VGICP_ACC_FP64, lam, fixed_pose=g["fixed"])
        c = out["cost"].cpu().numpy()
        if not costs:
            costs.append(c[0])
        if np.isfinite(c[1]) and c[1] < c[0]:
            poses, lam = out["poses"].clone(), min(max(lam * 0.1, 1e-12), 1e12)
            costs.append(c[1])
        else:
            lam = min(max(lam * 10.0, 1e-12), 1e12)
            costs.append(c[0])
    P = dev(g["poses"])
    lt = torch.tensor([1e-4], dtype=torch.float64, device="cuda")
    dc = band_batch.lm_iterate(P, lt, iters, V.VGICP_ACC_FP64, fixed_pose=g["fixed"])
    torch.cuda.synchronize()
    V.vgicp_sync_status()
    print(f"device iterations: costs {dc.cpu().numpy()}, lambda {lt.item():.1e}")
    assert torch.equal(P, poses)
    assert lt.item() == lam
    np.testing.assert_array_equal(dc.cpu().numpy(), np.array(costs))
    assert dc[-1] < dc[0]


def test_lm_iterate_reaches_the_truth(V, graph):
    b = gpu_batch(V, graph)
    P = dev(graph["start"])
    lt = torch.tensor([1e-4], dtype=torch.float64, device="cuda")
    c = b.lm_iterate(P, lt, 8, V.VGICP_ACC_FP64, fixed_pose=0).cpu().numpy()
    V.vgicp_sync_status()
    p = P.cpu().numpy()
    truth, start = graph["truth"], graph["start"]
    e0 = max(max(rot_err_deg(start[i], truth[i]), 10 * trans_err(start[i], truth[i]))
             for i in range(1, 9))
    e1 = max(max(rot_err_deg(p[i], truth[i]), 10 * trans_err(p[i], truth[i])) for i in range(1, 9))
    print(f"device LM: cost {c[0]:.1f} -> {c[-1]:.1f}; worst pose error {e0:.3f} -> {e1:.3f}")
    assert np.all(np.diff(c) <= 0) and e1 < 0.25 * e0
