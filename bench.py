"""Benchmark: batched VGICP factor linearization of one global-mapping LM iteration on one
MI355X, against the per-factor (plain) launch loop and the FP64 CPU oracle.

Workload (the global-mapping batch): 400 submaps of 10 consecutive 32-beam scans along a 2 km
loop, 10k-120k points each (log-uniform), voxel maps at 0.5 m, one binary factor for every
ordered pair of submaps whose origins lie within 50 m (~8,000 factors, ~3.5e8 source-point
linearizations per iteration). Inputs are synthetic and seeded (synth.global_batch) and are
resident in HBM before the timed region. A step is one linearization of every factor (graph
replay of the persistent kernel) at FP32 per-point math with FP64 accumulation.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "VGICP point linearizations/sec (batched vs plain) at H,b rel err ≤1e-4 vs FP64"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_kernel_global_traffic.json")
KERNEL_SOURCES = ["paper_2202_00242_amd/csrc/kernels.hip", "paper_2202_00242_amd/csrc/device_math.h",
                  "paper_2202_00242_amd/csrc/common.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_source_hash():
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_source_sha1") == kernel_source_hash():
            return t.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


class OracleSide:
    """The FP64 oracle over the same factors: voxel maps built once (untimed), then timed
    linearization of a bounded sample (the CPU baseline) whose results also check the GPU."""

    def __init__(self, data, res=0.5):
        import oracle

        self.data = data
        t0 = time.perf_counter()
        self.maps = [oracle.VoxelMap(x, c, res) for x, c in data["clouds"]]
        self.clouds = [oracle.Cloud.of(x, c) for x, c in data["clouds"]]
        self.build_s = time.perf_counter() - t0
        self.threads = oracle.max_threads()

    def run(self, idx, threads=None):
        import oracle

        return oracle.linearize_factors(self.maps, self.clouds, self.data["T"],
                                        self.data["factors"][idx],
                                        nthreads=threads or self.threads)

    def single_thread(self, budget_s=3.0):
        """The oracle on one host thread over a random sample of about budget_s seconds."""
        factors = self.data["factors"]
        n_of = np.array([self.clouds[int(f[1])].n for f in factors], np.int64)
        order = np.random.default_rng(8).permutation(len(factors))
        t0 = time.perf_counter()
        self.run(np.sort(order[:2]), threads=1)
        rate = n_of[order[:2]].sum() / (time.perf_counter() - t0)
        k = int(np.searchsorted(np.cumsum(n_of[order]), rate * budget_s)) + 1
        sample = np.sort(order[:min(k, len(order))])
        t0 = time.perf_counter()
        self.run(sample, threads=1)
        dt = time.perf_counter() - t0
        pts = int(n_of[sample].sum())
        return {"value": pts / dt, "unit": "points/s", "cores": 1,
                "sample": f"{len(sample)} random factors ({pts} source points) in {dt:.1f} s"}

    def baseline(self, budget_s):
        factors = self.data["factors"]
        n_of = np.array([self.clouds[int(f[1])].n for f in factors], np.int64)
        order = np.random.default_rng(7).permutation(len(factors))
        probe = np.sort(order[:max(2 * self.threads, 16)])
        t0 = time.perf_counter()
        self.run(probe)
        rate = n_of[probe].sum() / (time.perf_counter() - t0)
        want = rate * budget_s
        k = int(np.searchsorted(np.cumsum(n_of[order]), want)) + 1
        sample = np.sort(order[:min(k, len(order))])
        pts = int(n_of[sample].sum())
        t0 = time.perf_counter()
        ref = self.run(sample)
        passes = 1
        if k >= len(order):  # the whole batch takes less than the budget: repeat it
            t1 = time.perf_counter() - t0
            for _ in range(max(0, int(round(budget_s / t1)) - 1)):
                self.run(sample)
                passes += 1
        dt = time.perf_counter() - t0
        reps = f" x {passes} passes" if passes > 1 else ""
        info = {"value": passes * pts / dt, "unit": "points/s", "cores": self.threads,
                "kind": "oracle",
                "sample": f"{len(sample)} of {len(factors)} factors ({pts} source points){reps} "
                          f"in {dt:.1f} s; FP64, OpenMP over factors; voxel maps built "
                          f"beforehand ({self.build_s:.1f} s)"}
        return info, sample, ref


def factor_error_stats(out, ref, idx):
    """Per-factor max of (eps_H, eps_b, eps_e) of GPU outputs against oracle results."""
    from tests.metrics import factor_errors

    H = out["H"].cpu().numpy()[idx]
    b = out["b"].cpu().numpy()[idx]
    e = out["err"].cpu().numpy()[idx]
    nin = out["inliers"].cpu().numpy()[idx]
    errs = np.array([max(v for k, v in factor_errors(H[i], b[i], e[i], ref["H"][i], ref["b"][i],
                                                      ref["e"][i]).items() if k != "H_fro")
                     for i in range(len(idx))])
    return {"factors": int(len(idx)), "max_rel_err": float(errs.max()),
            "median_rel_err": float(np.median(errs)),
            "inlier_mismatch_factors": int(np.sum(nin != ref["inliers"])),
            "inlier_count_diff": int(np.abs(nin - ref["inliers"]).sum())}


def overlap_leg(V, data, maps, clouds, P, stream, orc):
    """The overlap-rate matrix of the submaps (every ordered pair, count-only kernel) at the
    same poses; inlier counts of a random sample of pairs checked against the oracle."""
    import torch

    S = len(clouds)
    ii, jj = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    keep = ii != jj
    src, tgt = ii[keep], jj[keep]
    pairs = np.stack([tgt, src, tgt, src, np.ones_like(src)], 1).astype(np.int32)
    t0 = time.perf_counter()
    ob = V.Batch(maps, clouds, pairs, P.shape[0])
    setup_s = time.perf_counter() - t0
    n_pts = int(sum(clouds[int(s_)][0].shape[1] for s_ in src))
    with torch.cuda.stream(stream):
        ov = ob.overlap(P)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            ov = ob.overlap(P)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    rates = ov["rates"].cpu().numpy()
    nin = ov["inliers"].cpu().numpy()
    out = {"pairs": int(len(pairs)), "ms": round(dt * 1e3, 3),
           "pairs_per_s": len(pairs) / dt, "points_per_s": n_pts / dt,
           "points": n_pts, "pairs_above_5pct": int((rates > 0.05).sum()),
           "batch_setup_s": round(setup_s, 2),
           "form": "count-only batched kernel over all ordered submap pairs"}
    if orc is not None:
        idx = np.sort(np.random.default_rng(9).choice(len(pairs), 300, replace=False))
        import oracle
        ref = oracle.linearize_factors(orc.maps, orc.clouds, orc.data["T"], pairs[idx],
                                       nthreads=orc.threads)
        out["vs_oracle"] = {"pairs": int(len(idx)),
                            "inlier_mismatch_pairs": int(np.sum(nin[idx] != ref["inliers"]))}
    del ob
    log(f"[bench] overlap matrix: {len(pairs)} pairs in {dt * 1e3:.2f} ms, "
        f"{(rates > 0.05).sum()} pairs above 5%")
    return out


def lm_leg(V, data, batch, P, prec, stream, orc, lam=1e-4):
    """One Levenberg-Marquardt step of the global graph (400 poses, pose 0 fixed): linearize,
    assemble, dense Cholesky solve, retract, evaluate; step and costs against the oracle."""
    import torch
    from oracle import lm

    with torch.cuda.stream(stream):
        out = batch.lm_step(P, prec, lam, fixed_pose=0)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(5)]
        for a, b in ev:
            a.record(stream)
            out = batch.lm_step(P, prec, lam, fixed_pose=0)
            b.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    d = out["delta"].cpu().numpy()
    c = out["cost"].cpu().numpy()
    res = {"ms": round(ms, 3), "poses": int(P.shape[0]), "unknowns": 6 * int(P.shape[0]),
           "lambda": lam, "cost_before": float(c[0]), "cost_after": float(c[1]),
           "form": "linearize + deterministic block assembly + dense FP64 Cholesky + "
                   "retraction + evaluation, all on the GPU"}
    t0 = time.perf_counter()
    ref = lm.lm_step(orc.maps, orc.clouds, data["T"], data["factors"], lam, 0, orc.threads)
    res["oracle_s"] = round(time.perf_counter() - t0, 2)
    res["vs_oracle"] = {
        "delta_max_rel_err": float(np.max(np.abs(d - ref["delta"])) / np.max(np.abs(ref["delta"]))),
        "cost_after_rel_err": float(abs(c[1] - ref["cost"][1]) / ref["cost"][1])}
    log(f"[bench] LM step: {ms:.2f} ms, cost {c[0]:.4g} -> {c[1]:.4g}, {res['vs_oracle']}")
    return res


def preprocess_leg(V, stream, orc):
    """Preprocessing of one raw sweep on the GPU (urban scene, 32 beams x 1,800 columns, ~53k
    hits with timestamps): voxel-grid filter at 0.25 m with the sweep-seam split, k = 10
    neighbours, plane-regularized covariances. Each call synchronises; median of 20 calls."""
    import torch
    import synth

    xyz, t = synth.raw_scan(0)
    c, s_ = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
    xyz = np.ascontiguousarray((R @ xyz.astype(np.float64)).astype(np.float32))
    dx, dt_ = torch.from_numpy(xyz).cuda(), torch.from_numpy(t).cuda()
    times = {"downsample": [], "knn": [], "covariances": []}
    with torch.cuda.stream(stream):
        for rep in range(23):
            t0 = time.perf_counter()
            ds, _ = V.vgicp_downsample(dx, 0.25, dt_, synth.SCAN_PERIOD, stream=stream)
            t1 = time.perf_counter()
            nbr = V.vgicp_knn(ds, 10, stream=stream)
            t2 = time.perf_counter()
            cov = V.vgicp_point_covariances(ds, nbr, stream=stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if rep >= 3:
                times["downsample"].append(t1 - t0)
                times["knn"].append(t2 - t1)
                times["covariances"].append(t3 - t2)
    V.vgicp_sync_status(stream)
    ms = {k: round(float(np.median(v)) * 1e3, 3) for k, v in times.items()}
    total = sum(ms.values())
    out = {"raw_points": int(xyz.shape[1]), "downsampled_points": int(ds.shape[1]),
           "ms": ms, "ms_per_sweep": round(total, 3), "sweeps_per_s": round(1e3 / total, 1),
           "form": "voxel-grid filter 0.25 m with timestamps + exact 10-NN + plane-regularized "
                   "covariances, all on the GPU (each call synchronises)"}
    if orc is not None:
        from oracle import preprocess as pp
        t0 = time.perf_counter()
        rx, _, _, _ = pp.downsample(xyz, 0.25, t, synth.SCAN_PERIOD)
        t_ds = time.perf_counter() - t0
        pts = ds.cpu().numpy()
        rows = np.sort(np.random.default_rng(5).choice(pts.shape[1], 1000, replace=False))
        t0 = time.perf_counter()
        rn = pp.knn(pts, 10, rows=rows)
        t_knn = (time.perf_counter() - t0) * pts.shape[1] / len(rows)
        nb = nbr.cpu().numpy()
        t0 = time.perf_counter()
        rc = pp.covariances(pts, nb)
        t_cov = time.perf_counter() - t0
        _, lam, _, _ = pp.normals(pts, nb)
        good = (lam[:, 1] - lam[:, 0]) / np.maximum(lam[:, 2], 1e-300) > 1e-6
        out["oracle_s"] = {"downsample": round(t_ds, 3), "knn_estimated_full": round(t_knn, 2),
                           "covariances": round(t_cov, 3),
                           "note": "NumPy oracle, brute-force neighbours timed on 1,000 "
                                   "sampled points and scaled to the sweep"}
        out["vs_oracle"] = {
            "downsample_bitwise_equal": bool(rx.shape == pts.shape and np.array_equal(rx, pts)),
            "knn_rows_checked": int(len(rows)),
            "knn_mismatch_rows": int(np.sum(np.any(nb[:, rows] != rn, axis=0))),
            "cov_max_abs_err_over_scale": float(np.abs(cov.cpu().numpy() - rc)[:, good].max()
                                                / 0.01)}
    log(f"[bench] preprocess: {ms} ms per sweep ({xyz.shape[1]} -> {ds.shape[1]} points)")
    return out


def imu_leg(V, stream, orc):
    """IMU factors of a 400 s trajectory at 10 Hz (4,000 factors of 20 samples at 200 Hz):
    batched preintegration with the noise covariance, then the Gauss-Newton blocks of every
    factor at perturbed states; a sample of factors against the oracle."""
    import torch
    from oracle import imu as oimu

    rng = np.random.default_rng(11)
    F, m = 4000, 20
    rows = np.zeros((F * m, 7))
    rows[:, :3] = rng.normal(size=(F * m, 3)) * 0.3
    rows[:, 3:6] = rng.normal(size=(F * m, 3)) * 1.0 + np.array([0.0, 0.0, 9.8])
    rows[:, 6] = 0.005
    seg = (np.arange(F + 1) * m).astype(np.int64)
    bias = rng.normal(size=(F, 6)) * 0.01
    poses = np.zeros((F + 1, 3, 4))
    for p_ in range(F + 1):
        w = rng.normal(size=3) * 0.5
        th = np.linalg.norm(w)
        K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) / th
        poses[p_, :, :3] = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
        poses[p_, :, 3] = rng.normal(size=3) * 10
    vels = rng.normal(size=(F + 1, 3))
    states = np.stack([np.arange(F), np.arange(1, F + 1)], 1).astype(np.int32)
    g = np.array([0.0, 0.0, -9.80665])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    drows, dseg, dbias, dst = d(rows), d(seg), d(bias), d(states)
    dpo, dve = d(poses.reshape(F + 1, 12)), d(vels)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(13)]
    with torch.cuda.stream(stream):
        for a, b, c in ev:
            a.record(stream)
            pre, cov = V.vgicp_imu_preintegrate(drows, dseg, dbias, 1.7e-3, 2e-2, stream=stream)
            b.record(stream)
            out = V.vgicp_imu_linearize(pre, cov, dst, dpo, dve, g, stream=stream)
            c.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    t_pre = float(np.median([a.elapsed_time(b) for a, b, _ in ev[3:]]))
    t_lin = float(np.median([b.elapsed_time(c) for _, b, c in ev[3:]]))
    res = {"factors": F, "samples_per_factor": m, "ms": {"preintegrate": round(t_pre, 4),
           "linearize": round(t_lin, 4)}, "factors_per_s": round(F / ((t_pre + t_lin) * 1e-3)),
           "form": "one thread per factor, FP64: preintegration + 9x9 noise covariance, "
                   "residual, Cholesky-whitened 18x18 blocks"}
    idx = np.linspace(0, F - 1, 40).astype(int)
    H, b_, e = out["H"].cpu().numpy(), out["b"].cpu().numpy(), out["err"].cpu().numpy()
    worst = 0.0
    t0 = time.perf_counter()
    for f in idx:
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], bias[f], 1.7e-3, 2e-2)
        lin = oimu.linearize(ref, poses[f], vels[f], poses[f + 1], vels[f + 1], g)
        dd = np.sqrt(np.diag(lin["H"]))
        worst = max(worst, np.max(np.abs(H[f] - lin["H"]) / np.outer(dd, dd)),
                    np.max(np.abs(b_[f] - lin["b"]) / (dd * np.sqrt(lin["e"]))),
                    abs(e[f] - lin["e"]) / lin["e"])
    res["oracle_s_per_factor"] = round((time.perf_counter() - t0) / len(idx), 5)
    res["vs_oracle"] = {"factors": int(len(idx)), "max_rel_err": float(worst)}
    log(f"[bench] IMU factors: {F} in {t_pre:.3f} + {t_lin:.3f} ms, vs oracle {worst:.2e}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="global", choices=["global", "precision"],
                    help="global: the loop near the world origin; precision: the same loop "
                         "4.3-5.0 km away (points stay submap-local FP32)")
    ap.add_argument("--submaps", type=int, default=400)
    ap.add_argument("--precision", default="acc_fp64",
                    choices=["acc_fp64", "kahan_fp32", "naive_world_fp32", "math_fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-overlap", action="store_true")
    ap.add_argument("--no-lm", action="store_true")
    ap.add_argument("--no-preprocess", action="store_true")
    ap.add_argument("--no-imu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB) after the "
                         "timed region, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the factor batch is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2202_00242_amd.vgicp as V

    prec = V.PRECISIONS[args.precision]
    t0 = time.perf_counter()
    make = synth.global_batch if args.workload == "global" else synth.precision_batch
    data = make(n_submaps=args.submaps)
    log(f"[bench] workload ready in {time.perf_counter() - t0:.1f} s: {len(data['clouds'])} "
        f"submaps, {len(data['factors'])} factors")
    dev = torch.device("cuda:0")
    clouds = [(torch.from_numpy(x).to(dev), torch.from_numpy(c).to(dev)) for x, c in data["clouds"]]
    P = torch.from_numpy(np.ascontiguousarray(data["T"])).to(dev)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    maps = [V.vgicp_build_voxelmap(x, c, 0.5) for x, c in clouds]
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    factors = data["factors"]
    F = len(factors)
    n_src = np.array([clouds[int(f[1])][0].shape[1] for f in factors], np.int64)
    total_points = int(n_src.sum())
    # voxels of every distinct target map of the batch (each is read from HBM once per
    # launch; its ~20 factors find it in L2 / Infinity Cache)
    vox = np.array([maps[t].size()[0] for t in np.unique(factors[:, 0])], np.int64)
    log(f"[bench] voxel maps built in {build_ms:.0f} ms; {total_points} source points per step")

    stream = torch.cuda.Stream()
    batch = V.Batch(maps, clouds, factors, P.shape[0])
    with torch.cuda.stream(stream):
        sched = batch.autotune(P, prec, cache_path=args.tune_cache)
        log(f"[bench] schedule (block, tile, blocks/CU, lookahead) = {sched}")
        out = batch.alloc_outputs()
        for _ in range(args.warmup):
            batch.linearize(P, prec, out=out)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            batch.linearize(P, prec, out=out)
            b.record(stream)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
    V.vgicp_sync_status(stream)
    wall = t_end - t_start
    ms_per_step = wall / args.steps * 1e3
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    value = total_points * args.steps / wall
    log(f"[bench] batched: {ms_per_step:.3f} ms/step wall, {launch_ms:.3f} ms/launch (events), "
        f"{value / 1e9:.1f} G points/s")

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 1 GiB read + 1 GiB written by one elementwise kernel")

    # algorithmic bytes per launch: every source point's position (12 B), every inlier's
    # covariance (24 B: a point outside every voxel needs none), every target map's voxel table
    # once (72 B per voxel), the outputs (736 B per binary factor). The 36 B-per-point count
    # (every covariance read) is reported beside it.
    n_inliers = int(out["inliers"].sum().item())
    alg_bytes = 12 * total_points + 24 * n_inliers + 72 * int(vox.sum()) + 736 * F
    alg_all_cov = 36 * total_points + 72 * int(vox.sum()) + 736 * F
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(),
                "kernel": "batch_kernel (graph: pose prep + persistent kernel + finalize)",
                "alg_bytes_per_launch": alg_bytes, "inliers_per_launch": n_inliers,
                "alg_bytes_every_covariance": alg_all_cov,
                "frac_every_covariance": round(alg_all_cov / (launch_ms * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4)}

    # the oracle on the host: CPU baseline, and the check of the timed outputs
    cpu = None
    ref_idx, ref = None, None
    if not args.no_cpu_baseline:
        orc = OracleSide(data)
        cpu, ref_idx, ref = orc.baseline(args.cpu_budget)
        cpu["cpu_model"] = cpu_model()
        cpu["single_thread"] = orc.single_thread()
        log(f"[bench] cpu baseline {cpu['value'] / 1e6:.1f} M points/s on {cpu['cores']} threads "
            f"({cpu['sample']})")
    if ref is None:
        orc = OracleSide(data)
        ref_idx = np.linspace(0, F - 1, 64).astype(int)
        ref = orc.run(ref_idx)
    parity = factor_error_stats(out, ref, ref_idx)
    log(f"[bench] parity of the timed outputs against the oracle: {parity}")

    extra = {}
    if not args.no_plain:
        # plain form: one launch pair per factor, from the host, FP64-accumulation form
        host_T = data["T"]
        outs = [{"H": torch.empty((12, 12), dtype=torch.float64, device=dev),
                 "b": torch.empty(12, dtype=torch.float64, device=dev),
                 "err": torch.empty(1, dtype=torch.float64, device=dev),
                 "inliers": torch.empty(1, dtype=torch.int64, device=dev), "corr": None}
                for _ in range(F)]
        pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(F)]
        with torch.cuda.stream(stream):
            for rep in range(2):
                torch.cuda.synchronize()
                tp = time.perf_counter()
                for f in range(F):
                    m, c, t, s_, bi = (int(x) for x in factors[f])
                    pe[f][0].record(stream)
                    V.vgicp_linearize(maps[m], *clouds[c], host_T[t], host_T[s_], bool(bi),
                                      V.VGICP_ACC_FP64, stream=stream, out=outs[f])
                    pe[f][1].record(stream)
                torch.cuda.synchronize()
                plain_s = time.perf_counter() - tp
        gpu_ms = float(sum(a.elapsed_time(b) for a, b in pe))
        extra["plain"] = {"value": total_points / plain_s, "ms_per_step": round(plain_s * 1e3, 2),
                          "gpu_busy_ms": round(gpu_ms, 2),
                          "value_gpu_busy": total_points / (gpu_ms * 1e-3),
                          "form": "per-factor launch loop from the host (vgicp_linearize), "
                                  "acc_fp64; gpu_busy_ms sums HIP-event time per factor"}
        extra["speedup_batched_vs_plain"] = round(value / (total_points / plain_s), 2)
        extra["speedup_batched_vs_plain_gpu_busy"] = round(gpu_ms / launch_ms, 2)
        log(f"[bench] plain loop: {plain_s * 1e3:.1f} ms/step wall, {gpu_ms:.1f} ms GPU busy")
    if not args.no_overlap:
        extra["overlap"] = overlap_leg(V, data, maps, clouds, P, stream, orc)
    if not args.no_lm:
        extra["lm_step"] = lm_leg(V, data, batch, P, prec, stream, orc)
    if not args.no_preprocess:
        extra["preprocess"] = preprocess_leg(V, stream, orc)
    if not args.no_imu:
        extra["imu"] = imu_leg(V, stream, orc)
    if not args.no_forms:
        forms = {}
        for name in ("acc_fp64", "kahan_fp32", "math_fp64", "naive_world_fp32"):
            p = V.PRECISIONS[name]
            with torch.cuda.stream(stream):
                sc = batch.autotune(P, p, cache_path=args.tune_cache)
                o2 = batch.alloc_outputs()
                batch.linearize(P, p, out=o2)
                torch.cuda.synchronize()
                tf = time.perf_counter()
                for _ in range(5):
                    batch.linearize(P, p, out=o2)
                torch.cuda.synchronize()
                dtf = (time.perf_counter() - tf) / 5
            st = factor_error_stats(o2, ref, ref_idx)
            forms[name] = {"value": total_points / dtf, "ms_per_step": round(dtf * 1e3, 3),
                           "schedule": list(sc), "vs_oracle": st}
            log(f"[bench] {name}: {dtf * 1e3:.3f} ms/step, {st}")
        extra["forms"] = forms
        if "plain" in extra:  # batched compensated-FP32 form over the plain FP64-accumulation loop
            extra["speedup_batched_kahan_vs_plain"] = round(
                extra["plain"]["ms_per_step"] / forms["kahan_fp32"]["ms_per_step"], 2)
        # restore the headline schedule
        batch.autotune(P, prec, cache_path=args.tune_cache)

    wl = ("global-mapping LM iteration: 400 submaps (10k-120k points, log-uniform) on a 2 km "
          "loop, binary VGICP factors between submaps within 50 m, voxel 0.5 m")
    if args.workload == "precision":
        wl += "; loop 4.3-5.0 km from the world origin (precision stress)"
    line = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": wl, "factors": F, "source_points_per_step": total_points,
                   "submaps": len(data["clouds"]),
                   "precision": args.precision + " (FP64 keys, transform, fused covariance, "
                                                 "inverse and residual; FP32 Gauss-Newton "
                                                 "terms; FP64 sums above 32-point FP32 lane "
                                                 "partials)",
                   "schedule": {"block": sched[0], "tile": sched[1], "blocks_per_cu": sched[2],
                                "lookahead": sched[3]},
                   "voxelmap_build_ms": round(build_ms, 1),
                   "parity_vs_oracle": parity},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
