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
VALU_FILE = os.path.join(ROOT, "profiles", "batch_kernel_global_valu.json")
# autotuned schedules of the global batch on MI355X (the launch the counter files describe)
SCHEDULES_FILE = os.path.join(ROOT, "paper_2202_00242_amd", "tuned_schedules.json")
# VALU issue peak: 256 CUs x 4 SIMDs, a wave64 instruction every 4 cycles per SIMD (16 lanes per
# cycle for FP32 and FP64 alike), at 2.4 GHz: 614.4 G wave instructions/s (39.3 T lane-ops/s)
VALU_PEAK_GIPS = 256 * 4 * 2.4e9 / 4 / 1e9
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


def counter_summary(path, sched):
    """A committed rocprofv3 counter summary, if it was taken on the current kernel source and
    with the same schedule (block, tile, blocks per CU, lookahead) as this launch."""
    try:
        with open(path) as f:
            t = json.load(f)
        if (t.get("kernel_source_sha1") == kernel_source_hash()
                and list(t.get("schedule", [])) == [int(x) for x in sched]):
            return t
    except (OSError, ValueError):
        pass
    return None


def measured_traffic(sched):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) or None."""
    t = counter_summary(TRAFFIC_FILE, sched)
    return None if t is None else t.get("bytes_per_launch")


def measured_valu(sched):
    """VALU instructions per launch (SQ_INSTS_VALU) or None."""
    return counter_summary(VALU_FILE, sched)


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

    def run_poses(self, poses, idx):
        import oracle

        return oracle.linearize_factors(self.maps, self.clouds, poses, self.data["factors"][idx],
                                        nthreads=self.threads)

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


def lm_leg(V, data, batch, P, prec, stream, orc, lam=1e-4, iters=5):
    """Levenberg-Marquardt on the global graph (400 poses, pose 0 fixed). One step (linearize,
    assemble, solve, retract, linearize at the new poses) against the oracle's dense NumPy step;
    then `iters` iterations decided on the device (one linearization and one solve each)."""
    import torch
    from oracle import lm

    banded, w = batch.lm_info()
    with torch.cuda.stream(stream):
        ramp(lambda: batch.lm_step(P, prec, lam, fixed_pose=0))
        for _ in range(3):
            out = batch.lm_step(P, prec, lam, fixed_pose=0)
        torch.cuda.synchronize()
        ev = _events(5)
        for a, b in ev:
            a.record(stream)
            out = batch.lm_step(P, prec, lam, fixed_pose=0)
            b.record(stream)
        torch.cuda.synchronize()
        # device-decided iterations from the same start, and the start's linearization alone
        Pi = P.clone()
        lt = torch.tensor([lam], dtype=torch.float64, device=P.device)
        batch.lm_iterate(Pi, lt, 3, prec, fixed_pose=0)
        Pi.copy_(P)
        lt.fill_(lam)
        e0, e1 = _events(1)[0]
        torch.cuda.synchronize()
        e0.record(stream)
        costs = batch.lm_iterate(Pi, lt, iters, prec, fixed_pose=0, stream=stream)
        e1.record(stream)
        lin = batch.alloc_outputs()
        batch.linearize(P, prec, out=lin, stream=stream)  # untimed: new outputs, new graph
        la, lb = _events(1)[0]
        la.record(stream)
        for _ in range(5):
            batch.linearize(P, prec, out=lin, stream=stream)
        lb.record(stream)
        # the same linearization at the poses the iterations reached (more inliers)
        lin_end = batch.alloc_outputs()
        batch.linearize(Pi, prec, out=lin_end, stream=stream)
        lc, ld = _events(1)[0]
        lc.record(stream)
        for _ in range(5):
            batch.linearize(Pi, prec, out=lin_end, stream=stream)
        ld.record(stream)
        torch.cuda.synchronize()
        one = None
        if banded == 2:
            # the same step and iterations with the banded system solved in one sweep
            batch.lm_solver(2)
            try:
                ramp(lambda: batch.lm_step(P, prec, lam, fixed_pose=0))
                for _ in range(3):
                    o1 = batch.lm_step(P, prec, lam, fixed_pose=0)
                Pj = P.clone()
                lj = torch.tensor([lam], dtype=torch.float64, device=P.device)
                batch.lm_iterate(Pj, lj, 3, prec, fixed_pose=0)
                Pj.copy_(P)
                lj.fill_(lam)
                f0, f1 = _events(1)[0]
                torch.cuda.synchronize()
                f0.record(stream)
                batch.lm_iterate(Pj, lj, iters, prec, fixed_pose=0, stream=stream)
                f1.record(stream)
                torch.cuda.synchronize()
                one = {"ms_per_iteration": round((f0.elapsed_time(f1) - lin_ms_of(la, lb)) / iters,
                                                 3),
                       "step_delta_rel_diff": float(
                           (o1["delta"] - out["delta"]).abs().max() / out["delta"].abs().max()),
                       "poses_rel_diff_after_iterations": float(
                           (Pj - Pi).abs().max() / Pi.abs().max())}
            finally:
                batch.lm_solver(0)
    V.vgicp_sync_status(stream)
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    it_total = e0.elapsed_time(e1)
    lin_ms = lin_ms_of(la, lb)
    d = out["delta"].cpu().numpy()
    c = out["cost"].cpu().numpy()
    res = {"ms": round(ms, 3), "poses": int(P.shape[0]), "unknowns": 6 * int(P.shape[0]),
           "lambda": lam, "cost_before": float(c[0]), "cost_after": float(c[1]),
           "solver": ({0: "dense blocked Cholesky",
                       1: f"banded, one sweep (half-bandwidth {w} unknowns after the pose "
                          f"ordering)",
                       2: f"banded from both ends (half-bandwidth {w} unknowns after the pose "
                          f"ordering; two workgroups, then the {w + 1}-unknown separator)"}
                      [banded]),
           "form": "linearize + deterministic block assembly + FP64 Cholesky + retraction + "
                   "linearize at the new poses, all on the GPU",
           "iterate": {"iterations": iters, "ms_total": round(it_total, 3),
                       "ms_per_iteration": round((it_total - lin_ms) / iters, 3),
                       "costs": [float(x) for x in costs.cpu().numpy()],
                       "lambda_after": float(lt.item()),
                       "form": "device-decided iterations: solve + retract + linearize at the "
                               "candidate + accept/reject on the GPU, the current "
                               "linearization reused"}}
    res["iterate"]["linearization"] = {
        "ms_at_start": round(lin_ms, 3), "inliers_at_start": int(lin["inliers"].sum().item()),
        "ms_at_result": round(lin_ms_of(lc, ld), 3),
        "inliers_at_result": int(lin_end["inliers"].sum().item())}
    if one is not None:
        res["iterate"]["one_sweep"] = one
    t0 = time.perf_counter()
    ref = lm.lm_step(orc.maps, orc.clouds, data["T"], data["factors"], lam, 0, orc.threads)
    res["oracle_s"] = round(time.perf_counter() - t0, 2)
    res["vs_oracle"] = {
        "delta_max_rel_err": float(np.max(np.abs(d - ref["delta"])) / np.max(np.abs(ref["delta"]))),
        "cost_after_rel_err": float(abs(c[1] - ref["cost"][1]) / ref["cost"][1])}
    log(f"[bench] LM step: {ms:.2f} ms, cost {c[0]:.4g} -> {c[1]:.4g}, {res['vs_oracle']}; "
        f"{iters} device iterations {it_total:.2f} ms")
    return res


def shard_leg(V, maps, clouds, factors, P, sched, prec, out_full, stream, n_shards=8):
    """One GPU's share of the global batch spread over n_shards GPUs (strong scaling, the
    exchange of the per-factor results not included): the factors partitioned by target map,
    groups dealt by decreasing source points to the least-loaded shard (so every voxel map lives
    on one GPU), and the largest shard run as a batch of its own with the same schedule. Its
    per-factor results are compared with the full batch's (same tiles, same order of sums)."""
    import torch
    n_src = np.array([clouds[int(f[1])][0].shape[1] for f in factors], np.int64)
    groups = {}
    for i, f in enumerate(factors):
        groups.setdefault(int(f[0]), []).append(i)
    order = sorted(groups, key=lambda t: (-int(n_src[groups[t]].sum()), t))
    load = np.zeros(n_shards, np.int64)
    members = [[] for _ in range(n_shards)]
    for t in order:
        k = int(np.argmin(load))
        load[k] += int(n_src[groups[t]].sum())
        members[k] += groups[t]
    big = int(np.argmax(load))
    idx = np.array(sorted(members[big]), np.int64)
    b = V.Batch(maps, clouds, factors[idx], P.shape[0])
    b.set_schedule(*sched)
    with torch.cuda.stream(stream):
        out = b.alloc_outputs()
        for _ in range(10):
            b.linearize(P, prec, out=out)
        ev = _events(20)
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            b.linearize(P, prec, out=out)
            e1.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    ti = torch.from_numpy(idx).to(out["H"].device)
    same = all(torch.equal(out[k], out_full[k].index_select(0, ti))
               for k in ("H", "b", "err", "inliers"))
    # the shard's own schedule (fewer work items may favour smaller tiles)
    with torch.cuda.stream(stream):
        tuned = b.autotune(P, prec)
        o2 = b.alloc_outputs()
        for _ in range(10):
            b.linearize(P, prec, out=o2)
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            b.linearize(P, prec, out=o2)
            e1.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    ms_tuned = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    dH = (out["H"] - out_full["H"].index_select(0, ti)).abs().max().item()
    res = {"shards": n_shards, "factors": int(len(idx)), "targets": int(
        len({int(factors[i][0]) for i in idx})), "points": int(load[big]),
        "load_max_over_mean": round(float(load.max() / load.mean()), 4), "ms": round(ms, 3),
        "points_per_s": load[big] / (ms * 1e-3),
        "projected_points_per_s": float(load.sum()) / (ms * 1e-3),
        "bitwise_equal_to_full_batch": bool(same), "max_abs_diff_H": dH,
        "tuned": {"schedule": list(tuned), "ms": round(ms_tuned, 3),
                  "points_per_s": load[big] / (ms_tuned * 1e-3),
                  "projected_points_per_s": float(load.sum()) / (ms_tuned * 1e-3)},
        "form": "the largest of the shards as its own batch (same schedule); the projection is "
                "the whole batch's points over this shard's time, without the exchange"}
    log(f"[bench] shard 1/{n_shards}: {len(idx)} factors, {ms:.3f} ms, "
        f"{res['points_per_s'] / 1e9:.1f} G points/s (tuned {tuned}: {ms_tuned:.3f} ms); "
        f"equal to the full batch: {same}")
    return res


def ramp(launch, ms=100.0):
    """Untimed launches for ~ms milliseconds: after host-side work the GPU has idled and its
    clocks take some load to come back up."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < ms * 1e-3:
        for _ in range(4):
            launch()
        torch.cuda.synchronize()


def lin_ms_of(a, b):
    """ms of one of the 5 linearizations timed between events a and b."""
    return a.elapsed_time(b) / 5


def _events(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(n)]


def room_leg(V, stream, check=True):
    """Single unary factor, plain method (room, 5,000 target and 5,000 source points, res
    1.0 m, walls on voxel faces) at the three linearization poses: the time of one
    vgicp_linearize call (HIP events on its stream, and host-to-host with a synchronisation),
    median of 50 calls after 5 warm-ups; outputs against the oracle."""
    import torch
    import synth
    from tests.metrics import factor_errors

    r = synth.room()
    (txyz, tcov), (sxyz, scov) = r["target"], r["source"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    tx, tc, sx, sc = d(txyz), d(tcov), d(sxyz), d(scov)
    m = V.vgicp_build_voxelmap(tx, tc, r["res"])
    n = int(sxyz.shape[1])
    om = None
    if check:
        import oracle
        om = oracle.VoxelMap(txyz, tcov, r["res"])
    res = {"points": n, "res": r["res"], "poses": {}}
    for name, Ts in r["T_source"].items():
        out = V.vgicp_linearize(m, sx, sc, r["T_target"], Ts, False, V.VGICP_ACC_FP64,
                                want_corr=True, stream=stream)
        ev = _events(55)
        host = []
        with torch.cuda.stream(stream):
            for i, (a, b) in enumerate(ev):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                a.record(stream)
                V.vgicp_linearize(m, sx, sc, r["T_target"], Ts, False, V.VGICP_ACC_FP64,
                                  stream=stream, out=out)
                b.record(stream)
                torch.cuda.synchronize()
                host.append(time.perf_counter() - t0)
        gpu_us = float(np.median([a.elapsed_time(b) for a, b in ev[5:]])) * 1e3
        host_us = float(np.median(host[5:])) * 1e6
        e = {"gpu_us": round(gpu_us, 1), "host_us": round(host_us, 1),
             "points_per_s": n / (gpu_us * 1e-6), "inliers": int(out["inliers"].item())}
        if om is not None:
            import oracle
            ref = oracle.linearize(om, sxyz, scov, r["T_target"], Ts, False)
            fe = factor_errors(out["H"].cpu().numpy(), out["b"].cpu().numpy(),
                               out["err"].item(), ref["H"], ref["b"], ref["e"])
            e["vs_oracle"] = {"corr_equal": bool(np.array_equal(out["corr"].cpu().numpy(),
                                                                 ref["corr"])),
                              "max_rel_err": max(fe["H"], fe["b"], fe["e"])}
        res["poses"][name] = e
    V.vgicp_sync_status(stream)
    log(f"[bench] room factor: {res['poses']}")
    return res


def urban_leg(V, stream, check=True):
    """Odometry-scale binary factors (urban scan of ~19k points against 8 keyframes of ~57k
    points at 0.25, 0.5 and 1.0 m: 24 factors): the 24 factors as one batch (graph replay) and
    as a loop of plain calls on the stream; outputs against the oracle."""
    import torch
    import synth
    from tests.metrics import factor_errors

    u = synth.urban(0)
    sxyz, scov = u["source"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    sx, sc = d(sxyz), d(scov)
    maps, facs, omaps = [], [], []
    for k, (txyz, tcov) in enumerate(u["targets"]):
        for r in (0.25, 0.5, 1.0):
            facs.append([len(maps), 0, k, 8, 1])
            maps.append(V.vgicp_build_voxelmap(d(txyz), d(tcov), r))
            if check:
                import oracle
                omaps.append(oracle.VoxelMap(txyz, tcov, r))
    poses = np.concatenate([np.stack([np.asarray(T).reshape(12) for T in u["T_targets"]]),
                            np.asarray(u["T_source"]).reshape(1, 12)])
    P = d(poses)
    facs = np.array(facs, np.int32)
    F = len(facs)
    n = int(sxyz.shape[1])
    b = V.Batch(maps, [(sx, sc)], facs, poses.shape[0])
    out = b.alloc_outputs()
    with torch.cuda.stream(stream):
        for _ in range(5):
            b.linearize(P, out=out, stream=stream)
        ev = _events(50)
        for a, e in ev:
            a.record(stream)
            b.linearize(P, out=out, stream=stream)
            e.record(stream)
        # the same factors as plain calls, enqueued back to back
        outs = [None] * F
        pe = _events(5)
        for rep, (a, e) in enumerate(pe):
            a.record(stream)
            for f in range(F):
                outs[f] = V.vgicp_linearize(maps[facs[f, 0]], sx, sc, poses[facs[f, 2]],
                                            poses[8], True, V.VGICP_ACC_FP64, stream=stream,
                                            out=outs[f] if rep else None)
            e.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    batch_us = float(np.median([a.elapsed_time(e) for a, e in ev])) * 1e3
    plain_us = float(np.median([a.elapsed_time(e) for a, e in pe[1:]])) * 1e3
    res = {"factors": F, "source_points": n, "target_points": [int(t[0].shape[1])
                                                                for t in u["targets"]],
           "batched_us": round(batch_us, 1), "batched_us_per_factor": round(batch_us / F, 2),
           "batched_points_per_s": F * n / (batch_us * 1e-6),
           "plain_loop_us": round(plain_us, 1),
           "plain_points_per_s": F * n / (plain_us * 1e-6)}
    if check:
        import oracle
        worst, mism = 0.0, 0
        for f in range(F):
            ref = oracle.linearize(omaps[f], sxyz, scov, poses[facs[f, 2]], poses[8], True)
            mism += int(out["inliers"][f].item() != ref["inliers"])
            fe = factor_errors(out["H"][f].cpu().numpy(), out["b"][f].cpu().numpy(),
                               out["err"][f].item(), ref["H"], ref["b"], ref["e"])
            worst = max(worst, fe["H"], fe["b"], fe["e"])
        res["vs_oracle"] = {"factors": F, "max_rel_err": worst, "inlier_mismatch_factors": mism}
    log(f"[bench] urban odometry: {res}")
    return res


def diff_leg(V, stream, check=True):
    """Differentiation set (32 urban scans x 8 keyframes = 256 binary factors at 0.5 m) as one
    batch: forward (costs) + backward (pose, factor and point gradients), median of 20 after 3
    warm-ups; gradients of a sample of scans against the oracle's exact gradient."""
    import torch
    import synth
    from tests.gpu_util import point_scales, scaled_point_error

    scenes = synth.diff_set()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    maps, clouds, sources, poses, facs, tg = [], [], [], [], [], []
    for si, sc in enumerate(scenes):
        sources.append(sc["source"])
        clouds.append((d(sc["source"][0]), d(sc["source"][1])))
        p0 = len(poses)
        poses.extend(np.asarray(T).reshape(12) for T in sc["T_targets"])
        poses.append(np.asarray(sc["T_source"]).reshape(12))
        for ki, r in sc["factors"]:
            txyz, tcov = sc["targets"][ki]
            facs.append([len(maps), si, p0 + ki, p0 + 8, 1])
            maps.append(V.vgicp_build_voxelmap(d(txyz), d(tcov), r))
            tg.append((txyz, tcov, r))
    poses = np.stack(poses)
    facs = np.array(facs, np.int32)
    F = len(facs)
    P = d(poses)
    n_pts = int(sum(sources[f[1]][0].shape[1] for f in facs))
    b = V.Batch(maps, clouds, facs, poses.shape[0])
    g_err = torch.ones(F, dtype=torch.float64, device="cuda")
    sched = b.autotune(P, V.VGICP_ACC_FP64)
    with torch.cuda.stream(stream):
        for _ in range(3):
            fw = b.evaluate(P, stream=stream)
            bw = b.backward(P, g_err, want_points=True, want_factors=True, stream=stream)
        ev = _events(20)
        mid = [torch.cuda.Event(enable_timing=True) for _ in range(20)]
        for (a, e), mm in zip(ev, mid):
            a.record(stream)
            fw = b.evaluate(P, stream=stream)
            mm.record(stream)
            bw = b.backward(P, g_err, want_points=True, want_factors=True, stream=stream)
            e.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    tot = float(np.median([a.elapsed_time(e) for a, e in ev]))
    t_bw = float(np.median([mm.elapsed_time(e) for (_, e), mm in zip(ev, mid)]))
    # algorithmic bytes of the backward pass: every source point's position and its gradient
    # row (12 + 12 B), every inlier's covariance and position (24 + 12 B), every voxel that some
    # point falls in (72 B, counted once per factor: each factor here has its own map), the
    # per-cloud sums (12 B per factor-point read, 12 B + 4 B per cloud point)
    n_in, n_vox = 0, 0
    for f in range(F):
        r = V.vgicp_evaluate(maps[facs[f, 0]], *clouds[facs[f, 1]], poses[facs[f, 2]],
                             poses[facs[f, 3]], want_corr=True)
        cc = r["corr"]
        n_in += int((cc >= 0).sum().item())
        n_vox += int(torch.unique(cc[cc >= 0]).numel())
    n_cloud = int(sum(x.shape[1] for x, _ in sources))
    alg = 24 * n_pts + 36 * n_in + 72 * n_vox + 12 * n_pts + 16 * n_cloud + 12 * 8 * F
    ach = alg / (t_bw * 1e-3) / 1e9
    res = {"factors": F, "points": n_pts, "ms_forward_backward": round(tot, 4),
           "ms_backward": round(t_bw, 4), "points_per_s": n_pts / (tot * 1e-3),
           "schedule": list(sched),
           "backward_roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                 "alg_bytes": alg, "inliers": n_in, "voxels_hit": n_vox,
                                 "time": "batched backward call (5 kernels), HIP events"},
           "form": "batched evaluate + batched backward (pose, factor and point gradients), "
                   "acc_fp64"}
    if check:
        import oracle
        worst_f, worst_p, worst_e = 0.0, 0.0, 0.0
        e = fw["err"].cpu().numpy()
        gf = bw["grad_factors"].cpu().numpy()
        for si in (0, len(scenes) // 2, len(scenes) - 1):
            xyz, cov = sources[si]
            gsum = np.zeros((3, xyz.shape[1]))
            scale = np.zeros(xyz.shape[1])
            for f in np.nonzero(facs[:, 1] == si)[0]:
                txyz, tcov, r = tg[f]
                om = oracle.VoxelMap(txyz, tcov, r)
                Tt, Ts = poses[facs[f, 2]], poses[facs[f, 3]]
                corr = oracle.evaluate(om, xyz, cov, Tt, Ts)["corr"]
                g = oracle.gradient(om, xyz, cov, Tt, Ts, True, corr)
                worst_e = max(worst_e, abs(e[f] - g["e"]) / g["e"])
                worst_f = max(worst_f, float(np.max(np.abs(gf[f] - g["g_xi"]))
                                             / np.linalg.norm(g["g_xi"])))
                gsum += g["g_points"]
                scale += point_scales(om, xyz, cov, Tt, Ts, corr)
            worst_p = max(worst_p, scaled_point_error(bw["grad_points"][si].cpu().numpy(), gsum,
                                                      scale))
        res["vs_oracle"] = {"scans_checked": 3, "factors_checked": 24,
                            "cost_max_rel_err": worst_e, "factor_grad_max_rel_err": worst_f,
                            "point_grad_max_scaled_err": worst_p}
    log(f"[bench] differentiation: {res}")
    return res, b, P


def precision_leg(V, batch, maps, clouds, data, stream, orc, tune_cache=None):
    """The global batch's loop moved 4.3-5.0 km from the world origin (points stay submap-local
    FP32; only the FP64 poses move), every precision form: time per step (median of 10 after 10
    warm-up launches, schedule autotuned per form) and the error of every factor against the
    oracle."""
    import torch
    import synth

    prec = synth.precision_batch()
    T4 = np.ascontiguousarray(prec["T"])
    P4 = torch.from_numpy(T4).cuda()
    factors = data["factors"]
    total = int(sum(clouds[int(f[1])][0].shape[1] for f in factors))
    t0 = time.perf_counter()
    ref = orc.run_poses(T4, np.arange(len(factors)))
    t_oracle = time.perf_counter() - t0
    forms = {}
    for name in ("acc_fp64", "kahan_fp32", "math_fp64", "naive_world_fp32"):
        p = V.PRECISIONS[name]
        with torch.cuda.stream(stream):
            sc = batch.autotune(P4, p, cache_path=tune_cache, stream=stream)
            o = batch.alloc_outputs()
            for _ in range(10):  # warm-up: clocks ramp up again after the host-side work
                batch.linearize(P4, p, out=o, stream=stream)
            ev = _events(10)
            for a, e in ev:
                a.record(stream)
                batch.linearize(P4, p, out=o, stream=stream)
                e.record(stream)
            torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(e) for a, e in ev]))
        st = factor_error_stats(o, ref, np.arange(len(factors)))
        forms[name] = {"ms_per_step": round(ms, 3), "value": total / (ms * 1e-3),
                       "schedule": list(sc), "vs_oracle": st}
        log(f"[bench] precision stress {name}: {ms:.3f} ms, {st}")
    V.vgicp_sync_status(stream)
    origin = np.linalg.norm(T4.reshape(-1, 3, 4)[:, :, 3], axis=1)
    return {"origin_distance_m": [round(float(origin.min()), 1), round(float(origin.max()), 1)],
            "factors": len(factors), "points_per_step": total, "oracle_s": round(t_oracle, 2),
            "forms": forms}


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
    # with bias states: preintegration with the bias derivatives, the 30-unknown factor
    biases = rng.normal(size=(F + 1, 6)) * 0.01
    dbi = d(biases)
    evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(13)]
    with torch.cuda.stream(stream):
        for a, b, c in evb:
            a.record(stream)
            preb, covb, jac = V.vgicp_imu_preintegrate_bias(drows, dseg, dbias, 1.7e-3, 2e-2,
                                                            stream=stream)
            b.record(stream)
            outb = V.vgicp_imu_linearize_bias(preb, covb, jac, dbias, dst, dpo, dve, dbi, g,
                                              3e-3, 2e-4, stream=stream)
            c.record(stream)
        torch.cuda.synchronize()
    V.vgicp_sync_status(stream)
    tb_pre = float(np.median([a.elapsed_time(b) for a, b, _ in evb[3:]]))
    tb_lin = float(np.median([b.elapsed_time(c) for _, b, c in evb[3:]]))
    Hb, bb, eb = outb["H"].cpu().numpy(), outb["b"].cpu().numpy(), outb["err"].cpu().numpy()
    worst_b = 0.0
    for f in idx:
        ref = oimu.preintegrate(rows[seg[f]:seg[f + 1]], bias[f], 1.7e-3, 2e-2)
        lin = oimu.linearize_bias(ref, poses[f], vels[f], biases[f], poses[f + 1], vels[f + 1],
                                  biases[f + 1], g, 3e-3, 2e-4)
        dd = np.sqrt(np.diag(lin["H"]))
        worst_b = max(worst_b, np.max(np.abs(Hb[f] - lin["H"]) / np.outer(dd, dd)),
                      np.max(np.abs(bb[f] - lin["b"]) / (dd * np.sqrt(lin["e"]))),
                      abs(eb[f] - lin["e"]) / lin["e"])
    res["bias_states"] = {
        "ms": {"preintegrate_with_bias_derivatives": round(tb_pre, 4),
               "linearize": round(tb_lin, 4)},
        "factors_per_s": round(F / ((tb_pre + tb_lin) * 1e-3)),
        "form": "bias derivatives of the preintegration, first-order bias correction, bias "
                "random walk: 15 residuals over 30 unknowns, one 64-thread block per factor",
        "vs_oracle": {"factors": int(len(idx)), "max_rel_err": float(worst_b)}}
    log(f"[bench] IMU factors: {F} in {t_pre:.3f} + {t_lin:.3f} ms, vs oracle {worst:.2e}; "
        f"with bias states {tb_pre:.3f} + {tb_lin:.3f} ms, vs oracle {worst_b:.2e}")
    return res


def plain_leg(V, data, maps, clouds, stream, total_points, value, launch_ms):
    """The plain form: one vgicp_linearize_noalloc call (two kernels) per factor, FP64
    accumulation. Timed twice: the host loop issuing the calls (wall time, host overhead
    included), and the same per-factor launches captured once into a HIP graph and replayed
    (GPU time of the per-factor kernels back to back, no host in the loop)."""
    import torch

    factors = data["factors"]
    host_T = data["T"]
    F = len(factors)
    dev = clouds[0][0].device
    outs = [{"H": torch.empty((12, 12), dtype=torch.float64, device=dev),
             "b": torch.empty(12, dtype=torch.float64, device=dev),
             "err": torch.empty(1, dtype=torch.float64, device=dev),
             "inliers": torch.empty(1, dtype=torch.int64, device=dev), "corr": None}
            for _ in range(F)]

    def issue(st):
        for f in range(F):
            m, c, t, s_, bi = (int(x) for x in factors[f])
            V.vgicp_linearize_noalloc(maps[m], *clouds[c], host_T[t], host_T[s_], bool(bi),
                                      V.VGICP_ACC_FP64, stream=st, out=outs[f])

    with torch.cuda.stream(stream):
        issue(stream)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        issue(stream)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - tp
    res = {"value": total_points / plain_s, "ms_per_step": round(plain_s * 1e3, 2),
           "form": "per-factor calls of vgicp_linearize_noalloc from a host loop, acc_fp64 "
                   "(2 kernels per factor)"}
    out = {"speedup_batched_vs_plain": round(value / (total_points / plain_s), 2)}
    try:
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=cap):
            issue(cap)
        g.replay()
        torch.cuda.synchronize()
        ev = _events(3)
        for a, e in ev:
            a.record(cap)
            with torch.cuda.stream(cap):
                g.replay()
            e.record(cap)
        torch.cuda.synchronize()
        gms = float(np.median([a.elapsed_time(e) for a, e in ev]))
        res["gpu_graph_ms"] = round(gms, 2)
        res["value_gpu_graph"] = total_points / (gms * 1e-3)
        res["gpu_form"] = ("the same per-factor launches captured into one HIP graph "
                           f"({2 * F} kernel nodes) and replayed: GPU time without the host")
        out["speedup_batched_vs_plain_gpu"] = round(gms / launch_ms, 2)
        del g
    except Exception as exc:  # the host-loop number stands alone
        res["gpu_graph_error"] = repr(exc)
    V.vgicp_sync_status(stream)
    log(f"[bench] plain: {res}")
    out["plain"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ramp-ms", type=float, default=100.0,
                    help="untimed launches before the warm-up steps, to bring the clocks up")
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
    ap.add_argument("--no-room", action="store_true")
    ap.add_argument("--no-urban", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-precision-stress", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--tune-cache", default=SCHEDULES_FILE,
                    help="schedule cache of the autotuner (default: the committed schedules, so "
                         "that the launch matches the committed counter summaries)")
    ap.add_argument("--retune", action="store_true", help="autotune without a schedule cache")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB) after the "
                         "timed region, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.retune:
        args.tune_cache = None
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
    torch.cuda.synchronize()
    tb = time.perf_counter()
    batch = V.Batch(maps, clouds, factors, P.shape[0])
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - tb) * 1e3
    log(f"[bench] batch created in {create_ms:.0f} ms (spatially ordered copies of "
        f"{len(clouds)} clouds)")
    with torch.cuda.stream(stream):
        sched = batch.autotune(P, prec, cache_path=args.tune_cache)
        log(f"[bench] schedule (block, tile, blocks/CU, lookahead) = {sched}")
        out = batch.alloc_outputs()
        # the GPU's clocks ramp up under sustained load: ~100 ms of untimed launches first (what
        # the autotuner's own launches did when the schedule was not cached), then the W
        # warm-up steps
        t_ramp = time.perf_counter()
        while time.perf_counter() - t_ramp < args.ramp_ms * 1e-3:
            for _ in range(8):
                batch.linearize(P, prec, out=out)
            torch.cuda.synchronize()
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
    # source-major accounting: every source cloud read once (36 B per point) for all of its
    # factors, the tables once, the outputs
    used = np.unique(factors[:, 1])
    alg_src_major = (36 * int(sum(clouds[int(c)][0].shape[1] for c in used))
                     + 72 * int(vox.sum()) + 736 * F)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(sched),
                "kernel": "batch_kernel (graph: pose prep + persistent kernel + finalize)",
                "alg_bytes_per_launch": alg_bytes, "inliers_per_launch": n_inliers,
                "alg_bytes_every_covariance": alg_all_cov,
                "frac_every_covariance": round(alg_all_cov / (launch_ms * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
                "alg_bytes_source_major": alg_src_major,
                "frac_source_major": round(alg_src_major / (launch_ms * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4)}
    vc = measured_valu(sched)
    if vc is not None:
        gips = vc["sq_insts_valu_per_dispatch"] / (launch_ms * 1e-3) / 1e9
        roofline["valu"] = {"bound": "alu", "achieved": round(gips, 1), "peak": VALU_PEAK_GIPS,
                            "unit": "G VALU instr/s", "frac": round(gips / VALU_PEAK_GIPS, 4),
                            "counters": os.path.relpath(VALU_FILE, ROOT)}
    else:
        roofline["valu"] = None

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
    if not args.no_shard:
        extra["shard"] = shard_leg(V, maps, clouds, factors, P, sched, prec, out, stream)
    if not args.no_plain:
        extra.update(plain_leg(V, data, maps, clouds, stream, total_points, value, launch_ms))
    if not args.no_overlap:
        extra["overlap"] = overlap_leg(V, data, maps, clouds, P, stream, orc)
    if not args.no_lm:
        extra["lm_step"] = lm_leg(V, data, batch, P, prec, stream, orc)
    if not args.no_preprocess:
        extra["preprocess"] = preprocess_leg(V, stream, orc)
    if not args.no_imu:
        extra["imu"] = imu_leg(V, stream, orc)
    if not args.no_room:
        extra["room"] = room_leg(V, stream)
    if not args.no_urban:
        extra["urban"] = urban_leg(V, stream)
    if not args.no_diff:
        extra["differentiation"], _, _ = diff_leg(V, stream)
    if not args.no_precision_stress:
        extra["precision_stress"] = precision_leg(V, batch, maps, clouds, data, stream, orc,
                                                  args.tune_cache)
    if not args.no_forms:
        forms = {}
        for name in ("acc_fp64", "kahan_fp32", "math_fp64", "naive_world_fp32"):
            p = V.PRECISIONS[name]
            with torch.cuda.stream(stream):
                sc = batch.autotune(P, p, cache_path=args.tune_cache)
                o2 = batch.alloc_outputs()
                # warm-up launches first (the GPU idled during the host-side checks and its
                # clocks ramp up again under load), then the median of 10 launches timed with
                # HIP events on the launch stream, as the headline's per-launch time
                for _ in range(10):
                    batch.linearize(P, p, out=o2)
                ev = _events(10)
                for a, e in ev:
                    a.record(stream)
                    batch.linearize(P, p, out=o2)
                    e.record(stream)
                torch.cuda.synchronize()
                dtf = float(np.median([a.elapsed_time(e) for a, e in ev])) * 1e-3
            st = factor_error_stats(o2, ref, ref_idx)
            forms[name] = {"value": total_points / dtf, "ms_per_step": round(dtf * 1e3, 3),
                           "schedule": list(sc), "vs_oracle": st}
            log(f"[bench] {name}: {dtf * 1e3:.3f} ms/step, {st}")
        extra["forms"] = forms
        if "plain" in extra:  # batched compensated-FP32 form over the plain FP64-accumulation loop
            extra["speedup_batched_kahan_vs_plain"] = round(
                extra["plain"]["ms_per_step"] / forms["kahan_fp32"]["ms_per_step"], 2)
            if extra["plain"].get("gpu_graph_ms"):
                extra["speedup_batched_kahan_vs_plain_gpu"] = round(
                    extra["plain"]["gpu_graph_ms"] / forms["kahan_fp32"]["ms_per_step"], 2)
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
                   "batch_create_ms": round(create_ms, 1),
                   "parity_vs_oracle": parity},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
