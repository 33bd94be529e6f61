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


def cpu_baseline(data, budget_s=15.0):
    """The oracle (C++ FP64, OpenMP over factors) on a bounded sample of the same factors."""
    import oracle

    clouds = data["clouds"]
    factors = data["factors"]
    res = 0.5
    order = np.random.default_rng(7).permutation(len(factors))
    # probe the rate on a few factors, then size the sample to the budget
    maps = {}

    def mk(j):
        if j not in maps:
            maps[j] = oracle.VoxelMap(*clouds[j], res)
        return maps[j]

    threads = oracle.max_threads()
    probe = order[:max(threads, 8)]
    for f in probe:
        mk(int(factors[f, 0]))
    t0 = time.perf_counter()
    run_oracle(probe, factors, clouds, mk, data["T"], threads)
    dt = time.perf_counter() - t0
    pts = sum(clouds[int(factors[f, 1])][0].shape[1] for f in probe)
    rate = pts / dt
    want = int(rate * budget_s)
    sample, acc = [], 0
    for f in order:
        sample.append(int(f))
        acc += clouds[int(factors[f, 1])][0].shape[1]
        if acc >= want:
            break
    for f in sample:
        mk(int(factors[f, 0]))
    t0 = time.perf_counter()
    run_oracle(sample, factors, clouds, mk, data["T"], threads)
    dt = time.perf_counter() - t0
    return {"value": acc / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} of {len(factors)} factors ({acc} source points), "
                      f"{dt:.1f} s wall, voxel maps built beforehand"}


def run_oracle(sample, factors, clouds, mk, poses, threads):
    import oracle

    maps, cl, fl = [], [], []
    mi, ci = {}, {}
    for f in sample:
        m, c, t, s, b = (int(x) for x in factors[f])
        if m not in mi:
            mi[m] = len(maps)
            maps.append(mk(m))
        if c not in ci:
            ci[c] = len(cl)
            cl.append(oracle.Cloud.of(*clouds[c]))
        fl.append([mi[m], ci[c], t, s, b])
    return oracle.linearize_factors(maps, cl, poses, np.array(fl, np.int32), nthreads=threads)


def parity_spot_check(data, out, n=16):
    """Max factor error of the timed outputs against the oracle on a few sampled factors."""
    import oracle
    from tests.metrics import factor_errors

    F = len(data["factors"])
    idx = np.linspace(0, F - 1, n).astype(int)
    worst = 0.0
    H = out["H"].cpu().numpy()
    b = out["b"].cpu().numpy()
    e = out["err"].cpu().numpy()
    nin = out["inliers"].cpu().numpy()
    for f in idx:
        m, c, t, s, bi = (int(x) for x in data["factors"][f])
        om = oracle.VoxelMap(*data["clouds"][m], 0.5)
        r = oracle.linearize(om, *data["clouds"][c], data["T"][t], data["T"][s], bool(bi))
        if int(nin[f]) != r["inliers"]:
            return {"factors": int(n), "max_rel_err": None, "inlier_mismatch": int(f)}
        err = factor_errors(H[f], b[f], e[f], r["H"], r["b"], r["e"])
        worst = max(worst, err["H"], err["b"], err["e"])
    return {"factors": int(n), "max_rel_err": worst}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--submaps", type=int, default=400)
    ap.add_argument("--precision", default="acc_fp64",
                    choices=["acc_fp64", "kahan_fp32", "naive_world_fp32", "math_fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one elementwise copy of 1 GiB (reads 1 GiB, writes 1 GiB) after the "
                         "timed region, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the factor batch is not sharded across GPUs in this "
              "build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2202_00242_amd.vgicp as V

    prec = V.PRECISIONS[args.precision]
    t0 = time.perf_counter()
    data = synth.global_batch(n_submaps=args.submaps)
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
    vox = np.array([maps[int(f[0])].size()[0] for f in factors], np.int64)
    log(f"[bench] voxel maps built in {build_ms:.0f} ms; {total_points} source points per step")

    stream = torch.cuda.Stream()
    batch = V.Batch(maps, clouds, factors, P.shape[0])
    with torch.cuda.stream(stream):
        sched = batch.autotune(P, prec, cache_path=args.tune_cache)
        log(f"[bench] schedule (block, tile, blocks/CU) = {sched}")
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

    parity = parity_spot_check(data, out)
    log(f"[bench] parity spot check: {parity}")

    # algorithmic bytes per launch: source stream, target tables once per factor, outputs
    alg_bytes = 36 * total_points + 72 * int(vox.sum()) + 736 * F
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(),
                "kernel": "batch_kernel (graph: pose prep + persistent kernel + finalize)",
                "alg_bytes_per_launch": alg_bytes}

    extra = {}
    if not args.no_plain:
        # plain form: one launch pair per factor, FP64 accumulation
        with torch.cuda.stream(stream):
            outs = [{"H": torch.empty((12, 12), dtype=torch.float64, device=dev),
                     "b": torch.empty(12, dtype=torch.float64, device=dev),
                     "err": torch.empty(1, dtype=torch.float64, device=dev),
                     "inliers": torch.empty(1, dtype=torch.int64, device=dev), "corr": None}
                    for _ in range(F)]
            host_T = data["T"]
            for rep in range(2):
                torch.cuda.synchronize()
                tp = time.perf_counter()
                for f in range(F):
                    m, c, t, s, bi = (int(x) for x in factors[f])
                    V.vgicp_linearize(maps[m], *clouds[c], host_T[t], host_T[s], bool(bi),
                                      V.VGICP_ACC_FP64, stream=stream, out=outs[f])
                torch.cuda.synchronize()
                plain_s = time.perf_counter() - tp
        extra["plain"] = {"value": total_points / plain_s, "ms_per_step": plain_s * 1e3,
                          "form": "per-factor launch loop, acc_fp64"}
        extra["speedup_batched_vs_plain"] = round(value / (total_points / plain_s), 2)
        log(f"[bench] plain loop: {plain_s * 1e3:.1f} ms/step, {total_points / plain_s / 1e9:.2f} "
            f"G points/s")
    if not args.no_forms:
        forms = {}
        for name in ("kahan_fp32", "math_fp64", "naive_world_fp32"):
            p = V.PRECISIONS[name]
            if p == prec:
                continue
            with torch.cuda.stream(stream):
                batch.autotune(P, p, cache_path=args.tune_cache)
                o2 = batch.alloc_outputs()
                batch.linearize(P, p, out=o2)
                torch.cuda.synchronize()
                tf = time.perf_counter()
                for _ in range(5):
                    batch.linearize(P, p, out=o2)
                torch.cuda.synchronize()
                dtf = (time.perf_counter() - tf) / 5
            forms[name] = {"value": total_points / dtf, "ms_per_step": round(dtf * 1e3, 3)}
            log(f"[bench] {name}: {dtf * 1e3:.3f} ms/step")
        extra["forms"] = forms

    cpu = None
    if not args.no_cpu_baseline:
        tc = time.perf_counter()
        cpu = cpu_baseline(data, args.cpu_budget)
        log(f"[bench] cpu baseline {cpu['value'] / 1e6:.2f} M points/s on {cpu['cores']} threads "
            f"({time.perf_counter() - tc:.1f} s)")

    line = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "global-mapping LM iteration: 400 submaps (10k-120k points, "
                               "log-uniform) on a 2 km loop, binary VGICP factors between "
                               "submaps within 50 m, voxel 0.5 m",
                   "factors": F, "source_points_per_step": total_points,
                   "submaps": len(data["clouds"]),
                   "precision": args.precision + " (FP64 keys, pose, residual and sums)",
                   "schedule": {"block": sched[0], "tile": sched[1], "blocks_per_cu": sched[2]},
                   "voxelmap_build_ms": round(build_ms, 1),
                   "parity": parity},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
