#!/usr/bin/env python3
"""Benchmark: numerical entanglement of batched integer convolution on one
MI355X.

Workload (the batched configuration): 64 groups of M = 3 streams, each
stream 1,048,576 int32 samples uniform in [-2^11, 2^11), each group with its
own 64-tap int32 kernel in the same range; full linear convolution. One step
is one pass of the whole method over the batch -- entangle (eq. (14)-(15)),
convolve every entangled stream (eq. (9)), recover every output (eq. (16)-
(19)) -- as one graph launch of the fused executor, inputs already resident
in HBM. The same batch is also run through the failure-intolerant plain
convolution (narrow and same-datapath) and the checksum method, and with one
stream lost per group.

Prints one JSON line. `value` is recovered output samples per second (Gout-
samples/s, whole job); `roofline` relates the dominant kernel's algorithmic
HBM bytes per launch to its average duration (HIP events on its stream);
`cpu_baseline` times the CPU oracle on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "entangled vs plain int conv Gout-samples/s; overhead %; % roofline; p99"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
CSRC = os.path.join(ROOT, "paper_1509_03838_amd", "csrc")
# Sources that define the fused convolution kernel and its launch.
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("fused_kernels.h", "fused.h", "fused_conv.hip",
                                               "conv_variants.h", "plan.hip")]
def traffic_file(config: str) -> str:
    return os.path.join(ROOT, "profiles", f"conv_fused_{config}_traffic.txt")


def parse():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--groups", type=int, default=64, help="stream-triples in the batch")
    p.add_argument("--no-baselines", action="store_true")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    p.add_argument("--conv-steps", type=int, default=0)
    p.add_argument("--stream-steps", type=int, default=0)
    p.add_argument("--no-autotune", action="store_true",
                   help="use the default tile steps instead of the autotuner's")
    p.add_argument("--config", default="batched",
                   choices=("batched", "small", "uneven", "long", "serve", "fig2", "chain", "gemm",
                            "ops", "w32"),
                   help="workload; the benchmark line is the batched one")
    p.add_argument("--jobs", type=int, default=2000, help="serving: number of jobs")
    p.add_argument("--rounds", type=int, default=3,
                   help="interleaved timing rounds per mode (each of --steps launches)")
    p.add_argument("--settle-ms", type=int, default=300,
                   help="untimed launches of every mode for this long before timing")
    p.add_argument("--single-launch", action="store_true",
                   help="the timed mode runs as one persistent launch (ne_tuning.single_launch)")
    p.add_argument("--by-category", action="store_true",
                   help="also time every (operation, M) category of the batch alone and the "
                        "widening copy of the batch's bytes (per-category roofline)")
    p.add_argument("--no-serving", action="store_true",
                   help="batched line: skip the short serving run")
    p.add_argument("--budget-mib", type=int, default=2048, help="serving: HBM budget")
    p.add_argument("--only", default=None,
                   choices=("entangled", "plain", "plain_same", "checksum", "checksum_same"),
                   help="time one mode only (profiling)")
    p.add_argument("--mfma-probe", action="store_true",
                   help="only launch the matrix-core reference with fixed and with random "
                        "operands, twice each (for its counters), and exit")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only widen an int32 buffer of this many MiB into int64 a few times "
                        "(ne_stream_widen, a kernel of known traffic, to calibrate the HBM byte "
                        "counters) and exit")
    return p.parse_args()


def source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(config: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload, if it was taken on the current kernel source; else None."""
    path = traffic_file(config)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each GPU would run a plan over its own share of the groups)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1509_03838_amd import ne
    from paper_1509_03838_amd import workloads as wl

    if args.mfma_probe:
        # the matrix-core reference alone (profiling): fixed, then random
        # operands, twice each
        ne.load()
        sink = torch.empty(4 * 2048, dtype=torch.int32, device="cuda:0")
        for varied in (False, True, False, True):
            ne.mfma_i8_peak(sink, 2048, 4096, varied)
            torch.cuda.synchronize()
        print(json.dumps({"kernel": "k_mfma_i8_peak", "launches": 4}))
        return

    if args.copy_calibration:
        # a kernel of known traffic for the HBM byte counters: the library's
        # widening copy reads 4 and writes 8 bytes per element
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty(n, dtype=torch.int64, device="cuda:0")
        ne.load()
        for _ in range(4):
            ne.stream_widen(src, dst)
        torch.cuda.synchronize()
        print(json.dumps({"kernel": "k_widen", "bytes_read": n * 4, "bytes_written": n * 8,
                          "launches": 4}))
        return

    dev = torch.device("cuda:0")
    ne.load()
    if args.config == "serve":
        return serve_line(args, wl)
    if args.config == "fig2":
        return fig2_line(args, wl)
    if args.config == "chain":
        return chain_line(args, wl)
    if args.config == "gemm":
        return gemm_line(args, wl)
    if args.config == "w32":
        return w32_line(args, wl)
    if args.config == "ops":
        return ops_line(args, wl)
    t_gen = time.perf_counter()
    cfg = CONFIGS[args.config]
    groups, in_bits, describe = cfg(wl, args)
    print(f"# generated {len(groups)} groups in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    c_dev = [[torch.from_numpy(row).to(dev) for row in g.c] for g in groups]
    k_dev = [None if g.op == "scale" else torch.from_numpy(g.operand).to(dev) for g in groups]
    n_outs = [ne.n_out(g.op, g.n, 0 if g.operand is None else g.operand.size) for g in groups]
    out = [[torch.empty(max(no, 1), dtype=torch.int64, device=dev)[:no] for _ in range(g.M)]
           for g, no in zip(groups, n_outs)]
    stream = torch.cuda.Stream()

    tuner = None
    if not args.no_autotune and not args.conv_steps and not args.stream_steps:
        from paper_1509_03838_amd.tune import DEFAULT_CACHE, Tuner
        tuner = Tuner(os.environ.get("NE_TUNE_CACHE", DEFAULT_CACHE))
    tuned = {}

    def make_plan(mode, lost=-1):
        # "<mode>@single": the mode as one persistent launch
        mode, _, how = mode.partition("@")
        single = how == "single" or (args.single_launch and mode == main_mode)
        specs = [ne.GroupSpec(g.op, c_dev[i], k_dev[i], out[i], g.scalar, lost, in_bits)
                 for i, g in enumerate(groups)]
        # the tuner times per-variant launches; the single launch keeps the
        # planner's strips (in a run whose tuner chose longer strips for many
        # classes the single launch took 6.64 ms against 5.1 with the planner's)
        if tuner is not None and not single:
            tuned.update(tuner.tune(specs, mode))
        plan = ne.Plan(specs, mode, conv_steps=args.conv_steps, stream_steps=args.stream_steps,
                       single_launch=single)
        plan.capture(stream)
        return plan

    def snapshot():
        return [[t[::997].cpu() for t in row] for row in out[:8]]

    # Every mode runs the same captured plan shape on the same buffers; their
    # timings are interleaved in rounds (the order rotating each round) so
    # that the clock and thermal state of the device does not favour the
    # mode timed first or last, and each mode's figure is the median round.
    main_mode = args.only or "entangled"
    runs = [(main_mode, -1)]
    if not args.no_baselines and not args.only:
        runs += [("plain", -1), ("plain_same", -1), ("checksum", -1), ("checksum_same", -1),
                 ("entangled", 1), ("checksum", 1)]
        if args.config in ("uneven", "batched") and not args.single_launch:
            runs += [("entangled@single", -1)]  # the whole batch in one persistent launch
    plans = {}
    for mode, lost in runs:
        plans[(mode, lost)] = make_plan(mode, lost)
    ent = plans[(main_mode, -1)]
    stats = ent.stats()
    # digit pairs each useful multiply-add takes on the matrix cores, per mode
    # (the datapath's cost; the Toeplitz padding comes on top)
    plan_digits = {name_of(k): round(p.stats()["limb_macs"] / max(1, p.stats()["macs"]), 3)
                   for k, p in plans.items()}
    # The device is brought to its steady clock before anything is timed:
    # untimed launches of every plan in turn for --settle-ms (a cold device
    # runs the first tens of launches about 10% slower), then the W warm-up
    # launches of each mode.
    t_settle = time.perf_counter() + args.settle_ms / 1e3
    with torch.cuda.stream(stream):
        while time.perf_counter() < t_settle:
            for p in plans.values():
                p.launch(stream)
            stream.synchronize()
    rounds = {k: [] for k in runs}
    walls = []
    out_ref = None
    for r in range(args.rounds):
        for j in range(len(runs)):
            key = runs[(j + r) % len(runs)]
            ms, wall = time_captured(torch, plans[key], stream, args.steps,
                                     args.warmup if r == 0 else 0)
            rounds[key].append(ms)
            if key == (main_mode, -1):
                walls.append(wall)
            if r == 0:
                if plans[key].flags():
                    raise SystemExit(f"device flags {plans[key].flags():#x} after the {key} run")
                snap = snapshot()
                if out_ref is None:
                    out_ref = snap
                elif not all(torch.equal(a, b) for ra, rb in zip(snap, out_ref)
                             for a, b in zip(ra, rb)):
                    raise SystemExit(f"{key} results differ from the {runs[0]} run")
    name = {k: name_of(k) for k in runs}
    results = {name[k]: float(np.median(v)) for k, v in rounds.items()}
    ms_ev = results[main_mode]
    ms_wall = float(np.median(walls))
    for k in runs:
        print(f"# {name[k]}: {results[name[k]]:.4f} ms/step (median of "
              f"{', '.join(f'{x:.4f}' for x in rounds[k])})", file=sys.stderr, flush=True)
    for p in plans.values():
        if p is not ent:
            p.close()

    samples = stats["out_samples"]
    value = samples / (ms_ev * 1e-3) / 1e9
    alg_bytes = stats["in_bytes"] + stats["out_bytes"]
    achieved = alg_bytes / (ms_ev * 1e-3) / 1e9
    # matrix-core rate on the useful digit products (no Toeplitz padding, no
    # sparse top digit); the issued rate is reported beside it
    mfma_tops = 2 * stats["limb_macs"] / (ms_ev * 1e-3) / 1e12
    mfma_issued_tops = 2 * stats["mfma_macs"] / (ms_ev * 1e-3) / 1e12
    hbm_frac, mfma_frac = achieved / HBM_PEAK_GBS, mfma_tops / INT8_PEAK_TOPS
    traffic = read_traffic(args.config) if main_mode == "entangled" else None

    def thr(ms):
        return samples / (ms * 1e-3) / 1e9

    single = len({(g.op, g.M) for g in groups}) == 1 and stats["launches"] == 1
    if hbm_frac >= mfma_frac:
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic}
    else:
        roof = {"bound": "mfma", "achieved": round(mfma_tops, 1), "peak": INT8_PEAK_TOPS,
                "unit": "TOP/s", "frac": round(mfma_frac, 4), "traffic": traffic}
    roof.update({
        "kernel": stats_kernel_name(stats, groups, main_mode) if single else
        f"all {stats['launches']} launches of the plan",
        "alg_bytes_per_launch": alg_bytes,
        "hbm_GBps": round(achieved, 1), "hbm_frac": round(hbm_frac, 4),
        "mfma_i8_tops": round(mfma_tops, 1), "mfma_frac": round(mfma_frac, 4),
        "mfma_i8_tops_issued": round(mfma_issued_tops, 1),
    })
    M0 = groups[0].M
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gout-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_ev, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": dict(workload=describe, groups=len(groups), mode=main_mode, w=64,
                       out_samples=samples, **({"l": ne.params(M0)[0]} if M0 >= 3 else {})),
        "roofline": roof,
        "wall_ms_per_step": round(ms_wall, 4),
        "tuned_steps": tuned_summary(tuned, main_mode),
    }
    if args.single_launch:
        line["config"]["single_launch"] = True
    line["timing"] = (f"median of {args.rounds} rounds of {args.steps} captured launches per "
                      f"mode, the modes interleaved with a rotating order, after {args.settle_ms} ms "
                      f"of untimed launches of every mode and {args.warmup} warm-up launches each")
    if not args.only and not args.no_baselines:
        def pct(a, b):
            return round(100 * (results[a] / results[b] - 1), 2)
        line["baselines"] = {
            "gout_per_s": {k: round(thr(v), 3) for k, v in results.items()},
            "ms_per_step": {k: round(v, 4) for k, v in results.items()},
            "rounds_ms": {name[k]: [round(x, 4) for x in v] for k, v in rounds.items()},
            # overhead = extra time relative to the failure-intolerant run;
            # plain_same and checksum_same run the entangled words' datapath
            # (digit planes), plain and checksum the fewest digits their
            # values need
            "overhead_pct_vs_plain_same": pct(main_mode, "plain_same"),
            "overhead_pct_vs_plain": pct(main_mode, "plain"),
            "checksum_same_overhead_pct_vs_plain_same": pct("checksum_same", "plain_same"),
            "checksum_overhead_pct_vs_plain": pct("checksum", "plain"),
            "checksum_overhead_pct_vs_plain_same": pct("checksum", "plain_same"),
            "digit_pairs_per_mac": plan_digits,
        }
        if "entangled_single_launch" in results:
            line["baselines"]["single_launch_pct_vs_per_variant_launches"] = pct(
                "entangled_single_launch", main_mode)
    if (args.config == "batched" and not args.only) or args.by_category:
        line["roofline"]["hbm_ceiling"] = hbm_ceiling(torch, ne, stream, stats, args, achieved)
    if args.by_category:
        line["categories"] = by_category(torch, ne, np, args, groups, c_dev, k_dev, out, in_bits,
                                         main_mode, stream, tuner)
    if roof["bound"] == "mfma" and not args.only:
        line["roofline"]["mfma_ceiling"] = mfma_ceiling(torch, ne, stream, mfma_tops)

    line["gpu"] = gpu_info(torch)
    if not args.no_cpu and args.config == "batched":
        line["cpu_baseline"] = cpu_baseline(groups, np)
    if args.config == "batched" and not args.only and not args.no_serving:
        line["serving"] = serving_summary(args, wl)
    print(json.dumps(line), flush=True)


def by_category(torch, ne, np, args, groups, c_dev, k_dev, out, in_bits, mode, stream, tuner):
    """Every (operation, M) category of the batch alone, as its own captured
    plan timed like the whole batch (median of the rounds): its time,
    algorithmic bytes (inputs and operands read once, outputs written once)
    and rate against the HBM peak."""
    cats = {}
    for i, g in enumerate(groups):
        cats.setdefault((g.op, g.M), []).append(i)
    rows = []
    for (op, M), idx in sorted(cats.items()):
        specs = [ne.GroupSpec(groups[i].op, c_dev[i], k_dev[i], out[i], groups[i].scalar, -1,
                              in_bits) for i in idx]
        if tuner is not None:
            tuner.tune(specs, mode)
        plan = ne.Plan(specs, mode, conv_steps=args.conv_steps, stream_steps=args.stream_steps)
        plan.capture(stream)
        ms = float(np.median([time_captured(torch, plan, stream, args.steps,
                                            args.warmup if r == 0 else 0)[0]
                              for r in range(args.rounds)]))
        st = plan.stats()
        plan.close()
        b = st["in_bytes"] + st["out_bytes"]
        gbps = b / (ms * 1e-3) / 1e9
        rows.append({"op": op, "M": M, "groups": len(idx), "ms": round(ms, 4), "alg_bytes": b,
                     "GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBS, 4),
                     "launches": st["launches"]})
    return rows


def name_of(key):
    mode, lost = key
    mode = mode.replace("@single", "_single_launch")
    return mode if lost < 0 else f"{mode}_one_lost"


def hbm_ceiling(torch, ne, stream, stats, args, achieved):
    """The practical HBM ceiling: ne_stream_widen (4 bytes read and 8 written
    per element, the fused convolution's mix, no arithmetic) over as many
    elements as the benchmark's algorithmic bytes, timed like the plan."""
    n = (stats["in_bytes"] + stats["out_bytes"]) // 12
    src = torch.ones(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty(n, dtype=torch.int64, device="cuda:0")
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            ne.stream_widen(src, dst, stream=stream)
        torch.cuda.synchronize()
        best = []
        for _ in range(args.rounds):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                ne.stream_widen(src, dst, stream=stream)
            e1.record(stream)
            e1.synchronize()
            best.append(e0.elapsed_time(e1) / args.steps)
    ms = float(sorted(best)[len(best) // 2])
    gbps = 12 * n / (ms * 1e-3) / 1e9
    return {"kernel": "k_widen (ne_stream_widen)", "bytes_per_launch": 12 * n,
            "ms": round(ms, 4), "GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBS, 4),
            "conv_frac_of_ceiling": round(achieved / gbps, 4)}


def mfma_ceiling(torch, ne, stream, achieved_tops):
    """The measured i8 matrix-core rate: ne_mfma_i8_peak, 8 workgroups of 4
    waves per compute unit issuing independent v_mfma_i32_16x16x64_i8, with
    fixed operands and with pseudo-random operands that change every product
    (as data digit planes do), each timed with HIP events (median of 3
    launches after one warm-up)."""
    blocks, iters = 256 * 8, 4096
    sink = torch.empty(4 * blocks, dtype=torch.int32, device="cuda:0")
    out = {"kernel": "k_mfma_i8_peak (ne_mfma_i8_peak)"}
    for key, varied in (("fixed_operands", False), ("random_operands", True)):
        times = []
        with torch.cuda.stream(stream):
            ops = ne.mfma_i8_peak(sink, blocks, iters, varied, stream=stream)
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ne.mfma_i8_peak(sink, blocks, iters, varied, stream=stream)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
        tops = ops / (sorted(times)[1] * 1e-3) / 1e12
        out[key] = {"TOPs": round(tops, 1), "frac_of_peak": round(tops / INT8_PEAK_TOPS, 4)}
    out["kernel_frac_of_random_operand_rate"] = round(
        achieved_tops / out["random_operands"]["TOPs"], 4)
    return out


def serving_summary(args, wl):
    """A short run of the serving workload (Poisson 2000 jobs/s, M in
    {3,4,5}, n log-uniform [2^10, 2^20], taps log-uniform [16, 1024], 1%
    drops, 4 lanes, 2 GiB budget), and the same job mix offered as a burst
    to one lane with a 256 MiB budget, where batches form and admissions
    wait for HBM footprint."""
    from paper_1509_03838_amd.serve import Server

    def rep_dict(rep):
        return {"jobs": rep.jobs, "jobs_per_s": round(rep.jobs_per_s, 1),
                "gout_per_s": round(rep.gout_per_s, 3), "p50_ms": round(rep.p50_ms, 3),
                "p99_ms": round(rep.p99_ms, 3), "max_ms": round(rep.max_ms, 3),
                "mean_batch": round(rep.mean_batch, 3), "batches": rep.batches,
                "deferred_jobs": rep.deferred_jobs, "peak_mib": round(rep.peak_bytes / 2**20, 1),
                "lost_jobs": rep.lost_jobs}
    srv = Server(hbm_budget=2 << 30, lanes=4, max_batch=64)
    srv.run(wl.serving_jobs(seed=wl.SEED_BASE + 40, count=200))  # warm-up traffic
    steady = srv.run(wl.serving_jobs(count=args.jobs), start_delay=0.0)
    del srv
    burst = Server(hbm_budget=256 << 20, lanes=1, max_batch=64)
    burst.run(wl.serving_jobs(seed=wl.SEED_BASE + 42, count=50, rate_hz=1e6))
    rep = burst.run(wl.serving_jobs(seed=wl.SEED_BASE + 43, count=400, rate_hz=1e6),
                    start_delay=0.0)
    return {"poisson_2000_per_s": rep_dict(steady),
            "burst_one_lane_256mib": rep_dict(rep)}


def time_captured(torch, plan, stream, steps, warmup):
    """(ms per launch by HIP events on the launch stream, ms per launch by the
    host clock) of a captured plan: `warmup` untimed launches, then `steps`
    timed ones, synchronized on both sides."""
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.launch(stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            plan.launch(stream)
        e1.record(stream)
        e1.synchronize()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def fig2_line(args, wl):
    """The paper's experiment (Sec. V, Fig. 2) on one GPU: M in {3, 8}
    streams of 10^6 samples convolved with K = 100 .. 4500 taps, no failures,
    the method against the failure-intolerant convolution (narrow and on the
    same datapath) and the checksum method. One group per point, its own
    captured plan; a step is one launch of every point's plan."""
    import numpy as np
    import torch
    from paper_1509_03838_amd import ne

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    tuner = None
    if not args.no_autotune and not args.conv_steps:
        from paper_1509_03838_amd.tune import DEFAULT_CACHE, Tuner
        tuner = Tuner(os.environ.get("NE_TUNE_CACHE", DEFAULT_CACHE))
    modes = ("entangled", "plain", "plain_same", "checksum")
    points, tot = [], {m: 0.0 for m in modes}
    samples_all = 0
    dominant = None
    for M in wl.FIG2_M:
        c = None
        for K in wl.FIG2_TAPS:
            g = wl.config_fig2(M, K)
            if c is None:  # the streams depend on M only
                c = [torch.from_numpy(np.ascontiguousarray(r)).to(dev) for r in g.c]
            k = torch.from_numpy(g.operand).to(dev)
            n_out = g.n + K - 1
            out = [torch.empty(n_out, dtype=torch.int64, device=dev) for _ in range(M)]
            ms, tuned, ref = {}, {}, None
            for mode in modes:
                spec = ne.GroupSpec("conv", c, k, out, 0, -1, wl.FIG2_BITS)
                if tuner is not None:
                    tuned.update(tuner.tune([spec], mode))
                plan = ne.Plan([spec], mode, conv_steps=args.conv_steps)
                plan.capture(stream)
                # a point runs for well under a millisecond: the first timed
                # pass doubles as warm-up, the second is kept
                time_captured(torch, plan, stream, args.steps, args.warmup)
                ms[mode], _ = time_captured(torch, plan, stream, args.steps, args.warmup)
                if mode == "entangled":
                    st = plan.stats()
                snap = torch.stack([o[::4999] for o in out]).cpu()
                if plan.flags() or (ref is not None and not torch.equal(snap, ref)):
                    raise SystemExit(f"fig2 M={M} K={K}: {mode} results differ or flagged")
                ref = snap
                plan.close()
            samples = M * n_out
            samples_all += samples
            for m in modes:
                tot[m] += ms[m]
            e = ms["entangled"]
            mfma = 2 * st["mfma_macs"] / (e * 1e-3) / 1e12
            pt = {
                "M": M, "K": K, "n": g.n,
                "ms": {m: round(v, 4) for m, v in ms.items()},
                "gout_per_s": {m: round(samples / (v * 1e-3) / 1e9, 3) for m, v in ms.items()},
                # the paper's measure: throughput lost against the plain run
                "throughput_loss_pct_vs_plain_same": round(100 * (1 - ms["plain_same"] / e), 2),
                "throughput_loss_pct_vs_plain": round(100 * (1 - ms["plain"] / e), 2),
                "checksum_throughput_loss_pct_vs_plain_same":
                    round(100 * (1 - ms["plain_same"] / ms["checksum"]), 2),
                "checksum_throughput_loss_pct_vs_plain":
                    round(100 * (1 - ms["plain"] / ms["checksum"]), 2),
                "mfma_i8_tops": round(mfma, 1), "mfma_frac": round(mfma / INT8_PEAK_TOPS, 4),
                "tuned": {kk.split("|", 1)[0]: v for kk, v in tuned.items()},
            }
            points.append(pt)
            print(f"# fig2 M={M} K={K}: " + ", ".join(f"{m} {v:.4f}" for m, v in ms.items()),
                  file=sys.stderr, flush=True)
            if dominant is None or e > dominant[0]:
                dominant = (e, pt, st)
            del out, k
    e, pt, st = dominant
    mfma = 2 * st["mfma_macs"] / (e * 1e-3) / 1e12
    hbm = (st["in_bytes"] + st["out_bytes"]) / (e * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(samples_all / (tot["entangled"] * 1e-3) / 1e9, 3),
        "unit": "Gout-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tot["entangled"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "fig2 sweep: one group per point, M in {3,8} streams x 10^6 "
                               "int32 samples uniform in [-2^14,2^14), K in "
                               f"{list(wl.FIG2_TAPS)} taps in the same range, no failures; "
                               "value = all points' outputs / the sum of their entangled times",
                   "points": len(points), "w": 64},
        "roofline": {"bound": "mfma", "achieved": round(mfma, 1), "peak": INT8_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(mfma / INT8_PEAK_TOPS, 4), "traffic": None,
                     "kernel": f"k_conv_fused at the longest point (M={pt['M']}, K={pt['K']})",
                     "hbm_GBps": round(hbm, 1)},
        "sweep_ms_total": {m: round(v, 4) for m, v in tot.items()},
        "sweep": points,
    }
    print(json.dumps(line), flush=True)


def chain_line(args, wl):
    """A series of operations on entangled streams (Sec. II): 3 streams of
    2^22 samples in [-2^9, 2^9); add a vector, scale, convolve with 64 taps,
    permute, add another vector (operands in the same range); one
    entanglement before the series and one extraction after it, against the
    same series on the raw streams. The line times ne_chain_run (three
    passes: entangle with [add, scale], conv, [perm, add] with the
    recovery); the three separate calls (entangle, ne_chain_apply, extract)
    are timed beside it."""
    import numpy as np
    import torch
    from paper_1509_03838_amd import ne

    dev = torch.device("cuda:0")
    M, n, bits = 3, 1 << 22, 10
    c = wl.uniform_i32(wl.rng(wl.SEED_BASE + 6), -(1 << (bits - 1)), 1 << (bits - 1), (M, n))
    ops = wl.chain_series(wl.rng(wl.SEED_BASE + 7), n, wl.CHAIN_RECIPE, bits=bits, K=64)
    l = ne.params(M)[0]
    stream = torch.cuda.Stream()

    def dev_ops(entangled):
        out = []
        for op, g, sc in ops:
            if op == "scale":
                out.append(ne.ChainOp(op, None, sc))
                continue
            dg = torch.from_numpy(np.ascontiguousarray(g)).to(dev)
            if op == "add":
                if entangled:
                    ge = torch.empty(g.size, dtype=torch.int64, device=dev)
                    ne.entangle_operand(dg, ge, l)
                    torch.cuda.synchronize()
                    dg = ge
                else:
                    dg = dg if out == [] else dg.to(torch.int64)
            out.append(ne.ChainOp(op, dg, sc, operand_bits=bits))
        return out

    ent_ops, plain_ops = dev_ops(True), dev_ops(False)
    n_out, bound = ne.chain_check(M, bits, n, ent_ops)
    cd = [torch.from_numpy(row).to(dev) for row in c]
    eps = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(M)]
    delta = [torch.empty(n_out, dtype=torch.int64, device=dev) for _ in range(M)]
    dhat = [torch.empty(n_out, dtype=torch.int64, device=dev) for _ in range(M)]
    first = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(M)]
    ws_e = torch.empty(ne.chain_workspace_size(M, n, ent_ops) + 256, dtype=torch.uint8, device=dev)
    ws_e = ws_e[(-ws_e.data_ptr()) % 256:]
    ws_p = torch.empty(ne.chain_workspace_size(M, n, plain_ops[1:]) + 256, dtype=torch.uint8,
                       device=dev)
    ws_p = ws_p[(-ws_p.data_ptr()) % 256:]
    ws_r = torch.empty(ne.chain_run_workspace_size(M, n, ent_ops) + 256, dtype=torch.uint8,
                       device=dev)
    ws_r = ws_r[(-ws_r.data_ptr()) % 256:]
    full = (1 << M) - 1

    def run_step(lost=-1):
        ne.chain_run(cd, ent_ops, dhat, lost, workspace=ws_r, stream=stream)

    def entangled_step(lost=-1):
        mask = full & ~(1 << lost) if lost >= 0 else full
        ne.entangle(cd, eps, l, stream=stream)
        ne.chain_apply(eps, ent_ops, delta, mask=mask, workspace=ws_e, stream=stream)
        ne.extract_recover([None if m == lost else delta[m] for m in range(M)], lost, dhat, l,
                           stream=stream)

    def plain_step():
        o0 = plain_ops[0]
        ne.plain_apply(o0.op, cd, o0.operand, first, o0.scalar, stream=stream)
        ne.chain_apply(first, plain_ops[1:], dhat, workspace=ws_p, stream=stream)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / args.steps

    t_plain = timed(plain_step)
    ref = torch.stack([t[::4099] for t in dhat]).cpu()
    same = True
    times = {}
    for name, fn in (("entangled", run_step), ("entangled_one_lost", lambda: run_step(1)),
                     ("entangled_three_calls", entangled_step),
                     ("entangled_three_calls_one_lost", lambda: entangled_step(1))):
        for t in dhat:
            t.fill_(0)
        times[name] = timed(fn)
        same = same and torch.equal(torch.stack([t[::4099] for t in dhat]).cpu(), ref)
    if not same:
        raise SystemExit("chain: entangled and plain results differ")
    t_ent, t_lost = times["entangled"], times["entangled_one_lost"]
    samples = M * n_out
    # algorithmic HBM bytes of one step of ne_chain_run: every pass reads its
    # inputs and operands once and writes its outputs once
    K = ops[2][1].size
    nb = (M * n * 4 + n * 8 + M * n * 8                       # entangle, add, scale
          + M * n * 8 + K * 4 + M * n_out * 8                 # conv
          + (M - 1) * n_out * 8 + n_out * (4 + 8) + M * n_out * 8)  # perm, add, recovery
    hbm = nb / (t_ent * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(samples / (t_ent * 1e-3) / 1e9, 3),
        "unit": "Gout-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_ent, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "series: 3 streams x 2^22 int32 samples in [-2^9,2^9), add -> "
                               "scale -> conv (64 taps) -> perm -> add, operands in the same range; "
                               "ne_chain_run: entanglement fused into the first run of "
                               "element-wise operations, recovery into the last",
                   "w": 64, "l": l, "worst_case_bound": bound},
        "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "all launches of the step (three passes)",
                     "alg_bytes_per_step": nb},
        "baselines": {"ms_per_step": dict({k: round(v, 4) for k, v in times.items()},
                                          plain=round(t_plain, 4)),
                      "overhead_pct_vs_plain": round(100 * (t_ent / t_plain - 1), 2),
                      "one_lost_overhead_pct_vs_plain": round(100 * (t_lost / t_plain - 1), 2)},
    }
    print(json.dumps(line), flush=True)


def _digits(neg: int, pos: int) -> int:
    """Fewest balanced base-256 digits covering [-neg, pos] (the kernels'
    digit rule, restated here to count the matrix-core work)."""
    R, p = 0, 1
    for L in range(1, 17):
        R += p
        p *= 256
        if 128 * R >= neg and 127 * R >= pos:
            return L
    return 17


def gemm_line(args, wl):
    """Entangled integer matrix product (Sec. IV's GEMM case): 3 blocks of
    4096 x 1024 int32 values times one 1024 x 4096 kernel matrix, values in
    [-2^11, 2^11); entangle on load, product on the i8 matrix cores, recover
    in registers, one launch; against the plain product (narrow and on the
    same datapath), the checksum method and one lost block."""
    import numpy as np
    import torch
    from paper_1509_03838_amd import ne

    dev = torch.device("cuda:0")
    c, g = wl.config_gemm()
    M, N, P = c.shape
    Q = g.shape[1]
    bits = wl.GEMM_BITS
    cd = [torch.from_numpy(np.ascontiguousarray(b)).to(dev) for b in c]
    gd = torch.from_numpy(g).to(dev)
    out = [torch.empty((N, Q), dtype=torch.int64, device=dev) for _ in range(M)]
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()

    wsz = max(ne.gemm_workspace_size(m, M, N, P, Q, bits)
              for m in ("entangled", "plain", "plain_same", "checksum"))
    ws_all = torch.empty(wsz + 256, dtype=torch.uint8, device=dev)
    ws_all = ws_all[(-ws_all.data_ptr()) % 256:][:wsz]

    def timed(mode, lost=-1, split=True):
        ws = ws_all[:ne.gemm_workspace_size(mode, M, N, P, Q, bits)] if split else None
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                ne.gemm(cd, gd, out, mode, lost, bits, flags=flags, stream=stream, workspace=ws)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                ne.gemm(cd, gd, out, mode, lost, bits, flags=flags, stream=stream, workspace=ws)
            e1.record(stream)
            e1.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms, ms_fused = {}, {}
    ref = None
    for split, table in ((True, ms), (False, ms_fused)):
        for mode in ("entangled", "plain", "plain_same", "checksum"):
            table[mode] = timed(mode, split=split)
            snap = torch.stack([o[::97, ::89] for o in out]).cpu()
            if int(flags.item()) or (ref is not None and not torch.equal(snap, ref)):
                raise SystemExit(f"gemm: {mode} results differ or flagged")
            ref = snap
        table["entangled_one_lost"] = timed("entangled", 1, split=split)
    B = 1 << (bits - 1)
    l = ne.params(M)[0]
    # the reference count: conventional digits of the entangled words (eq. (14)
    # words cut into base-256 digits) times the kernel matrix's digits; the
    # library issues fewer where it splits words into two fields
    la = _digits(B * ((1 << l) + 1), (B - 1) * ((1 << l) + 1))
    lb = _digits(B, B - 1)
    pairs = sum(1 for a in range(la) for b in range(lb) if a + b < 8)
    fs = _digits(B, B - 1)
    pairs_issued = 2 * fs * lb if 2 * fs < la and B <= 1 << (l - 1) else pairs
    pad = lambda x, t: (x + t - 1) // t * t
    mfma_ops = 2 * M * pad(N, 32) * pad(Q, 64) * pad(P, 64) * pairs
    issued_ops = 2 * M * pad(N, 32) * pad(Q, 64) * pad(P, 64) * pairs_issued
    useful_ops = 2 * M * N * P * Q
    e = ms["entangled"]
    tops = mfma_ops / (e * 1e-3) / 1e12
    samples = M * N * Q
    alg_bytes = M * N * P * 4 + P * Q * 4 + M * N * Q * 8
    line = {
        "metric": METRIC, "value": round(samples / (e * 1e-3) / 1e9, 3),
        "unit": "Gout-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(e, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"gemm: {M} blocks of {N}x{P} int32 values in [-2^11,2^11) times "
                               f"one {P}x{Q} kernel matrix, entangled (l={l}); two-phase form "
                               "(digit planes through workspace, then the matrix-core kernel)",
                   "w": 64, "digits": [la, lb]},
        "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": INT8_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(tops / INT8_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "digit planes + k_gemm_digits + recovery, whole call (i8 ops of the "
                               f"reference count: {pairs} digit pairs x padded tiles)",
                     "digit_pairs_issued": pairs_issued,
                     "issued_tops": round(issued_ops / (e * 1e-3) / 1e12, 1),
                     "useful_int_tops": round(useful_ops / (e * 1e-3) / 1e12, 2),
                     "hbm_GBps": round(alg_bytes / (e * 1e-3) / 1e9, 1)},
        "baselines": {"ms_per_step": {k: round(v, 4) for k, v in ms.items()},
                      "one_launch_form_ms_per_step": {k: round(v, 4) for k, v in ms_fused.items()},
                      "overhead_pct_vs_plain_same": round(100 * (e / ms["plain_same"] - 1), 2),
                      "overhead_pct_vs_plain": round(100 * (e / ms["plain"] - 1), 2),
                      "checksum_overhead_pct_vs_plain_same":
                          round(100 * (ms["checksum"] / ms["plain_same"] - 1), 2)},
    }
    print(json.dumps(line), flush=True)


def ops_line(args, wl):
    """The other operators of eq. (2) on the per-step path: for each of
    subtraction, element-by-element product, circular convolution (64 taps),
    cross-correlation (64 taps) and outer product (8 values), 3 streams of
    2^22 samples in [-2^9, 2^9) through entangle -> op -> extract, against
    the plain op on the raw streams; and the same operation in the fused
    executor (one pass, one captured launch)."""
    import numpy as np
    import torch
    from paper_1509_03838_amd import ne

    dev = torch.device("cuda:0")
    M, n, bits = 3, 1 << 22, 10
    rng = wl.rng(wl.SEED_BASE + 9)
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    c = wl.uniform_i32(rng, lo, hi, (M, n))
    l = ne.params(M)[0]
    stream = torch.cuda.Stream()
    cd = [torch.from_numpy(row).to(dev) for row in c]
    eps = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(M)]
    sizes = {"sub": n, "mul": n, "circ": 64, "xcorr": 64, "outer": 8}

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / args.steps

    rows, tot_samples, tot_ms, tot_bytes = {}, 0, 0.0, 0
    for op, K in sizes.items():
        g = wl.uniform_i32(rng, lo, hi, K)
        g32 = torch.from_numpy(g).to(dev)
        operand = g32
        if op == "sub":
            operand = torch.empty(n, dtype=torch.int64, device=dev)
            ne.entangle_operand(g32, operand, l, stream=stream)
        no = ne.n_out(op, n, K)
        delta = [torch.empty(no, dtype=torch.int64, device=dev) for _ in range(M)]
        dhat = [torch.empty(no, dtype=torch.int64, device=dev) for _ in range(M)]

        def ent():
            ne.entangle(cd, eps, l, stream=stream)
            ne.lsb_apply(op, eps, operand, delta, n_in=n, stream=stream)
            ne.extract_recover(delta, -1, dhat, l, stream=stream)

        def plain():
            ne.plain_apply(op, cd, g32, dhat, stream=stream)

        t_plain = timed(plain)
        ref = torch.stack([t[::4099] for t in dhat]).cpu()
        t_ent = timed(ent)
        if not torch.equal(torch.stack([t[::4099] for t in dhat]).cpu(), ref):
            raise SystemExit(f"ops: {op} entangled and plain results differ")
        fused = {}
        # the same operation in the fused executor: one pass, one captured launch
        for mode in ("entangled", "plain"):
            spec = ne.GroupSpec(op, cd, g32, dhat, 0, -1, bits)
            plan = ne.Plan([spec], mode)
            plan.capture(stream)
            fused[mode], _ = time_captured(torch, plan, stream, args.steps, args.warmup)
            same = torch.equal(torch.stack([t[::4099] for t in dhat]).cpu(), ref)
            if plan.flags() or not same:
                raise SystemExit(f"ops: fused {op} ({mode}) differs from the per-step result")
            plan.close()
        # algorithmic HBM bytes of the three launches: entangle, op, extract
        nb = (M * n * 12 + M * (n + no) * 8 + operand.numel() * operand.element_size() +
              (2 * M - 1) * no * 8)
        rows[op] = {"K": K, "n_out": no, "ms": {"entangled": round(t_ent, 4), "plain": round(t_plain, 4)},
                    "gout_per_s": round(M * no / (t_ent * 1e-3) / 1e9, 3),
                    "hbm_GBps": round(nb / (t_ent * 1e-3) / 1e9, 1),
                    "overhead_pct_vs_plain": round(100 * (t_ent / t_plain - 1), 2)}
        if fused:
            fb = M * n * 4 + g32.numel() * 4 + M * no * 8  # one pass: inputs in, outputs out
            rows[op]["fused_ms"] = {k: round(v, 4) for k, v in fused.items()}
            rows[op]["fused_gout_per_s"] = round(M * no / (fused["entangled"] * 1e-3) / 1e9, 3)
            rows[op]["fused_hbm_GBps"] = round(fb / (fused["entangled"] * 1e-3) / 1e9, 1)
        tot_samples += M * no
        tot_ms += t_ent
        tot_bytes += nb
        print(f"# ops {op}: per-step entangled {t_ent:.4f} ms, plain {t_plain:.4f} ms; fused "
              + ", ".join(f"{k} {v:.4f} ms" for k, v in fused.items()), file=sys.stderr, flush=True)
        del delta, dhat
    line = {
        "metric": METRIC, "value": round(tot_samples / (tot_ms * 1e-3) / 1e9, 3),
        "unit": "Gout-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tot_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "operators: 3 streams x 2^22 int32 samples in [-2^9,2^9); sub, mul, "
                               "circ (64 taps), xcorr (64 taps), outer (8 values); entangle -> op -> "
                               "extract per-step kernels; value = all outputs / the sum of times",
                   "w": 64, "l": l},
        "roofline": {"bound": "hbm", "achieved": round(tot_bytes / (tot_ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(tot_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "all launches of the five pipelines (per-operator rows below; the "
                               "convolution-like ones are bound by the vector ALUs)"},
        "ops": rows,
    }
    print(json.dumps(line), flush=True)


def w32_line(args, wl):
    """32-bit entangled words (the paper's practical w = 32, l = 11 for
    M = 3) on a workload whose range fits them: 3 streams of 2^22 samples in
    [-2^7, 2^7), 16-tap convolution (the small configuration's range, worst
    case 2^18 <= D = 1,046,528), stream 1 lost. The line times the fused
    executor with int32 outputs (one captured launch); baselines: the same
    with 64-bit words, the plain fused convolution with int32 outputs, and
    the per-step pipeline (entangle -> conv -> extract) in 32- and 64-bit
    words against the plain per-step convolution; and a series in these
    words (add -> conv -> perm -> add, worst case 2^19 + 2^7) through
    ne_chain_run32 against its three separate calls."""
    import numpy as np
    import torch
    from paper_1509_03838_amd import ne

    dev = torch.device("cuda:0")
    M, n, K = 3, 1 << 22, 16
    rng = wl.rng(wl.SEED_BASE + 11)
    c = wl.uniform_i32(rng, -128, 128, (M, n))
    g = wl.uniform_i32(rng, -128, 128, K)
    no = n + K - 1
    l32, l64 = ne.params(M, 32)[0], ne.params(M)[0]
    stream = torch.cuda.Stream()
    cd = [torch.from_numpy(row).to(dev) for row in c]
    gd = torch.from_numpy(g).to(dev)
    e32 = [torch.empty(n, dtype=torch.int32, device=dev) for _ in range(M)]
    d32 = [torch.empty(no, dtype=torch.int32, device=dev) for _ in range(M)]
    o32 = [torch.empty(no, dtype=torch.int32, device=dev) for _ in range(M)]
    e64 = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(M)]
    d64 = [torch.empty(no, dtype=torch.int64, device=dev) for _ in range(M)]
    o64 = [torch.empty(no, dtype=torch.int64, device=dev) for _ in range(M)]
    lost, mask = 1, 0b101

    def w32():
        ne.entangle32(cd, e32, l32, stream=stream)
        ne.lsb_apply32("conv", e32, gd, d32, mask=mask, stream=stream)
        ne.extract_recover32([d32[0], None, d32[2]], lost, o32, l32, stream=stream)

    def w64():
        ne.entangle(cd, e64, l64, stream=stream)
        ne.lsb_apply("conv", e64, gd, d64, mask=mask, stream=stream)
        ne.extract_recover([d64[0], None, d64[2]], lost, o64, l64, stream=stream)

    def plain():
        ne.plain_apply("conv", cd, gd, o64, stream=stream)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / args.steps

    t_plain = timed(plain)
    ref = torch.stack([t[::4099] for t in o64]).cpu()
    t64 = timed(w64)
    t32 = timed(w32)
    same = torch.equal(torch.stack([t[::4099] for t in o64]).cpu(), ref) and torch.equal(
        torch.stack([t[::4099] for t in o32]).cpu().to(torch.int64), ref)

    def fused(mode, word_bits):
        out = o32 if word_bits == 32 else o64
        spec = ne.GroupSpec("conv", cd, gd, out, 0, lost if mode == "entangled" else -1, 8,
                            word_bits=word_bits)
        plan = ne.Plan([spec], mode)
        plan.capture(stream)
        t, _ = time_captured(torch, plan, stream, args.steps, args.warmup)
        got = torch.stack([x[::4099] for x in out]).cpu().to(torch.int64)
        ok = not plan.flags() and torch.equal(got, ref)
        plan.close()
        return t, ok

    t_fused64, ok64 = fused("entangled", 0)
    t_fused32, ok32 = fused("entangled", 32)
    t_fplain32, okp = fused("plain", 32)
    if not (same and ok64 and ok32 and okp):
        raise SystemExit("w32: the 32-bit, 64-bit, fused and plain results differ")

    # a series in 32-bit words: one call against three
    sops = wl.chain_series(wl.rng(wl.SEED_BASE + 12), n, ("add", "conv", "perm", "add"), bits=8,
                           K=K)
    chain = []
    for op, gv, sc in sops:
        dg = torch.from_numpy(np.ascontiguousarray(gv)).to(dev)
        if op == "add":
            ge = torch.empty_like(dg)
            ne.entangle_operand32(dg, ge, l32)
            dg = ge
        chain.append(ne.ChainOp(op, dg, sc, operand_bits=8))
    torch.cuda.synchronize()
    sno, _ = ne.chain_check(M, 8, n, chain, w=32)
    s_one = [torch.empty(sno, dtype=torch.int32, device=dev) for _ in range(M)]
    s_three = [torch.empty(sno, dtype=torch.int32, device=dev) for _ in range(M)]
    s_delta = [torch.empty(sno, dtype=torch.int32, device=dev) for _ in range(M)]
    ws_run = torch.empty(ne.chain_run_workspace_size(M, n, chain, w=32) + 256, dtype=torch.uint8,
                         device=dev)
    ws_run = ws_run[(-ws_run.data_ptr()) % 256:]
    ws_apply = torch.empty(ne.chain_workspace_size(M, n, chain, w=32) + 256, dtype=torch.uint8,
                           device=dev)
    ws_apply = ws_apply[(-ws_apply.data_ptr()) % 256:]

    def series_one():
        ne.chain_run(cd, chain, s_one, lost, workspace=ws_run, stream=stream, w=32)

    def series_three():
        ne.entangle32(cd, e32, l32, stream=stream)
        ne.chain_apply(e32, chain, s_delta, mask=mask, workspace=ws_apply, stream=stream, w=32)
        ne.extract_recover32([s_delta[0], None, s_delta[2]], lost, s_three, l32, stream=stream)

    t_series1 = timed(series_one)
    t_series3 = timed(series_three)
    if not all(torch.equal(a, b) for a, b in zip(s_one, s_three)):
        raise SystemExit("w32: the series' one-call and three-call results differ")
    # algorithmic HBM bytes of the per-step launches (two streams computed)
    def nbytes(word):
        return (M * n * (4 + word) + (M - 1) * (n + no) * word + K * 4 +
                (M - 1) * no * word + M * no * word)
    b32, b64 = nbytes(4), nbytes(8)
    fb32 = M * n * 4 + K * 4 + M * no * 4  # the fused launch: inputs in, outputs out
    hbm = fb32 / (t_fused32 * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(M * no / (t_fused32 * 1e-3) / 1e9, 3),
        "unit": "Gout-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_fused32, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "32-bit words: 3 streams x 2^22 int32 samples in [-2^7,2^7), "
                               "16-tap conv, stream 1 lost; fused executor, one captured launch, "
                               "int32 outputs",
                   "w": 32, "l": l32, "D": ne.params(M, 32)[2]},
        "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_conv_fused (one launch)", "alg_bytes_per_launch": fb32},
        "baselines": {"ms_per_step": {"fused_w32": round(t_fused32, 4),
                                      "fused_w64": round(t_fused64, 4),
                                      "fused_plain_w32": round(t_fplain32, 4),
                                      "per_step_w32": round(t32, 4), "per_step_w64": round(t64, 4),
                                      "per_step_plain": round(t_plain, 4)},
                      "per_step_alg_bytes": {"w32": b32, "w64": b64},
                      "per_step_hbm_GBps_w32": round(b32 / (t32 * 1e-3) / 1e9, 1),
                      "speedup_w32_vs_w64": {"fused": round(t_fused64 / t_fused32, 3),
                                             "per_step": round(t64 / t32, 3)},
                      "series_w32": {"recipe": "add -> conv (16 taps) -> perm -> add, "
                                               "8-bit operands, stream 1 lost",
                                     "ms_per_step": {"ne_chain_run32": round(t_series1, 4),
                                                     "three_calls": round(t_series3, 4)}}},
    }
    print(json.dumps(line), flush=True)


def serve_line(args, wl):
    """Serving: Poisson arrivals (2000 jobs/s), M in {3,4,5}, n log-uniform
    [2^10, 2^20], taps log-uniform [16, 1024], 1% single-stream drops,
    admission by HBM footprint, continuous batching over 4 HIP streams."""
    from paper_1509_03838_amd.serve import Server
    srv = Server(hbm_budget=args.budget_mib << 20, lanes=4, max_batch=64)
    # warm-up traffic (other seeds) until the server is in a steady state:
    # kernel variants loaded, clocks up; the timed run follows at once
    srv.run(wl.serving_jobs(seed=wl.SEED_BASE + 40, count=200))
    srv.run(wl.serving_jobs(seed=wl.SEED_BASE + 41, count=400), start_delay=0.0)
    jobs = wl.serving_jobs(count=args.jobs)
    rep = srv.run(jobs, start_delay=0.0)
    line = {
        "metric": METRIC, "value": round(rep.gout_per_s, 3), "unit": "Gout-samples/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(rep.makespan_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson 2000 jobs/s, M in {3,4,5}, n log-uniform "
                               "[2^10,2^20] int32 in [-2^10,2^10), taps log-uniform [16,1024], "
                               "1% single-stream drops, HBM-footprint admission, 4 lanes",
                   "jobs": rep.jobs, "budget_mib": args.budget_mib},
        "latency_ms": {"p50": round(rep.p50_ms, 3), "p99": round(rep.p99_ms, 3),
                       "mean": round(rep.mean_ms, 3), "max": round(rep.max_ms, 3)},
        "serving": {k: (round(v, 4) if isinstance(v, float) else v)
                    for k, v in rep.as_dict().items()},
    }
    print(json.dumps(line), flush=True)


def tuned_summary(tuned, mode):
    """The autotuner's choices for the timed mode: the table itself when it
    is short, else a histogram {steps: classes}."""
    mine = {k: v for k, v in tuned.items() if k.startswith(mode + "|") and "|plan|" not in k}
    whole = [v for k, v in tuned.items() if k.startswith(mode + "|plan|")]
    if len(mine) <= 8:
        out = dict(mine)
    else:
        hist = {}
        for v in mine.values():
            hist[str(v)] = hist.get(str(v), 0) + 1
        out = {"classes": len(mine), "steps_histogram": hist}
    if whole:
        out["whole_plan"] = whole[-1]  # tuned choices kept, or the planner's defaults
    return out


def stats_kernel_name(stats, groups, mode):
    g = groups[0]
    return "k_conv_fused" if g.op == "conv" else "k_stream_fused"


def _batched(wl, args):
    groups = wl.config_batched(groups=args.groups)
    g = groups[0]
    return groups, 12, (f"batched M={g.M}: {len(groups)} stream-triples x {g.n:,} int32 samples "
                        f"uniform in [-2^11,2^11), {g.operand.size}-tap int32 kernels, full linear "
                        "convolution, entangle+conv+recover fused, one graph launch")


def _small(wl, args):
    return [wl.config_small()], 8, ("small: M=3 x 65,536 int32 samples uniform in [-128,127], "
                                    "16-tap kernel, full linear convolution")


def _uneven(wl, args):
    groups = wl.config_uneven(groups=args.groups if args.groups != 64 else 512)
    return groups, 10, (f"uneven: {len(groups)} groups, M in 3..8, n log-uniform [2^12,2^22], "
                        "int32 samples in [-2^9,2^9), conv taps log-uniform [8,512], ops mixed "
                        "(conv/scale/add/inner/perm), one graph launch")


def _long(wl, args):
    groups = wl.config_long_kernel(groups=args.groups if args.groups != 64 else 256)
    return groups, 16, (f"long kernel: {len(groups)} stream-triples x 262,144 int16-range samples "
                        "held as int32, 1024-tap kernels, i8-MFMA Toeplitz convolution")


CONFIGS = {"batched": _batched, "small": _small, "uneven": _uneven, "long": _long}


def gpu_info(torch) -> dict:
    """The device the line was measured on: name, architecture, compute units,
    memory, and its clocks as rocm-smi reports them (if it is there)."""
    import subprocess
    p = torch.cuda.get_device_properties(0)
    info = {"name": p.name, "arch": getattr(p, "gcnArchName", ""),
            "compute_units": p.multi_processor_count, "memory_GiB": round(p.total_memory / 2**30, 1)}
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=20)
        card = next(iter(json.loads(r.stdout).values()))
        info["clocks_rocm_smi"] = {k: v for k, v in card.items()
                                   if any(c in k for c in ("sclk", "mclk", "fclk", "socclk"))}
    except Exception:  # no rocm-smi, or output it cannot parse: the clocks stay out
        pass
    return info


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(groups, np):
    """The CPU oracle (entangle, convolve, recover; 128-bit C), one group per
    host thread: on all the host threads this job may use (at most 16, the
    CPU share of one GPU) over the whole batch, and on one thread over the
    first 4 groups."""
    import concurrent.futures as cf

    import oracle

    oracle.lib()

    def rate(gs, threads):
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            outs = list(ex.map(lambda g: oracle.pipeline(g.c, "conv", g.operand, r=1)[0].size,
                               gs))
        dt = time.perf_counter() - t0
        return sum(outs) / dt / 1e9, dt

    threads = max(1, min(16, os.cpu_count() or 1))
    v_all, dt_all = rate(groups, threads)
    one = groups[:4]
    v_one, dt_one = rate(one, 1)
    return {"value": round(v_all, 5), "unit": "Gout-samples/s", "cores": threads,
            "kind": "oracle",
            "sample": f"all {len(groups)} groups of the batch, one lost stream each, "
                      f"{threads} threads, {dt_all:.1f} s",
            "single_thread": {"value": round(v_one, 5), "cores": 1,
                              "sample": f"the first {len(one)} groups, one lost stream each, "
                                        f"{dt_one:.1f} s"},
            "host_logical_cpus": os.cpu_count(), "cpu_model": cpu_model()}


if __name__ == "__main__":
    main()
