"""Benchmark: bitmap-filtered exact self-join of 1,000,000 sets at Jaccard t = 4/5.

One step is one full ssj_self_join call on device-resident input: size sort,
Bitmap-Xor build (width per row-size class, chosen by the library), bitmap
filter over the length band, exact verification, sorting and copying the pairs
to host memory.  The metric is
length-band pairs per second of wall time (pairs the join accounts for, the
paper's GPU algorithm evaluates every one of them with the bitmap filter).
After the timed joins the default run adds, in the same line: the prepared
join's graph replay, the pair list's parity against the oracle's stored list,
the CPU oracle's rate on a row sample, the served form's p50/p99 latency
(query batches against a resident 5,000,000-set index under continuous
batching), and the batched form (256 uneven instances in one call against one
call each).

Other modes (not the default):
  --mode batch   256 uneven self-join instances: one ssj_self_join_batch call
                 per step, against the same instances as sequential calls;
  --mode serve   R-S query batches against a resident 5,000,000-set index
                 under continuous batching, Poisson arrivals at several loads:
                 p50/p99 latency, batches/s and pairs/s.

Prints one JSON line on stdout.  Details go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT_OPS = 256 * 64 * 2.4e9   # int32 lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
PEAK_FP4 = 10.1e15                # dense fp4 MFMA flop/s (published)
PEAK_HBM = 8.0e12                 # bytes/s
MFMA_BITS = (64, 128, 256)        # widths the matrix-core filter runs
MFMA_MIN_BAND = 1 << 26           # ... and b = 256 only for a class of at least this many band pairs
# arithmetic of the path: the matrix-core filter multiplies +-1 values held in
# fp4 and accumulates them in fp32 (exact integers); every other step is
# integer arithmetic on uint32 tokens, sizes and counts
DTYPE_MFMA = "fp4 (+-1) products, fp32 accumulation (exact); u32 elsewhere"
DTYPE_INT = "u32"

# HBM bytes per launch of the dominant filter launch (the b = 64 class of the
# 1,000,000-set workload at 4/5, matrix-core kernel), from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by what the
# same counters read for a 1 GiB device copy (FETCH_SIZE reads 0.5 GiB for
# it: factor 2.0; WRITE_SIZE 1 GiB: factor 1.0).  Valid only for the kernel
# sources they were taken with: any change to them makes the figure null
# until the counters are taken again.  The summary and commands are in
# profiles/.
TRAFFIC = {"sources_sha256": "ab9c8c822b76a9f0b4e156c8f4e139b0189aa582ecf7580c880fe594d9e5196a",
           "fetch_kib": 75345.3, "write_kib": 11357.7,
           "fetch_factor": 1.9999, "write_factor": 1.0000}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_filter.hip", "ssj_internal.h"):
        with open(os.path.join(ROOT, "paper_1711_07295_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes():
    t = TRAFFIC
    if not t["sources_sha256"] or t["sources_sha256"] != kernel_sources_sha256():
        return None
    return (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"]) * 1024


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(col, p, q, sim=0, fraction=0.005):
    """The oracle (banded, plain C, all host threads) on a deterministic sample:
    every 1/fraction-th row of the size order, each against its whole band."""
    import numpy as np
    import oracle
    threads = host_threads()
    order = oracle.size_order(col.offsets)
    step = int(round(1 / fraction))
    rows = np.arange(step // 2, col.n_sets, step, dtype=np.uint64)
    t0 = time.perf_counter()
    _, evaluated = oracle.self_join_banded(col.offsets, col.tokens, p, q, sim=sim, rows=rows,
                                           order=order, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": evaluated / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"{len(rows)} rows (every {step}th in size order) x their length band: "
                      f"{evaluated} pairs merged in {dt:.1f} s on {threads} threads"}


def host_threads():
    """Threads the oracle runs on: every CPU this process may use, at most 16
    (the host share that goes with one GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=("selfjoin", "batch", "serve"), default="selfjoin")
    ap.add_argument("--instances", type=int, default=256, help="batch mode: instances")
    ap.add_argument("--serve-batches", type=int, default=2000,
                    help="serve mode: measured batches per load (plus 100 warm-up)")
    ap.add_argument("--resident", type=int, default=5_000_000,
                    help="serve mode: sets in the resident index")
    ap.add_argument("--slots", type=int, default=2,
                    help="served form: calls in flight at once (continuous batching)")
    ap.add_argument("--batch-instances-default", type=int, default=256,
                    help="default mode: instances of the batched leg (0 disables it)")
    ap.add_argument("--serve-batches-default", type=int, default=1000,
                    help="default mode: measured query batches of the served leg "
                         "(0 = no served leg)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="selfjoin-1m")
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--q", type=int, default=5)
    ap.add_argument("--sim", choices=("jaccard", "dice", "cosine", "overlap"), default="jaccard")
    ap.add_argument("--bits", type=int, default=0,
                    help="bitmap width; 0 = automatic width per row-size class")
    ap.add_argument("--tile-cols", type=int, default=0, help="0 = the library default")
    ap.add_argument("--cutoff", action="store_true",
                    help="rows past the cutoff point take prefix-filtered candidates")
    ap.add_argument("--valu", action="store_true",
                    help="vector-ALU filter at every width (SSJ_FLAG_VALU) instead of the "
                         "matrix cores")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the join is measured on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1711_07295_amd as ssj

    torch.cuda.set_device(0)
    if args.mode == "batch":
        return run_batch(args)
    if args.mode == "serve":
        return run_serve(args)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n} bytes 3 times (read {n} and write {n} bytes per copy)")
        return
    t0 = time.perf_counter()
    col = gen.workload(args.workload)
    log(f"generated {args.workload}: {col.n_sets} sets, {col.n_tokens} tokens in "
        f"{time.perf_counter() - t0:.1f} s, checksum {col.checksum():#x}")
    dev = ssj.to_device(col.offsets, col.tokens)
    torch.cuda.synchronize()

    flags = (ssj.SSJ_FLAG_CUTOFF if args.cutoff else 0) | (ssj.SSJ_FLAG_VALU if args.valu else 0)
    sim = {"jaccard": ssj.SSJ_SIM_JACCARD, "dice": ssj.SSJ_SIM_DICE,
           "cosine": ssj.SSJ_SIM_COSINE, "overlap": ssj.SSJ_SIM_OVERLAP}[args.sim]

    def step():
        return ssj.ssj_self_join(dev, args.p, args.q, b_bits=args.bits, tile_cols=args.tile_cols,
                                 sim=sim, flags=flags)

    for w in range(args.warmup):
        pairs, st = step()
        log(f"warmup {w}: {len(pairs)} pairs, {st['ms_total']:.2f} ms")
    torch.cuda.synchronize()
    times, stats = [], []
    t_all = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        pairs, st = step()
        times.append(time.perf_counter() - t1)
        stats.append(st)
        log(f"step {k}: {times[-1] * 1e3:.2f} ms  filter {st['ms_filter']:.2f} ms  "
            f"verify {st['ms_verify']:.2f}  prepare {st['ms_prepare']:.2f}  "
            f"emit {st['ms_emit']:.2f}  survivors {st['survivors']}  results {st['results']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    graph = None
    if args.bits == 0 and not args.valu and args.sim == "jaccard":
        graph = graph_replay([dev], [args.p], [args.q], args, [pairs])

    band = stats[0]["band_pairs"]
    ms_per_step = total / args.steps * 1e3
    value = band / (total / args.steps)
    # roofline of the dominant kernel: the filter launch of the width class
    # with the most algorithmic work.  Per band pair the filter's algorithmic
    # work is b/32 xor + b/32 popcount-accumulate + 1 compare (int32
    # lane-ops) at the width of the pair's row class; the library reports that
    # work per class, and times every launch with events on its stream.
    s0 = stats[0]
    ncls = s0["n_classes"]
    roof = roofline_of(stats, args.steps, args.valu)
    dom = max(range(ncls), key=lambda k: s0["class_ops"][k])
    if (args.workload == "selfjoin-1m" and (args.p, args.q) == (4, 5) and args.bits == 0
            and args.sim == "jaccard" and s0["class_bits"][dom] == 64 and not args.valu
            and roof is not None):
        roof["traffic"] = traffic_bytes()
    classes = [{"max_set_size": m, "b_bits": b, "ops": o, "ms": sum(s["class_ms"][k]
                for s in stats) / args.steps}
               for k, (m, b, o) in enumerate(zip(s0["class_max_size"][:ncls],
                                                 s0["class_bits"][:ncls],
                                                 s0["class_ops"][:ncls]))]
    line = {
        "metric": "pairs/sec (bitmap-filtered join, 1M sets, J>=0.8) + p50/p99 query latency",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": (DTYPE_MFMA if s0["class_bits"][dom] in MFMA_BITS and not args.valu
                  else DTYPE_INT), "data": "synthetic",
        "config": {"workload": args.workload, "n_sets": col.n_sets,
                   "threshold": f"{args.p}/{args.q}", "similarity": args.sim,
                   "cutoff": args.cutoff, "filter": "valu" if args.valu else "mfma",
                   "b_bits": args.bits if args.bits else "auto", "width_classes": classes,
                   "generator": "Bitmap-Xor",
                   "band_pairs": band, "results": stats[0]["results"],
                   "checksum": f"{col.checksum():#x}"},
        "step_ms": {"p50": statistics.median(times) * 1e3,
                    "p99": float(np.percentile(np.array(times), 99)) * 1e3},
        "stage_ms": {k: statistics.mean(s[k] for s in stats)
                     for k in ("ms_prepare", "ms_filter", "ms_verify", "ms_emit")},
        "roofline": roof,
        "parity": golden_parity(args.workload, col.checksum(), args.sim, args.p, args.q, pairs),
        "cpu_baseline": None,
    }
    if graph:
        line["graph_replay"] = {**graph, "speedup_vs_call": ms_per_step / graph["ms_per_step"]}
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a 0.5% row sample ...")
        line["cpu_baseline"] = cpu_baseline(col, args.p, args.q, sim)
        log(f"cpu baseline: {line['cpu_baseline']}")
    if args.serve_batches_default:
        # the metric's latency half: query batches against the resident
        # 5,000,000-set index at 0.95 of the plain service rate
        del dev
        torch.cuda.empty_cache()
        sv = served_legs(args.resident, args.serve_batches_default, (0.95,), slots=args.slots)
        head = sv["loads"][0]
        line["latency"] = {"p50_ms": head["continuous"]["p50_ms"],
                           "p99_ms": head["continuous"]["p99_ms"], "rho": 0.95,
                           "workload": f"served-{sv['resident_sets']}",
                           "measured_batches": sv["batches"] - sv["warm_up_batches"],
                           "plain_p50_ms": head["plain"]["p50_ms"],
                           "plain_p99_ms": head["plain"]["p99_ms"],
                           "plain_service_rate": sv["plain_service_rate"]}
        line["served_vs_plain"] = {"p50": head["p50_plain_over_continuous"],
                                   "p99": head["p99_plain_over_continuous"]}
        line["served"] = sv
    if args.batch_instances_default:
        # the batched form: one call for many uneven instances against one
        # call per instance, and the prepared call replayed from a graph
        torch.cuda.empty_cache()
        line["batched"] = batched_leg(args.batch_instances_default)
    print(json.dumps(line), flush=True)


def batched_leg(n_instances, steps=3):
    """ssj_self_join_batch over the first ``n_instances`` batched instances
    (automatic widths) against the same instances one ssj_self_join call
    each, and the prepared call's replay; pairs must agree."""
    import numpy as np
    import torch

    import gen
    import paper_1711_07295_amd as ssj

    t0 = time.perf_counter()
    inst = gen.batched_instances(n_instances)
    log(f"batched leg: generated {len(inst)} instances in {time.perf_counter() - t0:.1f} s")
    devs = [ssj.to_device(c.offsets, c.tokens) for c, _ in inst]
    ps, qs = [t[0] for _, t in inst], [t[1] for _, t in inst]
    torch.cuda.synchronize()
    got, st = ssj.ssj_self_join_batch(devs, ps, qs)  # warm-up
    times = []
    for _ in range(steps):
        t1 = time.perf_counter()
        got, st = ssj.ssj_self_join_batch(devs, ps, qs)
        times.append(time.perf_counter() - t1)
    t1 = time.perf_counter()
    seq = [ssj.ssj_self_join(d, p, q, b_bits=0)[0] for d, p, q in zip(devs, ps, qs)]
    seq_ms = (time.perf_counter() - t1) * 1e3
    same = all(np.array_equal(a, b) for a, b in zip(got, seq))
    plan = ssj.Plan(devs, ps, qs)
    plan.execute()
    rt = []
    for _ in range(steps):
        t1 = time.perf_counter()
        again, _ = plan.execute()
        rt.append(time.perf_counter() - t1)
    plan.close()
    same = same and all(np.array_equal(a, b) for a, b in zip(got, again))
    ms = statistics.median(times) * 1e3
    out = {"workload": f"batched-{len(inst)}", "instances": len(inst),
           "n_sets": int(sum(c.n_sets for c, _ in inst)), "band_pairs": st["band_pairs"],
           "results": st["results"], "ms_per_call": ms, "pairs_per_s": st["band_pairs"] / (ms / 1e3),
           "sequential_ms": seq_ms, "speedup_vs_sequential": seq_ms / ms,
           "graph_replay_ms": statistics.median(rt) * 1e3,
           "graph_speedup_vs_sequential": seq_ms / (statistics.median(rt) * 1e3),
           "same_pairs": same}
    log(f"batched leg: {out}")
    return out


def golden_parity(workload, checksum, sim, p, q, pairs):
    """The timed join's pairs against the oracle's full pair list of the same
    workload and threshold (SHA-256 of the ascending (i, j) uint32 rows), when
    tests/golden holds one; None otherwise."""
    import hashlib

    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "full_golden.json")
    if sim != "jaccard" or not os.path.exists(path):
        return None
    with open(path) as fh:
        entry = json.load(fh).get(workload)
    if not entry or entry.get("rows") != "all" or entry.get("checksum") != f"{checksum:#x}":
        return None
    want = entry["thresholds"].get(f"{p}/{q}")
    if want is None:
        return None
    got = hashlib.sha256(np.ascontiguousarray(pairs, dtype="<u4").reshape(-1, 2).tobytes())
    return {"reference": "oracle pair list, tests/golden/full_golden.json",
            "pairs": int(len(pairs)), "expected_pairs": want["pairs"],
            "sha256_equal": got.hexdigest() == want["sha256"]}


def roofline_of(stats_list, steps, valu=False):
    """Roofline entry of the dominant filter launch (the width class with the
    most algorithmic work), from the library's per-class event timings.

    Matrix-core kernel (b = 64, 128, 256): per band pair the contraction of two
    +-1 vectors of b entries, 2b fp4 flops, against the dense fp4 peak.
    Vector-ALU kernel: per band pair b/32 xor + b/32 popcount-accumulate + 1
    compare, int32 lane-ops against the vector ALU peak (the library's
    filter_ops)."""
    s0 = stats_list[0]
    ncls = s0["n_classes"]
    dom = max(range(ncls), key=lambda k: s0["class_ops"][k])
    b = s0["class_bits"][dom]
    dom_ms = sum(s["class_ms"][dom] for s in stats_list) / steps
    launches = sum(s["filter_launches"] for s in stats_list) / steps / ncls
    filt_ms = sum(s["ms_filter"] for s in stats_list) / steps
    band = s0["class_ops"][dom] / (b // 16 + 1)  # band pairs of the class
    if dom_ms <= 0 or filt_ms <= 0:
        # a profiler that takes over the completion signals leaves the
        # library's event pairs without timestamps
        log("filter event timings read zero: no roofline entry for this run")
        return None
    stage = {"ops_per_step": s0["filter_ops"], "ms_per_step": filt_ms,
             "valu_equiv_frac": s0["filter_ops"] / (filt_ms / 1e3) / PEAK_INT_OPS}
    if b in MFMA_BITS and not valu and (b < 256 or band >= MFMA_MIN_BAND):
        achieved = band * 2 * b / (dom_ms / 1e3)
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP4 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP4, "traffic": None,
                "kernel": f"k_filter_mfma (b = {b} class, fp4 +-1 dot products)",
                "flops_per_launch": band * 2 * b / launches,
                "band_pairs_per_launch": band / launches, "avg_launch_ms": dom_ms / launches,
                "filter_stage": stage}
    achieved = s0["class_ops"][dom] / (dom_ms / 1e3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_OPS / 1e12,
            "unit": "Top/s", "frac": achieved / PEAK_INT_OPS, "traffic": None,
            "kernel": f"k_filter (b = {b} class, vector ALU)",
            "ops_per_launch": s0["class_ops"][dom] / launches,
            "band_pairs_per_launch": band / launches, "avg_launch_ms": dom_ms / launches,
            "filter_stage": stage}


def graph_replay(devs, ps, qs, args, want):
    """ssj_plan_self_join_batch once, then ssj_plan_execute per step (the
    first round replayed from a HIP graph); the pairs must equal ``want``
    (the unprepared call's)."""
    import numpy as np
    import torch

    import paper_1711_07295_amd as ssj

    t0 = time.perf_counter()
    plan = ssj.Plan(devs, ps, qs, b_bits=args.bits, tile_cols=args.tile_cols,
                    flags=ssj.SSJ_FLAG_CUTOFF if args.cutoff else 0)
    plan_ms = (time.perf_counter() - t0) * 1e3
    got, _ = plan.execute()
    same = len(got) == len(want) and all(np.array_equal(a, b) for a, b in zip(got, want))
    torch.cuda.synchronize()
    times = []
    for k in range(args.steps):
        t1 = time.perf_counter()
        got, st = plan.execute()
        times.append(time.perf_counter() - t1)
    plan.close()
    log(f"graph replay: {statistics.mean(times) * 1e3:.2f} ms per execution "
        f"(plan {plan_ms:.1f} ms), same pairs: {same}")
    return {"ms_per_step": statistics.mean(times) * 1e3, "plan_ms": plan_ms,
            "same_pairs": bool(same), "steps": args.steps}


def run_batch(args):
    import numpy as np
    import torch

    import gen
    import paper_1711_07295_amd as ssj

    t0 = time.perf_counter()
    inst = gen.batched_instances(args.instances)
    n_sets = sum(c.n_sets for c, _ in inst)
    n_tok = sum(c.n_tokens for c, _ in inst)
    log(f"generated {len(inst)} instances: {n_sets} sets, {n_tok} tokens in "
        f"{time.perf_counter() - t0:.1f} s")
    devs = [ssj.to_device(c.offsets, c.tokens) for c, _ in inst]
    ps, qs = [t[0] for _, t in inst], [t[1] for _, t in inst]
    torch.cuda.synchronize()

    flags = ssj.SSJ_FLAG_CUTOFF if args.cutoff else 0

    def batched():
        return ssj.ssj_self_join_batch(devs, ps, qs, b_bits=args.bits, tile_cols=args.tile_cols,
                                       flags=flags)

    def sequential():
        band, res = 0, 0
        for d, p, q in zip(devs, ps, qs):
            _, st = ssj.ssj_self_join(d, p, q, b_bits=args.bits, tile_cols=args.tile_cols,
                                      flags=flags)
            band += st["band_pairs"]
            res += st["results"]
        return band, res

    for w in range(args.warmup):
        got, st = batched()
        log(f"warmup {w}: {st['results']} pairs, {st['ms_total']:.2f} ms")
    sequential()
    torch.cuda.synchronize()
    times, stats = [], []
    for k in range(args.steps):
        t1 = time.perf_counter()
        got, st = batched()
        times.append(time.perf_counter() - t1)
        stats.append(st)
        log(f"batched step {k}: {times[-1] * 1e3:.2f} ms  filter {st['ms_filter']:.2f}  "
            f"verify {st['ms_verify']:.2f}  prepare {st['ms_prepare']:.2f}  "
            f"emit {st['ms_emit']:.2f}  survivors {st['survivors']}  results {st['results']}  "
            f"launches {st['filter_launches']}  classes {st['class_bits'][:st['n_classes']]} "
            f"ms {[round(x, 2) for x in st['class_ms'][:st['n_classes']]]}")
    torch.cuda.synchronize()
    seq_times = []
    for k in range(max(1, args.steps // 2)):
        t1 = time.perf_counter()
        band_seq, res_seq = sequential()
        seq_times.append(time.perf_counter() - t1)
        log(f"sequential step {k}: {seq_times[-1] * 1e3:.2f} ms")
    band = stats[0]["band_pairs"]
    assert band == band_seq and stats[0]["results"] == res_seq
    ms = statistics.mean(times) * 1e3
    seq_ms = statistics.mean(seq_times) * 1e3
    # the same instances prepared once, the first round replayed from a graph
    graph = graph_replay(devs, ps, qs, args, got)
    line = {
        "metric": "pairs/sec (batched bitmap-filtered self-joins)",
        "value": band / (ms / 1e3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_MFMA, "data": "synthetic",
        "config": {"workload": f"batched-{len(inst)}", "instances": len(inst),
                   "n_sets": n_sets, "n_tokens": n_tok,
                   "b_bits": args.bits if args.bits else "auto", "band_pairs": band,
                   "cutoff": args.cutoff,
                   "survivors": stats[0]["survivors"], "results": stats[0]["results"]},
        "sequential": {"ms_per_step": seq_ms, "value": band / (seq_ms / 1e3),
                       "calls": len(inst)},
        "speedup_vs_sequential": seq_ms / ms,
        "graph_replay": {**graph, "speedup_vs_call": ms / graph["ms_per_step"],
                         "speedup_vs_sequential": seq_ms / graph["ms_per_step"]},
        "step_ms": {"p50": statistics.median(times) * 1e3,
                    "p99": float(np.percentile(np.array(times), 99)) * 1e3},
        "stage_ms": {k: statistics.mean(s[k] for s in stats)
                     for k in ("ms_prepare", "ms_filter", "ms_verify", "ms_emit")},
        "roofline": roofline_of(stats, args.steps),
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def served_legs(resident, n_measured, rhos, warm=100, cutoff=False, bits=0, slots=2):
    """The served form on a resident index of ``resident`` sets: the plain
    service rate mu (one batch per call, back to back), then for each load
    rho Poisson arrivals at rho * mu served twice -- by the plain server (one
    call per batch, first come first served) and by continuous batching
    (``slots`` calls in flight, each admitting every waiting batch that fits
    the memory budget).  Latency is arrival to pairs in host memory; the
    first ``warm`` batches of every run are not measured."""
    import numpy as np
    import torch

    import gen
    import paper_1711_07295_amd as ssj
    from paper_1711_07295_amd.serve import ContinuousBatcher, poisson_arrivals

    t0 = time.perf_counter()
    sw = gen.served_workload(warm + n_measured, resident_sets=resident)
    log(f"generated resident {sw.resident.n_sets} sets and {len(sw.batches)} query batches "
        f"({sum(b.n_sets for b in sw.batches)} sets) in {time.perf_counter() - t0:.1f} s")
    t1 = time.perf_counter()
    idx = ssj.Index(ssj.to_device(sw.resident.offsets, sw.resident.tokens), b_bits=bits)
    torch.cuda.synchronize()
    log(f"index built in {time.perf_counter() - t1:.2f} s")
    flags = ssj.SSJ_FLAG_CUTOFF if cutoff else 0
    plain = ContinuousBatcher(idx, slots=1, max_batches_per_call=1, flags=flags)
    cont = ContinuousBatcher(idx, slots=slots, flags=flags)
    batches, thr = sw.batches, sw.thresholds
    n = len(batches)
    plain.run(batches[:warm], thr[:warm], np.zeros(warm))
    cont.run(batches[:warm], thr[:warm], np.zeros(warm))
    # plain service rate: one batch per call, back to back
    r = plain.run(batches[warm:], thr[warm:], np.zeros(n - warm))
    mu = (n - warm) / r.wall_s
    log(f"plain service rate: {mu:.1f} batches/s")

    def summary(r, rho):
        m = slice(warm, None)  # measured batches
        lat, wait = r.latency_s[m] * 1e3, r.wait_s[m] * 1e3
        ent = {"rho": rho, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
               "wait_p50_ms": float(np.percentile(wait, 50)),
               "wait_p99_ms": float(np.percentile(wait, 99)),
               "batches_per_s": n / r.wall_s, "pairs_per_s": r.band_pairs / r.wall_s,
               "calls": r.calls, "mean_batches_per_call": float(r.batches_per_call.mean()),
               "max_in_flight": r.max_in_flight, "peak_admitted_bytes": r.peak_bytes,
               "results": r.results}
        det = r.calls_detail
        ent["call_ms"] = {k: float(np.mean([d[k] for d in det]))
                          for k in ("wall_ms", "upload_ms", "ms_total", "ms_prepare", "ms_filter",
                                    "ms_verify", "ms_emit")}
        return ent

    loads = []
    for rho in rhos:
        arr = poisson_arrivals(n, rho * mu, seed=int(rho * 1000))
        ent = {"rho": rho, "arrival_rate": rho * mu,
               "plain": summary(plain.run(batches, thr, arr), rho),
               "continuous": summary(cont.run(batches, thr, arr), rho)}
        ent["p99_plain_over_continuous"] = ent["plain"]["p99_ms"] / ent["continuous"]["p99_ms"]
        ent["p50_plain_over_continuous"] = ent["plain"]["p50_ms"] / ent["continuous"]["p50_ms"]
        loads.append(ent)
        log(f"rho {rho}: plain p50/p99 {ent['plain']['p50_ms']:.2f}/{ent['plain']['p99_ms']:.2f} ms, "
            f"continuous {ent['continuous']['p50_ms']:.2f}/{ent['continuous']['p99_ms']:.2f} ms, "
            f"{ent['continuous']['calls']} calls, up to {ent['continuous']['max_in_flight']} in flight")
    idx.close()
    return {"resident_sets": sw.resident.n_sets, "batches": n, "warm_up_batches": warm,
            "slots": slots, "plain_service_rate": mu, "b_bits": bits if bits else "auto",
            "cutoff": cutoff, "loads": loads}


def run_serve(args):
    sv = served_legs(args.resident, args.serve_batches, (0.5, 0.8, 0.95, 1.2), cutoff=args.cutoff,
                     bits=args.bits, slots=args.slots)
    head = [e for e in sv["loads"] if e["rho"] == 0.95][0]
    c = head["continuous"]
    line = {
        "metric": "pairs/sec + p50/p99 query latency (served R-S joins, continuous batching)",
        "value": c["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.serve_batches, "warmup": sv["warm_up_batches"], "ms_per_step": c["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_MFMA,
        "data": "synthetic",
        "config": {"workload": f"served-{sv['resident_sets']}",
                   **{k: v for k, v in sv.items() if k != "loads"}},
        "latency": {"p50_ms": c["p50_ms"], "p99_ms": c["p99_ms"], "rho": 0.95,
                    "plain_p50_ms": head["plain"]["p50_ms"],
                    "plain_p99_ms": head["plain"]["p99_ms"]},
        "loads": sv["loads"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
