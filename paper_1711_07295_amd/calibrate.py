"""Measure the costs the width autotuner weighs, on the GPU at hand, and write
them to ``csrc/autotune_table.h`` (then rebuild the library).

The automatic mode gives the rows of each size a the bitmap width b(a) that
minimises the task's expected time,

    sum over a of  band(a) * (filter(b) + (1 - (1 - P)^s) * entry / s
                              + P * max(survivor, wave / tiles(a, b)))
    + the launch cost of every width used,

with P the chance of a false survivor at b from the binomial model of the
bits two unrelated Bitmap-Xor bitmaps differ in (Eq. 5 counts them; Section
3.4), s the pairs of one step of the width's filter kernel (a step with a
kept pair leaves the fast path once), and tiles(a, b) the filter tiles the
rows of size a fill (at most the grid's waves): survivors that few tiles
hold are staged by few waves, one after the other.  This script measures the costs
instead of assuming them, on subsets of the 1,000,000-set self-join
workload:

  filter(b)   ns of filter kernel time per band pair at width b (Jaccard
              4/5, the sets of 2..40 tokens, whose false survivors are rare
              at every width);
  entry,      ns of a slow-path entry and ns a survivor adds (its queue
  survivor    writes and verification), from the sets of 50..89 tokens:
              at 4/5, 64-bit bitmaps let many more dissimilar pairs through
              than 128-bit ones, nearly each in a step of its own; at 1/2,
              64-bit steps keep many pairs each.  The two times beyond the
              band pairs' filter cost give two linear equations;
  launch(b)   ns of a width class's launch on a few thousand sets (the cost
              that does not grow with the work);
  wave(b)     ns one filter wave takes to stage a survivor at width b: an
              R-S join of 64 sets against 2048 (one tile, one wave) of b
              random tokens each at Jaccard 1/2, where nearly every pair
              survives; the launch's time beyond its fixed cost, per
              survivor;
  tile width  of 1024, 2048 and 4096 columns, the one with the shortest
              filter time on the small sets.

Usage:  python -m paper_1711_07295_amd.calibrate [--steps N] [--out PATH] [--dry-run]
"""
from __future__ import annotations

import argparse
import datetime
import os
import statistics
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "autotune_table.h")
WIDTHS = (64, 128, 256, 512, 1024, 2048)
# pairs of one step of the filter kernel at each width: the matrix-core
# kernel scores 32 columns against 32 * RT rows (RT = 6 at 64 bits, 4 at 128,
# 5 at 256, 4 at 512, 2 at 1024), the vector-ALU kernel 64 * R rows against U
# columns (64 at 2048)
PAIRS_PER_STEP = {64: 6144, 128: 4096, 256: 5120, 512: 4096, 1024: 2048, 2048: 64}
MFMA_WIDTHS = (64, 128, 256, 512, 1024)
TILE_COLS = (1024, 2048, 4096)
P, Q = 4, 5


def _subset(col, lo, hi, limit=None):
    """The sets of col with lo..hi tokens (at most ``limit`` of them), as a
    new CSR collection."""
    import gen
    sizes = np.diff(col.offsets).astype(np.int64)
    keep = np.nonzero((sizes >= lo) & (sizes <= hi))[0]
    if limit is not None:
        keep = keep[:limit]
    n = sizes[keep]
    off = np.zeros(keep.shape[0] + 1, dtype=np.uint64)
    np.cumsum(n, out=off[1:])
    starts = col.offsets[:-1][keep].astype(np.int64)
    gather = np.repeat(starts - off[:-1].astype(np.int64), n) + np.arange(int(off[-1]))
    return gen.Collection(offsets=off, tokens=col.tokens[gather])


def _measure(dev, b, steps, tile_cols=0, p=P, q=Q):
    import paper_1711_07295_amd as ssj
    ssj.ssj_self_join(dev, p, q, b_bits=b, tile_cols=tile_cols)  # warm-up
    runs = [ssj.ssj_self_join(dev, p, q, b_bits=b, tile_cols=tile_cols)[1] for _ in range(steps)]
    return {"b": b, "tile_cols": tile_cols, "band": runs[0]["band_pairs"],
            "survivors": runs[0]["survivors"], "results": runs[0]["results"],
            "filter_ms": statistics.median(r["ms_filter"] for r in runs),
            "verify_ms": statistics.median(r["ms_verify"] for r in runs),
            "launches": runs[0]["filter_launches"],
            "tiles": sum(runs[0]["class_tiles"][:runs[0]["n_classes"]])}


def _crowded_tile(b, steps):
    """R-S join of 64 sets against 2048 sets of b random tokens each (one
    filter tile) at Jaccard 1/2 and width b: nearly every pair survives."""
    import paper_1711_07295_amd as ssj
    rng = np.random.default_rng(1000 + b)

    def sets(n):
        tok = np.sort(rng.choice(1 << 24, size=(n, b), replace=True), axis=1).astype(np.uint32)
        # distinct tokens per set: replace repeats by values above the range
        dup = np.zeros_like(tok, dtype=bool)
        dup[:, 1:] = tok[:, 1:] == tok[:, :-1]
        tok[dup] = (1 << 24) + np.arange(int(dup.sum()), dtype=np.uint32)
        tok.sort(axis=1)
        off = np.arange(n + 1, dtype=np.uint64) * np.uint64(b)
        return ssj.to_device(off, tok.reshape(-1))

    r, s = sets(64), sets(2048)
    flags = ssj.SSJ_FLAG_MFMA if b in MFMA_WIDTHS else 0
    ssj.ssj_rs_join(r, s, 1, 2, b_bits=b, tile_cols=2048, flags=flags)  # warm-up
    runs = [ssj.ssj_rs_join(r, s, 1, 2, b_bits=b, tile_cols=2048, flags=flags)[1]
            for _ in range(steps)]
    return {"b": b, "band": runs[0]["band_pairs"], "survivors": runs[0]["survivors"],
            "tiles": sum(runs[0]["class_tiles"][:runs[0]["n_classes"]]),
            "filter_ms": statistics.median(x["ms_filter"] for x in runs)}


def calibrate(steps=5, log=print):
    import torch

    import gen
    import paper_1711_07295_amd as ssj
    torch.cuda.set_device(0)
    full = gen.workload("selfjoin-1m")
    small = _subset(full, 2, 40)
    mid = _subset(full, 50, 89)
    tiny = _subset(full, 2, 40, limit=4000)
    d_small, d_mid, d_tiny = (ssj.to_device(c.offsets, c.tokens) for c in (small, mid, tiny))
    runs = {"small": {}, "mid": {}, "tiny": {}}
    for name, dev, widths in (("small", d_small, WIDTHS), ("mid", d_mid, (64, 128, 256, 512)),
                              ("tiny", d_tiny, WIDTHS)):
        for b in widths:
            m = _measure(dev, b, steps)
            runs[name][b] = m
            log(f"{name}, b = {b}: {m}")
    dense = _measure(d_mid, 64, max(1, steps // 2), p=1, q=2)
    runs["mid_dense"] = dense
    log(f"mid, b = 64, t = 1/2: {dense}")
    crowded = {}
    for b in WIDTHS:
        crowded[b] = _crowded_tile(b, steps)
        log(f"one crowded tile, b = {b}: {crowded[b]}")
    runs["crowded"] = crowded
    sm, md, ty = runs["small"], runs["mid"], runs["tiny"]
    launch_ns = {b: ty[b]["filter_ms"] * 1e6 / max(1, ty[b]["launches"]) for b in WIDTHS}
    # per band pair, net of the launch cost
    filt = {b: max(0.0, sm[b]["filter_ms"] * 1e6 - launch_ns[b] * sm[b]["launches"]) / sm[b]["band"]
            for b in WIDTHS}
    # the mid sets' band pairs cost a little differently (longer size
    # groups); scale the small sets' figures by the ratio the widths whose
    # survivors are rare on both subsets show
    ratio = statistics.mean(
        (md[b]["filter_ms"] * 1e6 - launch_ns[b] * md[b]["launches"]) / md[b]["band"] / filt[b]
        for b in (256, 512))

    def entries(m, b):
        """expected slow-path entries of a run: steps that keep a pair"""
        s = PAIRS_PER_STEP[b]
        pr = min(m["survivors"] / max(1, m["band"]), 1.0 - 1e-12)
        return m["band"] / s * -np.expm1(s * np.log1p(-pr))

    def extra(m, b):
        """ns of a run beyond its band pairs' filter cost"""
        return (m["filter_ms"] + m["verify_ms"]) * 1e6 - ratio * filt[b] * m["band"]

    # sparse: 64 against 128 bits at 4/5; dense: 64 bits at 1/2
    a = np.array([[entries(md[64], 64) - entries(md[128], 128),
                   md[64]["survivors"] - md[128]["survivors"]],
                  [entries(dense, 64), dense["survivors"]]], dtype=np.float64)
    y = np.array([extra(md[64], 64) - extra(md[128], 128), extra(dense, 64)], dtype=np.float64)
    entry_ns, survivor_ns = (max(0.0, float(v)) for v in np.linalg.solve(a, y))
    # one wave's staging time per survivor: the crowded tile's time beyond
    # the launch's fixed cost
    wave_ns = {b: max(0.0, m["filter_ms"] * 1e6 - launch_ns[b]) / max(1, m["survivors"])
               for b, m in crowded.items()}
    tiles = {}
    for b in WIDTHS:
        best = None
        for tc in TILE_COLS:
            m = _measure(d_small, b, steps, tile_cols=tc)
            log(f"small, b = {b}, tile_cols = {tc}: filter {m['filter_ms']:.3f} ms")
            if best is None or m["filter_ms"] < best[1]:
                best = (tc, m["filter_ms"])
        tiles[b] = best[0]
    props = torch.cuda.get_device_properties(0)
    return {"filter_ns": filt, "entry_ns": entry_ns, "survivor_ns": survivor_ns,
            "wave_ns": wave_ns, "launch_ns": launch_ns,
            "tile_cols": tiles, "mid_over_small": ratio, "runs": runs,
            "sets": {"small": small.n_sets, "mid": mid.n_sets, "tiny": tiny.n_sets},
            "device": f"{props.name} ({props.gcnArchName}, {props.multi_processor_count} CUs)"}


def write_table(res, path=TABLE):
    f, c, t = res["filter_ns"], res["launch_ns"], res["tile_cols"]
    s, e = res["survivor_ns"], res["entry_ns"]
    lines = [
        "// Costs the width autotuner weighs, measured by",
        "// paper_1711_07295_amd/calibrate.py on subsets of the 1,000,000-set",
        "// self-join workload at Jaccard 4/5 (fixed widths).",
        f"// Device: {res['device']}; {datetime.date.today().isoformat()}.",
        "// Per width b = 64 .. 2048: filter kernel ns per band pair (sets of 2..40",
        "// tokens); ns of a class launch that does not grow with its work (4,000",
        "// sets); the tile width (columns) with the shortest filter time; the pairs",
        "// of one step of the width's kernel.  And the ns of a slow-path entry and the",
        "// ns a survivor adds (queue writes, verification), from the sets of 50..89",
        "// tokens (64 against 128 bits at 4/5; 64 bits at 1/2); per width, the ns one",
        "// wave takes to stage a survivor, from one tile where nearly every pair",
        "// survives (64 x 2048 random sets of b tokens at 1/2).",
        "#pragma once",
        "#include <cstdint>",
        "",
        "namespace ssj {",
        "constexpr double kFilterNsPerPair[6] = {" + ", ".join(f"{f[b]:.4e}" for b in WIDTHS) + "};",
        "constexpr double kSlowEntryNs = " + f"{e:.4e}" + ";",
        "constexpr double kSurvivorNs = " + f"{s:.4e}" + ";",
        "constexpr double kSurvivorWaveNs[6] = {" + ", ".join(f"{res['wave_ns'][b]:.4e}" for b in WIDTHS) + "};",
        "constexpr double kPairsPerStep[6] = {" + ", ".join(f"{PAIRS_PER_STEP[b]}.0" for b in WIDTHS) + "};",
        "constexpr double kClassLaunchNs[6] = {" + ", ".join(f"{c[b]:.4e}" for b in WIDTHS) + "};",
        "constexpr uint32_t kClassTileCols[6] = {" + ", ".join(str(t[b]) for b in WIDTHS) + "};",
        "}  // namespace ssj",
        "",
    ]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))
    return path


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--dry-run", action="store_true", help="print the table, do not write it")
    ap.add_argument("--out", default=TABLE, help="where to write the table")
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    r = calibrate(a.steps, log=lambda m: print(m, file=sys.stderr, flush=True))
    print({k: v for k, v in r.items() if k != "runs"}, flush=True)
    if not a.dry_run:
        print("wrote", write_table(r, a.out), flush=True)
