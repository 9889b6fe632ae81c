"""Measure the costs the width autotuner weighs, on the GPU at hand, and write
them to ``csrc/autotune_table.h`` (then rebuild the library).

The automatic mode gives the rows of each size a the bitmap width b(a) that
minimises the task's expected time,

    sum over a of  band(a) * (filter(b) + P(false survivor at b) * survivor)
    + the launch cost of every width used,

with P from the binomial model of the bits two unrelated Bitmap-Xor bitmaps
differ in (Eq. 5 counts them; Section 3.4).  This script measures the costs
instead of assuming them, on subsets of the 1,000,000-set self-join
workload at Jaccard 4/5:

  filter(b)   ns of filter kernel time per band pair at width b, on the sets
              of 2..40 tokens, whose false survivors are rare at every width
              (the pairs that survive are nearly all similar pairs);
  survivor    ns a false survivor costs (the filter's slow path and queue
              writes, and its verification), from the sets of 50..89 tokens,
              where 64-bit bitmaps let many more dissimilar pairs through
              than 128-bit ones: the difference of the two widths' total
              time, less the difference of their band-pair costs, divided
              by the difference of their survivor counts;
  launch(b)   ns of a width class's launch on a few thousand sets (the cost
              that does not grow with the work);
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
WIDTHS = (64, 128, 256, 512)
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


def _measure(dev, b, steps, tile_cols=0):
    import paper_1711_07295_amd as ssj
    ssj.ssj_self_join(dev, P, Q, b_bits=b, tile_cols=tile_cols)  # warm-up
    runs = [ssj.ssj_self_join(dev, P, Q, b_bits=b, tile_cols=tile_cols)[1] for _ in range(steps)]
    return {"b": b, "tile_cols": tile_cols, "band": runs[0]["band_pairs"],
            "survivors": runs[0]["survivors"], "results": runs[0]["results"],
            "filter_ms": statistics.median(r["ms_filter"] for r in runs),
            "verify_ms": statistics.median(r["ms_verify"] for r in runs),
            "launches": runs[0]["filter_launches"]}


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
    for name, dev in (("small", d_small), ("mid", d_mid), ("tiny", d_tiny)):
        for b in WIDTHS:
            m = _measure(dev, b, steps)
            runs[name][b] = m
            log(f"{name}, b = {b}: {m}")
    sm, md, ty = runs["small"], runs["mid"], runs["tiny"]
    launch_ns = {b: ty[b]["filter_ms"] * 1e6 / max(1, ty[b]["launches"]) for b in WIDTHS}
    # per band pair, net of the launch cost
    filt = {b: max(0.0, sm[b]["filter_ms"] * 1e6 - launch_ns[b] * sm[b]["launches"]) / sm[b]["band"]
            for b in WIDTHS}
    # the mid sets' band pairs cost a little differently (longer size
    # groups); scale the small sets' figures by the ratio the widest widths,
    # whose survivors are rare on both subsets, show
    ratio = statistics.mean(
        (md[b]["filter_ms"] * 1e6 - launch_ns[b] * md[b]["launches"]) / md[b]["band"] / filt[b]
        for b in (256, 512))
    tot = {b: (md[b]["filter_ms"] + md[b]["verify_ms"]) * 1e6 for b in (64, 128)}
    ds = md[64]["survivors"] - md[128]["survivors"]
    survivor_ns = (tot[64] - tot[128] - ratio * (filt[64] - filt[128]) * md[64]["band"]) / ds \
        if ds > 0 else 0.0
    survivor_ns = max(survivor_ns, 0.0)
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
    return {"filter_ns": filt, "survivor_ns": survivor_ns, "launch_ns": launch_ns,
            "tile_cols": tiles, "mid_over_small": ratio, "runs": runs,
            "sets": {"small": small.n_sets, "mid": mid.n_sets, "tiny": tiny.n_sets},
            "device": f"{props.name} ({props.gcnArchName}, {props.multi_processor_count} CUs)"}


def write_table(res, path=TABLE):
    f, c, t = res["filter_ns"], res["launch_ns"], res["tile_cols"]
    s = res["survivor_ns"]
    lines = [
        "// Costs the width autotuner weighs, measured by",
        "// paper_1711_07295_amd/calibrate.py on subsets of the 1,000,000-set",
        "// self-join workload at Jaccard 4/5 (fixed widths).",
        f"// Device: {res['device']}; {datetime.date.today().isoformat()}.",
        "// Per width b = 64, 128, 256, 512: filter kernel ns per band pair (sets of",
        "// 2..40 tokens); ns of a class launch that does not grow with its work (4,000",
        "// sets); the tile width (columns) with the shortest filter time.  And ns per",
        "// false survivor (the filter's slow path and queue writes, and its",
        "// verification; from the sets of 50..89 tokens at b = 64 against b = 128).",
        "#pragma once",
        "#include <cstdint>",
        "",
        "namespace ssj {",
        "constexpr double kFilterNsPerPair[4] = {" + ", ".join(f"{f[b]:.4e}" for b in WIDTHS) + "};",
        "constexpr double kSurvivorNs = " + f"{s:.4e}" + ";",
        "constexpr double kClassLaunchNs[4] = {" + ", ".join(f"{c[b]:.4e}" for b in WIDTHS) + "};",
        "constexpr uint32_t kClassTileCols[4] = {" + ", ".join(str(t[b]) for b in WIDTHS) + "};",
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
