"""Writes the full-size expected pair lists of the self-join workloads.

Every value this script stores comes from the CPU oracle (``oracle/``) on the
seeded generator's input (``gen/``); nothing comes from the GPU library.

  selfjoin-1m   every similar pair, at Jaccard t = 1/2, 7/10, 4/5 and 9/10
  selfjoin-10m  every similar pair whose larger position in the size order
                (size, caller index) is a sampled row: every 100th position
                from position 50 (a 1% row sample), at t = 4/5 and 19/20

Method.  The join at the lowest threshold runs in full through the banded
oracle (Alg. 1 restricted by the length filter of Table 2: pairs it skips are
provably below t).  Its collection is first copied into size order, so that a
row's band of partners is contiguous in memory; the oracle then walks the
copy with the identity order, and its pairs are mapped back to caller
indices.  The lists at higher thresholds are the lowest threshold's pairs
that the oracle's own predicate (Table 1, ``oracle.check_pairs``) still
accepts: sim >= t2 implies sim >= t1 for t1 <= t2 (Eq. 1), so no pair at t2
is missing from the list at t1.

Outputs (next to this file):
  full_selfjoin-1m.npz, sample_selfjoin-10m.npz
      "pairs": the lowest threshold's list, (n, 2) uint32, ascending;
      "keep_P_Q": for each higher threshold P/Q, np.packbits of the mask that
      selects its pairs from "pairs" (so every list is stored once)
  full_golden.json    checksums, counts, SHA-256 of each list

Usage:  python tests/golden/make_full_golden.py [1m|10m|all] [--threads N]
Takes hours on 8 cores (about 3.4e7 band pairs/s for the 1M workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

MANIFEST = os.path.join(HERE, "full_golden.json")
SAMPLE_STEP, SAMPLE_FIRST = 100, 50


def pairs_sha256(pairs: np.ndarray) -> str:
    """SHA-256 of a pair list as little-endian uint32 (i, j) rows."""
    a = np.ascontiguousarray(pairs, dtype="<u4").reshape(-1, 2)
    return hashlib.sha256(a.tobytes()).hexdigest()


def size_ordered_copy(col):
    """The collection's sets in the oracle's size order, as a new CSR."""
    order = oracle.size_order(col.offsets)
    sizes = np.diff(col.offsets).astype(np.int64)[order]
    off = np.zeros(col.n_sets + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    starts = col.offsets[:-1][order].astype(np.int64)
    gather = np.repeat(starts - off[:-1].astype(np.int64), sizes) + np.arange(int(off[-1]))
    return order, off, col.tokens[gather]


def banded_pairs(col, p, q, rows=None, threads=None, chunks=16, log=print):
    """Oracle pairs (caller indices, ascending) of every row in ``rows``
    (size-order positions; None = all), each against its band."""
    order, off, tok = size_ordered_copy(col)
    ident = np.arange(col.n_sets, dtype=np.uint32)
    rows = np.arange(col.n_sets, dtype=np.uint64) if rows is None else np.asarray(rows, np.uint64)
    parts, evaluated = [], 0
    t0 = time.perf_counter()
    for k, part in enumerate(np.array_split(rows, chunks)):
        pr, ev = oracle.self_join_banded(off, tok, p, q, rows=part, order=ident, threads=threads)
        parts.append(pr)
        evaluated += ev
        log(f"  chunk {k + 1}/{chunks}: {len(pr)} pairs, {ev} band pairs merged, "
            f"{time.perf_counter() - t0:.0f} s")
    pr = np.concatenate(parts) if parts else np.zeros((0, 2), np.uint32)
    a = order[pr[:, 0]].astype(np.uint64)
    b = order[pr[:, 1]].astype(np.uint64)
    keys = np.unique((np.minimum(a, b) << np.uint64(32)) | np.maximum(a, b))
    out = np.empty((keys.shape[0], 2), dtype=np.uint32)
    out[:, 0] = (keys >> np.uint64(32)).astype(np.uint32)
    out[:, 1] = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out, evaluated, time.perf_counter() - t0


def derive(col, pairs, p, q):
    """The mask of the pairs of a higher threshold p/q: those the oracle still
    accepts."""
    return oracle.check_pairs(col.offsets, col.tokens, col.offsets, col.tokens, pairs, p, q)


def load(npz_path):
    """{(p, q): pairs} from a file this script wrote (thresholds as in its
    manifest entry; the lowest one is the stored list)."""
    z = np.load(npz_path)
    base = z["pairs"]
    out = {}
    for k in z.files:
        if k.startswith("keep_"):
            _, p, q = k.split("_")
            out[(int(p), int(q))] = base[np.unpackbits(z[k], count=base.shape[0]).astype(bool)]
    return base, out


def load_manifest():
    if os.path.exists(MANIFEST):
        with open(MANIFEST) as f:
            return json.load(f)
    return {}


def save(name, npz_name, col, lists, masks, extra, manifest):
    base = lists[min(lists, key=lambda t: t[0] / t[1])]
    np.savez_compressed(os.path.join(HERE, npz_name), pairs=base,
                        **{f"keep_{p}_{q}": np.packbits(m) for (p, q), m in masks.items()})
    manifest[name] = {
        "file": npz_name,
        "checksum": f"{col.checksum():#x}",
        "n_sets": col.n_sets,
        "n_tokens": col.n_tokens,
        "generator": gen.WORKLOADS[name]["gen"],
        "thresholds": {f"{p}/{q}": {"pairs": int(v.shape[0]), "sha256": pairs_sha256(v)}
                       for (p, q), v in lists.items()},
        **extra,
    }
    with open(MANIFEST, "w") as f:
        json.dump(manifest, f, indent=1, sort_keys=True)
        f.write("\n")


def run_1m(threads):
    col = gen.workload("selfjoin-1m")
    print(f"selfjoin-1m: {col.n_sets} sets, checksum {col.checksum():#x}", flush=True)
    base, ev, dt = banded_pairs(col, 1, 2, threads=threads,
                                log=lambda s: print(s, flush=True))
    print(f"t = 1/2: {len(base)} pairs, {ev} band pairs merged in {dt:.0f} s", flush=True)
    lists, masks = {(1, 2): base}, {}
    for p, q in ((7, 10), (4, 5), (9, 10)):
        masks[(p, q)] = derive(col, base, p, q)
        lists[(p, q)] = base[masks[(p, q)]]
        print(f"t = {p}/{q}: {len(lists[(p, q)])} pairs", flush=True)
    man = load_manifest()
    save("selfjoin-1m", "full_selfjoin-1m.npz", col, lists, masks,
         {"rows": "all", "base_threshold": "1/2", "band_pairs_merged": ev,
          "oracle_seconds": round(dt, 1), "threads": threads}, man)


def run_10m(threads):
    col = gen.workload("selfjoin-10m")
    print(f"selfjoin-10m: {col.n_sets} sets, checksum {col.checksum():#x}", flush=True)
    rows = np.arange(SAMPLE_FIRST, col.n_sets, SAMPLE_STEP, dtype=np.uint64)
    base, ev, dt = banded_pairs(col, 4, 5, rows=rows, threads=threads,
                                log=lambda s: print(s, flush=True))
    print(f"t = 4/5: {len(base)} pairs, {ev} band pairs merged in {dt:.0f} s", flush=True)
    masks = {(19, 20): derive(col, base, 19, 20)}
    lists = {(4, 5): base, (19, 20): base[masks[(19, 20)]]}
    print(f"t = 19/20: {len(lists[(19, 20)])} pairs", flush=True)
    man = load_manifest()
    save("selfjoin-10m", "sample_selfjoin-10m.npz", col, lists, masks,
         {"rows": {"size_order_positions": "every 100th from 50", "step": SAMPLE_STEP,
                   "first": SAMPLE_FIRST, "count": int(rows.shape[0])},
          "base_threshold": "4/5", "band_pairs_merged": ev, "oracle_seconds": round(dt, 1),
          "threads": threads}, man)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("1m", "10m", "all"), default="all", nargs="?")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    if a.which in ("1m", "all"):
        run_1m(a.threads)
    if a.which in ("10m", "all"):
        run_10m(a.threads)
