"""Continuous batching of R-S similarity queries against a resident index.

Query batches arrive over time (host CSR collections, each with its own
threshold).  Whenever the GPU is free, the scheduler admits the waiting
batches in arrival order, as many as fit the per-call device-memory budget,
uploads them in one host-to-device copy per array, and answers all of them
with one ``ssj_index_query`` call (one set of filter/verify launches for
every admitted batch).  Batches that arrive while a call runs wait for the
next call.  The candidate (survivor) buffer of a call is bounded by the
queue capacity: when it fills, the library drains and resumes, so the
budget bounds memory without ever changing a result.

Latency of a batch = time from its arrival to its pairs in host memory.
Every step of a join runs in the library's kernels; this module only
schedules and marshals.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import DeviceSets, Index

# Device bytes a call needs per admitted set and per token: offsets (8), four
# uint32 index arrays (16), two sort keys (16), bitmaps at up to 64+128+256+512
# bits (120); tokens 4 bytes each.
BYTES_PER_SET = 160
BYTES_PER_TOKEN = 4


def call_bytes(n_sets: int, n_tokens: int) -> int:
    """Device memory a query call needs for its row side (the candidate
    buffer excluded: it is fixed by the queue capacity)."""
    return BYTES_PER_SET * n_sets + BYTES_PER_TOKEN * n_tokens


@dataclass
class ServeResult:
    latency_s: np.ndarray         # per batch: completion - arrival
    wait_s: np.ndarray            # per batch: call start - arrival (admission wait)
    calls: int
    batches_per_call: np.ndarray  # per call
    wall_s: float                 # first arrival to last completion
    band_pairs: int
    results: int
    pairs: list = field(default_factory=list)  # per batch, when kept
    calls_detail: list = field(default_factory=list)  # per call: sizes and time split


class ContinuousBatcher:
    def __init__(self, index: Index, memory_budget: int = 256 << 20, queue_capacity: int = 0,
                 keep_pairs: bool = False, flags: int = 0):
        self.index = index
        self.memory_budget = memory_budget
        self.queue_capacity = queue_capacity
        self.keep_pairs = keep_pairs
        self.flags = flags

    def _call(self, batches, thresholds, device):
        import torch
        offs = [np.asarray(b.offsets, dtype=np.uint64) for b in batches]
        toks = [np.asarray(b.tokens, dtype=np.uint32) for b in batches]
        off_all = np.concatenate(offs).view(np.int64)
        tok_all = (np.concatenate(toks) if sum(t.size for t in toks) else
                   np.zeros(0, dtype=np.uint32)).view(np.int32)
        t0 = time.perf_counter()
        d_off = torch.from_numpy(off_all).to(device, non_blocking=False)
        d_tok = torch.from_numpy(tok_all).to(device, non_blocking=False)
        self._upload_s = time.perf_counter() - t0
        views, o_at, t_at = [], 0, 0
        for o, t in zip(offs, toks):
            views.append(DeviceSets(d_off[o_at:o_at + o.size], d_tok[t_at:t_at + t.size]))
            o_at += o.size
            t_at += t.size
        return self.index.query(views, [p for p, _ in thresholds], [q for _, q in thresholds],
                                queue_capacity=self.queue_capacity, flags=self.flags)

    def run(self, batches, thresholds, arrivals, device="cuda") -> ServeResult:
        """Serve ``batches`` (host Collections) arriving at ``arrivals``
        (seconds from the start, non-decreasing)."""
        n = len(batches)
        arrivals = np.asarray(arrivals, dtype=np.float64)
        done = np.zeros(n)
        start_of = np.zeros(n)
        per_call, band, results, detail = [], 0, 0, []
        kept = [None] * n if self.keep_pairs else []
        nxt = 0
        t0 = time.perf_counter()
        while nxt < n:
            now = time.perf_counter() - t0
            if arrivals[nxt] > now:
                time.sleep(arrivals[nxt] - now)
                now = time.perf_counter() - t0
            # admit the waiting batches in arrival order within the budget
            take, used = [], 0
            k = nxt
            while k < n and arrivals[k] <= now:
                need = call_bytes(batches[k].n_sets, batches[k].n_tokens)
                if take and used + need > self.memory_budget:
                    break
                take.append(k)
                used += need
                k += 1
            got, st = self._call([batches[i] for i in take], [thresholds[i] for i in take],
                                 device)
            end = time.perf_counter() - t0
            detail.append({"batches": len(take), "sets": sum(batches[i].n_sets for i in take),
                           "wall_ms": (end - now) * 1e3, "upload_ms": self._upload_s * 1e3,
                           **{f: st[f] for f in ("ms_total", "ms_prepare", "ms_filter",
                                                 "ms_verify", "ms_emit", "band_pairs",
                                                 "survivors", "results")}})
            for i, g in zip(take, got):
                done[i] = end
                start_of[i] = now
                if self.keep_pairs:
                    kept[i] = g
            per_call.append(len(take))
            band += st["band_pairs"]
            results += st["results"]
            nxt = k
        return ServeResult(latency_s=done - arrivals, wait_s=start_of - arrivals,
                           calls=len(per_call), batches_per_call=np.array(per_call),
                           wall_s=float(done.max() - arrivals.min()) if n else 0.0,
                           band_pairs=band, results=results, pairs=kept, calls_detail=detail)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))
