"""Continuous batching of R-S similarity queries against a resident index.

Query batches (host CSR collections, each with its own threshold) arrive
over time.  The scheduler keeps up to ``slots`` calls of ``ssj_index_query``
in flight, each on its own stream (all at the default priority) and its own
worker thread.  Whenever a slot is free it admits the waiting batches in
arrival order, as many as the free device memory allows, uploads them and
answers all of them with one call (one set of filter and verify launches
for every admitted batch).  Batches that arrive while calls run are
admitted into the next slot that frees up, so their host-side preparation
and their kernels overlap the calls already on the device.

Memory gate.  A call holds device memory for its row side (sets, tokens,
bitmaps of every width, sign planes), its survivor queue and its result
buffer (8 bytes each per queue slot), and the chunk rounding of the
library's allocator.  The scheduler passes the queue capacity on every call
and admits a call only when its estimate fits what the calls in flight leave
of the budget; the library's chunk cache never holds more than the calls in
flight took at once.  A full queue only makes the library drain and resume,
so the capacity bounds memory without changing a result.

Latency of a batch = time from its arrival to its pairs in host memory.
Every step of a join runs in the library's kernels; this module only
schedules and marshals.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import DeviceSets, Index

# Device bytes a call needs per admitted set and per token: the uploaded
# offsets (8) and tokens (4 per token); four uint32 index arrays (16), two
# sort keys and their scratch (24), bitmaps at 64, 128, ..., 2048 bits (504),
# sign planes of the matrix-core widths at up to 32+64+128+256+512 bytes
# (992; allocated for every set even where only some are written).
BYTES_PER_SET = 1544
BYTES_PER_TOKEN = 4
# Per queue slot: the (row, column) entry, a slot for a long pair that
# verification defers, and a result key, 8 bytes each.
BYTES_PER_QUEUE_SLOT = 24
# Plan, counters, tables, and the allocator's rounding: it hands out memory
# in chunks of 64 MiB and more, so a call may hold up to one chunk beyond
# what it uses, and its first chunk whole.
CALL_OVERHEAD = 128 << 20
DEFAULT_QUEUE = 1 << 22


def call_bytes(n_sets: int, n_tokens: int, queue_capacity: int = DEFAULT_QUEUE) -> int:
    """Device memory one query call may hold: its row side, its survivor
    queue and result buffer, and the fixed overhead."""
    return (BYTES_PER_SET * n_sets + BYTES_PER_TOKEN * n_tokens +
            BYTES_PER_QUEUE_SLOT * queue_capacity + CALL_OVERHEAD)


@dataclass
class ServeResult:
    latency_s: np.ndarray         # per batch: completion - arrival
    wait_s: np.ndarray            # per batch: call start - arrival (admission wait)
    calls: int
    batches_per_call: np.ndarray  # per call
    wall_s: float                 # first arrival to last completion
    band_pairs: int
    results: int
    max_in_flight: int = 0        # most calls on the device at once
    peak_bytes: int = 0           # largest admitted memory estimate in flight
    pairs: list = field(default_factory=list)  # per batch, when kept
    calls_detail: list = field(default_factory=list)  # per call: sizes and time split


class ContinuousBatcher:
    """Serves query batches against ``index`` with up to ``slots`` calls in
    flight and at most ``memory_budget`` bytes of call memory (estimated by
    ``call_bytes``) admitted at once.  ``slots=1`` is the plain server: one
    call at a time, each call admitting everything that waits."""

    def __init__(self, index: Index, slots: int = 2, memory_budget: int = 2 << 30,
                 queue_capacity: int = DEFAULT_QUEUE, keep_pairs: bool = False, flags: int = 0,
                 max_batches_per_call: int = 0):
        if slots < 1:
            raise ValueError("slots must be at least 1")
        self.index = index
        self.slots = slots
        self.memory_budget = memory_budget
        self.queue_capacity = queue_capacity
        self.keep_pairs = keep_pairs
        self.flags = flags
        self.max_batches_per_call = max_batches_per_call
        self._streams = None

    def _stream(self, slot, device):
        if device == "cpu":
            return None
        import torch
        if self._streams is None:
            # default priority for every stream
            self._streams = [torch.cuda.Stream(device=device) for _ in range(self.slots)]
        return self._streams[slot]

    def _call(self, slot, batches, thresholds, device):
        """One library call on the slot's stream: upload, query, pairs in host
        memory.  Returns (pairs per batch, stats, upload seconds)."""
        import contextlib
        offs = [np.asarray(b.offsets, dtype=np.uint64) for b in batches]
        toks = [np.asarray(b.tokens, dtype=np.uint32) for b in batches]
        off_all = np.concatenate(offs).view(np.int64)
        tok_all = (np.concatenate(toks) if sum(t.size for t in toks) else
                   np.zeros(0, dtype=np.uint32)).view(np.int32)
        stream = self._stream(slot, device)
        ctx = contextlib.nullcontext()
        if stream is not None:
            import torch
            ctx = torch.cuda.stream(stream)
        with ctx:
            import torch
            t0 = time.perf_counter()
            d_off = torch.from_numpy(off_all).to(device)
            d_tok = torch.from_numpy(tok_all).to(device)
            upload_s = time.perf_counter() - t0
            views, o_at, t_at = [], 0, 0
            for o, t in zip(offs, toks):
                views.append(DeviceSets(d_off[o_at:o_at + o.size], d_tok[t_at:t_at + t.size]))
                o_at += o.size
                t_at += t.size
            kw = {"queue_capacity": self.queue_capacity, "flags": self.flags}
            if stream is not None:
                kw["stream"] = stream
            got, st = self.index.query(views, [p for p, _ in thresholds],
                                       [q for _, q in thresholds], **kw)
        return got, st, upload_s

    def run(self, batches, thresholds, arrivals, device="cuda") -> ServeResult:
        """Serve ``batches`` (host Collections) arriving at ``arrivals``
        (seconds from the start, non-decreasing)."""
        n = len(batches)
        arrivals = np.asarray(arrivals, dtype=np.float64)
        done = np.zeros(n)
        start_of = np.zeros(n)
        kept = [None] * n if self.keep_pairs else []
        need = [BYTES_PER_SET * b.n_sets + BYTES_PER_TOKEN * b.n_tokens for b in batches]
        fixed = BYTES_PER_QUEUE_SLOT * self.queue_capacity + CALL_OVERHEAD
        cv = threading.Condition()
        state = {"used": 0, "in_flight": 0, "max_in_flight": 0, "peak": 0,
                 "band": 0, "results": 0, "error": None}
        free_slots = list(range(self.slots - 1, -1, -1))
        per_call, detail = [], []
        t0 = time.perf_counter()

        def work(slot, take, est, started):
            try:
                got, st, up = self._call(slot, [batches[i] for i in take],
                                         [thresholds[i] for i in take], device)
            except BaseException as e:  # handed to the dispatcher
                with cv:
                    state["error"] = e
                    state["used"] -= est
                    state["in_flight"] -= 1
                    free_slots.append(slot)
                    cv.notify_all()
                return
            end = time.perf_counter() - t0
            with cv:
                for i, g in zip(take, got):
                    done[i] = end
                    if self.keep_pairs:
                        kept[i] = g
                per_call.append(len(take))
                detail.append({"slot": slot, "batches": len(take),
                               "sets": sum(batches[i].n_sets for i in take),
                               "wall_ms": (end - started) * 1e3, "upload_ms": up * 1e3,
                               **{f: st[f] for f in ("ms_total", "ms_prepare", "ms_filter",
                                                     "ms_verify", "ms_emit", "band_pairs",
                                                     "survivors", "results")}})
                state["band"] += st["band_pairs"]
                state["results"] += st["results"]
                state["used"] -= est
                state["in_flight"] -= 1
                free_slots.append(slot)
                cv.notify_all()

        nxt = 0
        with ThreadPoolExecutor(self.slots) as pool:
            with cv:
                while True:
                    if state["error"] is not None:
                        break
                    now = time.perf_counter() - t0
                    # admit the waiting batches in arrival order while a slot
                    # and memory are free; a batch too large for the whole
                    # budget still runs, alone on the device
                    while free_slots and nxt < n and arrivals[nxt] <= now:
                        take, est = [], fixed
                        k = nxt
                        while k < n and arrivals[k] <= now:
                            if self.max_batches_per_call and len(take) >= self.max_batches_per_call:
                                break
                            over = state["used"] + est + need[k] > self.memory_budget
                            if over and (take or state["in_flight"]):
                                break
                            take.append(k)
                            est += need[k]
                            k += 1
                        if not take:
                            break  # waits for memory
                        slot = free_slots.pop()
                        state["used"] += est
                        state["peak"] = max(state["peak"], state["used"])
                        state["in_flight"] += 1
                        state["max_in_flight"] = max(state["max_in_flight"], state["in_flight"])
                        for i in take:
                            start_of[i] = now
                        pool.submit(work, slot, take, est, now)
                        nxt = k
                    if nxt >= n and state["in_flight"] == 0:
                        break
                    # sleep until the next arrival (if a slot could take it)
                    # or until a call completes
                    timeout = None
                    if nxt < n and free_slots:
                        timeout = max(0.0, arrivals[nxt] - (time.perf_counter() - t0))
                    cv.wait(timeout)
        if state["error"] is not None:
            raise state["error"]
        return ServeResult(latency_s=done - arrivals, wait_s=start_of - arrivals,
                           calls=len(per_call), batches_per_call=np.array(per_call),
                           wall_s=float(done.max() - arrivals.min()) if n else 0.0,
                           band_pairs=state["band"], results=state["results"],
                           max_in_flight=state["max_in_flight"], peak_bytes=state["peak"],
                           pairs=kept, calls_detail=detail)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))
