"""Seeded synthetic token-set collections (CSR), shared input for the oracle and
the GPU library.  Holds no join arithmetic: it only draws sets.

The recipe is documented in ``ssjgen.c``.  Named workloads follow the shape of
the paper's collections (Section 5, Table 4): Zipf-like token occurrence,
tokens renumbered by ascending global frequency, sets sorted ascending.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libssjgen.so")

SIZE_UNIFORM, SIZE_LOGNORMAL, SIZE_POISSON = 0, 1, 2
SEED_BASE = 0x1711072950000000


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_sets", ctypes.c_uint64),
        ("universe", ctypes.c_uint32),
        ("zipf_s", ctypes.c_double),
        ("size_dist", ctypes.c_int32),
        ("size_a", ctypes.c_double),
        ("size_b", ctypes.c_double),
        ("size_lo", ctypes.c_uint32),
        ("size_hi", ctypes.c_uint32),
        ("planted_frac", ctypes.c_double),
        ("cluster_lo", ctypes.c_uint32),
        ("cluster_hi", ctypes.c_uint32),
        ("swap_frac", ctypes.c_double),
        ("relabel", ctypes.c_int32),
        ("shuffle", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("n_threads", ctypes.c_int32),
    ]


class _Out(ctypes.Structure):
    _fields_ = [
        ("n_sets", ctypes.c_uint64),
        ("n_tokens", ctypes.c_uint64),
        ("offsets", ctypes.POINTER(ctypes.c_uint64)),
        ("tokens", ctypes.POINTER(ctypes.c_uint32)),
        ("n_distinct", ctypes.c_uint32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ssjgen_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.POINTER(_Out)]
        lib.ssjgen_generate.restype = ctypes.c_int
        lib.ssjgen_free.argtypes = [ctypes.POINTER(_Out)]
        lib.ssjgen_free.restype = None
        lib.ssjgen_checksum.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        lib.ssjgen_checksum.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class Collection:
    """A token-set collection in CSR form (caller order)."""
    offsets: np.ndarray  # uint64[N+1]
    tokens: np.ndarray   # uint32[T]
    n_distinct: int = 0
    params: dict | None = None

    @property
    def n_sets(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_tokens(self) -> int:
        return int(self.tokens.shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def set(self, k: int) -> np.ndarray:
        return self.tokens[self.offsets[k]:self.offsets[k + 1]]

    def checksum(self) -> int:
        return checksum(self.offsets, self.tokens)

    def subset(self, idx) -> "Collection":
        """Sets ``idx`` (in that order) as a new collection."""
        idx = np.asarray(idx, dtype=np.int64)
        return from_lists([self.set(int(k)) for k in idx])


def checksum(offsets: np.ndarray, tokens: np.ndarray) -> int:
    lib = _load()
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    tokens = np.ascontiguousarray(tokens, dtype=np.uint32)
    if tokens.size == 0:
        tokens = np.zeros(1, dtype=np.uint32)
    return int(lib.ssjgen_checksum(offsets.ctypes.data, offsets.shape[0] - 1, tokens.ctypes.data))


def from_lists(sets) -> Collection:
    """CSR collection from an iterable of token sequences (kept as given)."""
    sets = [np.asarray(s, dtype=np.uint32) for s in sets]
    sizes = np.array([s.shape[0] for s in sets], dtype=np.uint64)
    offsets = np.zeros(len(sets) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    tokens = np.concatenate(sets) if sets else np.zeros(0, dtype=np.uint32)
    return Collection(offsets=offsets, tokens=tokens.astype(np.uint32))


def generate(n_sets: int, universe: int, zipf_s: float, size_dist: int = SIZE_UNIFORM,
             size_a: float = 0.0, size_b: float = 0.0, size_lo: int = 1, size_hi: int = 50,
             planted_frac: float = 0.0, cluster_lo: int = 2, cluster_hi: int = 20,
             swap_frac: float = 0.1, relabel: bool = True, shuffle: bool = True,
             seed: int = SEED_BASE, n_threads: int | None = None) -> Collection:
    lib = _load()
    if n_threads is None:
        n_threads = min(16, os.cpu_count() or 1)
    cfg = _Cfg(n_sets, universe, zipf_s, size_dist, size_a, size_b, size_lo, size_hi,
               planted_frac, cluster_lo, cluster_hi, swap_frac, int(relabel), int(shuffle),
               seed & 0xFFFFFFFFFFFFFFFF, n_threads)
    out = _Out()
    rc = lib.ssjgen_generate(ctypes.byref(cfg), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"ssjgen_generate failed with code {rc}")
    try:
        n = int(out.n_sets)
        t = int(out.n_tokens)
        offsets = np.ctypeslib.as_array(out.offsets, shape=(n + 1,)).copy()
        tokens = (np.ctypeslib.as_array(out.tokens, shape=(t,)).copy() if t
                  else np.zeros(0, dtype=np.uint32))
        nd = int(out.n_distinct)
    finally:
        lib.ssjgen_free(ctypes.byref(out))
    params = dict(n_sets=n_sets, universe=universe, zipf_s=zipf_s, size_dist=size_dist,
                  size_a=size_a, size_b=size_b, size_lo=size_lo, size_hi=size_hi,
                  planted_frac=planted_frac, cluster_lo=cluster_lo, cluster_hi=cluster_hi,
                  swap_frac=swap_frac, relabel=relabel, shuffle=shuffle, seed=seed)
    return Collection(offsets=offsets, tokens=tokens, n_distinct=nd, params=params)


# Named workloads.  Thresholds are exact rationals (p, q); b is the bitmap width.
WORKLOADS = {
    # 10,000 sets, universe 10,000, Zipf 1.0, sizes uniform 5..50
    "selfjoin-10k": dict(gen=dict(n_sets=10_000, universe=10_000, zipf_s=1.0,
                                  size_dist=SIZE_UNIFORM, size_lo=5, size_hi=50,
                                  seed=SEED_BASE + 0),
                         thresholds=[(4, 5)], bits=[64]),
    # 1,000,000 sets, universe 1,000,000, Zipf 1.1, log-normal(median 20, sigma 0.8)
    # clipped to 2..500, 5% of sets in near-duplicate clusters of 2..20 with 10% swaps
    "selfjoin-1m": dict(gen=dict(n_sets=1_000_000, universe=1_000_000, zipf_s=1.1,
                                 size_dist=SIZE_LOGNORMAL, size_a=20.0, size_b=0.8,
                                 size_lo=2, size_hi=500, planted_frac=0.05,
                                 seed=SEED_BASE + 1),
                        thresholds=[(1, 2), (7, 10), (4, 5), (9, 10)], bits=[64, 128, 256]),
    # 10,000,000 sets, universe 5,000,000, Zipf 1.0, log-normal(12, 0.6) clipped 2..200,
    # 2% planted
    "selfjoin-10m": dict(gen=dict(n_sets=10_000_000, universe=5_000_000, zipf_s=1.0,
                                  size_dist=SIZE_LOGNORMAL, size_a=12.0, size_b=0.6,
                                  size_lo=2, size_hi=200, planted_frac=0.02,
                                  seed=SEED_BASE + 2),
                         thresholds=[(4, 5), (19, 20)], bits=[128]),
    # resident collection for R-S queries: 5,000,000 sets, universe 2,000,000, Zipf 1.1,
    # log-normal(median 30, sigma 0.8) clipped 2..500
    "resident-5m": dict(gen=dict(n_sets=5_000_000, universe=2_000_000, zipf_s=1.1,
                                 size_dist=SIZE_LOGNORMAL, size_a=30.0, size_b=0.8,
                                 size_lo=2, size_hi=500, seed=SEED_BASE + 4),
                        thresholds=[(7, 10), (9, 10)], bits=[128]),
}


def workload(name: str, n_sets: int | None = None, seed: int | None = None) -> Collection:
    """Generate a named workload; ``n_sets`` scales it down (same distributions)."""
    g = dict(WORKLOADS[name]["gen"])
    if n_sets is not None:
        scale = n_sets / g["n_sets"]
        g["universe"] = max(64, int(round(g["universe"] * scale)))
        g["n_sets"] = n_sets
    if seed is not None:
        g["seed"] = seed
    return generate(**g)


# ---------------------------------------------------------------- batched form
BATCH_THRESHOLDS = [(1, 2), (7, 10), (4, 5), (9, 10)]


def batched_instances(n_instances: int = 256, seed: int = SEED_BASE + 3, n_min: int = 1_000,
                      n_max: int = 200_000, size_hi: int = 2000):
    """Many uneven self-join instances: ``[(Collection, (p, q)), ...]``.

    Instance k: N_k = round(exp(U[ln n_min, ln n_max])) sets, log-normal sizes
    with median m_k = exp(U[ln 5, ln 200]) and sigma 0.8 clipped to
    2..size_hi, universe max(N_k, 50 m_k), Zipf exponent U[0.8, 1.3], 5% of
    the sets in near-duplicate clusters, threshold drawn from 1/2, 7/10, 4/5,
    9/10.  Instance parameters come from one seeded stream; each instance's
    sets from its own seed."""
    rng = np.random.Generator(np.random.PCG64(seed & 0xFFFFFFFFFFFFFFFF))
    out = []
    for k in range(n_instances):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        m = float(np.exp(rng.uniform(np.log(5.0), np.log(200.0))))
        s = float(rng.uniform(0.8, 1.3))
        t = BATCH_THRESHOLDS[int(rng.integers(len(BATCH_THRESHOLDS)))]
        u = max(n, int(round(50 * m)))
        col = generate(n_sets=n, universe=u, zipf_s=s, size_dist=SIZE_LOGNORMAL, size_a=m,
                       size_b=0.8, size_lo=2, size_hi=size_hi, planted_frac=0.05,
                       seed=seed + ((k + 1) << 24))
        out.append((col, t))
    return out


# ----------------------------------------------------------------- served form
SERVE_THRESHOLDS = [(7, 10), (9, 10)]


@dataclass
class Served:
    resident: Collection
    batches: list          # [Collection]
    thresholds: list       # [(p, q)] per batch
    copies: list           # per batch: bool array, True where the set is a perturbed copy


def _csr_slice(col: Collection, a: int, b: int) -> Collection:
    off = col.offsets[a:b + 1]
    return Collection(offsets=(off - off[0]).astype(np.uint64),
                      tokens=col.tokens[int(off[0]):int(off[-1])].copy())


def served_workload(n_batches: int, resident_sets: int = 5_000_000, seed: int = SEED_BASE + 4,
                    max_batch: int = 10_000, copy_frac: float = 0.2, swap_frac: float = 0.1,
                    universe: int = 2_000_000) -> Served:
    """A resident collection and query batches against it.

    One generated collection (Zipf 1.1, log-normal sizes median 30, sigma 0.8,
    clipped 2..500) supplies both, so the token ids of resident and fresh sets
    share one frequency order: the first ``resident_sets`` sets are resident,
    the rest are fresh query sets.  Batch sizes are round(exp(U[0, ln
    max_batch])); each query set is, with probability ``copy_frac``, a copy of
    a uniformly chosen resident set with round(swap_frac * n) tokens replaced
    by token occurrences drawn uniformly from the whole collection (so they
    follow the global token frequencies), else the next fresh set.  The
    threshold of each batch is 7/10 or 9/10."""
    rng = np.random.Generator(np.random.PCG64((seed + 0x5E) & 0xFFFFFFFFFFFFFFFF))
    sizes = np.round(np.exp(rng.uniform(0.0, np.log(max_batch), n_batches))).astype(np.int64)
    is_copy = [rng.random(int(n)) < copy_frac for n in sizes]
    n_fresh = int(sum(int((~c).sum()) for c in is_copy))
    scale = (resident_sets + n_fresh) / 5_000_000
    col = generate(n_sets=resident_sets + n_fresh, universe=max(64, int(round(universe * scale))),
                   zipf_s=1.1, size_dist=SIZE_LOGNORMAL, size_a=30.0, size_b=0.8, size_lo=2,
                   size_hi=500, seed=seed)
    resident = _csr_slice(col, 0, resident_sets)
    fresh_at = resident_sets
    batches, thresholds = [], []
    for b in range(n_batches):
        sets = []
        for cp in is_copy[b]:
            if cp:
                k = int(rng.integers(resident_sets))
                base = resident.set(k)
                n = base.shape[0]
                n_swap = int(round(swap_frac * n))
                keep = np.sort(rng.choice(n, size=n - n_swap, replace=False)) if n_swap else \
                    np.arange(n)
                cur = set(int(x) for x in base[keep])
                while len(cur) < n:
                    cur.add(int(col.tokens[int(rng.integers(col.n_tokens))]))
                sets.append(np.array(sorted(cur), dtype=np.uint32))
            else:
                sets.append(col.set(fresh_at))
                fresh_at += 1
        batches.append(from_lists(sets))
        thresholds.append(SERVE_THRESHOLDS[int(rng.integers(len(SERVE_THRESHOLDS)))])
    return Served(resident=resident, batches=batches, thresholds=thresholds, copies=is_copy)
