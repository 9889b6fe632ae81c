"""CPU oracle for the exact set similarity join -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct integer code (``oracle.c``) written from the
paper (Sandes, Teodoro, Melo, arXiv 1711.07295): the naive join of Alg. 1 with
the similarity functions of Table 1, the length filter of Table 2, the bitmap
generators of Alg. 3-5, the overlap bound of Theorem 1 (Eq. 2) and the filter
decision of Alg. 7.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

Every pin of this oracle lives in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

JACCARD, DICE, COSINE, OVERLAP = 0, 1, 2, 3
BM_XOR, BM_SET, BM_NEXT, BM_COMBINED = 0, 1, 2, 3

_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, u64, i64, c_int = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        lib.oracle_merge_count.argtypes = [vp, u64, vp, u64, vp, vp]
        lib.oracle_merge_count.restype = None
        lib.oracle_similar.argtypes = [c_int, u64, u64, u64, u64, u64, u64]
        lib.oracle_similar.restype = c_int
        lib.oracle_length_ok.argtypes = [c_int, u64, u64, u64, u64]
        lib.oracle_length_ok.restype = c_int
        lib.oracle_self_join.argtypes = [vp, vp, u64, c_int, u64, u64, c_int, ctypes.POINTER(_u64p)]
        lib.oracle_self_join.restype = i64
        lib.oracle_rs_join.argtypes = [vp, vp, u64, vp, vp, u64, c_int, u64, u64, c_int,
                                       ctypes.POINTER(_u64p)]
        lib.oracle_rs_join.restype = i64
        lib.oracle_self_join_rows.argtypes = [vp, vp, u64, vp, u64, c_int, u64, u64, c_int,
                                              ctypes.POINTER(_u64p)]
        lib.oracle_self_join_rows.restype = i64
        lib.oracle_size_order.argtypes = [vp, u64, vp]
        lib.oracle_size_order.restype = c_int
        lib.oracle_self_join_banded.argtypes = [vp, vp, u64, vp, vp, u64, c_int, u64, u64, c_int,
                                                ctypes.POINTER(_u64p), vp]
        lib.oracle_self_join_banded.restype = i64
        lib.oracle_band_pairs.argtypes = [vp, u64, c_int, u64, u64]
        lib.oracle_band_pairs.restype = u64
        lib.oracle_bitmap_one.argtypes = [vp, u64, c_int, ctypes.c_uint32, vp]
        lib.oracle_bitmap_one.restype = c_int
        lib.oracle_bitmaps.argtypes = [vp, vp, u64, c_int, ctypes.c_uint32, vp]
        lib.oracle_bitmaps.restype = c_int
        lib.oracle_overlap_ub.argtypes = [u64, u64, u64]
        lib.oracle_overlap_ub.restype = u64
        lib.oracle_bitmap_survives.argtypes = [u64, u64, u64, u64, u64]
        lib.oracle_bitmap_survives.restype = c_int
        lib.oracle_bitmap_survives_sim.argtypes = [c_int, u64, u64, u64, u64, u64]
        lib.oracle_bitmap_survives_sim.restype = c_int
        lib.oracle_combined_method.argtypes = [u64, u64]
        lib.oracle_combined_method.restype = c_int
        lib.oracle_survivors.argtypes = [vp, u64, vp, ctypes.c_uint32, vp, c_int, u64, u64, c_int,
                                         vp, ctypes.POINTER(_u64p)]
        lib.oracle_survivors.restype = i64
        lib.oracle_check_pairs.argtypes = [vp, vp, vp, vp, vp, u64, c_int, u64, u64, vp]
        lib.oracle_check_pairs.restype = None
        lib.oracle_free.argtypes = [vp]
        lib.oracle_free.restype = None
        _lib = lib
    return _lib


def _threads(n):
    return n if n else min(16, os.cpu_count() or 1)


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a if a.size else np.zeros(1, dtype=np.uint32)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def _take_pairs(ptr, n) -> np.ndarray:
    """(n, 2) uint32 array of (i, j) from a malloc'd (i << 32 | j) buffer."""
    lib = _load()
    if n < 0:
        raise MemoryError("oracle failed")
    try:
        keys = (np.ctypeslib.as_array(ptr, shape=(n,)).copy() if n
                else np.zeros(0, dtype=np.uint64))
    finally:
        lib.oracle_free(ctypes.cast(ptr, ctypes.c_void_p))
    out = np.empty((n, 2), dtype=np.uint32)
    out[:, 0] = (keys >> np.uint64(32)).astype(np.uint32)
    out[:, 1] = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out


def merge_count(r, s) -> tuple[int, int]:
    """(|r n s|, |r u s|) of two strictly increasing token arrays, by one merge."""
    lib = _load()
    ra = np.ascontiguousarray(r, dtype=np.uint32)
    sa = np.ascontiguousarray(s, dtype=np.uint32)
    rb = ra if ra.size else np.zeros(1, dtype=np.uint32)
    sb = sa if sa.size else np.zeros(1, dtype=np.uint32)
    o, u = ctypes.c_uint64(), ctypes.c_uint64()
    lib.oracle_merge_count(rb.ctypes.data, ra.size, sb.ctypes.data, sa.size,
                           ctypes.byref(o), ctypes.byref(u))
    return int(o.value), int(u.value)


def similar(sim: int, o: int, u: int, nr: int, ns: int, p: int, q: int) -> bool:
    return bool(_load().oracle_similar(sim, o, u, nr, ns, p, q))


def length_ok(sim: int, nr: int, ns: int, p: int, q: int) -> bool:
    return bool(_load().oracle_length_ok(sim, nr, ns, p, q))


def self_join(offsets, tokens, p: int, q: int, sim: int = JACCARD, threads: int | None = None):
    """All (i, j), i < j, with sim >= p/q (Alg. 1).  (n, 2) uint32, ascending."""
    lib = _load()
    off, tok = _u64(offsets), _u32(tokens)
    ptr = _u64p()
    n = lib.oracle_self_join(off.ctypes.data, tok.ctypes.data, off.shape[0] - 1, sim, p, q,
                             _threads(threads), ctypes.byref(ptr))
    return _take_pairs(ptr, n)


def rs_join(r_offsets, r_tokens, s_offsets, s_tokens, p: int, q: int, sim: int = JACCARD,
            threads: int | None = None):
    """All (i in R, j in S) with sim >= p/q (Alg. 1).  (n, 2) uint32, ascending."""
    lib = _load()
    ro, rt, so, st = _u64(r_offsets), _u32(r_tokens), _u64(s_offsets), _u32(s_tokens)
    ptr = _u64p()
    n = lib.oracle_rs_join(ro.ctypes.data, rt.ctypes.data, ro.shape[0] - 1,
                           so.ctypes.data, st.ctypes.data, so.shape[0] - 1,
                           sim, p, q, _threads(threads), ctypes.byref(ptr))
    return _take_pairs(ptr, n)


def self_join_rows(offsets, tokens, rows, p: int, q: int, sim: int = JACCARD,
                   threads: int | None = None):
    """Every similar pair (min, max) that involves one of ``rows`` (caller indices)."""
    lib = _load()
    off, tok = _u64(offsets), _u32(tokens)
    rows = _u64(rows)
    rb = rows if rows.size else np.zeros(1, dtype=np.uint64)
    ptr = _u64p()
    n = lib.oracle_self_join_rows(off.ctypes.data, tok.ctypes.data, off.shape[0] - 1,
                                  rb.ctypes.data, rows.size, sim, p, q, _threads(threads),
                                  ctypes.byref(ptr))
    return _take_pairs(ptr, n)


def size_order(offsets) -> np.ndarray:
    """Positions sorted by (set size, caller index)."""
    lib = _load()
    off = _u64(offsets)
    n = off.shape[0] - 1
    order = np.empty(max(n, 1), dtype=np.uint32)
    lib.oracle_size_order(off.ctypes.data, n, order.ctypes.data)
    return order[:n]


def self_join_banded(offsets, tokens, p: int, q: int, sim: int = JACCARD, rows=None,
                     order=None, threads: int | None = None):
    """Banded self-join (length filter skips, same result).  ``rows`` are
    size-order positions to process (None = all).  Returns (pairs, evaluated)."""
    lib = _load()
    off, tok = _u64(offsets), _u32(tokens)
    if order is None:
        order = size_order(off)
    order = _u32(order)
    ptr = _u64p()
    ev = ctypes.c_uint64()
    if rows is None:
        rows_ptr, nrows = None, 0
    else:
        rows = _u64(rows)
        rb = rows if rows.size else np.zeros(1, dtype=np.uint64)
        rows_ptr, nrows = rb.ctypes.data, rows.size
    n = lib.oracle_self_join_banded(off.ctypes.data, tok.ctypes.data, off.shape[0] - 1,
                                    order.ctypes.data, rows_ptr, nrows, sim, p, q,
                                    _threads(threads), ctypes.byref(ptr), ctypes.byref(ev))
    return _take_pairs(ptr, n), int(ev.value)


def band_pairs(sizes, p: int, q: int, sim: int = JACCARD) -> int:
    """Unordered pairs of non-empty sets that pass the length filter (Table 2)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    mx = int(sizes.max()) if sizes.size else 0
    hist = np.bincount(sizes, minlength=mx + 1).astype(np.uint64)
    return int(_load().oracle_band_pairs(hist.ctypes.data, mx, sim, p, q))


def band_pairs_rs(r_sizes, s_sizes, p: int, q: int, sim: int = JACCARD) -> int:
    """Pairs (i in R, j in S) of non-empty sets that pass the length filter
    (Table 2), from the two size histograms."""
    hr = np.bincount(np.asarray(r_sizes, dtype=np.int64))
    hs = np.bincount(np.asarray(s_sizes, dtype=np.int64))
    total = 0
    for a in range(1, hr.shape[0]):
        if not hr[a]:
            continue
        for c in range(1, hs.shape[0]):
            if hs[c] and length_ok(sim, a, c, p, q):
                total += int(hr[a]) * int(hs[c])
    return total


def combined_method(p: int, q: int) -> int:
    """The generator Bitmap-Combined (Alg. 6) takes for a Jaccard threshold
    t = p/q: Next, Set or Xor by the normalized threshold 2t/(1+t)."""
    return int(_load().oracle_combined_method(p, q))


def _method(method: int, p, q) -> int:
    if method != BM_COMBINED:
        return method
    if not p or not q:
        raise ValueError("Bitmap-Combined needs the threshold p/q")
    return combined_method(p, q)


def bitmap(tokens, b: int, method: int = BM_XOR, p: int | None = None,
           q: int | None = None) -> np.ndarray:
    """One set's bitmap, b/64 uint64 words (Alg. 3/4/5, h(t) = t mod b;
    Alg. 6 with the Jaccard threshold p/q)."""
    lib = _load()
    method = _method(method, p, q)
    t = np.ascontiguousarray(tokens, dtype=np.uint32)
    tb = t if t.size else np.zeros(1, dtype=np.uint32)
    out = np.zeros(b // 64, dtype=np.uint64)
    rc = lib.oracle_bitmap_one(tb.ctypes.data, t.size, method, b, out.ctypes.data)
    if rc:
        raise ValueError("bad bitmap width or method")
    return out


def bitmaps(offsets, tokens, b: int, method: int = BM_XOR, p: int | None = None,
            q: int | None = None) -> np.ndarray:
    """(N, b/64) uint64 bitmaps of every set, caller order (Bitmap-Combined:
    the generator Alg. 6 picks for the Jaccard threshold p/q)."""
    lib = _load()
    method = _method(method, p, q)
    off, tok = _u64(offsets), _u32(tokens)
    n = off.shape[0] - 1
    out = np.zeros((max(n, 1), b // 64), dtype=np.uint64)
    rc = lib.oracle_bitmaps(off.ctypes.data, tok.ctypes.data, n, method, b, out.ctypes.data)
    if rc:
        raise ValueError("bad bitmap width or method")
    return out[:n]


def overlap_ub(nr: int, ns: int, hamming: int) -> int:
    """Eq. 2: floor((|r| + |s| - popcount(b_r xor b_s)) / 2)."""
    return int(_load().oracle_overlap_ub(nr, ns, hamming))


def bitmap_survives(nr: int, ns: int, hamming: int, p: int, q: int, sim: int | None = None) -> bool:
    """Alg. 7's decision for a threshold p/q: not pruned.  Without ``sim``
    the Jaccard-only form; with it, the form for any function of Table 1."""
    if sim is None:
        return bool(_load().oracle_bitmap_survives(nr, ns, hamming, p, q))
    return bool(_load().oracle_bitmap_survives_sim(sim, nr, ns, hamming, p, q))


def survivors(offsets, bms, b: int, p: int, q: int, order=None, listing: bool = False,
              threads: int | None = None, sim: int = JACCARD):
    """Survivors of the bitmap filter over the length band of the function
    ``sim``.  Returns (count, band_pairs, pairs or None)."""
    lib = _load()
    off = _u64(offsets)
    n = off.shape[0] - 1
    bm = np.ascontiguousarray(bms, dtype=np.uint64)
    if bm.size == 0:
        bm = np.zeros((1, b // 64), dtype=np.uint64)
    if order is None:
        order = size_order(off)
    order = _u32(order)
    band = ctypes.c_uint64()
    ptr = _u64p()
    cnt = lib.oracle_survivors(off.ctypes.data, n, bm.ctypes.data, b, order.ctypes.data, sim, p,
                               q, _threads(threads), ctypes.byref(band),
                               ctypes.byref(ptr) if listing else None)
    if cnt < 0:
        raise MemoryError("oracle failed")
    pairs = _take_pairs(ptr, int(cnt)) if listing else None
    return int(cnt), int(band.value), pairs


def check_pairs(r_offsets, r_tokens, s_offsets, s_tokens, pairs, p: int, q: int,
                sim: int = JACCARD) -> np.ndarray:
    """Boolean array: sim >= p/q for each (i, j) row of ``pairs`` (R x S)."""
    lib = _load()
    ro, rt, so, st = _u64(r_offsets), _u32(r_tokens), _u64(s_offsets), _u32(s_tokens)
    pr = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    ok = np.zeros(max(len(pr), 1), dtype=np.uint8)
    pb = pr if pr.size else np.zeros((1, 2), dtype=np.uint32)
    lib.oracle_check_pairs(ro.ctypes.data, rt.ctypes.data, so.ctypes.data, st.ctypes.data,
                           pb.ctypes.data, len(pr), sim, p, q, ok.ctypes.data)
    return ok[:len(pr)].astype(bool)


# ---- Section 3.4: expected bound (Eqs. 4-6) and the cutoff point ------------
# Eq. 5 is evaluated as printed, as its sum over odd k, each term in log space
# (the binomial coefficients of 2n up to 2^20 do not fit a double).

def expected_bound(method: int, b: int, n: int) -> float:
    """E(b, n): the expected overlap bound (Eq. 2 without the floor) of two
    sets of n random tokens each (Eqs. 4, 5, 6)."""
    import math
    b, n = int(b), int(n)
    if method == BM_SET:      # Eq. 4
        return n + math.exp(2 * n * math.log(b - 1) - (2 * n - 1) * math.log(b)) \
            - math.exp(n * math.log(b - 1) - (n - 1) * math.log(b))
    if method == BM_XOR:      # Eq. 5
        from scipy.special import gammaln
        k = np.arange(1, 2 * n + 1, 2, dtype=np.float64)
        m = 2.0 * n
        log_terms = (gammaln(m + 1) - gammaln(k + 1) - gammaln(m - k + 1)
                     - k * math.log(b) + (m - k) * math.log((b - 1) / b))
        return n - b / 2 * float(np.exp(log_terms).sum())
    if method == BM_NEXT:     # Eq. 6
        return min(n * n / b, float(n))
    raise ValueError(method)


def expected_bound_exact(method: int, b: int, n: int):
    """E(b, n) as an exact Fraction, for the comparisons the floating value
    cannot decide.  Eq. 5's sum over odd k of C(2n, k) (b-1)^(2n-k) is the
    odd half of the binomial expansion of (1 + (b-1))^(2n), i.e.
    (b^(2n) - (b-2)^(2n)) / 2 -- an identity the tests check against the
    term-by-term sum."""
    from fractions import Fraction
    if method == BM_SET:
        return Fraction(n) + Fraction((b - 1) ** (2 * n), b ** (2 * n - 1)) \
            - Fraction((b - 1) ** n, b ** (n - 1))
    if method == BM_XOR:
        odd = (b ** (2 * n) - (b - 2) ** (2 * n)) // 2
        return Fraction(n) - Fraction(b, 2) * Fraction(odd, b ** (2 * n))
    return min(Fraction(n * n, b), Fraction(n))


def normalized_threshold(sim: int, p: int, q: int):
    """The overlap fraction o/n two sets of n tokens need to reach sim >= p/q
    (the normalized scale of Fig. 5), exactly: Jaccard 2t/(1+t), Dice and
    Cosine t."""
    from fractions import Fraction
    t = Fraction(p, q)
    if sim == JACCARD:
        return 2 * t / (1 + t)
    if sim in (DICE, COSINE):
        return t
    raise ValueError("no normalized threshold for Overlap")


def cutoff(method: int, b: int, tau, n_max: int = 1 << 20) -> int:
    """Section 3.4: the cutoff point, the largest set size n at which the
    expected normalized bound E(b, n)/n is still at most tau; Alg. 7 applies
    the filter to sets up to this size.  E(b, n)/n grows with n, so the
    largest such n is found by bisection.  0 when n = 1 already exceeds tau.
    tau: a Fraction, or a decimal given as a string or float."""
    from fractions import Fraction
    tau = Fraction(str(tau)) if isinstance(tau, float) else Fraction(tau)

    def ok(n):
        v = expected_bound(method, b, n) / n
        if abs(v - float(tau)) > 1e-9:
            return v <= float(tau)
        return expected_bound_exact(method, b, n) / n <= tau

    if not ok(1):
        return 0
    lo, hi = 1, n_max          # ok(lo); the answer is below hi or is n_max
    if ok(hi):
        return hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo
