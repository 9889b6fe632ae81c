"""Exact set similarity join with the Bitmap Filter on AMD Instinct MI355X.

Python binding of ``libssj.so`` (the C ABI declared in ``include/ssj.h``).
This module only marshals arguments: every step of a join runs in the
library's HIP kernels.  PyTorch provides device memory and streams.

Method: Sandes, Teodoro, Melo, "Bitmap Filter: Speeding up Exact Set
Similarity Joins with Bitwise Operations" (arXiv 1711.07295).
"""
from __future__ import annotations

import ctypes
import weakref
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssj.so")

SSJ_OK, SSJ_E_INVALID, SSJ_E_UNSORTED, SSJ_E_NOMEM, SSJ_E_DEVICE, SSJ_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
SSJ_SIM_JACCARD, SSJ_SIM_DICE, SSJ_SIM_COSINE, SSJ_SIM_OVERLAP = 0, 1, 2, 3
SSJ_BM_XOR, SSJ_BM_SET, SSJ_BM_NEXT, SSJ_BM_COMBINED = 0, 1, 2, 3
SSJ_FLAG_SURVIVORS_ONLY = 1
SSJ_FLAG_CUTOFF = 2
SSJ_FLAG_VALU = 4
SSJ_FLAG_MFMA = 8
SSJ_NOALLOC_MAX_SETS = 4_000_000
ABI_VERSION = 4  # SSJ_ABI_VERSION of include/ssj.h

EXPORTS = ("ssj_build_bitmaps", "ssj_build_bitmaps_noalloc", "ssj_self_join", "ssj_rs_join", "ssj_self_join_batch",
           "ssj_index_create", "ssj_index_query", "ssj_index_destroy", "ssj_cutoff",
           "ssj_free_pairs",
           "ssj_status_string", "ssj_abi_version", "ssj_memory_limit",
           "ssj_plan_self_join_batch", "ssj_plan_execute", "ssj_plan_destroy")


class ssj_sets(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("tokens", ctypes.c_void_p),
                ("n_sets", ctypes.c_uint64), ("n_tokens", ctypes.c_uint64)]


class ssj_pair(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32)]


class ssj_pairs(ctypes.Structure):
    _fields_ = [("pairs", ctypes.POINTER(ssj_pair)), ("count", ctypes.c_uint64)]


class ssj_stats(ctypes.Structure):
    _fields_ = [("band_pairs", ctypes.c_uint64), ("survivors", ctypes.c_uint64),
                ("results", ctypes.c_uint64), ("filter_ops", ctypes.c_uint64),
                ("queue_slots", ctypes.c_uint64),
                ("filter_launches", ctypes.c_uint32), ("b_bits", ctypes.c_uint32),
                ("n_classes", ctypes.c_uint32), ("class_bits", ctypes.c_uint32 * 8),
                ("class_max_size", ctypes.c_uint32 * 8), ("class_ops", ctypes.c_uint64 * 8),
                ("class_tiles", ctypes.c_uint64 * 8),
                ("class_ms", ctypes.c_float * 8), ("ms_total", ctypes.c_float),
                ("ms_prepare", ctypes.c_float), ("ms_filter", ctypes.c_float),
                ("ms_verify", ctypes.c_float), ("ms_emit", ctypes.c_float)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class ssj_options(ctypes.Structure):
    _fields_ = [("queue_capacity", ctypes.c_uint64), ("tile_cols", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class SsjError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """The built library.  Raises when it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1711_07295_amd/build.py`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, c_int = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sp = ctypes.POINTER(ssj_sets)
        lib.ssj_build_bitmaps.argtypes = [sp, u32, c_int, u32, u32, vp, vp]
        lib.ssj_build_bitmaps.restype = c_int
        lib.ssj_build_bitmaps_noalloc.argtypes = [sp, u32, c_int, u32, u32, vp, vp]
        lib.ssj_build_bitmaps_noalloc.restype = c_int
        lib.ssj_self_join.argtypes = [sp, vp, u32, c_int, u32, u32, ctypes.POINTER(ssj_options),
                                      ctypes.POINTER(ssj_pairs), ctypes.POINTER(ssj_stats), vp]
        lib.ssj_self_join.restype = c_int
        lib.ssj_rs_join.argtypes = [sp, vp, sp, vp, u32, c_int, u32, u32,
                                    ctypes.POINTER(ssj_options), ctypes.POINTER(ssj_pairs),
                                    ctypes.POINTER(ssj_stats), vp]
        lib.ssj_rs_join.restype = c_int
        u32p, u64p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
        lib.ssj_self_join_batch.argtypes = [sp, u32, u32p, u32p, u32, c_int,
                                            ctypes.POINTER(ssj_options), ctypes.POINTER(ssj_pairs),
                                            u64p, ctypes.POINTER(ssj_stats), vp]
        lib.ssj_self_join_batch.restype = c_int
        lib.ssj_index_create.argtypes = [sp, u32, ctypes.POINTER(vp), vp]
        lib.ssj_index_create.restype = c_int
        lib.ssj_index_query.argtypes = [vp, sp, u32, u32p, u32p, c_int,
                                        ctypes.POINTER(ssj_options), ctypes.POINTER(ssj_pairs),
                                        u64p, ctypes.POINTER(ssj_stats), vp]
        lib.ssj_index_query.restype = c_int
        lib.ssj_index_destroy.argtypes = [vp]
        lib.ssj_index_destroy.restype = None
        lib.ssj_cutoff.argtypes = [u32, c_int, c_int, u32, u32, u32p]
        lib.ssj_cutoff.restype = c_int
        lib.ssj_free_pairs.argtypes = [ctypes.POINTER(ssj_pairs)]
        lib.ssj_free_pairs.restype = None
        lib.ssj_status_string.argtypes = [c_int]
        lib.ssj_status_string.restype = ctypes.c_char_p
        lib.ssj_memory_limit.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        lib.ssj_memory_limit.restype = c_int
        lib.ssj_plan_self_join_batch.argtypes = [sp, u32, u32p, u32p, u32, c_int,
                                                 ctypes.POINTER(ssj_options), ctypes.POINTER(vp),
                                                 vp]
        lib.ssj_plan_self_join_batch.restype = c_int
        lib.ssj_plan_execute.argtypes = [vp, ctypes.POINTER(ssj_pairs),
                                         ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ssj_stats), vp]
        lib.ssj_plan_execute.restype = c_int
        lib.ssj_plan_destroy.argtypes = [vp]
        lib.ssj_plan_destroy.restype = None
        lib.ssj_abi_version.argtypes = []
        lib.ssj_abi_version.restype = c_int
        if lib.ssj_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has C ABI {lib.ssj_abi_version()}, this binding "
                               f"needs {ABI_VERSION}: rebuild it")
        _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().ssj_status_string(status).decode()


def ssj_abi_version() -> int:
    return load().ssj_abi_version()


@dataclass
class DeviceSets:
    """A collection in device memory (CSR), kept alive with its tensors."""
    offsets: object  # torch uint64 tensor [N+1] on the GPU
    tokens: object   # torch int32/uint32 tensor [T] on the GPU

    @property
    def n_sets(self) -> int:
        return int(self.offsets.numel()) - 1

    @property
    def n_tokens(self) -> int:
        return int(self.tokens.numel())

    def c(self) -> ssj_sets:
        return ssj_sets(self.offsets.data_ptr() if self.offsets.numel() else None,
                        self.tokens.data_ptr() if self.tokens.numel() else None,
                        self.n_sets, self.n_tokens)


def to_device(offsets, tokens, device="cuda") -> DeviceSets:
    """Upload a host CSR collection (uint64 offsets, uint32 tokens)."""
    import torch
    off = np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)
    tok = np.ascontiguousarray(tokens, dtype=np.uint32).view(np.int32)
    return DeviceSets(torch.from_numpy(off.copy()).to(device),
                      torch.from_numpy(tok.copy()).to(device))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _release(address: int, count: int) -> None:
    load().ssj_free_pairs(ctypes.byref(ssj_pairs(ctypes.cast(address, ctypes.POINTER(ssj_pair)),
                                                 count)))


def _take(out: ssj_pairs) -> np.ndarray:
    """The pairs as an (n, 2) uint32 array over the library's own buffer (no
    copy); the buffer goes back to the library when the array and every view
    of it are gone."""
    n = int(out.count)
    if n == 0:
        load().ssj_free_pairs(ctypes.byref(out))
        return np.zeros((0, 2), dtype=np.uint32)
    address = ctypes.cast(out.pairs, ctypes.c_void_p).value
    buf = (ctypes.c_uint32 * (2 * n)).from_address(address)
    done = weakref.finalize(buf, _release, address, n)
    done.atexit = False  # at exit the process returns the memory
    return np.frombuffer(buf, dtype=np.uint32).reshape(n, 2)


def _opts(queue_capacity=0, tile_cols=0, flags=0):
    if not (queue_capacity or tile_cols or flags):
        return None
    return ssj_options(queue_capacity, tile_cols, flags)


def ssj_build_bitmaps(sets: DeviceSets, b_bits: int, method: int = SSJ_BM_XOR, p: int = 0,
                      q: int = 0, out=None, stream=None):
    """Bitmaps of every set (caller order) as a (N, b/64) int64 tensor.
    ``p, q``: the Jaccard threshold Bitmap-Combined chooses its generator by
    (read only for SSJ_BM_COMBINED)."""
    import torch
    if out is None:
        out = torch.empty((sets.n_sets, b_bits // 64), dtype=torch.int64,
                          device=sets.offsets.device)
    cs = sets.c()
    st = load().ssj_build_bitmaps(ctypes.byref(cs), b_bits, method, p, q,
                                  out.data_ptr() if out.numel() else None, _stream(stream))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_build_bitmaps")
    return out


def ssj_build_bitmaps_noalloc(sets: DeviceSets, b_bits: int, out, method: int = SSJ_BM_XOR,
                              p: int = 0, q: int = 0, stream=None):
    """ssj_build_bitmaps into the caller's ``out`` ((N, b/64) int64 device
    tensor), through the entry point that allocates no device memory: its
    working memory is the library's fixed per-device array, which limits the
    collection to SSJ_NOALLOC_MAX_SETS sets."""
    if tuple(out.shape) != (sets.n_sets, b_bits // 64):
        raise ValueError(f"out must be ({sets.n_sets}, {b_bits // 64}), not {tuple(out.shape)}")
    cs = sets.c()
    st = load().ssj_build_bitmaps_noalloc(ctypes.byref(cs), b_bits, method, p, q,
                                          out.data_ptr() if out.numel() else None,
                                          _stream(stream))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_build_bitmaps_noalloc")
    return out


def ssj_self_join(sets: DeviceSets, p: int, q: int, b_bits: int = 64, bitmaps=None,
                  sim: int = SSJ_SIM_JACCARD, queue_capacity: int = 0, tile_cols: int = 0,
                  flags: int = 0, stream=None):
    """All pairs (i, j), i < j, with sim >= p/q.  Returns ((n, 2) uint32 array, stats dict)."""
    cs = sets.c()
    out, stats = ssj_pairs(), ssj_stats()
    o = _opts(queue_capacity, tile_cols, flags)
    st = load().ssj_self_join(ctypes.byref(cs), _ptr(bitmaps), b_bits, sim, p, q,
                              ctypes.byref(o) if o else None, ctypes.byref(out),
                              ctypes.byref(stats), _stream(stream))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_self_join")
    return _take(out), stats.as_dict()


def ssj_rs_join(r: DeviceSets, s: DeviceSets, p: int, q: int, b_bits: int = 64, r_bitmaps=None,
                s_bitmaps=None, sim: int = SSJ_SIM_JACCARD, queue_capacity: int = 0,
                tile_cols: int = 0, flags: int = 0, stream=None):
    """All pairs (i in R, j in S) with sim >= p/q.  Returns (pairs, stats dict)."""
    cr, cs = r.c(), s.c()
    out, stats = ssj_pairs(), ssj_stats()
    o = _opts(queue_capacity, tile_cols, flags)
    st = load().ssj_rs_join(ctypes.byref(cr), _ptr(r_bitmaps), ctypes.byref(cs),
                            _ptr(s_bitmaps), b_bits, sim, p, q, ctypes.byref(o) if o else None,
                            ctypes.byref(out), ctypes.byref(stats), _stream(stream))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_rs_join")
    return _take(out), stats.as_dict()


def _tasks(cols, p, q):
    n = len(cols)
    if len(p) != n or len(q) != n:
        raise ValueError("one threshold (p, q) per instance")
    arr = (ssj_sets * max(n, 1))(*[c.c() for c in cols])
    pa = (ctypes.c_uint32 * max(n, 1))(*[int(v) for v in p])
    qa = (ctypes.c_uint32 * max(n, 1))(*[int(v) for v in q])
    starts = (ctypes.c_uint64 * (n + 1))()
    return n, arr, pa, qa, starts


def _split(pairs: np.ndarray, starts, n: int):
    st = np.ctypeslib.as_array(starts, shape=(n + 1,)).astype(np.int64)
    return [pairs[st[k]:st[k + 1]] for k in range(n)]


def ssj_self_join_batch(instances, p, q, b_bits: int = 0, sim: int = SSJ_SIM_JACCARD,
                        queue_capacity: int = 0, tile_cols: int = 0, flags: int = 0,
                        stream=None):
    """Self-join of every instance (DeviceSets) at its own threshold p[k]/q[k],
    all in one call.  Returns ([pairs of instance k], totals stats dict)."""
    n, arr, pa, qa, starts = _tasks(instances, p, q)
    out, stats = ssj_pairs(), ssj_stats()
    o = _opts(queue_capacity, tile_cols, flags)
    st = load().ssj_self_join_batch(arr, n, pa, qa, b_bits, sim, ctypes.byref(o) if o else None,
                                    ctypes.byref(out), starts, ctypes.byref(stats),
                                    _stream(stream))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_self_join_batch")
    return _split(_take(out), starts, n), stats.as_dict()


class Plan:
    """A prepared self-join of one or more instances (ssj_plan_*): planned
    once, its first round replayed from a HIP graph by every execute().  The
    instances' buffers must stay alive and their offsets unchanged; the
    tokens may change between executions."""

    def __init__(self, instances, p, q, b_bits: int = 0, sim: int = SSJ_SIM_JACCARD,
                 queue_capacity: int = 0, tile_cols: int = 0, flags: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        n, arr, pa, qa, _ = _tasks(instances, p, q)
        self._keep = (list(instances), arr, pa, qa)
        self.n = n
        o = _opts(queue_capacity, tile_cols, flags)
        st = load().ssj_plan_self_join_batch(arr, n, pa, qa, b_bits, sim,
                                             ctypes.byref(o) if o else None,
                                             ctypes.byref(self._h), _stream(stream))
        if st != SSJ_OK:
            self._h = ctypes.c_void_p()
            raise SsjError(st, "ssj_plan_self_join_batch")

    def execute(self, stream=None):
        """Returns ([pairs of instance k], totals stats dict)."""
        if not self._h:
            raise RuntimeError("plan is closed")
        out, stats = ssj_pairs(), ssj_stats()
        starts = (ctypes.c_uint64 * (self.n + 1))()
        st = load().ssj_plan_execute(self._h, ctypes.byref(out), starts, ctypes.byref(stats),
                                     _stream(stream))
        if st != SSJ_OK:
            raise SsjError(st, "ssj_plan_execute")
        return _split(_take(out), starts, self.n), stats.as_dict()

    def close(self):
        if self._h:
            load().ssj_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Index:
    """A resident collection S for repeated R-S queries (ssj_index_*)."""

    def __init__(self, sets: DeviceSets, b_bits: int = 0, stream=None):
        self._h = ctypes.c_void_p()
        cs = sets.c()
        st = load().ssj_index_create(ctypes.byref(cs), b_bits, ctypes.byref(self._h),
                                     _stream(stream))
        if st != SSJ_OK:
            self._h = ctypes.c_void_p()
            raise SsjError(st, "ssj_index_create")
        self.n_sets = sets.n_sets
        self.b_bits = b_bits

    def query(self, batches, p, q, sim: int = SSJ_SIM_JACCARD, queue_capacity: int = 0,
              tile_cols: int = 0, flags: int = 0, stream=None):
        """R-S join of every batch (DeviceSets) against S at p[k]/q[k], in one
        call.  Returns ([pairs of batch k], totals stats dict)."""
        if not self._h:
            raise RuntimeError("index is closed")
        n, arr, pa, qa, starts = _tasks(batches, p, q)
        out, stats = ssj_pairs(), ssj_stats()
        o = _opts(queue_capacity, tile_cols, flags)
        st = load().ssj_index_query(self._h, arr, n, pa, qa, sim, ctypes.byref(o) if o else None,
                                    ctypes.byref(out), starts, ctypes.byref(stats),
                                    _stream(stream))
        if st != SSJ_OK:
            raise SsjError(st, "ssj_index_query")
        return _split(_take(out), starts, n), stats.as_dict()

    def close(self):
        if self._h:
            load().ssj_index_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssj_memory_limit(limit_bytes: int) -> int:
    """Caps the device memory of the library's per-call working memory on
    each device (0: no cap); returns the bytes the current device's chunks
    hold now."""
    held = ctypes.c_uint64(0)
    st = load().ssj_memory_limit(int(limit_bytes), ctypes.byref(held))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_memory_limit")
    return int(held.value)


def ssj_cutoff(b_bits: int, p: int, q: int, method: int = SSJ_BM_XOR,
               sim: int = SSJ_SIM_JACCARD) -> int:
    """The cutoff point omega(b, p/q) of Section 3.5 (host computation)."""
    out = ctypes.c_uint32()
    st = load().ssj_cutoff(b_bits, method, sim, p, q, ctypes.byref(out))
    if st != SSJ_OK:
        raise SsjError(st, "ssj_cutoff")
    return int(out.value)


def ssj_free_pairs(out: ssj_pairs) -> None:
    load().ssj_free_pairs(ctypes.byref(out))
