// The bitmap filter over the length band -- the hot loop of the join.
//
// For every pair (i, j) of the band it evaluates the overlap bound of
// Theorem 1 (Eq. 2), UB = floor((|r| + |s| - popcount(b_r xor b_s)) / 2),
// and keeps the pair when UB reaches the overlap that the threshold needs
// (Table 1; Alg. 7 without the cutoff, as the paper's GPU algorithm, Alg. 8,
// runs it).  With L = |r| + |s| and omin(L) the least overlap that reaches
// t, UB >= omin(L)  <=>  popcount(b_r xor b_s) <= L - 2 omin(L) = slack(L),
// so each pair costs b/32 xor, b/32 accumulating popcounts and one compare.
//
// Work decomposition (size-ordered rows and columns, Section 2.3.2):
//   - a wave owns 64*R consecutive rows, R per lane, with their bitmaps in
//     VGPRs for the whole tile;
//   - the wave walks the tile's columns in order; every column's bitmap is
//     wave-uniform and is read with scalar loads;
//   - columns of equal size form a group; at a group start each lane
//     derives its threshold from the row and column sizes, folding the
//     length filter in (threshold -1 = never kept), so the per-pair work is
//     exactly the xor/popcount/compare;
//   - the compare lands in a wave mask (ballot); only when some lane keeps a
//     pair does the wave leave the fast path, reserve queue slots with one
//     atomic and write the (row, column) pairs at their ballot ranks;
//   - self-join diagonal tiles add the triangle condition j < i.
// Waves are persistent and take tiles from an atomic cursor.  When the
// survivor queue is full the wave marks its reserved slots as sentinels,
// records (tile, column) to resume from, sets the overflow flag and stops;
// the host verifies the queue and relaunches with the resume list.
#include "ssj_internal.h"

namespace ssj {
namespace {

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long rfl64(unsigned long long v) {
  uint32_t lo = rfl((uint32_t)v), hi = rfl((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

template <int W, int R>
struct Rows {
  uint32_t bits[R][2 * W];
  uint32_t size[R];
  uint32_t cmn[R];
  uint32_t cmx[R];
  uint32_t idx[R];
};

struct Sink {
  uint2 *queue;
  JoinCounters *ctr;
  Resume *resume_out;
  unsigned long long cap;
  uint32_t tile;
  uint32_t resume_cap;
};

// popcount(x) + acc as one v_bcnt_u32_b32.  Written out so that the sum over
// a bitmap's words stays one accumulating chain (the compiler would otherwise
// split it into parallel chains joined by an extra add).
__device__ __forceinline__ uint32_t bcnt_first(uint32_t x) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, 0" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

template <int W, int R, bool DIAG>
__device__ __forceinline__ bool keep(const Rows<W, R> &rw, const uint32_t *cb, int r,
                                     int32_t thr, uint32_t j) {
  uint32_t h = bcnt_first(rw.bits[r][0] ^ cb[0]);
#pragma unroll
  for (int e = 1; e < 2 * W; ++e) h = bcnt_acc(rw.bits[r][e] ^ cb[e], h);
  bool k = (int32_t)h <= thr;
  if (DIAG) k = k && (j < rw.idx[r]);
  return k;
}

// Slow path: write the kept pairs of columns [j, j+U).  Returns false when
// the queue is full (the tile is to be resumed at column j).
template <int W, int R, int U, bool DIAG>
__device__ __forceinline__ bool emit(const Rows<W, R> &rw, const int32_t (&thr)[R],
                                               const uint32_t (&cb)[U][2 * W], uint32_t j,
                                               const Sink &sink) {
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long m[U][R];
  uint32_t total = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      m[u][r] = __ballot(keep<W, R, DIAG>(rw, cb[u], r, thr[r], j + u));
      total += (uint32_t)__popcll(m[u][r]);
    }
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&sink.ctr->queue_count, (unsigned long long)total);
  base = rfl64(base);
  const bool fits = base + total <= sink.cap;
  const unsigned long long below = __lanemask_lt();
  unsigned long long off = base;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if ((m[u][r] >> lane) & 1ull) {
        unsigned long long pos = off + (unsigned long long)__popcll(m[u][r] & below);
        if (pos < sink.cap)
          sink.queue[pos] = fits ? make_uint2(rw.idx[r], j + u) : make_uint2(kSentinel, kSentinel);
      }
      off += (unsigned long long)__popcll(m[u][r]);
    }
  if (!fits) {
    if (lane == 0) {
      atomicOr(&sink.ctr->overflow, 1u);
      uint32_t k = atomicAdd(&sink.ctr->n_resume, 1u);
      Resume rs;
      rs.tile = sink.tile;
      rs.col = j;
      if (k < sink.resume_cap) sink.resume_out[k] = rs;
    }
    return false;
  }
  return true;
}

// Columns [j, g1) of one size group.
template <int W, int R, int U, bool DIAG>
__device__ __forceinline__ bool sweep(const uint64_t *__restrict__ bm_cols, const Rows<W, R> &rw,
                                      const int32_t (&thr)[R], uint32_t j, uint32_t g1,
                                      const Sink &sink) {
  // Scalar loads may return out of order, so a wave can only wait for all
  // of them; the next step's columns are therefore requested right after the
  // wait for the current step and arrive while the current step computes.
  uint32_t nb[U][2 * W];
  if (j + U <= g1) {
    const uint32_t *p = reinterpret_cast<const uint32_t *>(bm_cols + (size_t)j * W);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 2 * W; ++e) nb[u][e] = p[u * 2 * W + e];
  }
  for (; j + U <= g1; j += U) {
    uint32_t cb[U][2 * W];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 2 * W; ++e) cb[u][e] = nb[u][e];
    if (j + 2 * U <= g1) {
      const uint32_t *p = reinterpret_cast<const uint32_t *>(bm_cols + (size_t)(j + U) * W);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) nb[u][e] = p[u * 2 * W + e];
    }
    unsigned long long any = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) any |= __ballot(keep<W, R, DIAG>(rw, cb[u], r, thr[r], j + u));
    if (any) {
      if (!emit<W, R, U, DIAG>(rw, thr, cb, j, sink)) return false;
    }
  }
  for (; j < g1; ++j) {
    uint32_t cb[1][2 * W];
    const uint32_t *p = reinterpret_cast<const uint32_t *>(bm_cols + (size_t)j * W);
#pragma unroll
    for (int e = 0; e < 2 * W; ++e) cb[0][e] = p[e];
    unsigned long long any = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) any |= __ballot(keep<W, R, DIAG>(rw, cb[0], r, thr[r], j));
    if (any) {
      if (!emit<W, R, 1, DIAG>(rw, thr, cb, j, sink)) return false;
    }
  }
  return true;
}

template <int W, int R, int U>
__global__ __launch_bounds__(kBlock) void k_filter(
    const uint64_t *__restrict__ bm_rows, const uint64_t *__restrict__ bm_cols,
    const uint32_t *__restrict__ size_rows, const uint32_t *__restrict__ size_cols,
    const uint32_t *__restrict__ sstart_cols, const int32_t *__restrict__ slack,
    const uint32_t *__restrict__ cmin, const uint32_t *__restrict__ cmax,
    const RowBlock *__restrict__ blocks, const uint32_t *__restrict__ tile_block,
    uint2 *__restrict__ queue, JoinCounters *__restrict__ ctr,
    const Resume *__restrict__ resume_in, Resume *__restrict__ resume_out, FilterConfig cfg) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = rfl(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
  Sink sink;
  sink.queue = queue;
  sink.ctr = ctr;
  sink.resume_out = resume_out;
  sink.cap = cfg.cap;
  sink.resume_cap = cfg.resume_cap;

  bool resumed = wave < cfg.n_resume_in && wave < cfg.resume_cap;
  uint32_t t = 0, col = 0;
  if (resumed) {
    t = rfl(resume_in[wave].tile);
    col = rfl(resume_in[wave].col);
  }
  // Workgroups are dispatched to the XCDs round-robin: start in this XCD's
  // partition of the tile list, move on to the others when it runs dry.
  uint32_t part = blockIdx.x % kParts, parts_left = kParts;
  for (;;) {
    if (!resumed) {
      if (__hip_atomic_load(&ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
      bool got = false;
      while (parts_left) {
        const uint32_t p0 = (uint32_t)(((uint64_t)cfg.n_tiles * part) / kParts);
        const uint32_t p1 = (uint32_t)(((uint64_t)cfg.n_tiles * (part + 1)) / kParts);
        uint32_t tt = 0;
        if (lane == 0) tt = atomicAdd(&ctr->tile_next[part][0], 1u);
        tt = rfl(tt);
        if (tt < p1 - p0) {
          t = p0 + tt;
          got = true;
          break;
        }
        part = part + 1 == kParts ? 0 : part + 1;
        --parts_left;
      }
      if (!got) return;
    }
    // decode the tile
    const uint32_t b = rfl(tile_block[t]);
    if (b >= cfg.n_blocks) return;
    const uint32_t row0 = rfl(blocks[b].row0);
    const uint32_t cbeg = rfl(blocks[b].col_begin);
    const uint32_t cend = rfl(blocks[b].col_end);
    const uint32_t k = t - rfl(blocks[b].tile_begin);
    uint32_t c0, c1;
    bool diag = false;
    if (cfg.self) {
      const uint32_t n_int = (row0 - cbeg + cfg.tile_cols - 1) / cfg.tile_cols;
      if (k < n_int) {
        c0 = cbeg + k * cfg.tile_cols;
        c1 = min(c0 + cfg.tile_cols, row0);
      } else {
        c0 = row0;
        c1 = cend;
        diag = true;
      }
    } else {
      c0 = cbeg + k * cfg.tile_cols;
      c1 = min(c0 + cfg.tile_cols, cend);
    }
    if (resumed) c0 = col;
    resumed = false;
    sink.tile = t;

    // the wave's rows
    Rows<W, R> rw;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = row0 + 64u * r + lane;
      rw.idx[r] = i;
      if (i < cfg.n_rows) {
        const uint32_t a = size_rows[i];
        rw.size[r] = a;
        rw.cmn[r] = cmin[a];
        rw.cmx[r] = cmax[a];
        const uint32_t *src = reinterpret_cast<const uint32_t *>(bm_rows + (size_t)i * W);
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) rw.bits[r][e] = src[e];
      } else {
        rw.size[r] = 0;
        rw.cmn[r] = 0xFFFFFFFFu;
        rw.cmx[r] = 0;
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) rw.bits[r][e] = 0;
      }
    }

    bool ok = true;
    uint32_t j = c0;
    while (j < c1) {
      const uint32_t c = rfl(size_cols[j]);
      const uint32_t g1 = min(max(rfl(sstart_cols[c + 1]), j + 1), c1);  // always advances
      int32_t thr[R];
      bool any_ok = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool in_band = c >= rw.cmn[r] && c <= rw.cmx[r];
        thr[r] = in_band ? slack[rw.size[r] + c] : -1;
        any_ok |= in_band;
      }
      if (__ballot(any_ok)) {
        ok = diag ? sweep<W, R, U, true>(bm_cols, rw, thr, j, g1, sink)
                  : sweep<W, R, U, false>(bm_cols, rw, thr, j, g1, sink);
        if (!ok) break;
      }
      j = g1;
    }
    if (!ok) return;
  }
}

template <int W, int R, int U>
hipError_t launch_w(dim3 grid, hipStream_t st, const uint64_t *bm_rows, const uint64_t *bm_cols,
                    const uint32_t *size_rows, const uint32_t *size_cols,
                    const uint32_t *sstart_cols, const int32_t *slack, const uint32_t *cmin,
                    const uint32_t *cmax, const RowBlock *blocks, const uint32_t *tile_block,
                    uint2 *queue, JoinCounters *ctr, const Resume *resume_in,
                    Resume *resume_out, FilterConfig cfg) {
  hipLaunchKernelGGL((k_filter<W, R, U>), grid, dim3(kBlock), 0, st, bm_rows, bm_cols, size_rows,
                     size_cols, sstart_cols, slack, cmin, cmax, blocks, tile_block, queue, ctr,
                     resume_in, resume_out, cfg);
  return hipGetLastError();
}

// (padded words, rows per lane, columns per step)
#define SSJ_FILTER_SHAPES(X) \
  X(1, 2, 8)                 \
  X(2, 2, 4)                 \
  X(3, 2, 2)                 \
  X(4, 2, 2)                 \
  X(5, 1, 2)                 \
  X(6, 1, 2)                 \
  X(7, 1, 2)                 \
  X(8, 1, 2)                 \
  X(10, 1, 1)                \
  X(12, 1, 1)                \
  X(16, 1, 1)                \
  X(20, 1, 1)                \
  X(24, 1, 1)                \
  X(32, 1, 1)                \
  X(40, 1, 1)                \
  X(48, 1, 1)                \
  X(64, 1, 1)

}  // namespace

uint32_t filter_padded_words(uint32_t words) {
#define X(w, r, u) \
  if (words <= (w)) return (w);
  SSJ_FILTER_SHAPES(X)
#undef X
  return 0;
}

FilterShape filter_shape(uint32_t padded_words) {
  FilterShape s{0, 0, 0};
#define X(w, r, u)       \
  if (padded_words == (w)) { \
    s.words = (w);       \
    s.rows = 64 * (r);   \
    s.batch = 64 * (r) * (u); \
  }
  SSJ_FILTER_SHAPES(X)
#undef X
  return s;
}

int filter_grid_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus * 8;  // 32 waves per CU
}

hipError_t launch_filter(uint32_t padded_words, const uint64_t *bm_rows, const uint64_t *bm_cols,
                         const uint32_t *size_rows, const uint32_t *size_cols,
                         const uint32_t *sstart_cols, const int32_t *slack,
                         const uint32_t *cmin, const uint32_t *cmax, const RowBlock *blocks,
                         const uint32_t *tile_block, uint2 *queue, JoinCounters *ctr,
                         const Resume *resume_in, Resume *resume_out, FilterConfig cfg,
                         hipStream_t st) {
  dim3 grid(filter_grid_blocks());
#define X(w, r, u)                                                                           \
  if (padded_words == (w))                                                                   \
    return launch_w<w, r, u>(grid, st, bm_rows, bm_cols, size_rows, size_cols, sstart_cols, \
                             slack, cmin, cmax, blocks, tile_block, queue, ctr, resume_in,   \
                             resume_out, cfg);
  SSJ_FILTER_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace ssj
