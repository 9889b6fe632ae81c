// The bitmap filter over the length band -- the hot loop of the join.
//
// For every pair (i, j) of the band it evaluates the overlap bound of
// Theorem 1 (Eq. 2), UB = floor((|r| + |s| - popcount(b_r xor b_s)) / 2),
// and keeps the pair when UB reaches the overlap that the threshold needs
// (Table 1; Alg. 7, as the paper's GPU algorithm, Alg. 8, runs it).  With
// L = |r| + |s| and omin the least overlap that reaches t,
// UB >= omin  <=>  popcount(b_r xor b_s) <= L - 2 omin = slack,
// so each pair costs b/32 xor, b/32 accumulating popcounts and a compare.
//
// Work decomposition (size-ordered rows and columns, Section 2.3.2):
//   - a wave owns 64*R consecutive rows of one task, R per lane, with their
//     bitmaps in VGPRs for the whole tile;
//   - the wave walks the tile's columns in order; every column's bitmap is
//     wave-uniform and is read with scalar loads, one step of U columns
//     ahead, into two alternating register buffers;
//   - columns of equal size form a group; at a group start each lane
//     derives its threshold from the row and column sizes, folding the
//     length filter in (threshold -1 = never kept);
//   - the compare is folded into the popcount: the chain starts at
//     -(slack + 1), so a kept pair has a negative sum; the sums of a step's
//     U*R pairs are ORed and one ballot of the sign bit decides whether the
//     wave leaves the fast path to stage the kept (row, column) pairs at
//     their ballot ranks in its LDS buffer, which goes to the queue with one
//     reservation when full and at the end of every tile;
//   - self-join diagonal tiles add the triangle condition j < i.
// Waves are persistent and take tiles from cursors split per XCD.  When the
// survivor queue is full the wave marks its reserved slots as sentinels,
// records (tile, column, row slab) of its first staged pair to resume from,
// sets the overflow flag and stops; the host verifies the queue and
// relaunches with the resume list.
#include <algorithm>

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

// Kept pairs are staged per wave in LDS and written to the queue in runs:
// one queue reservation per run instead of one per (column, row slab) mask,
// since same-address atomics from every XCD serialise.  A run never spans
// tiles, so the first staged entry always names a point of the current tile.
constexpr uint32_t kStage = 256;

struct Sink {
  uint2 *queue;
  JoinCounters *ctr;
  unsigned long long cap;
  uint2 *stage;         // this wave's kStage LDS entries
  uint32_t fill;        // entries staged (wave-uniform)
  uint32_t first_col;   // (column, row slab) of the first staged entry
  uint32_t first_slab;
  uint32_t fail_col;    // resume point, set when the queue fills
  uint32_t fail_slab;
};

// Reserve queue slots for the staged entries and copy them out.  When they
// do not fit, the reserved slots that exist become sentinels, the first
// staged entry's point is left as the resume point and false is returned:
// every pair before that point is in the queue, none after it.
__device__ __forceinline__ bool flush(Sink &s) {
  const uint32_t n = rfl(s.fill);
  if (n == 0) return true;
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&s.ctr->queue_count, (unsigned long long)n);
  base = rfl64(base);
  const bool fits = base + n <= s.cap;
  __builtin_amdgcn_wave_barrier();
  for (uint32_t x = lane; x < n; x += 64) {
    const unsigned long long pos = base + x;
    if (pos < s.cap) s.queue[pos] = fits ? s.stage[x] : make_uint2(kSentinel, kSentinel);
  }
  __builtin_amdgcn_wave_barrier();
  s.fill = 0;
  if (!fits) {
    s.fail_col = s.first_col;
    s.fail_slab = s.first_slab;
    return false;
  }
  return true;
}

// popcount(x) + acc as one v_bcnt_u32_b32.  Written out so that the sum over
// a bitmap's words stays one accumulating chain (the compiler would otherwise
// split it into parallel chains joined by an extra add).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// bias + popcount(b_r xor b_c) with bias = -(slack + 1): negative exactly
// when the pair is kept.  The compare is folded into the popcount chain's
// starting value, so the sign bits of many pairs can be ORed together and
// tested once.
template <int W, int R>
__device__ __forceinline__ uint32_t biased_distance(const Rows<W, R> &rw, const uint32_t *cb,
                                                    int r, uint32_t bias) {
  uint32_t h = bcnt_acc(rw.bits[r][0] ^ cb[0], bias);
#pragma unroll
  for (int e = 1; e < 2 * W; ++e) h = bcnt_acc(rw.bits[r][e] ^ cb[e], h);
  return h;
}

// Slow path: stage the kept pairs of columns [j, j+U), one (column, row
// slab) mask at a time in (column, slab) order, from the biased distances
// the step computed.  False when the queue filled (resume point in the
// sink).
template <int W, int R, int U>
__device__ __forceinline__ bool emit(const Rows<W, R> &rw, const uint32_t (&d)[U][R], uint32_t j,
                                     Sink &sink) {
  const unsigned long long below = __lanemask_lt();
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool kp = (int32_t)d[u][r] < 0;
      const unsigned long long m = __ballot(kp);
      if (!m) continue;
      const uint32_t cnt = (uint32_t)__popcll(m);
      if (sink.fill + cnt > kStage && !flush(sink)) return false;
      if (sink.fill == 0) {
        sink.first_col = j + u;
        sink.first_slab = r;
      }
      if (kp) sink.stage[sink.fill + (uint32_t)__popcll(m & below)] = make_uint2(rw.idx[r], j + u);
      sink.fill += cnt;
    }
  return true;
}

// Column bitmaps are read through the constant address space: they are not
// written while the kernel runs, and uniform loads from that space always
// become scalar loads (s_load), whatever the slow path stores.
typedef const __attribute__((address_space(4))) uint32_t *const_u32_ptr;

__device__ __forceinline__ const_u32_ptr as_const(const uint64_t *p) {
  return (const_u32_ptr)(p);
}

// Bitmaps of columns [j, j + U) into SGPRs.
template <int W, int U>
__device__ __forceinline__ void load_cols(const uint64_t *__restrict__ bm_cols, uint32_t j,
                                          uint32_t (&cb)[U][2 * W]) {
  const_u32_ptr p = as_const(bm_cols + (size_t)j * W);
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < 2 * W; ++e) cb[u][e] = p[u * 2 * W + e];
}

// j, once every scalar load issued so far (the current step's columns)
// has arrived: the next step's load is then issued after that wait, on
// every path.
__device__ __forceinline__ uint32_t after(uint32_t j) {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0); vmcnt, expcnt untouched
  return j;
}

// One step: columns [j, j + U) against the wave's rows.  The biased
// distances of its U*R pairs are ORed and one ballot of the sign bit tells
// whether any is kept; only then does the slow path stage them.  On a
// diagonal tile a pair off the lower triangle (j >= i) is made positive.
// False when the queue filled.
template <int W, int R, int U, bool DIAG>
__device__ __forceinline__ bool step(const Rows<W, R> &rw, const uint32_t (&bias)[R],
                                     const uint32_t (&cb)[U][2 * W], uint32_t j, Sink &sink) {
  uint32_t d[U][R];
  uint32_t acc = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint32_t h = biased_distance<W, R>(rw, cb[u], r, bias[r]);
      if (DIAG) h = j + u < rw.idx[r] ? h : 0u;
      d[u][r] = h;
      acc |= h;
    }
  if (__ballot((int32_t)acc < 0)) return emit<W, R, U>(rw, d, j, sink);
  return true;
}

// Columns [j, g1) of one size group.
template <int W, int R, int U, bool DIAG>
__device__ __forceinline__ bool sweep(const uint64_t *__restrict__ bm_cols, const Rows<W, R> &rw,
                                      const int32_t (&thr)[R], uint32_t j, uint32_t g1,
                                      Sink &sink) {
  uint32_t bias[R];
#pragma unroll
  for (int r = 0; r < R; ++r) bias[r] = (uint32_t)(-thr[r] - 1);
  // Scalar loads may return out of order, so a wave can only wait for all
  // of them.  Two register buffers alternate: the wait for the current
  // step's columns comes before the next step's load is issued (the next
  // address is made to depend on the current columns), so the next load
  // is in flight while the current step computes, and no registers are
  // copied between steps.
  uint32_t ba[U][2 * W], bb[U][2 * W];
  if (j + U <= g1) load_cols<W, U>(bm_cols, j, ba);
  for (;;) {
    if (j + U > g1) break;
    const uint32_t jb = after(j + U);
    if (jb + U <= g1) load_cols<W, U>(bm_cols, jb, bb);
    if (!step<W, R, U, DIAG>(rw, bias, ba, j, sink)) return false;
    j += U;
    if (j + U > g1) break;
    const uint32_t ja = after(j + U);
    if (ja + U <= g1) load_cols<W, U>(bm_cols, ja, ba);
    if (!step<W, R, U, DIAG>(rw, bias, bb, j, sink)) return false;
    j += U;
  }
  for (; j < g1; ++j) {
    uint32_t cb[1][2 * W];
    load_cols<W, 1>(bm_cols, j, cb);
    if (!step<W, R, 1, DIAG>(rw, bias, cb, j, sink)) return false;
  }
  return true;
}

// One tile: rows [row0, row_end) of a row block (at most 64*R of them, R per
// lane, interleaved by 64), columns [c0, c1).  Returns false when the queue
// filled (a resume point has been recorded).
template <int W, int R, int U, bool COS>
__device__ __forceinline__ bool run_tile(
    const uint64_t *__restrict__ bm_rows, const uint64_t *__restrict__ bm_cols,
    const uint32_t *__restrict__ size_rows, const uint32_t *__restrict__ size_cols,
    const uint32_t *__restrict__ sstart_cols, uint32_t col_base,
    const int32_t *__restrict__ slack, const uint32_t *__restrict__ cmin,
    const uint32_t *__restrict__ cmax, bool cosine, uint32_t p, uint32_t q, uint32_t row0,
    uint32_t row_end, uint32_t c0, uint32_t c1, bool diag, uint32_t first_slab, Sink &sink) {
  const uint32_t lane = threadIdx.x & 63;
  Rows<W, R> rw;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = row0 + 64u * r + lane;
    rw.idx[r] = i;
    if (i < row_end) {
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
  uint32_t j = c0;
  while (j < c1) {
    const uint32_t c = rfl(size_cols[j]);
    const uint32_t g1 = min(max(col_base + rfl(sstart_cols[c + 1]), j + 1), c1);  // advances
    int32_t thr[R];
    bool any_ok = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in_band = c >= rw.cmn[r] && c <= rw.cmx[r];
      if (!in_band) thr[r] = -1;
      else if (COS && cosine) thr[r] = cosine_slack(rw.size[r], c, p, q);
      else thr[r] = slack[rw.size[r] + c];
      any_ok |= in_band;
    }
    // resumed inside column j: its slabs below first_slab are already queued,
    // so column j runs alone with those slabs masked off
    const uint32_t gend = first_slab ? j + 1 : g1;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if ((uint32_t)r < first_slab) thr[r] = -1;
    first_slab = 0;
    if (__ballot(any_ok)) {
      const bool ok =
          diag ? sweep<W, R, U, true>(bm_cols, rw, thr, j, gend, sink)
               : sweep<W, R, U, false>(bm_cols, rw, thr, j, gend, sink);
      if (!ok) return false;
    }
    j = gend;
  }
  // the tile's staged pairs go out before the next tile
  return flush(sink);
}

// Persistent filter for one bitmap width (W words, R rows per lane, U
// columns per step) over the tiles [cfg.tile_lo, cfg.tile_hi) of the plan.
// Waves first take the resume entries of a previous launch that fall in
// that range (entry k goes to wave k), then tiles from the partitioned
// cursors, until the range is exhausted or the queue has filled.
template <int W, int R, int U, bool COS>
__global__ __launch_bounds__(kBlock) void k_filter(
    const uint64_t *__restrict__ bm_rows, const uint64_t *__restrict__ bm_cols,
    const uint32_t *__restrict__ size_rows, const uint32_t *__restrict__ size_cols,
    const uint32_t *__restrict__ sstart_cols, const uint32_t *__restrict__ tables,
    const TaskDesc *__restrict__ tasks, const RowBlock *__restrict__ blocks,
    const uint32_t *__restrict__ tile_block,
    uint2 *__restrict__ queue, JoinCounters *__restrict__ ctr,
    const Resume *__restrict__ resume_in, Resume *__restrict__ resume_out, FilterConfig cfg) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = rfl(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
  __shared__ uint2 stage[kBlock / 64][kStage];
  Sink sink;
  sink.queue = queue;
  sink.ctr = ctr;
  sink.cap = cfg.cap;
  sink.stage = stage[threadIdx.x >> 6];
  sink.fill = 0;
  sink.first_col = 0;
  sink.first_slab = 0;
  sink.fail_col = 0;
  sink.fail_slab = 0;

  bool resumed = false;
  uint32_t t = 0, col = 0, slab = 0;
  if (wave < cfg.n_resume_in && wave < cfg.resume_cap) {
    t = rfl(resume_in[wave].tile);
    col = rfl(resume_in[wave].col);
    slab = rfl(resume_in[wave].slab);
    resumed = t >= cfg.tile_lo && t < cfg.tile_hi;
  }
  const uint32_t n_tiles = cfg.tile_hi - cfg.tile_lo;
  uint32_t *cursors = &ctr->tile_next[cfg.cls][0][0];
  // Workgroups are dispatched to the XCDs round-robin: start in this XCD's
  // partition of the tile range, move on to the others when it runs dry.
  uint32_t part = blockIdx.x % kParts, parts_left = kParts;
  for (;;) {
    if (!resumed) {
      if (__hip_atomic_load(&ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
      bool got = false;
      while (parts_left) {
        const uint32_t p0 = (uint32_t)(((uint64_t)n_tiles * part) / kParts);
        const uint32_t p1 = (uint32_t)(((uint64_t)n_tiles * (part + 1)) / kParts);
        // a relaxed read first: exhausted partitions cost no atomic
        uint32_t tt = p1 - p0;
        if (lane == 0 &&
            __hip_atomic_load(&cursors[part * 32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                p1 - p0)
          tt = atomicAdd(&cursors[part * 32], 1u);
        tt = rfl(tt);
        if (tt < p1 - p0) {
          t = cfg.tile_lo + p0 + tt;
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
    const uint32_t row_end = rfl(blocks[b].row_end);
    const uint32_t cbeg = rfl(blocks[b].col_begin);
    const uint32_t cend = rfl(blocks[b].col_end);
    const uint32_t k = t - rfl(blocks[b].tile_begin);
    const uint32_t task = rfl(blocks[b].task);
    const bool self = rfl(blocks[b].self) != 0;
    const TaskDesc *td = tasks + task;
    const int32_t *slack = reinterpret_cast<const int32_t *>(tables + rfl(td->slack_off));
    const uint32_t *cmin = tables + rfl(td->cmin_off);
    const uint32_t *cmax = tables + rfl(td->cmax_off);
    const uint32_t *sstart = sstart_cols + rfl64(td->col_sstart_off);
    const uint32_t col_base = rfl(td->col_base);
    const bool cosine = rfl(td->sim) == SSJ_SIM_COSINE;
    const uint32_t tp = rfl(td->p), tq = rfl(td->q);
    uint32_t c0, c1;
    bool diag = false;
    if (self) {
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
    uint32_t first_slab = 0;
    if (resumed) {
      c0 = col;
      first_slab = slab;
    }
    resumed = false;
    if (!run_tile<W, R, U, COS>(bm_rows, bm_cols, size_rows, size_cols, sstart, col_base, slack, cmin,
                           cmax, cosine, tp, tq, row0, min(row_end, cfg.n_rows), c0,
                           min(c1, cfg.n_cols), diag, first_slab, sink)) {
      // the queue is full: record where this tile resumes, and stop
      const uint32_t fcol = rfl(sink.fail_col), fslab = rfl(sink.fail_slab);
      if (lane == 0) {
        atomicOr(&ctr->overflow, 1u);
        const uint32_t q = atomicAdd(&ctr->n_resume, 1u);
        Resume rs;
        rs.tile = t;
        rs.col = fcol;
        rs.slab = fslab;
        rs.pad = 0;
        if (q < cfg.resume_cap) resume_out[q] = rs;
      }
      return;
    }
  }
}

template <int W, int R, int U, bool COS>
hipError_t launch_shape(dim3 grid, hipStream_t st, const FilterArgs &a) {
  hipLaunchKernelGGL((k_filter<W, R, U, COS>), grid, dim3(kBlock), 0, st, a.bm_rows, a.bm_cols,
                     a.size_rows, a.size_cols, a.sstart_cols, a.tables, a.tasks, a.blocks,
                     a.tile_block, a.queue, a.ctr, a.resume_in, a.resume_out, a.cfg);
  return hipGetLastError();
}

// Fixed-width kernels: (padded words, rows per lane, columns per step)
#define SSJ_FILTER_SHAPES(X) \
  X(1, 4, 4)                 \
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
#define X(w, r, u)            \
  if (padded_words == (w)) {  \
    s.words = (w);            \
    s.rows = 64 * (r);        \
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

hipError_t launch_filter(uint32_t padded_words, bool cosine, const FilterArgs &a,
                         hipStream_t st) {
  // a persistent grid, but no more waves than the launch has tiles or resume
  // entries to hand out (small width classes would otherwise start thousands
  // of waves that find nothing to do); wave k takes resume entry k
  const uint64_t need = std::max<uint64_t>(
      std::max<uint64_t>(a.cfg.tile_hi - a.cfg.tile_lo, a.cfg.n_resume_in), 1);
  const uint64_t waves_per_block = kBlock / 64;
  dim3 grid((unsigned)std::min<uint64_t>((uint64_t)filter_grid_blocks(),
                                         (need + waves_per_block - 1) / waves_per_block));
#define X(w, r, u)                                              \
  if (padded_words == (w))                                      \
    return cosine ? launch_shape<w, r, u, true>(grid, st, a)    \
                  : launch_shape<w, r, u, false>(grid, st, a);
  SSJ_FILTER_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace ssj
