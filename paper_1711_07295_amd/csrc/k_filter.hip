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

// Kept pairs are staged per wave in LDS and written to the queue in runs.
// Queue slots come from a chunk the wave reserves for itself (cfg.chunk
// slots per reservation), so reservations are few: same-address atomics
// from every XCD serialise at the memory side, and one per run would cost
// more than the filter.  A run never spans tiles, so the first staged entry
// always names a point of the current tile.  The unused end of a chunk is
// filled with sentinels (verification skips them) when the wave takes a
// new chunk and when it exits.
constexpr uint32_t kStage = kFilterStage;

struct Sink {
  uint2 *queue;
  JoinCounters *ctr;
  unsigned long long cap;
  uint32_t chunk;              // slots per reservation (>= kStage)
  uint2 *stage;                // this wave's kStage LDS entries
  uint32_t fill;               // entries staged (wave-uniform)
  uint32_t first_col;          // (column, row slab) of the first staged entry
  uint32_t first_slab;
  uint32_t fail_col;           // resume point, set when the queue fills
  uint32_t fail_slab;
  unsigned long long pos, end; // the wave's reserved slots [pos, end), end <= cap
};

// Sentinels into the rest of the wave's chunk.
__device__ __forceinline__ void sink_pad(Sink &s) {
  const uint32_t lane = threadIdx.x & 63;
  for (unsigned long long x = s.pos + lane; x < s.end; x += 64)
    s.queue[x] = make_uint2(kSentinel, kSentinel);
  s.pos = s.end;
}

// Copy the staged entries into the wave's chunk, reserving a new chunk
// when they do not fit in the current one.  When the queue has no room
// for them, the reserved slots become sentinels, the first staged entry's
// point is left as the resume point and false is returned: every pair
// before that point is in the queue, none after it.
__device__ __forceinline__ bool flush(Sink &s) {
  const uint32_t n = rfl(s.fill);
  if (n == 0) return true;
  const uint32_t lane = threadIdx.x & 63;
  if (s.pos + n > s.end) {
    sink_pad(s);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&s.ctr->queue_count, (unsigned long long)s.chunk);
    base = rfl64(base);
    s.pos = base < s.cap ? base : s.cap;
    s.end = base + s.chunk < s.cap ? base + s.chunk : s.cap;
    if (s.pos + n > s.end) {
      sink_pad(s);
      s.fill = 0;
      s.fail_col = s.first_col;
      s.fail_slab = s.first_slab;
      return false;
    }
  }
  __builtin_amdgcn_wave_barrier();
  for (uint32_t x = lane; x < n; x += 64) s.queue[s.pos + x] = s.stage[x];
  __builtin_amdgcn_wave_barrier();
  s.pos += n;
  s.fill = 0;
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
  static_assert(U * R <= 32, "one word holds the step's kept flags");
  const unsigned long long below = __lanemask_lt();
  // bit u*R + r: this lane's pair (column j + u, row slab r) is kept; one
  // loop then stages the masks, so the staging code exists once
  uint32_t kb = 0;
#pragma unroll
  for (int x = U * R - 1; x >= 0; --x)
    kb = (kb << 1) | ((int32_t)d[x / R][x % R] < 0 ? 1u : 0u);
  const uint32_t row_slab0 = rw.idx[0];  // this lane's row in slab r: + 64 r
#pragma unroll 1
  for (uint32_t x = 0; x < (uint32_t)(U * R); ++x) {
    const bool kp = (kb >> x) & 1u;
    const unsigned long long m = __ballot(kp);
    if (!m) continue;
    const uint32_t u = x / R, r = x - u * R;
    const uint32_t cnt = (uint32_t)__popcll(m);
    if (sink.fill + cnt > kStage && !flush(sink)) return false;
    if (sink.fill == 0) {
      sink.first_col = j + u;
      sink.first_slab = r;
    }
    if (kp)
      sink.stage[sink.fill + (uint32_t)__popcll(m & below)] =
          make_uint2(row_slab0 + 64u * r, j + u);
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

// What a wave needs to run one tile.
struct TileJob {
  uint32_t row0, row_end, c0, c1;
  bool diag;
  uint32_t first;  // resumed inside the tile: first slab (vector ALU) or pairs to skip (MFMA)
  const int32_t *slack;
  const uint32_t *cmin, *cmax, *sstart;
  uint32_t col_base;
  bool cosine;
  uint32_t p, q;
};

// The persistent loop both kernels share, over the tiles [cfg.tile_lo,
// cfg.tile_hi) of the plan.  Waves first take the resume entries of a
// previous launch that fall in that range (entry k goes to wave k), then
// tiles from the partitioned cursors, until the range is exhausted or the
// queue has filled.  run(job) runs one tile and returns false when the
// queue filled, with the resume point in the sink.
template <class Run>
__device__ __forceinline__ void persistent(const uint32_t *__restrict__ tables,
                                           const TaskDesc *__restrict__ tasks,
                                           const RowBlock *__restrict__ blocks,
                                           const uint32_t *__restrict__ tile_block,
                                           const uint32_t *__restrict__ sstart_cols,
                                           JoinCounters *__restrict__ ctr,
                                           const Resume *__restrict__ resume_in,
                                           Resume *__restrict__ resume_out,
                                           const FilterConfig &cfg, Sink &sink, Run &&run) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = rfl(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
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
  // Each XCD owns one contiguous region of the tile range, so that its
  // waves sweep neighbouring row blocks whose columns stay in its L2.
  // Inside a region the tiles are dealt to kSub sub-cursors in blocks of
  // kDeal, so that the cursors' atomics spread over kSub addresses (atomics
  // on one address from every XCD serialise) while the region is still
  // swept as one front.  Workgroups are dispatched to the XCDs round-robin:
  // a workgroup starts on its own XCD's region, takes that region's other
  // sub-cursors when its own runs dry, and then the other regions.
  constexpr uint32_t kSub = kParts / kXcds, kDeal = 4;
  const uint32_t xcd0 = blockIdx.x % kXcds, sub0 = (blockIdx.x / kXcds) % kSub;
  uint32_t visit = 0;
  for (;;) {
    if (!resumed) {
      if (__hip_atomic_load(&ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      bool got = false;
      while (visit < kParts) {
        const uint32_t x = (xcd0 + visit / kSub) % kXcds, k = (sub0 + visit) % kSub;
        const uint32_t r0 = (uint32_t)(((uint64_t)n_tiles * x) / kXcds);
        const uint32_t len = (uint32_t)(((uint64_t)n_tiles * (x + 1)) / kXcds) - r0;
        // tiles of the region sub-cursor k owns: blocks k, k + kSub, ...
        const uint32_t rounds = len / (kSub * kDeal), rem = len - rounds * kSub * kDeal;
        const uint32_t owned =
            rounds * kDeal + min(kDeal, rem > k * kDeal ? rem - k * kDeal : 0u);
        uint32_t *cur = &cursors[(x * kSub + k) * 32];
        // a relaxed read first: exhausted sub-cursors cost no atomic
        uint32_t c = owned;
        if (lane == 0 &&
            __hip_atomic_load(cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < owned)
          c = atomicAdd(cur, 1u);
        c = rfl(c);
        if (c < owned) {
          t = cfg.tile_lo + r0 + ((c / kDeal) * kSub + k) * kDeal + c % kDeal;
          got = true;
          break;
        }
        ++visit;
      }
      if (!got) break;
    }
    // decode the tile
    const uint32_t b = rfl(tile_block[t]);
    if (b >= cfg.n_blocks) break;
    TileJob job;
    job.row0 = rfl(blocks[b].row0);
    job.row_end = min(rfl(blocks[b].row_end), cfg.n_rows);
    const uint32_t cbeg = rfl(blocks[b].col_begin);
    const uint32_t cend = rfl(blocks[b].col_end);
    const uint32_t k = t - rfl(blocks[b].tile_begin);
    const uint32_t task = rfl(blocks[b].task);
    const bool self = rfl(blocks[b].self) != 0;
    const TaskDesc *td = tasks + task;
    job.slack = reinterpret_cast<const int32_t *>(tables + rfl(td->slack_off));
    job.cmin = tables + rfl(td->cmin_off);
    job.cmax = tables + rfl(td->cmax_off);
    job.sstart = sstart_cols + rfl64(td->col_sstart_off);
    job.col_base = rfl(td->col_base);
    job.cosine = rfl(td->sim) == SSJ_SIM_COSINE;
    job.p = rfl(td->p);
    job.q = rfl(td->q);
    uint32_t c0, c1;
    job.diag = false;
    if (self) {
      const uint32_t n_int = (job.row0 - cbeg + cfg.tile_cols - 1) / cfg.tile_cols;
      if (k < n_int) {
        c0 = cbeg + k * cfg.tile_cols;
        c1 = min(c0 + cfg.tile_cols, job.row0);
      } else {
        c0 = job.row0;
        c1 = cend;
        job.diag = true;
      }
    } else {
      c0 = cbeg + k * cfg.tile_cols;
      c1 = min(c0 + cfg.tile_cols, cend);
    }
    job.first = 0;
    if (resumed) {
      c0 = col;
      job.first = slab;
    }
    resumed = false;
    job.c0 = c0;
    job.c1 = min(c1, cfg.n_cols);
    if (!run(job)) {
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
      break;
    }
  }
  sink_pad(sink);
}

__device__ __forceinline__ void sink_init(Sink &sink, uint2 *queue, JoinCounters *ctr,
                                          const FilterConfig &cfg, uint2 *stage) {
  sink.queue = queue;
  sink.ctr = ctr;
  sink.cap = cfg.cap;
  sink.chunk = max(cfg.chunk, kStage);
  sink.pos = 0;
  sink.end = 0;
  sink.stage = stage;
  sink.fill = 0;
  sink.first_col = 0;
  sink.first_slab = 0;
  sink.fail_col = 0;
  sink.fail_slab = 0;
}

// Vector-ALU filter for one bitmap width (W words, R rows per lane, U
// columns per step).
template <int W, int R, int U, bool COS>
__global__ __launch_bounds__(kBlock) void k_filter(
    const uint64_t *__restrict__ bm_rows, const uint64_t *__restrict__ bm_cols,
    const uint32_t *__restrict__ size_rows, const uint32_t *__restrict__ size_cols,
    const uint32_t *__restrict__ sstart_cols, const uint32_t *__restrict__ tables,
    const TaskDesc *__restrict__ tasks, const RowBlock *__restrict__ blocks,
    const uint32_t *__restrict__ tile_block, uint2 *__restrict__ queue,
    JoinCounters *__restrict__ ctr, const Resume *__restrict__ resume_in,
    Resume *__restrict__ resume_out, FilterConfig cfg) {
  __shared__ uint2 stage[kBlock / 64][kStage];
  Sink sink;
  sink_init(sink, queue, ctr, cfg, stage[threadIdx.x >> 6]);
  persistent(tables, tasks, blocks, tile_block, sstart_cols, ctr, resume_in, resume_out, cfg,
             sink, [&](const TileJob &jb) {
               return run_tile<W, R, U, COS>(bm_rows, bm_cols, size_rows, size_cols, jb.sstart,
                                             jb.col_base, jb.slack, jb.cmin, jb.cmax, jb.cosine,
                                             jb.p, jb.q, jb.row0, jb.row_end, jb.c0, jb.c1,
                                             jb.diag, jb.first, sink);
             });
}

// ---------------------------------------------------------------------------
// Matrix-core filter (b = 64, 128, 256, 512, 1024).
//
// With every bit of a bitmap mapped to +1 (set) or -1 (clear), the dot
// product of two such vectors over K bits is K - 2 popcount(b_r xor b_s), so
// the test of Theorem 1 reads dot >= T = K - 2 slack.  The values +-1 are
// exact in fp4 (e2m1) and the dot products are small integers, exact in the
// fp32 accumulator, so the decision is the same as the vector-ALU kernel's.
// One v_mfma_scale_f32_32x32x64_f8f6f4 scores 32 columns against 32 rows
// over 64 bits:
//   - MFMA rows (A) are 32 consecutive columns of the sweep (one step),
//     loaded per step from the column sign planes, the next step's while
//     the current one computes;
//   - MFMA columns (B) are 32 of the wave's rows, RT such row tiles, held in
//     registers for the whole tile;
//   - lane l holds row l%32 of every row tile and 16 of the step's columns,
//     8(v/4) + 4(l/32) + v%4 for v = 0..15.  Steps never cross a size group
//     (a group's last step is partial; lanes past its end load zeros), so
//     one threshold per lane and row tile covers all 16 values: the max of
//     the 16 dot products against T is the whole fast-path test.
// The slow path stages the kept pairs in a fixed order (row tile, then v,
// then lane), so a step resumed after a full queue skips exactly the pairs
// it had written.

typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef float v16f_t __attribute__((ext_vector_type(16)));

constexpr float kNever = 1.0e30f;  // threshold of a row that no column of the group pairs with

template <int W, int RT>
struct MRows {
  uint4 sg[RT][W];  // this lane's half of every 64-bit block of its row in each row tile
  float thr[RT];    // dot threshold for the current size group
  // the same threshold for the fast test, which compares the bit patterns
  // of the dot products as integers: for a positive threshold those order
  // like the values (every value is an exact integer, +0 included, and the
  // negative ones fall below every positive pattern); a threshold of 0 or
  // less becomes INT32_MIN, so that every step goes to the exact test
  int32_t thr_bits[RT];
  uint32_t size[RT];
  uint32_t cmn[RT];
  uint32_t cmx[RT];
  uint32_t idx;     // this lane's row in row tile 0 (row tile rt: idx + 32 rt)
};

__device__ __forceinline__ v16f_t mfma_pm1(const uint4 &a, const uint4 &b, const v16f_t &c) {
  const v8i_t x = {(int)a.x, (int)a.y, (int)a.z, (int)a.w, 0, 0, 0, 0};
  const v8i_t y = {(int)b.x, (int)b.y, (int)b.z, (int)b.w, 0, 0, 0, 0};
  // formats 4/4: fp4 (e2m1) for A and B; scales 2^0 (e8m0 127)
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y, c, 4, 4, 0, 127, 0, 127);
}

// This lane's half of every block of column `col`, or zeros when !ok: the
// planes hold n + 1 columns, column n all zero, so every lane loads and no
// load sits behind a branch.
// This lane's half of set `col`'s sign planes (set n, all zero, when !ok).
template <int W>
__device__ __forceinline__ void load_signs(const uint4 *__restrict__ planes, uint32_t n,
                                           uint32_t col, bool ok, uint32_t h, uint4 (&a)[W]) {
  const size_t c = ok ? col : n;
#pragma unroll
  for (int kb = 0; kb < W; ++kb) a[kb] = planes[((size_t)kb * (n + kSignPad) + c) * 2 + h];
}

// The columns j0 + (lane % 32) of one step: a uniform address (j0 is the
// same in every lane) plus the lane's byte offset loff = 32 (lane % 32) +
// 16 h.  No bounds test: the zero padding past set n - 1 covers loads up to
// 95 columns past a column below n, and the pairs of columns past the size
// group's end are dropped by the exact test.
template <int W>
__device__ __forceinline__ void load_cols(const uint4 *__restrict__ planes, uint32_t n,
                                          uint32_t j0, uint32_t loff, uint4 (&a)[W]) {
#pragma unroll
  for (int kb = 0; kb < W; ++kb) {
    const uint4 *p = planes + ((size_t)kb * (n + kSignPad) + j0) * 2;
    a[kb] = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(p) + loff);
  }
}

// Stage one ballot mask of kept pairs (row `row` of the lanes' row tile is
// the caller's; column per lane): `skip` pairs are dropped first, `done`
// counts the step's pairs in order.
__device__ __forceinline__ bool stage_mask(unsigned long long m, uint32_t row, uint32_t col,
                                           uint32_t j0, uint32_t &skip, uint32_t &done,
                                           Sink &sink) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t cnt = (uint32_t)__popcll(m);
  if (skip) {
    if (skip >= cnt) {
      skip -= cnt;
      done += cnt;
      return true;
    }
    for (uint32_t x = 0; x < skip; ++x) m &= m - 1;  // drop the lowest `skip` lanes
    done += skip;
    cnt -= skip;
    skip = 0;
  }
  if (sink.fill + cnt > kStage && !flush(sink)) return false;
  if (sink.fill == 0) {
    sink.first_col = j0;
    sink.first_slab = done;
  }
  if ((m >> lane) & 1ull)
    sink.stage[sink.fill + (uint32_t)__popcll(m & __lanemask_lt())] = make_uint2(row, col);
  sink.fill += cnt;
  done += cnt;
  return true;
}

// Slow path of one step at columns [j0, j0 + 32) of a group ending at gend:
// stage the kept pairs.  Only row tiles whose best value reaches their
// threshold are looked at; in them each lane packs its kept values into the
// bits of one word.  Few lanes with kept values (the usual case): the wave
// walks those lanes and their set bits, one pair at a time, in the order
// (lane, v).  Many: one ballot per value v stages whole masks, in the order
// (v, lane).  The choice depends only on the step's values, so a step
// resumed after a full queue takes the same order and skips exactly the
// `skip` pairs it had written.
template <int W, int RT>
__device__ __forceinline__ bool emit_mfma(const MRows<W, RT> &rw, const uint4 (&a)[W],
                                          const int32_t (&mx)[RT], uint32_t j0, uint32_t gend,
                                          bool diag, uint32_t &skip, Sink &sink) {
  constexpr uint32_t kFewLanes = 4;
  const uint32_t lane = threadIdx.x & 63, h = lane >> 5;
  const uint32_t cb = j0 + 4u * h;  // this lane's column for v is cb + 8(v/4) + v%4
  const uint32_t row0 = (uint32_t)__builtin_amdgcn_readlane((int)rw.idx, 0);  // lane 0: row0
  uint32_t done = 0;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if (!__ballot(mx[rt] >= rw.thr_bits[rt])) continue;
    // the step's dot products of this row tile again (the fast path does
    // not keep them: registers are what limits the waves per SIMD)
    v16f_t d = {};
#pragma unroll
    for (int kb = 0; kb < W; ++kb) d = mfma_pm1(a[kb], rw.sg[rt][kb], d);
    const uint32_t my_row = rw.idx + 32u * rt;
    uint32_t k = 0;  // bit v: value v kept (built by shifting: no wide constants)
#pragma unroll
    for (int v = 15; v >= 0; --v) {
      const uint32_t col = cb + 8u * (v / 4) + (uint32_t)(v % 4);
      const bool kp = d[v] >= rw.thr[rt] && col < gend && (!diag || col < my_row);
      k = (k << 1) | (kp ? 1u : 0u);
    }
    unsigned long long lm = __ballot(k != 0);
    if ((uint32_t)__popcll(lm) > kFewLanes) {
#pragma unroll 1
      for (uint32_t v = 0; v < 16; ++v) {
        const unsigned long long m = __ballot((k >> v) & 1u);
        if (m && !stage_mask(m, my_row, cb + 8u * (v >> 2) + (v & 3u), j0, skip, done, sink))
          return false;
      }
      continue;
    }
    while (lm) {
      const uint32_t L = (uint32_t)__builtin_ctzll(lm);
      lm &= lm - 1;
      uint32_t kk = (uint32_t)__builtin_amdgcn_readlane((int)k, (int)L);
      const uint32_t row = row0 + 32u * rt + (L & 31u);
      const uint32_t cL = j0 + 4u * (L >> 5);
      while (kk) {
        const uint32_t v = (uint32_t)__builtin_ctz(kk);
        kk &= kk - 1;
        if (skip) {
          --skip;
          ++done;
          continue;
        }
        if (sink.fill == kStage && !flush(sink)) return false;
        if (sink.fill == 0) {
          sink.first_col = j0;
          sink.first_slab = done;
        }
        if (lane == 0) sink.stage[sink.fill] = make_uint2(row, cL + 8u * (v >> 2) + (v & 3u));
        ++sink.fill;
        ++done;
      }
    }
  }
  return true;
}

// The dot products of the step's columns `a` with row tile rt.
template <int W, int RT>
__device__ __forceinline__ v16f_t products(const uint4 (&a)[W], const MRows<W, RT> &rw, int rt) {
  v16f_t t = {};
#pragma unroll
  for (int kb = 0; kb < W; ++kb) t = mfma_pm1(a[kb], rw.sg[rt][kb], t);
  return t;
}

// Largest of the 16 dot products of a lane (one row, 16 columns) as a bit
// pattern compared as an integer: a tree of 3-input maxima.
__device__ __forceinline__ int32_t max16(const v16f_t &x) {
  int32_t b[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) b[v] = __float_as_int(x[v]);
  int32_t m0 = max(max(b[0], b[1]), b[2]);
  int32_t m1 = max(max(b[3], b[4]), b[5]);
  int32_t m2 = max(max(b[6], b[7]), b[8]);
  int32_t m3 = max(max(b[9], b[10]), b[11]);
  int32_t m4 = max(max(b[12], b[13]), b[14]);
  m0 = max(max(m0, m1), m2);
  m3 = max(max(m3, m4), b[15]);
  return max(m0, m3);
}

// Fast path of one step: columns [j0, j0 + 32) (operands `a`) against the
// wave's rows.  Leaves each row tile's largest bit pattern (as an integer)
// in mx and returns whether one reaches its threshold (thr_bits).  Integer
// maxima: float maxima would first quiet possible signalling NaNs, two
// more instructions per row tile.
//
// The products run one row tile ahead of their reduction, across steps:
// product number k (row tile k mod RT of step k / RT) goes into
// accumulator k mod 3 and is reduced while product k + 1 runs on the
// matrix cores; the last row tile's reduction overlaps the first product
// of the next step (operands `an`, the next step's columns, already
// loaded).  K is the step's place in the three-step unrolled loop, so that
// every accumulator index is a constant; on entry accumulator (K RT) mod 3
// holds this step's first product.  When the sweep ends after this step,
// that last product is simply dropped.
template <int W, int RT, int K>
__device__ __forceinline__ bool fast_mfma(const uint4 (&a)[W], const uint4 (&an)[W],
                                          const MRows<W, RT> &rw, v16f_t (&acc)[3],
                                          int32_t (&mx)[RT]) {
  unsigned long long hit = 0;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    constexpr int base = K * RT;
    const int cur = (base + rt) % 3, nxt = (base + rt + 1) % 3;
    acc[nxt] = rt + 1 < RT ? products<W, RT>(a, rw, rt + 1) : products<W, RT>(an, rw, 0);
    __builtin_amdgcn_sched_barrier(0);
    mx[rt] = max16(acc[cur]);
    hit |= __ballot(mx[rt] >= rw.thr_bits[rt]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // the next step's first product stays ahead of the branch that ends the
  // step (the compiler would otherwise sink it below, into the next step)
  asm volatile("" ::"v"(acc[(K * RT + RT) % 3]));
  return hit != 0;
}

// The steps of columns [j, g1) of one size group.  Column loads run two
// steps ahead in a ring of three register buffers; the loop is unrolled by
// three so that the ring turns without register copies (a copy of a buffer
// still being loaded would wait for that load) and the accumulators of the
// fast path keep constant indices.  A step that keeps something leaves the
// loop for the one slow path, laid out once (instruction cache: the kernel
// stays small); the slow path turns the ring by register moves so that the
// loop goes on at the next step with the buffers already loaded.  Every
// branch leaves the loop, none enters it in the middle, and every buffer
// is read on both sides of each exit: the compiler keeps the ring in fixed
// registers and leaves the loads where they are.
template <int W, int RT>
__device__ __forceinline__ bool sweep_mfma(const uint4 *__restrict__ sg_cols, uint32_t n_cols,
                                           const MRows<W, RT> &rw, uint32_t j, uint32_t g1,
                                           bool diag, uint32_t &skip, Sink &sink) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t loff = (lane & 31u) * 32u + (lane >> 5) * 16u;
  uint4 b0[W], b1[W], b2[W];
  int32_t mx[RT];
  v16f_t acc[3];
  uint32_t j0 = j;
  load_cols<W>(sg_cols, n_cols, j0, loff, b0);
  load_cols<W>(sg_cols, n_cols, j0 + 32, loff, b1);
  for (;;) {
    int phase;  // the ring buffer that holds the columns of step j0
    // The step's columns for the slow path, copied on the way out of the
    // loop from the one buffer that holds them: selecting among the three
    // would read the buffer whose load the step has just issued, and wait
    // for it (a whole memory round trip per slow-path entry).
    uint4 cur[W];
    acc[0] = products<W, RT>(b0, rw, 0);
    for (;;) {
      load_cols<W>(sg_cols, n_cols, j0 + 64, loff, b2);
      if (__builtin_expect(fast_mfma<W, RT, 0>(b0, b1, rw, acc, mx), 0)) {
        phase = 0;
#pragma unroll
        for (int kb = 0; kb < W; ++kb) cur[kb] = b0[kb];
        break;
      }
      skip = 0;
      if ((j0 += 32) >= g1) return true;
      load_cols<W>(sg_cols, n_cols, j0 + 64, loff, b0);
      if (__builtin_expect(fast_mfma<W, RT, 1>(b1, b2, rw, acc, mx), 0)) {
        phase = 1;
#pragma unroll
        for (int kb = 0; kb < W; ++kb) cur[kb] = b1[kb];
        break;
      }
      skip = 0;
      if ((j0 += 32) >= g1) return true;
      load_cols<W>(sg_cols, n_cols, j0 + 64, loff, b1);
      if (__builtin_expect(fast_mfma<W, RT, 2>(b2, b0, rw, acc, mx), 0)) {
        phase = 2;
#pragma unroll
        for (int kb = 0; kb < W; ++kb) cur[kb] = b2[kb];
        break;
      }
      skip = 0;
      if ((j0 += 32) >= g1) return true;
    }
    if (!emit_mfma<W, RT>(rw, cur, mx, j0, g1, diag, skip, sink)) return false;
    skip = 0;
    if ((j0 += 32) >= g1) return true;
    // b0 and b1 take the columns of steps j0 and j0 + 32
#pragma unroll
    for (int kb = 0; kb < W; ++kb) {
      const uint4 x0 = phase == 0 ? b1[kb] : phase == 1 ? b2[kb] : b0[kb];
      const uint4 x1 = phase == 0 ? b2[kb] : phase == 1 ? b0[kb] : b1[kb];
      b0[kb] = x0;
      b1[kb] = x1;
    }
  }
}

// One tile on the matrix cores: rows [row0, row_end) (at most 32*RT),
// columns [c0, c1).
template <int W, int RT, bool COS>
__device__ __forceinline__ bool run_tile_mfma(const uint4 *__restrict__ sg_rows,
                                              const uint4 *__restrict__ sg_cols, uint32_t n_rows,
                                              uint32_t n_cols, const uint32_t *__restrict__ size_rows,
                                              const uint32_t *__restrict__ size_cols,
                                              const TileJob &jb, Sink &sink) {
  const uint32_t lane = threadIdx.x & 63, h = lane >> 5, jr = lane & 31;
  constexpr int32_t K = 64 * W;
  MRows<W, RT> rw;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const uint32_t i = jb.row0 + 32u * rt + jr;
    if (rt == 0) rw.idx = i;
    if (i < jb.row_end) {
      const uint32_t a = size_rows[i];
      rw.size[rt] = a;
      rw.cmn[rt] = jb.cmin[a];
      rw.cmx[rt] = jb.cmax[a];
    } else {
      rw.size[rt] = 0;
      rw.cmn[rt] = 0xFFFFFFFFu;
      rw.cmx[rt] = 0;
    }
    load_signs<W>(sg_rows, n_rows, i, i < jb.row_end, h, rw.sg[rt]);
  }
  uint32_t skip = jb.first;
  uint32_t j = jb.c0;
  while (j < jb.c1) {
    const uint32_t c = rfl(size_cols[j]);
    const uint32_t g1 =
        min(max(jb.col_base + rfl(jb.sstart[c + 1]), j + 1), jb.c1);  // advances
    bool any_ok = false;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const bool in_band = c >= rw.cmn[rt] && c <= rw.cmx[rt];
      int32_t sl = 0;
      if (in_band) sl = (COS && jb.cosine) ? cosine_slack(rw.size[rt], c, jb.p, jb.q)
                                           : jb.slack[rw.size[rt] + c];
      const int32_t t = K - 2 * sl;
      rw.thr[rt] = in_band ? (float)t : kNever;
      rw.thr_bits[rt] = !in_band ? __float_as_int(kNever)
                        : t > 0  ? __float_as_int((float)t)
                                 : INT32_MIN;
      any_ok |= in_band;
    }
    if (__ballot(any_ok)) {
      if (!sweep_mfma<W, RT>(sg_cols, n_cols, rw, j, g1, jb.diag, skip, sink)) return false;
    }
    skip = 0;
    j = g1;
  }
  // the tile's staged pairs go out before the next tile
  return flush(sink);
}

template <int W, int RT, bool COS>
__global__ __launch_bounds__(kBlock) void k_filter_mfma(
    const uint4 *__restrict__ sg_rows, const uint4 *__restrict__ sg_cols,
    const uint32_t *__restrict__ size_rows, const uint32_t *__restrict__ size_cols,
    const uint32_t *__restrict__ sstart_cols, const uint32_t *__restrict__ tables,
    const TaskDesc *__restrict__ tasks, const RowBlock *__restrict__ blocks,
    const uint32_t *__restrict__ tile_block, uint2 *__restrict__ queue,
    JoinCounters *__restrict__ ctr, const Resume *__restrict__ resume_in,
    Resume *__restrict__ resume_out, FilterConfig cfg) {
  __shared__ uint2 stage[kBlock / 64][kStage];
  Sink sink;
  sink_init(sink, queue, ctr, cfg, stage[threadIdx.x >> 6]);
  persistent(tables, tasks, blocks, tile_block, sstart_cols, ctr, resume_in, resume_out, cfg,
             sink, [&](const TileJob &jb) {
               return run_tile_mfma<W, RT, COS>(sg_rows, sg_cols, cfg.n_rows, cfg.n_cols,
                                                size_rows, size_cols, jb, sink);
             });
}

template <int W, int R, int U, bool COS>
hipError_t launch_shape(dim3 grid, hipStream_t st, const FilterArgs &a) {
  hipLaunchKernelGGL((k_filter<W, R, U, COS>), grid, dim3(kBlock), 0, st, a.bm_rows, a.bm_cols,
                     a.size_rows, a.size_cols, a.sstart_cols, a.tables, a.tasks, a.blocks,
                     a.tile_block, a.queue, a.ctr, a.resume_in, a.resume_out, a.cfg);
  return hipGetLastError();
}

template <int W, int RT, bool COS>
hipError_t launch_mfma(dim3 grid, hipStream_t st, const FilterArgs &a) {
  hipLaunchKernelGGL((k_filter_mfma<W, RT, COS>), grid, dim3(kBlock), 0, st, a.sg_rows,
                     a.sg_cols, a.size_rows, a.size_cols, a.sstart_cols, a.tables, a.tasks,
                     a.blocks, a.tile_block, a.queue, a.ctr, a.resume_in, a.resume_out, a.cfg);
  return hipGetLastError();
}

// Vector-ALU kernels: (padded words, rows per lane, columns per step)
#define SSJ_FILTER_SHAPES(X) \
  X(1, 4, 4)                 \
  X(2, 2, 4)                 \
  X(3, 2, 2)                 \
  X(4, 2, 2)                 \
  X(5, 1, 1)                 \
  X(6, 1, 1)                 \
  X(7, 1, 1)                 \
  X(8, 1, 1)                 \
  X(10, 1, 1)                \
  X(12, 1, 1)                \
  X(16, 1, 1)                \
  X(20, 1, 1)                \
  X(24, 1, 1)                \
  X(32, 1, 1)                \
  X(40, 1, 1)                \
  X(48, 1, 1)                \
  X(64, 1, 1)

// Matrix-core kernels: (words, row tiles of 32 per wave).  At b = 64 six row
// tiles (three waves per SIMD) beat four (four waves per SIMD): a column
// step's loads, loop control and tests serve six products instead of four.
// At b = 128 four row tiles (three waves per SIMD) and at b = 256 five (two
// waves per SIMD) are the most the registers allow at that occupancy; six,
// at one wave fewer per SIMD, were slower.  At b = 512 and 1024 a column step streams b/2 bytes of sign planes per
// column, shared by the 32 RT rows of the wave: four and two row tiles
// (one wave per SIMD, the register file's other half holding rows and
// column buffers) keep that stream within what L2 delivers, and beat the
// vector ALUs by 3.2x and 1.8x.  b = 2048 stays on the vector ALUs: its
// ring of column buffers alone would fill the registers.
#define SSJ_MFMA_SHAPES(X) \
  X(1, 6)                  \
  X(2, 4)                  \
  X(4, 5)                  \
  X(8, 4)                  \
  X(16, 2)

}  // namespace

uint32_t filter_padded_words(uint32_t words) {
#define X(w, r, u) \
  if (words <= (w)) return (w);
  SSJ_FILTER_SHAPES(X)
#undef X
  return 0;
}

FilterShape filter_shape(uint32_t padded_words, bool mfma) {
  FilterShape s{0, 0, false};
#define X(w, r, u)           \
  if (padded_words == (w)) { \
    s.words = (w);           \
    s.rows = 64 * (r);       \
  }
  SSJ_FILTER_SHAPES(X)
#undef X
  if (mfma) {
#define X(w, rt)                           \
  if (padded_words == (w)) {               \
    s.rows = 32 * (rt);                    \
    s.mfma = true;                         \
  }
    SSJ_MFMA_SHAPES(X)
#undef X
  }
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
  if (a.sg_rows || a.sg_cols) {
    if (!a.sg_rows || !a.sg_cols) return hipErrorInvalidValue;
#define X(w, rt)                                                \
  if (padded_words == (w))                                      \
    return cosine ? launch_mfma<w, rt, true>(grid, st, a)       \
                  : launch_mfma<w, rt, false>(grid, st, a);
    SSJ_MFMA_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
  }
#define X(w, r, u)                                              \
  if (padded_words == (w))                                      \
    return cosine ? launch_shape<w, r, u, true>(grid, st, a)    \
                  : launch_shape<w, r, u, false>(grid, st, a);
  SSJ_FILTER_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace ssj
