// Exact verification of the bitmap filter's survivors (the verify step the
// paper's GPU algorithm leaves to the host, Alg. 8, done here on the GPU).
//
// Each queue entry (i, j) names a row and a column (global size-order
// indices of the row and column spaces); the sets are the caller's CSR sets
// perm[i] of side side_of[i] and perm[j] of side side_of[j], and the task is
// the one of the row's side.  The overlap o = |r n s| comes from one sorted merge
// that stops as soon as even matching every remaining token could not reach
// omin(|r|, |s|), the least overlap that meets the task's threshold
// (Table 1, integer form).  A qualifying pair is written as a 64-bit key
// (task, caller i, caller j), (min, max) for a self-join task and (r, s) for
// an R-S task, so that one radix sort orders the results of every task.
//
// Before the merge, a survivor can be tested once more with wider bitmaps
// of both sets (the cascade width, the widest a call has built): the bound
// of Theorem 1 holds at any width, and a wider one prunes most of the false
// survivors of a narrow class for a few dozen operations.  Pairs of sets too
// large for that width (its bits saturate) are tested again at the wide
// width, 4096 bits, when both sets have wide bitmaps.
//
// Each wave packs the real entries of its windows of the queue (the
// filter's chunks end in sentinels) so that every lane verifies a survivor;
// results are appended with one atomic per wave and round (ballot + lane
// rank).
#include <atomic>

#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr int kWin = 8;  // tokens per merge window

// Load tokens [at, at + kWin) of a set of n tokens; slots past the end are
// marked invalid.  The loads are independent, so a refill costs one round trip.
__host__ __device__ __forceinline__ void load_window(const uint32_t *__restrict__ t, uint32_t n,
                                            uint32_t at, uint32_t (&w)[kWin]) {
#pragma unroll
  for (int k = 0; k < kWin; ++k) w[k] = at + k < n ? t[at + k] : 0u;
}

// |r n s| >= need for two strictly increasing token lists, by a windowed
// merge: count the common tokens of the current windows, then drop the
// window whose last token is smaller (both when equal).  A common token sits
// in both current windows at some step and leaves with the dropped window,
// so it is counted once.  Stops as soon as the count reaches need, or the
// tokens left cannot reach it.
__host__ __device__ __forceinline__ bool overlap_reaches(const uint32_t *__restrict__ rp, uint32_t a,
                                                const uint32_t *__restrict__ sp, uint32_t c,
                                                uint32_t need) {
  uint32_t ia = 0, ic = 0, o = 0;
  uint32_t rw[kWin], sw[kWin];
  load_window(rp, a, 0, rw);
  load_window(sp, c, 0, sw);
  while (ia < a && ic < c) {
    if (o >= need) return true;
    if (o + min(a - ia, c - ic) < need) return false;
    const uint32_t nr = min(a - ia, (uint32_t)kWin), ns = min(c - ic, (uint32_t)kWin);
#pragma unroll
    for (int x = 0; x < kWin; ++x)
#pragma unroll
      for (int y = 0; y < kWin; ++y)
        o += ((uint32_t)x < nr && (uint32_t)y < ns && rw[x] == sw[y]) ? 1u : 0u;
    // last valid token of each window
    uint32_t rmax = rw[0], smax = sw[0];
#pragma unroll
    for (int k = 1; k < kWin; ++k) {
      if ((uint32_t)k < nr) rmax = rw[k];
      if ((uint32_t)k < ns) smax = sw[k];
    }
    if (rmax <= smax) {
      ia += nr;
      load_window(rp, a, ia, rw);
    }
    if (smax <= rmax) {
      ic += ns;
      load_window(sp, c, ic, sw);
    }
  }
  return o >= need;
}

// |r n s| with the whole wave, for one pair of long sets (the same on every
// lane).  Lane l takes r's tokens [a l / 64, a (l + 1) / 64) and counts
// those that s holds.  s is cut by 64 splitters s[c j / 64], one load per
// lane; a lane finds the last splitter not above its first token by a
// binary search over the lanes' splitters (six shuffles) and merges its
// tokens with s from there.  Tokens of s before that splitter are smaller
// than every token of the lane's, so each token of r is counted exactly
// when s holds it.  About four memory round trips, against one per eight
// tokens for a lane's own merge.
__device__ __forceinline__ uint32_t wave_overlap(const uint32_t *__restrict__ rp, uint32_t a,
                                                 const uint32_t *__restrict__ sp, uint32_t c) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t lo = (uint32_t)(((uint64_t)a * lane) >> 6);
  const uint32_t hi = (uint32_t)(((uint64_t)a * (lane + 1)) >> 6);
  const uint32_t sj = (uint32_t)(((uint64_t)c * lane) >> 6);  // < c
  const uint32_t sv = sp[sj];
  const bool has = lo < hi;
  const uint32_t first = has ? rp[lo] : 0u;
  int j = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const uint32_t cand = (uint32_t)__shfl((int)sv, j + step, 64);
    if (cand <= first) j += step;
  }
  const uint32_t from = (uint32_t)(((uint64_t)c * (uint32_t)j) >> 6);
  uint32_t o = 0;
  if (has) {
    const uint32_t na = hi - lo, nc = c - from;
    const uint32_t *__restrict__ r = rp + lo, *__restrict__ t = sp + from;
    uint32_t ia = 0, ic = 0;
    uint32_t rw[kWin], sw[kWin];
    load_window(r, na, 0, rw);
    load_window(t, nc, 0, sw);
    while (ia < na && ic < nc) {
      const uint32_t nr = min(na - ia, (uint32_t)kWin), ns = min(nc - ic, (uint32_t)kWin);
#pragma unroll
      for (int x = 0; x < kWin; ++x)
#pragma unroll
        for (int y = 0; y < kWin; ++y)
          o += ((uint32_t)x < nr && (uint32_t)y < ns && rw[x] == sw[y]) ? 1u : 0u;
      uint32_t rmax = rw[0], smax = sw[0];
#pragma unroll
      for (int k = 1; k < kWin; ++k) {
        if ((uint32_t)k < nr) rmax = rw[k];
        if ((uint32_t)k < ns) smax = sw[k];
      }
      if (rmax <= smax) {
        ia += nr;
        load_window(r, na, ia, rw);
      }
      if (smax <= rmax) {
        ic += ns;
        load_window(t, nc, ic, sw);
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) o += (uint32_t)__shfl_xor((int)o, d, 64);
  return o;
}

// Hamming distance of two bitmaps of W 64-bit words (W even: both start on
// a 16-byte boundary), every load issued before the first popcount so that
// the test costs one round trip.
template <int W>
__device__ __forceinline__ uint32_t distance(const uint64_t *__restrict__ x,
                                             const uint64_t *__restrict__ y) {
  static_assert(W % 2 == 0, "pairs of words per 16-byte load");
  const uint4 *a = reinterpret_cast<const uint4 *>(x), *b = reinterpret_cast<const uint4 *>(y);
  uint4 p[W / 2], q[W / 2];
#pragma unroll
  for (int k = 0; k < W / 2; ++k) {
    p[k] = a[k];
    q[k] = b[k];
  }
  uint32_t h = 0;
#pragma unroll
  for (int k = 0; k < W / 2; ++k)
    h += (uint32_t)__popc(p[k].x ^ q[k].x) + (uint32_t)__popc(p[k].y ^ q[k].y) +
         (uint32_t)__popc(p[k].z ^ q[k].z) + (uint32_t)__popc(p[k].w ^ q[k].w);
  return h;
}

// The wide test's distance, kWideWords words in batches of 8.
__device__ __forceinline__ uint32_t wide_distance(const uint64_t *__restrict__ x,
                                                  const uint64_t *__restrict__ y) {
  uint32_t h = 0;
#pragma unroll 1
  for (uint32_t k = 0; k < kWideWords; k += 8) h += distance<8>(x + k, y + k);
  return h;
}

// Pairs whose sizes sum to more than kLongMerge, and that pass the cascade
// test, are merged by a whole wave (wave_overlap) in a second launch: a
// lane's own merge takes a memory round trip per eight tokens, and one long
// true pair would hold its whole round that long.
constexpr uint32_t kLongMerge = 128;

// Result keys a verification wave stages in LDS.
constexpr uint32_t kWaveResults = 256;

struct VerifyArgs {
  VerifySpace rows, cols;
  const uint32_t *side_task;
  const TaskDesc *tasks;
  const uint32_t *tables;
  int ib, jb;
  uint32_t survivors_only;
  uint2 *longq;  // the deferred long pairs (capacity: the queue's), or NULL
};

// What verify_entry reads of a call's one task (ONE): its descriptor, the
// CSR of its row and column sides and their wide ranges, read once per
// wave.
struct OneTask {
  TaskDesc td;
  const uint64_t *r_off, *c_off;
  const uint32_t *r_tok, *c_tok;
  uint32_t r_wlo, c_wlo, r_wslot, c_wslot;
};

__device__ __forceinline__ OneTask one_task(const VerifyArgs &va) {
  OneTask one{};
  one.td = va.tasks[0];
  const SideDesc &dr = va.rows.sides[one.td.row_side], &dc = va.cols.sides[one.td.col_side];
  one.r_off = dr.offsets;
  one.r_tok = dr.tokens;
  one.c_off = dc.offsets;
  one.c_tok = dc.tokens;
  if (va.rows.bmw) {
    one.r_wlo = va.rows.wide_lo[one.td.row_side];
    one.c_wlo = va.cols.wide_lo[one.td.col_side];
    one.r_wslot = va.rows.wide_slot[one.td.row_side];
    one.c_wslot = va.cols.wide_slot[one.td.col_side];
  }
  return one;
}

// Verify one survivor (row x, column y of the two spaces): its result key,
// or false.  Sizes, the task's least overlap and the cascade bitmaps (W2
// words per set, 0: no cascade) come from arrays indexed by the queue entry
// itself, so the false survivors that the wider bitmaps reject (most of
// them) never touch the caller's offsets or tokens.  Every load that needs
// only (x, y) -- sides, positions, sizes, cascade bitmaps -- is issued
// first, so that a survivor's chain of dependent round trips before its
// merge is short.  ONE: the call has one task, whose descriptor, sides and
// wide ranges are uniform and come from `one`.
// Result key of a qualifying pair: (task, caller i, caller j), (min, max)
// for a self-join task.
__device__ __forceinline__ unsigned long long result_key(uint32_t px, uint32_t py,
                                                         const TaskDesc &td, uint32_t task,
                                                         int ib, int jb) {
  uint32_t ki = px, kj = py;
  if (td.self && kj < ki) {
    const uint32_t t = ki;
    ki = kj;
    kj = t;
  }
  unsigned long long key = ((unsigned long long)ki << jb) | kj;
  if (ib + jb < 64) key |= (unsigned long long)task << (ib + jb);
  return key;
}

template <int W2, bool ONE>
__device__ __forceinline__ bool verify_entry(uint32_t x, uint32_t y, const VerifyArgs &va,
                                             const OneTask &one, bool &defer,
                                             unsigned long long &key) {
  const VerifySpace &rows = va.rows, &cols = va.cols;
  const uint32_t sr = ONE ? 0u : rows.side_of[x], sc = ONE ? 0u : cols.side_of[y];
  const uint32_t px = rows.perm[x], py = cols.perm[y];
  const uint32_t a = rows.sizes[x], c = cols.sizes[y];
  uint32_t h2 = 0;
  if (W2) h2 = distance<W2 ? W2 : 2>(rows.bm2 + (size_t)x * W2, cols.bm2 + (size_t)y * W2);
  const uint32_t task = ONE ? 0u : va.side_task[sr];
  const TaskDesc td = ONE ? one.td : va.tasks[task];
  // with one task the CSR offsets come with the least overlap (a few bytes
  // per survivor); otherwise only pairs that pass the bitmap tests read them
  uint64_t r0 = 0, s0 = 0;
  if (ONE) {
    r0 = one.r_off[px];
    s0 = one.c_off[py];
  }
  bool hit = true;
  if (!va.survivors_only) {
    // the table entry is read for every function (Cosine's one unused
    // entry for Cosine) so that its load is not held back by the branch
    const bool cosine = td.sim == SSJ_SIM_COSINE;
    const uint32_t t_need = va.tables[td.omin_off + (cosine ? 0u : a + c)];
    const uint32_t need = cosine ? cosine_omin(a, c, td.p, td.q) : t_need;
    const int64_t slack = (int64_t)a + c - 2 * (int64_t)need;
    // second bitmap test at the cascade width (Theorem 1 holds at every
    // width): most false survivors of a narrow class end here
    hit = a != 0 && c != 0 && slack >= 0 && (int64_t)h2 <= slack;
    // and at the wide width when both sets have wide bitmaps (sets too
    // large for the cascade width, whose bits saturate)
    if (hit && rows.bmw) {
      const uint32_t lr = ONE ? one.r_wlo : rows.wide_lo[sr];
      const uint32_t lc = ONE ? one.c_wlo : cols.wide_lo[sc];
      if (x >= lr && y >= lc) {
        const uint32_t wr = ONE ? one.r_wslot : rows.wide_slot[sr];
        const uint32_t wc = ONE ? one.c_wslot : cols.wide_slot[sc];
        hit = (int64_t)wide_distance(rows.bmw + (size_t)(wr + (x - lr)) * kWideWords,
                                     cols.bmw + (size_t)(wc + (y - lc)) * kWideWords) <= slack;
      }
    }
    // pairs of long sets go to the wave-cooperative merge
    if (hit && va.longq && a + c > kLongMerge) {
      defer = true;
      return false;
    }
    if (hit) {
      if (!ONE) {
        r0 = rows.sides[sr].offsets[px];
        s0 = cols.sides[sc].offsets[py];
      }
      const uint32_t *rt = ONE ? one.r_tok : rows.sides[sr].tokens;
      const uint32_t *ct = ONE ? one.c_tok : cols.sides[sc].tokens;
      hit = overlap_reaches(rt + r0, a, ct + s0, c, need);
    }
  }
  if (hit) key = result_key(px, py, td, task, va.ib, va.jb);
  return hit;
}

// The queue holds the filter waves' chunks, whose unused ends are
// sentinels.  Wave w reads the queue's 64-entry windows w, w + W, w + 2W, ...
// (W waves; a run of full chunks is spread over many waves), packs the real
// entries into an LDS list and verifies them 64 at a time, so that every
// lane of a verification round has a survivor (the round's length is that
// of its longest merge).
template <int W2, bool ONE>
__global__ __launch_bounds__(kBlock) void k_verify(const uint2 *__restrict__ queue,
                                                   unsigned long long cap, VerifyArgs va,
                                                   unsigned long long *__restrict__ results,
                                                   unsigned long long results_cap,
                                                   JoinCounters *__restrict__ ctr) {
  __shared__ uint2 pend[kBlock / 64][128];
  // result keys, staged per wave and written with one reservation per
  // workgroup at the end (or per wave when a wave's list fills): one
  // same-address atomic per workgroup instead of one per round
  __shared__ unsigned long long rkeys[kBlock / 64][kWaveResults];
  __shared__ unsigned long long rbase[kBlock / 64];
  __shared__ uint32_t block_surv;
  uint2 *buf = pend[threadIdx.x >> 6];
  unsigned long long *rk = rkeys[threadIdx.x >> 6];
  uint32_t rfill = 0;
  const uint32_t lane = threadIdx.x & 63;
  if (threadIdx.x == 0) block_surv = 0;
  unsigned long long count = ctr->queue_count;
  if (count > cap) count = cap;
  const unsigned long long windows = (count + 63) / 64;
  const unsigned long long n_waves = (unsigned long long)gridDim.x * (kBlock / 64);
  const unsigned long long wave = (unsigned long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  uint32_t fill = 0, surv = 0;
  const OneTask one = ONE ? one_task(va) : OneTask{};
  auto round = [&](uint2 qe, bool ok) {
    unsigned long long key = 0;
    bool defer = false;
    const bool hit = ok && verify_entry<W2, ONE>(qe.x, qe.y, va, one, defer, key);
    const unsigned long long dm = __ballot(defer);
    if (dm) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&ctr->long_count, (unsigned long long)__popcll(dm));
      base = __shfl(base, 0, 64);
      if (defer) {
        const unsigned long long pos = base + (unsigned long long)__popcll(dm & __lanemask_lt());
        if (pos < cap) va.longq[pos] = qe;
      }
    }
    const unsigned long long m = __ballot(hit);
    if (m) {
      const uint32_t n = (uint32_t)__popcll(m);
      if (rfill + n > kWaveResults) {
        // this wave's list is full: write it out on its own
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&ctr->results, (unsigned long long)rfill);
        base = __shfl(base, 0, 64);
        for (uint32_t x = lane; x < rfill; x += 64)
          if (base + x < results_cap) results[base + x] = rk[x];
        __builtin_amdgcn_wave_barrier();
        rfill = 0;
      }
      if (hit) rk[rfill + (uint32_t)__popcll(m & __lanemask_lt())] = key;
      rfill += n;
    }
  };
  // the next window's entry is loaded before the current one is used
  auto entry = [&](unsigned long long w) {
    const unsigned long long e = w * 64 + lane;
    return w < windows && e < count ? queue[e] : make_uint2(kSentinel, kSentinel);
  };
  uint2 next = entry(wave);
  for (unsigned long long w = wave; w < windows; w += n_waves) {
    const uint2 qe = next;
    next = entry(w + n_waves);
    const bool valid = qe.x < va.rows.n && qe.y < va.cols.n;
    const unsigned long long m = __ballot(valid);
    if (valid) buf[fill + (uint32_t)__popcll(m & __lanemask_lt())] = qe;
    fill += (uint32_t)__popcll(m);  // < 128: at most 63 were left over
    if (fill >= 64) {
      __builtin_amdgcn_wave_barrier();
      const uint2 mine = buf[lane], carry = buf[64 + lane];
      __builtin_amdgcn_wave_barrier();
      fill -= 64;
      if (lane < fill) buf[lane] = carry;
      __builtin_amdgcn_wave_barrier();
      ++surv;
      round(mine, true);
    }
  }
  if (fill) {
    __builtin_amdgcn_wave_barrier();
    const uint2 mine = buf[lane];
    surv += lane < fill ? 1u : 0u;
    round(mine, lane < fill);
  }
  // survivors seen and the staged results: one atomic each per workgroup
  // (same-address atomics from every XCD are served one at a time)
  const uint32_t wv = threadIdx.x >> 6;
  uint32_t s = surv;
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  __syncthreads();  // block_surv was cleared at the start
  if (lane == 0) {
    if (s) atomicAdd(&block_surv, s);
    rbase[wv] = rfill;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (block_surv) atomicAdd(&ctr->survivors, (unsigned long long)block_surv);
    unsigned long long total = 0;
    for (uint32_t k = 0; k < kBlock / 64; ++k) total += rbase[k];
    unsigned long long at = total ? atomicAdd(&ctr->results, total) : 0ull;
    for (uint32_t k = 0; k < kBlock / 64; ++k) {
      const unsigned long long nk = rbase[k];
      rbase[k] = at;
      at += nk;
    }
  }
  __syncthreads();
  const unsigned long long base = rbase[wv];
  for (uint32_t x = lane; x < rfill; x += 64)
    if (base + x < results_cap) results[base + x] = rk[x];
}

// The deferred long pairs (their bitmap tests passed).  A few of them (up to
// kLaneMode per wave): one wave per pair, the pairs dealt to the waves in
// turn, so that each takes a few round trips.  Many: a lane per pair, 64 at
// a time, which takes longer per pair but costs the wave less (a wave's
// merge of one pair is about eight times the work of a lane's).
constexpr uint32_t kLaneMode = 8;

template <bool ONE>
__global__ __launch_bounds__(kBlock) void k_verify_long(unsigned long long cap, VerifyArgs va,
                                                        unsigned long long *__restrict__ results,
                                                        unsigned long long results_cap,
                                                        JoinCounters *__restrict__ ctr) {
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long count = ctr->long_count;
  if (count > cap) count = cap;
  const unsigned long long n_waves = (unsigned long long)gridDim.x * (kBlock / 64);
  const unsigned long long wave = (unsigned long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const OneTask one = ONE ? one_task(va) : OneTask{};
  const VerifySpace &rows = va.rows, &cols = va.cols;
  if (count >= (unsigned long long)kLaneMode * n_waves) {
    for (unsigned long long e0 = wave * 64; e0 < count; e0 += n_waves * 64) {
      const unsigned long long e = e0 + lane;
      bool hit = false;
      unsigned long long key = 0;
      if (e < count) {
        const uint2 qe = va.longq[e];
        const uint32_t x = qe.x, y = qe.y;
        const uint32_t sr = ONE ? 0u : rows.side_of[x], sc = ONE ? 0u : cols.side_of[y];
        const uint32_t px = rows.perm[x], py = cols.perm[y];
        const uint32_t a = rows.sizes[x], c = cols.sizes[y];
        const uint32_t task = ONE ? 0u : va.side_task[sr];
        const TaskDesc td = ONE ? one.td : va.tasks[task];
        const uint32_t need = td.sim == SSJ_SIM_COSINE ? cosine_omin(a, c, td.p, td.q)
                                                       : va.tables[td.omin_off + a + c];
        const uint64_t r0 = ONE ? one.r_off[px] : rows.sides[sr].offsets[px];
        const uint64_t s0 = ONE ? one.c_off[py] : cols.sides[sc].offsets[py];
        const uint32_t *rt = ONE ? one.r_tok : rows.sides[sr].tokens;
        const uint32_t *ct = ONE ? one.c_tok : cols.sides[sc].tokens;
        hit = overlap_reaches(rt + r0, a, ct + s0, c, need);
        if (hit) key = result_key(px, py, td, task, va.ib, va.jb);
      }
      const unsigned long long m = __ballot(hit);
      if (m) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&ctr->results, (unsigned long long)__popcll(m));
        base = __shfl(base, 0, 64);
        if (hit) {
          const unsigned long long pos = base + (unsigned long long)__popcll(m & __lanemask_lt());
          if (pos < results_cap) results[pos] = key;
        }
      }
    }
    return;
  }
  for (unsigned long long e = wave; e < count; e += n_waves) {
    const uint2 qe = va.longq[e];
    const uint32_t x = (uint32_t)__builtin_amdgcn_readfirstlane((int)qe.x);
    const uint32_t y = (uint32_t)__builtin_amdgcn_readfirstlane((int)qe.y);
    const uint32_t sr = ONE ? 0u : rows.side_of[x], sc = ONE ? 0u : cols.side_of[y];
    const uint32_t px = rows.perm[x], py = cols.perm[y];
    const uint32_t a = rows.sizes[x], c = cols.sizes[y];
    const uint32_t task = ONE ? 0u : va.side_task[sr];
    const TaskDesc td = ONE ? one.td : va.tasks[task];
    const uint32_t need = td.sim == SSJ_SIM_COSINE ? cosine_omin(a, c, td.p, td.q)
                                                   : va.tables[td.omin_off + a + c];
    const uint64_t r0 = ONE ? one.r_off[px] : rows.sides[sr].offsets[px];
    const uint64_t s0 = ONE ? one.c_off[py] : cols.sides[sc].offsets[py];
    const uint32_t *rt = ONE ? one.r_tok : rows.sides[sr].tokens;
    const uint32_t *ct = ONE ? one.c_tok : cols.sides[sc].tokens;
    const uint32_t o = wave_overlap(rt + r0, a, ct + s0, c);
    if (o >= need && lane == 0) {
      const unsigned long long pos = atomicAdd(&ctr->results, 1ull);
      if (pos < results_cap) results[pos] = result_key(px, py, td, task, va.ib, va.jb);
    }
  }
}

// Sorted keys -> pairs, and the first result of every task: the key at x
// opens tasks (task(x-1), task(x)]; the last key closes the rest.
__global__ __launch_bounds__(kBlock) void k_split_results(
    const unsigned long long *__restrict__ keys, uint64_t n, int ib, int jb, uint32_t n_tasks,
    ssj_pair *__restrict__ out, uint64_t *__restrict__ task_start) {
  const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x >= n) return;
  const int tshift = ib + jb;
  auto task_of = [&](unsigned long long k) -> uint32_t {
    return tshift < 64 ? (uint32_t)(k >> tshift) : 0u;
  };
  const unsigned long long k = keys[x];
  const uint32_t t = task_of(k);
  ssj_pair pr;
  pr.i = (uint32_t)((k >> jb) & ((1ull << ib) - 1));
  pr.j = (uint32_t)(k & ((1ull << jb) - 1));
  out[x] = pr;
  const uint32_t t_prev = x ? task_of(keys[x - 1]) : 0u;
  for (uint32_t u = x ? t_prev + 1 : 0u; u <= t && u <= n_tasks; ++u) task_start[u] = x;
  if (x + 1 == n)
    for (uint32_t u = t + 1; u <= n_tasks; ++u) task_start[u] = n;
}

}  // namespace

// Blocks of a k_verify instance resident at once on the current device
// (queried once per instance and device).  The grid strides over the queue
// with a fixed share per lane: blocks beyond what the compute units hold
// would start only when the first ones end, and the launch would take two
// rounds of its latency-bound loop instead of one.
constexpr int kVerifyDevices = 64;

template <int W2, bool ONE>
static int verify_grid_blocks() {
  static std::atomic<int> cached[kVerifyDevices];
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (dev >= 0 && dev < kVerifyDevices) {
    const int c = cached[dev].load(std::memory_order_relaxed);
    if (c) return c;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_verify<W2, ONE>, kBlock, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  if (dev >= 0 && dev < kVerifyDevices) cached[dev].store(cus * per_cu, std::memory_order_relaxed);
  return cus * per_cu;
}

template <bool ONE>
static int verify_long_grid_blocks() {
  static std::atomic<int> cached[kVerifyDevices];
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (dev >= 0 && dev < kVerifyDevices) {
    const int c = cached[dev].load(std::memory_order_relaxed);
    if (c) return c;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_verify_long<ONE>, kBlock, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  if (dev >= 0 && dev < kVerifyDevices) cached[dev].store(cus * per_cu, std::memory_order_relaxed);
  return cus * per_cu;
}

template <int W2, bool ONE>
static void launch_verify_as(const uint2 *queue, unsigned long long cap, const VerifyArgs &va,
                             unsigned long long *results, unsigned long long results_cap,
                             JoinCounters *ctr, hipStream_t st) {
  hipLaunchKernelGGL((k_verify<W2, ONE>), dim3(verify_grid_blocks<W2, ONE>()), dim3(kBlock), 0,
                     st, queue, cap, va, results, results_cap, ctr);
  if (va.longq)
    hipLaunchKernelGGL((k_verify_long<ONE>), dim3(verify_long_grid_blocks<ONE>()), dim3(kBlock),
                       0, st, cap, va, results, results_cap, ctr);
}

hipError_t launch_verify(const uint2 *queue, uint2 *longq, unsigned long long cap,
                         VerifySpace rows, VerifySpace cols, const uint32_t *side_task,
                         const TaskDesc *tasks, uint32_t n_tasks, const uint32_t *tables, int ib,
                         int jb, uint32_t survivors_only, uint32_t w2,
                         unsigned long long *results, unsigned long long results_cap,
                         JoinCounters *ctr, hipStream_t st) {
  if ((rows.bm2 == nullptr) != (cols.bm2 == nullptr) || (rows.bm2 && !w2))
    return hipErrorInvalidValue;
  if ((rows.bmw == nullptr) != (cols.bmw == nullptr)) return hipErrorInvalidValue;
  if (!rows.bm2) w2 = 0;
  if (w2 != 0 && w2 != 2 && w2 != 4 && w2 != 8) return hipErrorInvalidValue;
  if (n_tasks == 0) return hipErrorInvalidValue;
  // only pairs that passed a cascade test are deferred: they are nearly all
  // true pairs, which a lane's merge cannot leave early; without a cascade
  // most survivors are false, and a lane's merge rejects them in a few
  // windows
  const VerifyArgs va{rows, cols, side_task, tasks, tables, ib, jb, survivors_only,
                      survivors_only || !rows.bm2 ? nullptr : longq};
  const bool one = n_tasks == 1;
  switch (w2 * 2 + (one ? 1 : 0)) {
    case 0: launch_verify_as<0, false>(queue, cap, va, results, results_cap, ctr, st); break;
    case 1: launch_verify_as<0, true>(queue, cap, va, results, results_cap, ctr, st); break;
    case 4: launch_verify_as<2, false>(queue, cap, va, results, results_cap, ctr, st); break;
    case 5: launch_verify_as<2, true>(queue, cap, va, results, results_cap, ctr, st); break;
    case 8: launch_verify_as<4, false>(queue, cap, va, results, results_cap, ctr, st); break;
    case 9: launch_verify_as<4, true>(queue, cap, va, results, results_cap, ctr, st); break;
    case 16: launch_verify_as<8, false>(queue, cap, va, results, results_cap, ctr, st); break;
    default: launch_verify_as<8, true>(queue, cap, va, results, results_cap, ctr, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_split_results(const unsigned long long *keys, uint64_t n, int ib, int jb,
                                uint32_t n_tasks, ssj_pair *out, uint64_t *task_start,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (ib < 1 || jb < 1 || ib > 32 || jb > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_results, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, st, keys, n, ib, jb, n_tasks, out, task_start);
  return hipGetLastError();
}

}  // namespace ssj
