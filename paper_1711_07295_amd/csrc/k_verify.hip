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
// so it is counted once.  Stops as soon as the tokens left cannot reach need.
__host__ __device__ __forceinline__ bool overlap_reaches(const uint32_t *__restrict__ rp, uint32_t a,
                                                const uint32_t *__restrict__ sp, uint32_t c,
                                                uint32_t need) {
  uint32_t ia = 0, ic = 0, o = 0;
  uint32_t rw[kWin], sw[kWin];
  load_window(rp, a, 0, rw);
  load_window(sp, c, 0, sw);
  while (ia < a && ic < c) {
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

// Hamming distance of two bitmaps of w 64-bit words, two words per
// 16-byte load (both bitmaps start on a 16-byte boundary when w is even).
__device__ __forceinline__ uint32_t distance(const uint64_t *__restrict__ x,
                                             const uint64_t *__restrict__ y, uint32_t w) {
  uint32_t h = 0;
  if ((w & 1u) == 0) {
    const uint4 *a = reinterpret_cast<const uint4 *>(x), *b = reinterpret_cast<const uint4 *>(y);
    for (uint32_t k = 0; k < w / 2; ++k) {
      const uint4 p = a[k], q = b[k];
      h += (uint32_t)__popc(p.x ^ q.x) + (uint32_t)__popc(p.y ^ q.y) +
           (uint32_t)__popc(p.z ^ q.z) + (uint32_t)__popc(p.w ^ q.w);
    }
  } else {
    for (uint32_t k = 0; k < w; ++k) h += (uint32_t)__popcll(x[k] ^ y[k]);
  }
  return h;
}

// Verify one survivor (row x, column y of the two spaces): its result key,
// or false.  Sizes, the task's least overlap and the cascade bitmaps come
// from arrays indexed by the queue entry itself, so the false survivors
// that the wider bitmaps reject (most of them) never touch the caller's
// offsets or tokens.
__device__ __forceinline__ bool verify_entry(uint32_t x, uint32_t y, const VerifySpace &rows,
                                             const VerifySpace &cols,
                                             const uint32_t *__restrict__ side_task,
                                             const TaskDesc *__restrict__ tasks,
                                             const uint32_t *__restrict__ tables, int ib, int jb,
                                             uint32_t survivors_only, uint32_t w2,
                                             unsigned long long &key) {
  const uint32_t sr = rows.side_of[x], sc = cols.side_of[y];
  const uint32_t a = rows.sizes[x], c = cols.sizes[y];
  const uint32_t task = side_task[sr];
  const TaskDesc &td = tasks[task];
  bool hit = true;
  if (!survivors_only) {
    const uint32_t need = td.sim == SSJ_SIM_COSINE ? cosine_omin(a, c, td.p, td.q)
                                                   : tables[td.omin_off + a + c];
    const int64_t slack = (int64_t)a + c - 2 * (int64_t)need;
    // second bitmap test at the cascade width (Theorem 1 holds at every
    // width): most false survivors of a narrow class end here
    hit = a != 0 && c != 0 && slack >= 0;
    if (hit && rows.bm2)
      hit = (int64_t)distance(rows.bm2 + (size_t)x * w2, cols.bm2 + (size_t)y * w2, w2) <= slack;
    // and at the wide width when both sets have wide bitmaps (sets too
    // large for the cascade width, whose bits saturate)
    if (hit && rows.bmw) {
      const uint32_t lr = rows.wide_lo[sr], lc = cols.wide_lo[sc];
      if (x >= lr && y >= lc)
        hit = (int64_t)distance(rows.bmw + (size_t)(rows.wide_slot[sr] + (x - lr)) * kWideWords,
                                cols.bmw + (size_t)(cols.wide_slot[sc] + (y - lc)) * kWideWords,
                                kWideWords) <= slack;
    }
    if (hit) {
      const SideDesc &dr = rows.sides[sr], &dc = cols.sides[sc];
      const uint64_t r0 = dr.offsets[rows.perm[x]], s0 = dc.offsets[cols.perm[y]];
      hit = overlap_reaches(dr.tokens + r0, a, dc.tokens + s0, c, need);
    }
  }
  if (hit) {
    uint32_t ki = rows.perm[x], kj = cols.perm[y];
    if (td.self && kj < ki) {
      const uint32_t t = ki;
      ki = kj;
      kj = t;
    }
    key = ((unsigned long long)ki << jb) | kj;
    if (ib + jb < 64) key |= (unsigned long long)task << (ib + jb);
  }
  return hit;
}

// The queue holds the filter waves' chunks, whose unused ends are
// sentinels.  Wave w reads the queue's 64-entry windows w, w + W, w + 2W, ...
// (W waves; a run of full chunks is spread over many waves), packs the real
// entries into an LDS list and verifies them 64 at a time, so that every
// lane of a verification round has a survivor (the round's length is that
// of its longest merge).
__global__ __launch_bounds__(kBlock) void k_verify(
    const uint2 *__restrict__ queue, unsigned long long cap, VerifySpace rows, VerifySpace cols,
    const uint32_t *__restrict__ side_task, const TaskDesc *__restrict__ tasks,
    const uint32_t *__restrict__ tables, int ib, int jb, uint32_t survivors_only, uint32_t w2,
    unsigned long long *__restrict__ results, unsigned long long results_cap,
    JoinCounters *__restrict__ ctr) {
  __shared__ uint2 pend[kBlock / 64][128];
  uint2 *buf = pend[threadIdx.x >> 6];
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long count = ctr->queue_count;
  if (count > cap) count = cap;
  const unsigned long long windows = (count + 63) / 64;
  const unsigned long long n_waves = (unsigned long long)gridDim.x * (kBlock / 64);
  const unsigned long long wave = (unsigned long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  uint32_t fill = 0, surv = 0;
  auto round = [&](uint2 qe, bool ok) {
    unsigned long long key = 0;
    const bool hit = ok && verify_entry(qe.x, qe.y, rows, cols, side_task, tasks, tables, ib, jb,
                                        survivors_only, w2, key);
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
  };
  for (unsigned long long w = wave; w < windows; w += n_waves) {
    const unsigned long long e = w * 64 + lane;
    uint2 qe = make_uint2(kSentinel, kSentinel);
    if (e < count) qe = queue[e];
    const bool valid = qe.x < rows.n && qe.y < cols.n;
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
  // survivors seen, one atomic per wave
  uint32_t s = surv;
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0 && s) atomicAdd(&ctr->survivors, (unsigned long long)s);
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

// Blocks of k_verify resident at once on the current device.  The grid
// strides over the queue with a fixed share per lane: blocks beyond what
// the compute units hold would start only when the first ones end, and the
// launch would take two rounds of its latency-bound loop instead of one.
static int verify_grid_blocks() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_verify, kBlock, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  return cus * per_cu;
}

hipError_t launch_verify(const uint2 *queue, unsigned long long cap, VerifySpace rows,
                         VerifySpace cols, const uint32_t *side_task, const TaskDesc *tasks,
                         const uint32_t *tables, int ib, int jb, uint32_t survivors_only,
                         uint32_t w2, unsigned long long *results,
                         unsigned long long results_cap, JoinCounters *ctr, hipStream_t st) {
  if ((rows.bm2 == nullptr) != (cols.bm2 == nullptr) || (rows.bm2 && !w2))
    return hipErrorInvalidValue;
  if ((rows.bmw == nullptr) != (cols.bmw == nullptr)) return hipErrorInvalidValue;
  dim3 grid(verify_grid_blocks());
  hipLaunchKernelGGL(k_verify, grid, dim3(kBlock), 0, st, queue, cap, rows, cols, side_task,
                     tasks, tables, ib, jb, survivors_only, w2, results, results_cap,
                     ctr);
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
