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
// Grid-stride over the queue, one survivor per lane; results are appended
// with one atomic per wave (ballot + lane rank).
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

__global__ __launch_bounds__(kBlock) void k_verify(
    const uint2 *__restrict__ queue, unsigned long long cap, VerifySpace rows, VerifySpace cols,
    const uint32_t *__restrict__ side_task, const TaskDesc *__restrict__ tasks,
    const uint32_t *__restrict__ tables, int ib, int jb, uint32_t survivors_only, uint32_t w2,
    unsigned long long *__restrict__ results, unsigned long long results_cap,
    JoinCounters *__restrict__ ctr) {
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long count = ctr->queue_count;
  if (count > cap) count = cap;
  const unsigned long long stride = (unsigned long long)gridDim.x * kBlock;
  const unsigned long long start = (unsigned long long)blockIdx.x * kBlock + threadIdx.x;
  // every lane of a wave runs the same number of iterations
  const unsigned long long wave0 = start - lane;
  const int tshift = ib + jb;
  uint32_t surv = 0;
  for (unsigned long long e0 = wave0; e0 < count; e0 += stride) {
    const unsigned long long e = e0 + lane;
    bool hit = false;
    unsigned long long key = 0;
    if (e < count) {
      const uint2 qe = queue[e];
      if (qe.x < rows.n && qe.y < cols.n) {
        ++surv;
        const uint32_t sr = rows.side_of[qe.x], sc = cols.side_of[qe.y];
        const SideDesc dr = rows.sides[sr];
        const SideDesc dc = cols.sides[sc];
        const uint32_t task = side_task[sr];
        const uint32_t x = rows.perm[qe.x], y = cols.perm[qe.y];
        const uint64_t r0 = dr.offsets[x], r1 = dr.offsets[x + 1];
        const uint64_t s0 = dc.offsets[y], s1 = dc.offsets[y + 1];
        const uint32_t a = (uint32_t)(r1 - r0), c = (uint32_t)(s1 - s0);
        if (survivors_only) {
          hit = true;
        } else {
          const TaskDesc &td = tasks[task];
          const uint32_t need = td.sim == SSJ_SIM_COSINE ? cosine_omin(a, c, td.p, td.q)
                                                         : tables[td.omin_off + a + c];
          // second bitmap test at the cascade width (Theorem 1 holds at
          // every width): most false survivors of a narrow class end here
          bool pass = true;
          if (rows.bm2) {
            const uint64_t *bx = rows.bm2 + (size_t)qe.x * w2;
            const uint64_t *by = cols.bm2 + (size_t)qe.y * w2;
            uint32_t h = 0;
            for (uint32_t w = 0; w < w2; ++w) h += (uint32_t)__popcll(bx[w] ^ by[w]);
            pass = (int64_t)h <= (int64_t)a + c - 2 * (int64_t)need;
          }
          // and at the wide width when both sets have wide bitmaps (sets too
          // large for the cascade width, whose bits saturate)
          if (pass && rows.bmw) {
            const uint32_t lr = rows.wide_lo[sr], lc = cols.wide_lo[sc];
            if (qe.x >= lr && qe.y >= lc) {
              const uint4 *bx = reinterpret_cast<const uint4 *>(
                  rows.bmw + (size_t)(rows.wide_slot[sr] + (qe.x - lr)) * kWideWords);
              const uint4 *by = reinterpret_cast<const uint4 *>(
                  cols.bmw + (size_t)(cols.wide_slot[sc] + (qe.y - lc)) * kWideWords);
              uint32_t h = 0;
              for (uint32_t w = 0; w < kWideWords / 2; ++w) {
                const uint4 p = bx[w], q = by[w];
                h += (uint32_t)__popc(p.x ^ q.x) + (uint32_t)__popc(p.y ^ q.y) +
                     (uint32_t)__popc(p.z ^ q.z) + (uint32_t)__popc(p.w ^ q.w);
              }
              pass = (int64_t)h <= (int64_t)a + c - 2 * (int64_t)need;
            }
          }
          hit = a != 0 && c != 0 && pass &&
                overlap_reaches(dr.tokens + r0, a, dc.tokens + s0, c, need);
        }
        if (hit) {
          uint32_t ki = x, kj = y;
          if (tasks[task].self && y < x) {
            ki = y;
            kj = x;
          }
          key = ((unsigned long long)ki << jb) | kj;
          if (tshift < 64) key |= (unsigned long long)task << tshift;
        }
      }
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
