// Exact verification of the bitmap filter's survivors (the verify step the
// paper's GPU algorithm leaves to the host, Alg. 8, done here on the GPU).
//
// Each queue entry (i, j) names a row and a column in size order; the
// sets are the caller's CSR sets perm_rows[i] and perm_cols[j].  The overlap
// o = |r n s| comes from one sorted merge that stops as soon as even
// matching every remaining token could not reach omin(|r| + |s|), the least
// overlap that meets the threshold (Table 1, integer form).  A qualifying
// pair is written as a 64-bit key of caller indices, (min, max) for the
// self-join and (r, s) for the R-S join.
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
    const uint2 *__restrict__ queue, unsigned long long cap,
    const uint64_t *__restrict__ off_rows, const uint32_t *__restrict__ tok_rows,
    const uint32_t *__restrict__ perm_rows, const uint64_t *__restrict__ off_cols,
    const uint32_t *__restrict__ tok_cols, const uint32_t *__restrict__ perm_cols,
    const uint32_t *__restrict__ omin, uint32_t n_rows, uint32_t n_cols, uint32_t self,
    uint32_t survivors_only,
    unsigned long long *__restrict__ results, unsigned long long results_cap,
    JoinCounters *__restrict__ ctr) {
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long count = ctr->queue_count;
  if (count > cap) count = cap;
  const unsigned long long stride = (unsigned long long)gridDim.x * kBlock;
  const unsigned long long start = (unsigned long long)blockIdx.x * kBlock + threadIdx.x;
  // every lane of a wave runs the same number of iterations
  const unsigned long long wave0 = start - lane;
  uint32_t surv = 0;
  for (unsigned long long e0 = wave0; e0 < count; e0 += stride) {
    const unsigned long long e = e0 + lane;
    bool hit = false;
    unsigned long long key = 0;
    if (e < count) {
      const uint2 qe = queue[e];
      if (qe.x < n_rows && qe.y < n_cols) {
        ++surv;
        const uint32_t x = perm_rows[qe.x], y = perm_cols[qe.y];
        const uint64_t r0 = off_rows[x], r1 = off_rows[x + 1];
        const uint64_t s0 = off_cols[y], s1 = off_cols[y + 1];
        const uint32_t a = (uint32_t)(r1 - r0), c = (uint32_t)(s1 - s0);
        if (survivors_only) {
          hit = true;
        } else {
          hit = a != 0 && c != 0 && overlap_reaches(tok_rows + r0, a, tok_cols + s0, c,
                                                   omin[a + c]);
        }
        if (hit) {
          if (self) {
            const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
            key = ((unsigned long long)lo << 32) | hi;
          } else {
            key = ((unsigned long long)x << 32) | y;
          }
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

}  // namespace

hipError_t launch_verify(const uint2 *queue, unsigned long long cap, const uint64_t *off_rows,
                         const uint32_t *tok_rows, const uint32_t *perm_rows,
                         const uint64_t *off_cols, const uint32_t *tok_cols,
                         const uint32_t *perm_cols, const uint32_t *omin, uint32_t n_rows,
                         uint32_t n_cols, uint32_t self,
                         uint32_t survivors_only, unsigned long long *results,
                         unsigned long long results_cap, JoinCounters *ctr, hipStream_t st) {
  dim3 grid(filter_grid_blocks());
  hipLaunchKernelGGL(k_verify, grid, dim3(kBlock), 0, st, queue, cap, off_rows, tok_rows,
                     perm_rows, off_cols, tok_cols, perm_cols, omin, n_rows, n_cols, self,
                     survivors_only,
                     results, results_cap, ctr);
  return hipGetLastError();
}

}  // namespace ssj
