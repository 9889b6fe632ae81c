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
          const uint32_t need = omin[a + c];
          const uint32_t *rp = tok_rows + r0;
          const uint32_t *sp = tok_cols + s0;
          uint32_t ia = 0, ic = 0, o = 0;
          uint32_t u = a ? rp[0] : 0, v = c ? sp[0] : 0;
          while (ia < a && ic < c) {
            const uint32_t rest = min(a - ia, c - ic);
            if (o + rest < need) break;
            if (u == v) {
              ++o;
              ++ia;
              ++ic;
              if (ia < a) u = rp[ia];
              if (ic < c) v = sp[ic];
            } else if (u < v) {
              ++ia;
              if (ia < a) u = rp[ia];
            } else {
              ++ic;
              if (ic < c) v = sp[ic];
            }
          }
          hit = a != 0 && c != 0 && o >= need;
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
