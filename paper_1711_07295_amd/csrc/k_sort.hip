// Stable LSD radix sort of 64-bit keys (8-bit digits) and a device-wide
// exclusive scan.  Used for the size sort of the collections and for the
// final ordering of the result pairs.
//
// Per pass: (1) every workgroup counts the digits of its kTile keys,
// (2) the digit-major table of counts is scanned (by the scatter itself
// when there are few workgroups), (3) every workgroup
// ranks its keys stably -- wave by wave, 64 keys at a time, peers with
// the same digit found by eight ballots -- and scatters them.
#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr int kItems = 8;                 // keys per thread
constexpr int kTile = kBlock * kItems;    // keys per workgroup
constexpr int kWaves = kBlock / 64;
constexpr int kWaveKeys = kTile / kWaves; // contiguous keys per wave
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;
// Sort blocks up to which a pass's scatter sums the digit counts itself.
constexpr uint64_t kFoldBlocks = 64;

__device__ __forceinline__ uint32_t digit_of(unsigned long long k, int shift) {
  return (uint32_t)(k >> shift) & 0xFFu;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const unsigned long long *__restrict__ keys,
                                                       uint64_t n, int shift, uint32_t nblocks,
                                                       uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[kWaves][256];
  const int w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * 256; d += kBlock) (&cnt[0][0])[d] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * kTile;
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    uint64_t x = base + (uint64_t)it * kBlock + threadIdx.x;
    if (x < n) atomicAdd(&cnt[w][digit_of(keys[x], shift)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kBlock) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) s += cnt[v][d];
    hist[(uint64_t)d * nblocks + blockIdx.x] = s;
  }
}

// FOLD (few sort blocks): hist holds the blocks' raw digit counts, and each
// block sums its digit's row itself (its offset and the digit's total), so
// that a pass needs no scan launch; otherwise hist holds the scanned counts
// and totals the digit totals (k_radix_digit_scan).
template <bool FOLD>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const unsigned long long *__restrict__ keys, unsigned long long *__restrict__ out, uint64_t n,
    int shift, uint32_t nblocks, const uint32_t *__restrict__ hist_scanned,
    const uint32_t *__restrict__ totals) {
  static_assert(kBlock == 256, "one thread per digit");
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t gbase[256];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * 256; d += kBlock) (&wcnt[0][0])[d] = 0;
  // digit bases: exclusive scan of the 256 digit totals, plus this block's
  // offset inside its digit
  {
    __shared__ uint32_t wtot[kWaves];
    const int d = threadIdx.x;  // kBlock == 256 digits
    uint32_t tot = 0, mine = 0;
    if (FOLD) {
      const uint32_t *__restrict__ row = hist_scanned + (uint64_t)d * nblocks;
      for (uint32_t b = 0; b < nblocks; ++b) {
        const uint32_t v = row[b];
        mine += b < blockIdx.x ? v : 0u;
        tot += v;
      }
    } else {
      tot = totals[d];
      mine = hist_scanned[(uint64_t)d * nblocks + blockIdx.x];
    }
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int v = 0; v < w; ++v) pre += wtot[v];
    gbase[d] = pre + inc - tot + mine;
  }
  __syncthreads();

  const uint64_t wbase = (uint64_t)blockIdx.x * kTile + (uint64_t)w * kWaveKeys;
  const unsigned long long below = __lanemask_lt();
  unsigned long long key[kItems];
  uint32_t dig[kItems], rank[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    uint64_t x = wbase + (uint64_t)it * 64 + lane;
    bool valid = x < n;
    key[it] = valid ? keys[x] : 0ull;
    uint32_t d = digit_of(key[it], shift);
    dig[it] = d;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long set = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? set : ~set;
    }
    uint32_t prior = wcnt[w][d];
    uint32_t r = prior + (uint32_t)__popcll(peers & below);
    rank[it] = r;
    // the highest lane of each peer group advances the wave's count
    if (valid && (peers >> lane) == 1ull) wcnt[w][d] = prior + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kBlock) {
    uint32_t run = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) {
      uint32_t c = wcnt[v][d];
      wcnt[v][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    uint64_t x = wbase + (uint64_t)it * 64 + lane;
    if (x < n) {
      const uint64_t pos = (uint64_t)gbase[dig[it]] + wcnt[w][dig[it]] + rank[it];
      if (pos < n) out[pos] = key[it];
    }
  }
}

// One workgroup per digit: exclusive scan, in place, of that digit's counts
// over all sort blocks (hist[d * nblocks + b]), and the digit's total.
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t *__restrict__ hist,
                                                             uint32_t nblocks,
                                                             uint32_t *__restrict__ totals) {
  __shared__ uint32_t wsum[kWaves];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  uint32_t *row = hist + (uint64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nblocks; base += kScanTile) {
    const uint32_t first = base + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tsum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = first + i < nblocks ? row[first + i] : 0u;
      tsum += v[i];
    }
    uint32_t inc = tsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
#pragma unroll
    for (int v2 = 0; v2 < kWaves; ++v2) {
      uint32_t s2 = wsum[v2];
      if (v2 < w) wpre += s2;
      total += s2;
    }
    uint32_t run = carry + wpre + inc - tsum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (first + i < nblocks) row[first + i] = run;
      run += v[i];
    }
    carry += total;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace

uint64_t radix_scratch_words(uint64_t n) {
  uint64_t nb = cdiv(n ? n : 1, kTile);
  return 256 * nb + 256;
}

hipError_t radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n,
                          const int *shifts, int n_shifts, uint32_t *scratch, hipStream_t st,
                          unsigned long long **result) {
  *result = keys;
  if (n <= 1 || n_shifts == 0) return hipSuccess;
  uint64_t nb = cdiv(n, kTile);
  if (nb > 0xFFFFFFFFull / 256) return hipErrorInvalidValue;
  uint32_t *hist = scratch;
  uint32_t *totals = scratch + 256 * nb;
  unsigned long long *src = keys, *dst = tmp;
  for (int p = 0; p < n_shifts; ++p) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, st, src, n, shifts[p],
                       (uint32_t)nb, hist);
    if (nb <= kFoldBlocks) {
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nb), dim3(kBlock), 0, st, src,
                         dst, n, shifts[p], (uint32_t)nb, hist, totals);
    } else {
      hipLaunchKernelGGL(k_radix_digit_scan, dim3(256), dim3(kBlock), 0, st, hist, (uint32_t)nb,
                         totals);
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nb), dim3(kBlock), 0, st, src,
                         dst, n, shifts[p], (uint32_t)nb, hist, totals);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long *t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return hipSuccess;
}

}  // namespace ssj
