// Stable LSD radix sort of 64-bit keys (8-bit digits) and a device-wide
// exclusive scan.  Used for the size sort of the collections and for the
// final ordering of the result pairs.
//
// Per pass: (1) every workgroup counts the digits of its kTile keys,
// (2) the digit-major table of counts is scanned, (3) every workgroup
// ranks its keys stably -- wave by wave, 64 keys at a time, peers with
// the same digit found by eight ballots -- and scatters them.
#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr int kItems = 8;                 // keys per thread
constexpr int kTile = kBlock * kItems;    // keys per workgroup
constexpr int kWaves = kBlock / 64;
constexpr int kWaveKeys = kTile / kWaves; // contiguous keys per wave
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

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

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const unsigned long long *__restrict__ keys, unsigned long long *__restrict__ out, uint64_t n,
    int shift, uint32_t nblocks, const uint32_t *__restrict__ hist_scanned) {
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t gbase[256];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * 256; d += kBlock) (&wcnt[0][0])[d] = 0;
  for (int d = threadIdx.x; d < 256; d += kBlock)
    gbase[d] = hist_scanned[(uint64_t)d * nblocks + blockIdx.x];
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

// exclusive scan of kScanTile entries per workgroup; block totals to `sums`
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *__restrict__ data, uint64_t m,
                                                       uint32_t *__restrict__ sums) {
  __shared__ uint32_t wsum[kWaves];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t tsum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < m ? data[base + i] : 0u;
    tsum += v[i];
  }
  // inclusive wave scan of the thread totals
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
    uint32_t s = wsum[v2];
    if (v2 < w) wpre += s;
    total += s;
  }
  uint32_t run = wpre + inc - tsum;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < m) data[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *__restrict__ data, uint64_t m,
                                                     const uint32_t *__restrict__ sums) {
  uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t add = sums[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kBlock)
    if (base + i < m) data[base + i] += add;
}

inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

uint64_t scan_scratch_words(uint64_t m) {
  uint64_t total = 0;
  while (m > (uint64_t)kScanTile) {
    m = cdiv(m, kScanTile);
    total += m;
  }
  return total + 1;
}

// in-place exclusive scan of data[0..m); scratch holds scan_scratch_words(m)
hipError_t scan_exclusive(uint32_t *data, uint64_t m, uint32_t *scratch, hipStream_t st) {
  if (m == 0) return hipSuccess;
  uint64_t nb = cdiv(m, kScanTile);
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, st, data, m, (uint32_t *)nullptr);
    return hipGetLastError();
  }
  uint32_t *sums = scratch;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kBlock), 0, st, data, m, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(sums, nb, scratch + nb, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, st, data, m, sums);
  return hipGetLastError();
}

}  // namespace

uint64_t radix_scratch_words(uint64_t n) {
  uint64_t nb = cdiv(n ? n : 1, kTile);
  uint64_t m = 256 * nb;
  return m + scan_scratch_words(m);
}

hipError_t radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n,
                          const int *shifts, int n_shifts, uint32_t *scratch, hipStream_t st,
                          unsigned long long **result) {
  *result = keys;
  if (n <= 1 || n_shifts == 0) return hipSuccess;
  uint64_t nb = cdiv(n, kTile);
  if (nb > 0xFFFFFFFFull / 256) return hipErrorInvalidValue;
  uint32_t *hist = scratch;
  uint32_t *sscr = scratch + 256 * nb;
  unsigned long long *src = keys, *dst = tmp;
  for (int p = 0; p < n_shifts; ++p) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, st, src, n, shifts[p],
                       (uint32_t)nb, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive(hist, 256 * nb, sscr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, st, src, dst, n,
                       shifts[p], (uint32_t)nb, hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long *t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return hipSuccess;
}

}  // namespace ssj
