// Prefix-filtered candidate generation for the rows past the cutoff point
// (Section 3.5): rows whose sets are too large for their bitmaps to tell
// dissimilar pairs apart skip the bitmap filter (Alg. 7 applies it only up
// to the cutoff) and take their candidates from an inverted index of set
// prefixes instead (the prefix filter of Section 2.3).
//
// With one global token order (the ascending token ids; rarest first when
// the collection is relabelled by frequency), two sets that share at least
// alpha tokens share one among the first |x| - alpha + 1 tokens of each.
// Every indexed column set contributes (token, column) entries for its
// prefix; the entries are sorted by token, with columns ascending inside a
// token's run.  A probing row then finds, for each of its prefix tokens, the
// run of columns inside its length band with two binary searches.
// Candidates are deduplicated by sorting and go to the verification queue.
#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kScanItems = 8;
constexpr uint32_t kScanTile = kBlock * kScanItems;

// ---------------------------------------------------------------- scan
// Exclusive scan of uint32 counts into uint64 offsets, in three launches:
// per-tile sums, one workgroup scanning the tile sums, per-tile scans.

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total
// through *total.
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v,
                                                              unsigned long long *total) {
  __shared__ unsigned long long wsum[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long inc = wave_incl_scan(v, lane);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  unsigned long long pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    if (k < w) pre += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(const uint32_t *__restrict__ in,
                                                           uint64_t n,
                                                           unsigned long long *__restrict__ sums) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  unsigned long long tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place, and the total.
__global__ __launch_bounds__(kBlock) void k_scan_tile_offsets(unsigned long long *__restrict__ sums,
                                                              uint64_t n_tiles,
                                                              unsigned long long *__restrict__ total) {
  unsigned long long carry = 0;
  for (uint64_t b = 0; b < n_tiles; b += kBlock) {
    const uint64_t i = b + threadIdx.x;
    const unsigned long long v = i < n_tiles ? sums[i] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan(v, &tot);
    if (i < n_tiles) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *__restrict__ in, uint64_t n,
                                                       const unsigned long long *__restrict__ sums,
                                                       unsigned long long *__restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  unsigned long long tot;
  unsigned long long run = sums[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------- index

// Prefix length of every column (0: not indexed) from its side's table.
__global__ __launch_bounds__(kBlock) void k_index_len(const uint32_t *__restrict__ sizes,
                                                      const uint32_t *__restrict__ side_of,
                                                      const uint32_t *__restrict__ ilen,
                                                      uint32_t stride, uint64_t n,
                                                      uint32_t *__restrict__ len) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g < n) len[g] = ilen[(uint64_t)side_of[g] * stride + sizes[g]];
}

// Entries (token << 32 | column) of every indexed column's prefix, one wave
// per column, written at the column's offset.
__global__ __launch_bounds__(kBlock) void k_index_fill(const SideDesc *__restrict__ sides,
                                                       const uint32_t *__restrict__ side_of,
                                                       const uint32_t *__restrict__ perm,
                                                       const uint32_t *__restrict__ len,
                                                       const unsigned long long *__restrict__ off,
                                                       uint64_t n,
                                                       unsigned long long *__restrict__ keys) {
  const uint64_t g = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63;
  if (g >= n) return;
  const uint32_t m = len[g];
  if (!m) return;
  const SideDesc sd = sides[side_of[g]];
  const uint32_t *t = sd.tokens + sd.offsets[perm[g]];
  const unsigned long long o = off[g];
  for (uint32_t k = lane; k < m; k += 64) keys[o + k] = ((unsigned long long)t[k] << 32) | g;
}

// ---------------------------------------------------------------- probe

__device__ __forceinline__ uint64_t lower_bound(const unsigned long long *__restrict__ keys,
                                                uint64_t n, unsigned long long v) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (keys[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Run of a probe row (list position x): the last run whose `first` <= x.
__device__ __forceinline__ uint32_t run_of(const PrefixRun *__restrict__ runs, uint32_t n_runs,
                                           uint64_t x) {
  uint32_t lo = 0, hi = n_runs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (runs[mid].first <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// One wave per probe row.  COUNT: the number of (row, column) candidates,
// duplicates included, into counts[x].  Fill: the candidate keys
// (row << 32 | column) of rows [x0, x1) at out[row_off[x] - base ...].
template <bool COUNT>
__global__ __launch_bounds__(kBlock) void k_probe(
    ProbeArgs a, uint64_t x0, uint64_t x1, const unsigned long long *__restrict__ row_off,
    unsigned long long base, uint32_t *__restrict__ counts, unsigned long long *__restrict__ out) {
  const uint64_t x = x0 + (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (x >= x1) return;
  const PrefixRun run = a.runs[run_of(a.runs, a.n_runs, x)];
  const uint32_t r = run.row_begin + (uint32_t)(x - run.first);
  const TaskDesc td = a.tasks[run.task];
  const uint32_t sz = a.size_rows[r];
  const uint32_t plen = a.tables[run.plen_off + sz];
  // the row's band in global column positions
  const uint32_t cmn = a.tables[td.cmin_off + sz], cmx = a.tables[td.cmax_off + sz];
  const uint32_t *ss = a.sstart_cols + td.col_sstart_off;
  const uint32_t col_n = ss[a.col_max_size + 1];  // the column side's size
  uint32_t lo_c = cmn > a.col_max_size ? col_n : ss[cmn];
  uint32_t hi_c = cmx >= a.col_max_size ? col_n : ss[cmx + 1];
  lo_c += td.col_base;
  hi_c += td.col_base;
  if (td.self && hi_c > r) hi_c = r;  // columns before the row in size order
  uint64_t mine = 0;
  if (plen && hi_c > lo_c) {
    const SideDesc sd = a.row_sides[a.side_of_rows[r]];
    const uint32_t *t = sd.tokens + sd.offsets[a.perm_rows[r]];
    for (uint32_t k = lane; k < plen; k += 64) {
      const unsigned long long tok = (unsigned long long)t[k] << 32;
      mine += lower_bound(a.keys, a.n_keys, tok | hi_c) - lower_bound(a.keys, a.n_keys, tok | lo_c);
    }
  }
  if (COUNT) {
    unsigned long long s = mine;
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) counts[x] = s >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s;  // saturated
    return;
  }
  // fill: each lane writes its candidates after those of lower lanes
  const unsigned long long inc = wave_incl_scan(mine, lane);
  unsigned long long pos = row_off[x] - base + inc - mine;
  if (!(plen && hi_c > lo_c)) return;
  const SideDesc sd = a.row_sides[a.side_of_rows[r]];
  const uint32_t *t = sd.tokens + sd.offsets[a.perm_rows[r]];
  for (uint32_t k = lane; k < plen; k += 64) {
    const unsigned long long tok = (unsigned long long)t[k] << 32;
    const uint64_t b = lower_bound(a.keys, a.n_keys, tok | lo_c);
    const uint64_t e = lower_bound(a.keys, a.n_keys, tok | hi_c);
    for (uint64_t i = b; i < e; ++i)
      out[pos++] = ((unsigned long long)r << 32) | (uint32_t)a.keys[i];
  }
}

// Sorted candidate keys -> distinct (row, column) entries of the queue.
__global__ __launch_bounds__(kBlock) void k_unique_to_queue(const unsigned long long *__restrict__ keys,
                                                            uint64_t n, uint2 *__restrict__ queue,
                                                            JoinCounters *__restrict__ ctr) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool first = i < n && (i == 0 || keys[i] != keys[i - 1]);
  const unsigned long long m = __ballot(first);
  if (!m) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&ctr->queue_count, (unsigned long long)__popcll(m));
  base = __shfl(base, 0, 64);
  if (first) {
    const unsigned long long k = keys[i];
    queue[base + __popcll(m & __lanemask_lt())] = make_uint2((uint32_t)(k >> 32), (uint32_t)k);
  }
}

inline unsigned grid_for(uint64_t n, uint64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

uint64_t scan_scratch_words(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, unsigned long long *out,
                           unsigned long long *total, unsigned long long *scratch,
                           hipStream_t st) {
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles) {
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)tiles), dim3(kBlock), 0, st, in, n,
                       scratch);
  }
  hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(kBlock), 0, st, scratch, tiles, total);
  if (tiles) {
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kBlock), 0, st, in, n, scratch,
                       out);
  }
  return hipGetLastError();
}

hipError_t launch_index_len(const uint32_t *sizes, const uint32_t *side_of, const uint32_t *ilen,
                            uint32_t stride, uint64_t n, uint32_t *len, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_index_len, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, sizes, side_of,
                     ilen, stride, n, len);
  return hipGetLastError();
}

hipError_t launch_index_fill(const SideDesc *sides, const uint32_t *side_of, const uint32_t *perm,
                             const uint32_t *len, const unsigned long long *off, uint64_t n,
                             unsigned long long *keys, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_index_fill, dim3(grid_for(n, kWaves)), dim3(kBlock), 0, st, sides, side_of,
                     perm, len, off, n, keys);
  return hipGetLastError();
}

hipError_t launch_probe_count(const ProbeArgs &a, uint64_t n_rows, uint32_t *counts,
                              hipStream_t st) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe<true>, dim3(grid_for(n_rows, kWaves)), dim3(kBlock), 0, st, a,
                     (uint64_t)0, n_rows, (const unsigned long long *)nullptr, 0ull, counts,
                     (unsigned long long *)nullptr);
  return hipGetLastError();
}

hipError_t launch_probe_fill(const ProbeArgs &a, uint64_t x0, uint64_t x1,
                             const unsigned long long *row_off, unsigned long long base,
                             unsigned long long *out, hipStream_t st) {
  if (x1 <= x0) return hipSuccess;
  hipLaunchKernelGGL(k_probe<false>, dim3(grid_for(x1 - x0, kWaves)), dim3(kBlock), 0, st, a, x0,
                     x1, row_off, base, (uint32_t *)nullptr, out);
  return hipGetLastError();
}

hipError_t launch_unique_to_queue(const unsigned long long *keys, uint64_t n, uint2 *queue,
                                  JoinCounters *ctr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unique_to_queue, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, keys, n,
                     queue, ctr);
  return hipGetLastError();
}

}  // namespace ssj
