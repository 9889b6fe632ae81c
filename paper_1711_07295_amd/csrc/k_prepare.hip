// Preparation kernels: set sizes and offset validation, the size sort of
// every side (collection) of a space, the per-size group starts of each
// size-ordered side, and small helpers (counter resets, tile expansion).
//
// The paper sorts every collection by set size before joining (Section 5,
// collection preprocessing) and the length filter (Section 2.3.2, Table 2)
// then bounds each row's partners to a contiguous range of that order.
//
// A space holds one or more sides one after the other: side s owns global
// indices [base_s, base_s + n_s).  Before the sort, global index g is the
// side's caller index g - base_s; after it, the side's sets in size order.
#include "ssj_internal.h"

namespace ssj {

namespace {

// sizes[g] of every set of every side; offsets checked; largest size.
__global__ __launch_bounds__(kBlock) void k_set_sizes(const SideDesc *__restrict__ sides,
                                                      uint32_t n_sides, uint64_t n_total,
                                                      uint32_t *__restrict__ sizes,
                                                      uint32_t *__restrict__ side_of,
                                                      JoinCounters *__restrict__ ctr) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t err = 0, sz32 = 0;
  if (g < n_total) {
    const uint32_t s = side_of_index(sides, n_sides, g);
    const SideDesc sd = sides[s];
    const uint64_t k = g - sd.base;
    const uint64_t o0 = sd.offsets[k], o1 = sd.offsets[k + 1];
    if (k == 0 && o0 != 0) err |= kErrOffsets;
    if (k == sd.n - 1 && o1 != sd.n_tokens) err |= kErrOffsets;
    if (o1 < o0 || o1 > sd.n_tokens) {
      err |= kErrOffsets;
    } else {
      const uint64_t sz = o1 - o0;
      if (sz >= 0xFFFFFFFFull) err |= kErrTooBig;
      else sz32 = (uint32_t)sz;
    }
    sizes[g] = sz32;
    side_of[g] = s;
  }
  // workgroup reduction, then at most one atomic per workgroup, skipped when
  // the running maximum is already as large
  __shared__ uint32_t wmax[kBlock / 64], werr[kBlock / 64];
  uint32_t m = sz32;
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t o = __shfl_xor(m, d, 64);
    m = o > m ? o : m;
  }
  uint32_t e = err;
  for (int d = 32; d >= 1; d >>= 1) e |= __shfl_xor(e, d, 64);
  if ((threadIdx.x & 63) == 0) {
    wmax[threadIdx.x >> 6] = m;
    werr[threadIdx.x >> 6] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      m = wmax[w] > m ? wmax[w] : m;
      e |= werr[w];
    }
    if (m > __hip_atomic_load(&ctr->max_size, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&ctr->max_size, m);
    if (e) atomicOr(&ctr->error, e);
  }
}

// sort key of set g: (side, size, caller index within the side)
__global__ __launch_bounds__(kBlock) void k_make_keys(const SideDesc *__restrict__ sides,
                                                      const uint32_t *__restrict__ sizes,
                                                      const uint32_t *__restrict__ side_of,
                                                      uint64_t n_total, int size_bits,
                                                      unsigned long long *__restrict__ keys) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n_total) return;
  const uint32_t s = side_of[g];
  const uint64_t k = g - sides[s].base;
  keys[g] = ((unsigned long long)s << (32 + size_bits)) | ((unsigned long long)sizes[g] << 32) | k;
}

// sorted keys -> sizes and caller index (perm) in size order; sides keep
// their ranges because the side is the key's most significant part
__global__ __launch_bounds__(kBlock) void k_unpack_keys(const unsigned long long *__restrict__ keys,
                                                        uint64_t n, int size_bits,
                                                        uint32_t *__restrict__ sizes,
                                                        uint32_t *__restrict__ perm) {
  const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x < n) {
    const unsigned long long k = keys[x];
    sizes[x] = (uint32_t)(k >> 32) & (uint32_t)((1ull << size_bits) - 1);
    perm[x] = (uint32_t)k;
  }
}

// sstart[s * stride + v] = first position of side s (counted from its base)
// whose size is >= v, for v in [0, max_size + 1]
__global__ __launch_bounds__(kBlock) void k_group_starts(const SideDesc *__restrict__ sides,
                                                         const uint32_t *__restrict__ sizes,
                                                         const uint32_t *__restrict__ side_of,
                                                         uint64_t n_total, uint32_t max_size,
                                                         uint32_t stride,
                                                         uint32_t *__restrict__ sstart) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n_total) return;
  const uint32_t s = side_of[g];
  const SideDesc sd = sides[s];
  const uint32_t x = (uint32_t)(g - sd.base);
  uint32_t *tab = sstart + (uint64_t)s * stride;
  const int64_t lo = x == 0 ? -1 : (int64_t)sizes[g - 1];
  const int64_t hi = (int64_t)min(sizes[g], max_size + 1);
  for (int64_t v = lo + 1; v <= hi; ++v) tab[v] = x;
  if (x + 1 == sd.n)
    for (int64_t v = hi + 1; v <= (int64_t)max_size + 1; ++v) tab[v] = sd.n;
}

// rank[base_s + perm[g]] = g: the size-order position of every caller set
__global__ __launch_bounds__(kBlock) void k_invert_perm(const SideDesc *__restrict__ sides,
                                                        const uint32_t *__restrict__ perm,
                                                        const uint32_t *__restrict__ side_of,
                                                        uint64_t n_total,
                                                        uint32_t *__restrict__ rank) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n_total) return;
  const SideDesc sd = sides[side_of[g]];
  const uint32_t k = perm[g];
  if (k < sd.n) rank[sd.base + k] = (uint32_t)g;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, uint64_t n,
                                                     uint32_t v) {
  const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x < n) p[x] = v;
}

__global__ void k_reset_round(JoinCounters *ctr) {
  if (threadIdx.x == 0) {
    ctr->queue_count = 0;
    ctr->long_count = 0;
    ctr->overflow = 0;
    ctr->n_resume = 0;
  }
}

__global__ void k_reset_all(JoinCounters *ctr) {
  uint32_t *w = reinterpret_cast<uint32_t *>(ctr);
  for (uint32_t i = threadIdx.x; i < sizeof(JoinCounters) / 4; i += blockDim.x) w[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_copy_u64(const unsigned long long *__restrict__ in,
                                                     uint64_t n,
                                                     unsigned long long *__restrict__ out) {
  uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x < n) out[x] = in[x];
}

// one wave per row block writes its tiles' block index
__global__ __launch_bounds__(kBlock) void k_expand_tiles(const RowBlock *__restrict__ blocks,
                                                         uint32_t n_blocks, uint32_t n_tiles,
                                                         uint32_t *__restrict__ tile_block) {
  uint32_t b = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (b >= n_blocks) return;
  uint32_t t0 = blocks[b].tile_begin;
  uint32_t t1 = b + 1 < n_blocks ? blocks[b + 1].tile_begin : n_tiles;
  for (uint32_t t = t0 + (threadIdx.x & 63); t < t1; t += 64) tile_block[t] = b;
}

inline unsigned grid_for(uint64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_set_sizes(const SideDesc *sides, uint32_t n_sides, uint64_t n_total,
                            uint32_t *sizes, uint32_t *side_of, JoinCounters *ctr,
                            hipStream_t st) {
  if (n_total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_sizes, dim3(grid_for(n_total)), dim3(kBlock), 0, st, sides, n_sides,
                     n_total, sizes, side_of, ctr);
  return hipGetLastError();
}

hipError_t launch_make_keys(const SideDesc *sides, const uint32_t *sizes, const uint32_t *side_of,
                            uint64_t n_total, int size_bits, unsigned long long *keys,
                            hipStream_t st) {
  if (n_total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n_total)), dim3(kBlock), 0, st, sides, sizes,
                     side_of, n_total, size_bits, keys);
  return hipGetLastError();
}

hipError_t launch_unpack_keys(const unsigned long long *keys, uint64_t n, int size_bits,
                              uint32_t *sizes, uint32_t *perm, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_keys, dim3(grid_for(n)), dim3(kBlock), 0, st, keys, n, size_bits,
                     sizes, perm);
  return hipGetLastError();
}

hipError_t launch_group_starts(const SideDesc *sides, const uint32_t *sizes,
                               const uint32_t *side_of, uint64_t n_total, uint32_t max_size,
                               uint32_t stride, uint32_t n_sides, uint32_t *sstart,
                               hipStream_t st) {
  // empty sides keep the fill value 0 (= their n) everywhere
  const uint64_t tab = (uint64_t)n_sides * stride;
  if (tab == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(tab)), dim3(kBlock), 0, st, sstart, tab, 0u);
  if (n_total)
    hipLaunchKernelGGL(k_group_starts, dim3(grid_for(n_total)), dim3(kBlock), 0, st, sides,
                       sizes, side_of, n_total, max_size, stride, sstart);
  return hipGetLastError();
}

hipError_t launch_invert_perm(const SideDesc *sides, const uint32_t *perm,
                              const uint32_t *side_of, uint64_t n_total, uint32_t *rank,
                              hipStream_t st) {
  if (n_total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(n_total)), dim3(kBlock), 0, st, sides, perm,
                     side_of, n_total, rank);
  return hipGetLastError();
}

hipError_t launch_reset_round(JoinCounters *ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_round, dim3(1), dim3(64), 0, st, ctr);
  return hipGetLastError();
}

hipError_t launch_reset_all(JoinCounters *ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_all, dim3(1), dim3(64), 0, st, ctr);
  return hipGetLastError();
}

hipError_t launch_copy_u64(const unsigned long long *in, uint64_t n, unsigned long long *out,
                           hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, in, n, out);
  return hipGetLastError();
}

hipError_t launch_expand_tiles(const RowBlock *blocks, uint32_t n_blocks, uint32_t n_tiles,
                               uint32_t *tile_block, hipStream_t st) {
  if (n_blocks == 0 || n_tiles == 0) return hipSuccess;
  unsigned grid = (n_blocks + (kBlock / 64) - 1) / (kBlock / 64);
  hipLaunchKernelGGL(k_expand_tiles, dim3(grid), dim3(kBlock), 0, st, blocks, n_blocks, n_tiles,
                     tile_block);
  return hipGetLastError();
}

}  // namespace ssj
