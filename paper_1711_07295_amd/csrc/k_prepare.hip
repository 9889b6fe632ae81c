// Preparation kernels: set sizes and offset validation, the size-sort keys,
// the per-size group starts of the size-ordered collection, and small
// helpers (counter resets, key unpacking, tile expansion).
//
// The paper sorts every collection by set size before joining (Section 5,
// collection preprocessing) and the length filter (Section 2.3.2, Table 2)
// then bounds each row's partners to a contiguous range of that order.
#include "ssj_internal.h"

namespace ssj {
namespace {

__global__ __launch_bounds__(kBlock) void k_set_sizes(const uint64_t *__restrict__ offsets,
                                                      uint64_t n, uint64_t n_tokens,
                                                      unsigned long long *__restrict__ keys,
                                                      JoinCounters *__restrict__ ctr) {
  uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t err = 0, sz32 = 0;
  if (k < n) {
    uint64_t o0 = offsets[k], o1 = offsets[k + 1];
    if (k == 0 && o0 != 0) err |= kErrOffsets;
    if (k == n - 1 && o1 != n_tokens) err |= kErrOffsets;
    if (o1 < o0 || o1 > n_tokens) {
      err |= kErrOffsets;
    } else {
      uint64_t sz = o1 - o0;
      if (sz >= 0xFFFFFFFFull) err |= kErrTooBig;
      else sz32 = (uint32_t)sz;
    }
    keys[k] = ((unsigned long long)sz32 << 32) | k;
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

__global__ __launch_bounds__(kBlock) void k_unpack_keys(const unsigned long long *__restrict__ keys,
                                                        uint64_t n, uint32_t *__restrict__ sizes,
                                                        uint32_t *__restrict__ perm) {
  uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x < n) {
    unsigned long long k = keys[x];
    sizes[x] = (uint32_t)(k >> 32);
    perm[x] = (uint32_t)k;
  }
}

// sstart[s] for s in (size[x-1], size[x]] is x; for s above the last size it is n.
__global__ __launch_bounds__(kBlock) void k_group_starts(const uint32_t *__restrict__ sizes,
                                                         uint64_t n, uint32_t max_size,
                                                         uint32_t *__restrict__ sstart) {
  uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x > n) return;
  int64_t lo = x == 0 ? -1 : (int64_t)sizes[x - 1];
  int64_t hi = x == n ? (int64_t)max_size + 1 : (int64_t)sizes[x];
  if (hi > (int64_t)max_size + 1) hi = (int64_t)max_size + 1;
  for (int64_t s = lo + 1; s <= hi; ++s) sstart[s] = (uint32_t)x;
}

__global__ void k_reset_round(JoinCounters *ctr) {
  if (threadIdx.x == 0) {
    ctr->queue_count = 0;
    ctr->overflow = 0;
    ctr->n_resume = 0;
  }
}

__global__ void k_reset_all(JoinCounters *ctr) {
  uint32_t *w = reinterpret_cast<uint32_t *>(ctr);
  for (uint32_t i = threadIdx.x; i < sizeof(JoinCounters) / 4; i += blockDim.x) w[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_keys_to_pairs(const unsigned long long *__restrict__ keys,
                                                          uint64_t n, ssj_pair *__restrict__ out) {
  uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x < n) {
    unsigned long long k = keys[x];
    ssj_pair p;
    p.i = (uint32_t)(k >> 32);
    p.j = (uint32_t)k;
    out[x] = p;
  }
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

hipError_t launch_set_sizes(const uint64_t *offsets, uint64_t n, uint64_t n_tokens,
                            unsigned long long *keys, JoinCounters *ctr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_sizes, dim3(grid_for(n)), dim3(kBlock), 0, st, offsets, n, n_tokens,
                     keys, ctr);
  return hipGetLastError();
}

hipError_t launch_unpack_keys(const unsigned long long *keys, uint64_t n, uint32_t *sizes,
                              uint32_t *perm, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_keys, dim3(grid_for(n)), dim3(kBlock), 0, st, keys, n, sizes, perm);
  return hipGetLastError();
}

hipError_t launch_group_starts(const uint32_t *sizes, uint64_t n, uint32_t max_size,
                               uint32_t *sstart, hipStream_t st) {
  hipLaunchKernelGGL(k_group_starts, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, sizes, n,
                     max_size, sstart);
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

hipError_t launch_keys_to_pairs(const unsigned long long *keys, uint64_t n, ssj_pair *out,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys_to_pairs, dim3(grid_for(n)), dim3(kBlock), 0, st, keys, n, out);
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
