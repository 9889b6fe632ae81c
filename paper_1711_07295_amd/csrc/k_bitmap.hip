// Bitmap generation (Section 3.2) and the strict-order check of the input
// sets.  The hash is h(t) = t mod b (Section 5.1); bit k of a bitmap is bit
// k % 64 of 64-bit word k / 64.
//
//   Bitmap-Xor (Alg. 4): flip bit h(t) for every token -- bit k ends set iff
//     an odd number of tokens hash to k.  The join's default.
//   Bitmap-Set (Alg. 3): set bit h(t) for every token.
//   Bitmap-Next (Alg. 5): all ones when n >= b; otherwise each token takes
//     bit h(t) or the next free bit after it, cyclically.  The occupied
//     bits do not depend on the order the tokens are taken in.
//
// The sets come from one or more sides (collections) laid out one after the
// other in a space of global indices (see SideDesc).
//
// One wave per set: lanes stride over the set's tokens (coalesced reads of
// the CSR token array), combine their bits in a per-wave LDS bitmap with
// LDS atomics, and lane w writes word w.  The kernel is bound by HBM reads
// of the tokens (4 bytes per token) and writes of b/8 bytes per set.
#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr int kWavesPerBlock = kBlock / 64;

// Side of workgroup blk of the segmented build: the last side whose first
// workgroup is <= blk (empty sides share it with the next side).
__device__ __forceinline__ uint32_t side_of_block(const SideDesc *__restrict__ sides,
                                                  uint32_t n_sides, uint32_t blk) {
  uint32_t lo = 0, hi = n_sides;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sides[mid].blk0 <= blk) lo = mid; else hi = mid;
  }
  return lo;
}

// One wave per output row x: in size order (perm/side_of given) the set
// perm[x] of side side_of[x], otherwise the caller set x - base of the side
// holding global index x.
template <int METHOD, bool POW2>
__global__ __launch_bounds__(kBlock) void k_build_bitmaps(
    const SideDesc *__restrict__ sides, uint32_t n_sides, const uint32_t *__restrict__ perm,
    const uint32_t *__restrict__ side_of, uint64_t n, uint32_t b_bits, uint32_t out_words,
    uint64_t *__restrict__ out, JoinCounters *__restrict__ ctr) {
  __shared__ uint32_t lbits[kWavesPerBlock][2 * kMaxWords];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const uint64_t x = (uint64_t)blockIdx.x * kWavesPerBlock + w;
  if (x >= n) return;  // whole wave leaves together
  uint32_t *bits = lbits[w];
  for (uint32_t i = lane; i < 2 * out_words; i += 64) bits[i] = 0;
  const uint32_t sid = perm ? side_of[x] : side_of_index(sides, n_sides, x);
  const SideDesc sd = sides[sid];
  const uint64_t k = perm ? perm[x] : x - sd.base;
  if (k >= sd.n) return;
  const uint32_t *__restrict__ tokens = sd.tokens;
  const uint64_t o0 = sd.offsets[k], o1 = sd.offsets[k + 1];
  const uint32_t nt = (uint32_t)(o1 - o0);
  const uint32_t mask = b_bits - 1;
  bool unsorted = false;
  if (METHOD == SSJ_BM_NEXT) {
    // Alg. 5: saturated when n >= b, else linear probing by one lane.
    for (uint64_t t = o0 + lane; t + 1 < o1; t += 64)
      unsorted |= !(tokens[t] < tokens[t + 1]);
    if (nt >= b_bits) {
      for (uint32_t i = lane; i < 2 * (b_bits / 64); i += 64) bits[i] = 0xFFFFFFFFu;
    } else if (lane == 0) {
      for (uint64_t t = o0; t < o1; ++t) {
        uint32_t v = tokens[t];
        uint32_t s = POW2 ? (v & mask) : (v % b_bits);
        while ((bits[s >> 5] >> (s & 31)) & 1u) s = (s + 1 == b_bits) ? 0 : s + 1;
        bits[s >> 5] |= 1u << (s & 31);
      }
    }
  } else {
    for (uint64_t t = o0 + lane; t < o1; t += 64) {
      uint32_t v = tokens[t];
      if (t + 1 < o1) unsorted |= !(v < tokens[t + 1]);
      uint32_t s = POW2 ? (v & mask) : (v % b_bits);
      if (METHOD == SSJ_BM_XOR) atomicXor(&bits[s >> 5], 1u << (s & 31));
      else atomicOr(&bits[s >> 5], 1u << (s & 31));
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  uint64_t *dst = out + x * out_words;
  for (uint32_t i = lane; i < out_words; i += 64)
    dst[i] = (uint64_t)bits[2 * i] | ((uint64_t)bits[2 * i + 1] << 32);
  if (__ballot(unsorted) && lane == 0) atomicOr(&ctr->error, kErrUnsorted);
}

// Bitmaps of up to 8 words, and of 16 and 32, XOR or SET: a workgroup takes
// kSegSets consecutive sets in caller order, whose tokens are one contiguous
// run of the CSR array, and reads that run fully coalesced (in passes of as
// many sets as 16 KB of LDS bitmaps hold).  Each token finds its
// set by binary search over the segment's offsets in LDS and flips (or sets)
// its bit in the set's LDS bitmap; the bitmaps are then written to their
// output rows (rank[k] when the output is in size order).
constexpr uint32_t kSegSets = 256;

// Sets of a segment one pass of the build holds in LDS: 16 KB of bitmaps
// (256 sets up to 8 words, 128 at 16 words, 64 at 32), so that wide widths
// keep as many workgroups per compute unit as narrow ones.
template <int WO>
constexpr uint32_t seg_pass_sets() {
  return kSegSets * 8 / (WO > 8 ? WO : 8);
}

template <int WO, int METHOD, bool POW2>
__global__ __launch_bounds__(kBlock) void k_build_bitmaps_seg(
    const SideDesc *__restrict__ sides, uint32_t n_sides, const uint32_t *__restrict__ rank,
    uint64_t n, uint32_t b_bits, uint64_t *__restrict__ out, FoldOut fold,
    JoinCounters *__restrict__ ctr) {
  constexpr uint32_t kPass = seg_pass_sets<WO>();
  __shared__ uint64_t soff[kPass + 1];
  __shared__ uint32_t sbits[kPass * 2 * WO];
  const SideDesc sd = sides[side_of_block(sides, n_sides, blockIdx.x)];
  const uint64_t seg0 = (uint64_t)(blockIdx.x - sd.blk0) * kSegSets;
  if (seg0 >= sd.n) return;  // whole workgroup leaves together
  const uint32_t nseg = (uint32_t)min((uint64_t)kSegSets, sd.n - seg0);
  const uint64_t *__restrict__ offsets = sd.offsets;
  const uint32_t *__restrict__ tokens = sd.tokens;
  const uint32_t mask = b_bits - 1;
  bool unsorted = false;
  for (uint32_t p0 = 0; p0 < nseg; p0 += kPass) {
    const uint64_t s0 = seg0 + p0;
    const uint32_t ns = min(kPass, nseg - p0);
    const uint64_t t0 = offsets[s0];
    if (p0) __syncthreads();  // the previous pass has read soff and sbits
    for (uint32_t i = threadIdx.x; i <= ns; i += kBlock) soff[i] = offsets[s0 + i] - t0;
    for (uint32_t i = threadIdx.x; i < ns * 2 * WO; i += kBlock) sbits[i] = 0;
    __syncthreads();
    const uint64_t nt = soff[ns];
    // Each thread takes four consecutive tokens at a time, from the
    // 16-byte boundary at or before the run's start: one 16-byte load
    // (scalar loads at the array's end or for an unaligned array), one
    // binary search for the first token's set, then a step to the next set
    // wherever a set ends.  Each token is checked against the one before it
    // in its set.
    const uint64_t head = t0 & 3, a0 = t0 - head;  // tokens[a0] is 16-byte aligned
    const bool vec = (reinterpret_cast<uintptr_t>(tokens) & 15) == 0;
    for (uint64_t c = (uint64_t)threadIdx.x * 4; c < nt + head; c += 4 * kBlock) {
      uint32_t v[4];
      if (vec && a0 + c + 4 <= sd.n_tokens) {
        const uint4 q = *reinterpret_cast<const uint4 *>(tokens + a0 + c);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = a0 + c + k < sd.n_tokens ? tokens[a0 + c + k] : 0u;
      }
      // tokens g = c + k - head of the run, for k with 0 <= g < nt
      const uint64_t kfirst = c < head ? head - c : 0;
      const uint64_t gfirst = c + kfirst - head;
      uint32_t lo = 0, hi = ns;  // soff[lo] <= gfirst < soff[hi]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (soff[mid] <= gfirst) lo = mid; else hi = mid;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((uint64_t)k < kfirst) continue;
        const uint64_t g = c + k - head;
        if (g >= nt) break;
        while (soff[lo + 1] <= g) ++lo;
        if (g > soff[lo]) {
          const uint32_t prev = (uint64_t)k > kfirst ? v[k - 1] : tokens[t0 + g - 1];
          unsorted |= !(prev < v[k]);
        }
        const uint32_t s = POW2 ? (v[k] & mask) : (v[k] % b_bits);
        if (METHOD == SSJ_BM_XOR) atomicXor(&sbits[lo * 2 * WO + (s >> 5)], 1u << (s & 31));
        else atomicOr(&sbits[lo * 2 * WO + (s >> 5)], 1u << (s & 31));
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < ns * WO; i += kBlock) {
      const uint32_t x = i / WO, w = i - x * WO;
      const uint64_t row = rank ? rank[sd.base + s0 + x] : sd.base + s0 + x;
      if (row < n)
        out[row * WO + w] = (uint64_t)sbits[x * 2 * WO + 2 * w] |
                            ((uint64_t)sbits[x * 2 * WO + 2 * w + 1] << 32);
    }
    // Narrower widths b' = b / 2^k from the same pass: bit k' of b' collects
    // the tokens with t mod b' = k', i.e. bits k' + m b' of b, so word i of
    // b' combines (xor for Bitmap-Xor, or for Bitmap-Set) words i + m (b'/64).
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const uint32_t wf = (uint32_t)WO >> (f + 1);
      if (wf == 0 || fold.out[f] == nullptr) continue;
      for (uint32_t i = threadIdx.x; i < ns * wf; i += kBlock) {
        const uint32_t x = i / wf, w = i - x * wf;
        uint64_t v = 0;
        for (uint32_t m = 0; m < (uint32_t)WO / wf; ++m) {
          const uint32_t src = w + m * wf;
          const uint64_t word = (uint64_t)sbits[x * 2 * WO + 2 * src] |
                                ((uint64_t)sbits[x * 2 * WO + 2 * src + 1] << 32);
          v = METHOD == SSJ_BM_XOR ? (v ^ word) : (v | word);
        }
        const uint64_t row = rank ? rank[sd.base + s0 + x] : sd.base + s0 + x;
        if (row < n) fold.out[f][row * wf + w] = v;
      }
    }
  }
  if (__ballot(unsorted) && (threadIdx.x & 63) == 0) atomicOr(&ctr->error, kErrUnsorted);
}

// Bitmap-Xor bitmaps at 16 or 32 words (and the narrower widths of `fold`)
// of only the sets whose size lies in their side's window: the wide width
// classes are read by few sets, whose tokens are a fraction of the
// collection's.  A workgroup takes the segment of kSegSets sets in caller
// order that the segmented build takes, lists the sets of the segment that
// fall in the window, and its waves take the listed sets one at a time:
// the lanes stride over the set's tokens (these sets are long), flip their
// bits in the wave's LDS bitmap and write it to the set's size-order row.
// The token order is not checked here: a full build of the same sets does.
template <int WO>
__global__ __launch_bounds__(kBlock) void k_build_bitmaps_window(
    const SideDesc *__restrict__ sides, uint32_t n_sides, const uint32_t *__restrict__ rank,
    const SizeWindow *__restrict__ win, uint64_t n, uint64_t *__restrict__ out, FoldOut fold) {
  __shared__ uint32_t listed[kSegSets];
  __shared__ uint32_t n_listed;
  __shared__ uint32_t lbits[kWavesPerBlock][2 * WO];
  const uint32_t sid = side_of_block(sides, n_sides, blockIdx.x);
  const SideDesc sd = sides[sid];
  const uint64_t seg0 = (uint64_t)(blockIdx.x - sd.blk0) * kSegSets;
  const SizeWindow w = win[sid];
  if (seg0 >= sd.n || w.lo > w.hi) return;  // whole workgroup leaves together
  const uint32_t nseg = (uint32_t)min((uint64_t)kSegSets, sd.n - seg0);
  const uint64_t *__restrict__ offsets = sd.offsets;
  const uint32_t *__restrict__ tokens = sd.tokens;
  if (threadIdx.x == 0) n_listed = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nseg; i += kBlock) {
    const uint64_t size = offsets[seg0 + i + 1] - offsets[seg0 + i];
    if (size >= w.lo && size <= w.hi) listed[atomicAdd(&n_listed, 1u)] = i;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6, count = n_listed;
  uint32_t *bits = lbits[wv];
  constexpr uint32_t kMask = 64 * WO - 1;
  for (uint32_t e = wv; e < count; e += kWavesPerBlock) {
    const uint32_t x = listed[e];
    for (uint32_t i = lane; i < 2 * WO; i += 64) bits[i] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const uint64_t o0 = offsets[seg0 + x], o1 = offsets[seg0 + x + 1];
    // four loads in flight per lane before their bits are flipped
    for (uint64_t t = o0 + lane; t < o1; t += 256) {
      uint32_t v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = t + 64 * k < o1 ? tokens[t + 64 * k] : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (t + 64 * k < o1) atomicXor(&bits[(v[k] & kMask) >> 5], 1u << (v[k] & 31));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const uint64_t row = rank[sd.base + seg0 + x];
    if (row < n) {
      if (lane < (uint32_t)WO)
        out[row * WO + lane] = (uint64_t)bits[2 * lane] | ((uint64_t)bits[2 * lane + 1] << 32);
      // narrower widths b / 2^(f+1): word i combines words i + m (b'/64)
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const uint32_t wf = (uint32_t)WO >> (f + 1);
        if (wf == 0 || fold.out[f] == nullptr || lane >= wf) continue;
        uint64_t v = 0;
        for (uint32_t m = 0; m < (uint32_t)WO / wf; ++m) {
          const uint32_t src = lane + m * wf;
          v ^= (uint64_t)bits[2 * src] | ((uint64_t)bits[2 * src + 1] << 32);
        }
        fold.out[f][row * wf + lane] = v;
      }
    }
    // every lane has read the bitmap before the next set clears it
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(kBlock) void k_check_sorted(const uint64_t *__restrict__ offsets,
                                                         const uint32_t *__restrict__ tokens,
                                                         uint64_t n, JoinCounters *__restrict__ ctr) {
  const int lane = threadIdx.x & 63;
  const uint64_t k = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (k >= n) return;
  const uint64_t o0 = offsets[k], o1 = offsets[k + 1];
  bool unsorted = false;
  for (uint64_t t = o0 + lane; t + 1 < o1; t += 64) unsorted |= !(tokens[t] < tokens[t + 1]);
  if (__ballot(unsorted) && lane == 0) atomicOr(&ctr->error, kErrUnsorted);
}

__global__ __launch_bounds__(kBlock) void k_gather_bitmaps(const uint64_t *__restrict__ in,
                                                           const uint32_t *__restrict__ perm,
                                                           uint64_t n, uint32_t in_words,
                                                           uint32_t out_words,
                                                           uint64_t *__restrict__ out) {
  const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t x = e / out_words;
  const uint32_t w = (uint32_t)(e - x * out_words);
  if (x >= n) return;
  const uint64_t k = perm[x];
  out[e] = (w < in_words && k < n) ? in[k * in_words + w] : 0ull;
}

template <int WO, int METHOD>
hipError_t launch_seg(bool pow2, hipStream_t st, const SideDesc *sides, uint32_t n_sides,
                      uint32_t seg_blocks, const uint32_t *rank, uint64_t n, uint32_t b_bits,
                      uint64_t *out, const FoldOut &fold, JoinCounters *ctr) {
  dim3 grid(seg_blocks);
  if (pow2)
    hipLaunchKernelGGL((k_build_bitmaps_seg<WO, METHOD, true>), grid, dim3(kBlock), 0, st,
                       sides, n_sides, rank, n, b_bits, out, fold, ctr);
  else
    hipLaunchKernelGGL((k_build_bitmaps_seg<WO, METHOD, false>), grid, dim3(kBlock), 0, st,
                       sides, n_sides, rank, n, b_bits, out, fold, ctr);
  return hipGetLastError();
}

template <int METHOD>
hipError_t launch_method(bool pow2, hipStream_t st, const SideDesc *sides, uint32_t n_sides,
                         uint32_t seg_blocks, uint64_t n, const uint32_t *perm,
                         const uint32_t *rank, const uint32_t *side_of, uint32_t b_bits,
                         uint32_t out_words, uint64_t *out, const FoldOut &fold,
                         JoinCounters *ctr) {
  if (METHOD != SSJ_BM_NEXT && (rank || !perm) && seg_blocks) {
#define SSJ_SEG(wo)                                                                     \
  case wo:                                                                              \
    return launch_seg<wo, METHOD>(pow2, st, sides, n_sides, seg_blocks, rank, n, b_bits, \
                                  out, fold, ctr);
    switch (out_words) {
      SSJ_SEG(1) SSJ_SEG(2) SSJ_SEG(3) SSJ_SEG(4) SSJ_SEG(5) SSJ_SEG(6) SSJ_SEG(7) SSJ_SEG(8)
      SSJ_SEG(16) SSJ_SEG(32)
      default: break;
    }
#undef SSJ_SEG
  }
  dim3 grid((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock));
  if (pow2)
    hipLaunchKernelGGL((k_build_bitmaps<METHOD, true>), grid, dim3(kBlock), 0, st, sides,
                       n_sides, perm, side_of, n, b_bits, out_words, out, ctr);
  else
    hipLaunchKernelGGL((k_build_bitmaps<METHOD, false>), grid, dim3(kBlock), 0, st, sides,
                       n_sides, perm, side_of, n, b_bits, out_words, out, ctr);
  return hipGetLastError();
}

// fp4 nibbles of one 32-bit half x of a bitmap block: +1 (0x2) for a set
// bit, -1 (0xA) for a clear one; bit 8e+m of the half in nibble m of dword e.
__device__ __forceinline__ uint4 sign_nibbles(uint32_t x) {
  uint32_t d[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t spread = 0;  // bit m of byte e at bit 4m
#pragma unroll
    for (int m = 0; m < 8; ++m) spread |= ((x >> (8 * e + m)) & 1u) << (4 * m);
    d[e] = 0xAAAAAAAAu ^ (spread << 3);
  }
  return make_uint4(d[0], d[1], d[2], d[3]);
}

// Sign planes of set s, half h (zeros for s >= n): the thread reads the
// set's words in turn and writes block kb's half to plane kb, so that the
// threads of a wave (consecutive sets and halves) write one contiguous run
// of each plane.
__device__ __forceinline__ void expand_set(const uint64_t *__restrict__ bm, uint32_t words,
                                           uint64_t n, uint64_t s, uint32_t h,
                                           uint4 *__restrict__ planes) {
  for (uint32_t kb = 0; kb < words; ++kb) {
    const uint4 out = s < n ? sign_nibbles((uint32_t)(bm[s * words + kb] >> (32 * h)))
                            : make_uint4(0u, 0u, 0u, 0u);
    planes[((uint64_t)kb * (n + kSignPad) + s) * 2 + h] = out;
  }
}

// Sign planes: one thread per (set, half), for n + kSignPad sets: the sets
// from n on are all zero.
__global__ __launch_bounds__(kBlock) void k_expand_signs(const uint64_t *__restrict__ bm,
                                                          uint32_t words, uint64_t n,
                                                          uint4 *__restrict__ planes) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (n + kSignPad) * 2) return;
  expand_set(bm, words, n, t >> 1, (uint32_t)(t & 1), planes);
}

// Sign planes of the sets in the ranges only (the padding sets n .. n +
// kSignPad - 1 are one of them), one thread per (set, half): element e of
// the ranges' concatenation is position ranges[r].lo + e - ranges[r].first
// of the range r holding it.
__global__ __launch_bounds__(kBlock) void k_expand_signs_ranges(
    const uint64_t *__restrict__ bm, uint32_t words, uint64_t n,
    const PosRange *__restrict__ ranges, uint32_t n_ranges, uint64_t total,
    uint4 *__restrict__ planes) {
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= total * 2) return;
  const uint64_t e = t >> 1;
  uint32_t lo = 0, hi = n_ranges;  // the last range whose first element is <= e
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ranges[mid].first <= e) lo = mid;
    else hi = mid;
  }
  expand_set(bm, words, n, ranges[lo].lo + (e - ranges[lo].first), (uint32_t)(t & 1), planes);
}

// The wide ranges of every side from its group starts, on the device (one
// workgroup): side s holds the sets from its first position of size above
// kWideMin to its end, at slots after those of the sides before it; a side
// with none gets an empty range, wide_lo ~0u and the slot the next side
// starts at.
__global__ __launch_bounds__(kBlock) void k_wide_ranges(const SideDesc *__restrict__ sides,
                                                         uint32_t n_sides,
                                                         const uint32_t *__restrict__ sstart,
                                                         uint32_t stride, uint32_t max_size,
                                                         WideRange *__restrict__ ranges,
                                                         uint32_t *__restrict__ wide_lo,
                                                         uint32_t *__restrict__ wide_slot) {
  __shared__ uint32_t count[kBlock];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t s0 = 0; s0 < n_sides; s0 += kBlock) {
    const uint32_t s = s0 + threadIdx.x;
    uint32_t first = 0, n = 0;
    if (s < n_sides) {
      n = sides[s].n;
      first = kWideMin + 1 <= max_size ? sstart[(uint64_t)s * stride + kWideMin + 1] : n;
      first = min(first, n);
    }
    count[threadIdx.x] = n - first;
    __syncthreads();
    if (threadIdx.x == 0) {
      // exclusive scan of the chunk's counts, after the sides before it
      uint32_t run = carry;
      for (uint32_t i = 0; i < kBlock; ++i) {
        const uint32_t c = count[i];
        count[i] = run;
        run += c;
      }
      carry = run;
    }
    __syncthreads();
    if (s < n_sides) {
      const uint32_t base = (uint32_t)sides[s].base, slot = count[threadIdx.x];
      WideRange r;
      r.lo = base + first;
      r.hi = base + n;
      r.slot = slot;
      r.side = s;
      ranges[s] = r;
      wide_lo[s] = first < n ? base + first : 0xFFFFFFFFu;
      wide_slot[s] = slot;
    }
    __syncthreads();  // count is rewritten by the next chunk
  }
}

// Wide Bitmap-Xor bitmaps of the sets in the wide ranges: one wave per set,
// built in LDS (4096 bits per wave) and written out whole.
__global__ __launch_bounds__(kBlock) void k_build_wide(const SideDesc *__restrict__ sides,
                                                        const uint32_t *__restrict__ perm,
                                                        const WideRange *__restrict__ ranges,
                                                        uint32_t n_ranges, uint64_t total,
                                                        uint64_t *__restrict__ out) {
  __shared__ uint32_t acc[kWavesPerBlock][kWideWords * 2];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t w = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
  if (w >= total) return;
  uint32_t *a = acc[wv];
  for (uint32_t x = lane; x < kWideWords * 2; x += 64) a[x] = 0u;
  __builtin_amdgcn_wave_barrier();
  // the last range whose first slot is <= w
  uint32_t lo = 0, hi = n_ranges;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (ranges[mid].slot <= w) lo = mid;
    else hi = mid;
  }
  const WideRange r = ranges[lo];
  const uint64_t g = r.lo + (w - r.slot);
  const SideDesc sd = sides[r.side];
  const uint32_t x = perm[g];
  const uint64_t o0 = sd.offsets[x], o1 = sd.offsets[x + 1];
  for (uint64_t t = o0 + lane; t < o1; t += 64) {
    const uint32_t bit = sd.tokens[t] & (kWideWords * 64 - 1);
    atomicXor(&a[bit >> 5], 1u << (bit & 31));
  }
  __builtin_amdgcn_wave_barrier();
  uint64_t *dst = out + w * kWideWords;
  for (uint32_t k = lane; k < kWideWords; k += 64)
    dst[k] = (uint64_t)a[2 * k] | ((uint64_t)a[2 * k + 1] << 32);
}

}  // namespace

uint32_t bitmap_seg_blocks(uint64_t n) { return (uint32_t)((n + kSegSets - 1) / kSegSets); }

hipError_t launch_build_bitmaps(const SideDesc *sides, uint32_t n_sides, uint32_t seg_blocks,
                                uint64_t n_total, const uint32_t *perm, const uint32_t *rank,
                                const uint32_t *side_of, uint32_t b_bits, int method,
                                uint32_t out_words, uint64_t *out, JoinCounters *ctr,
                                hipStream_t st, const FoldOut *fold_in) {
  if (n_total == 0) return hipSuccess;
  if (out_words > kMaxWords || out_words < b_bits / 64) return hipErrorInvalidValue;
  if (perm && !side_of) return hipErrorInvalidValue;
  FoldOut fold{};
  if (fold_in) {
    // folding needs a power-of-two width built at exactly its words, by the
    // segmented kernel (Xor or Set, at most kMaxFoldWords words)
    const bool pow2w = (out_words & (out_words - 1)) == 0 && b_bits == 64 * out_words;
    if (!pow2w || method == SSJ_BM_NEXT || out_words > kMaxFoldWords || !(rank || !perm) ||
        !seg_blocks)
      return hipErrorInvalidValue;
    fold = *fold_in;
  }
  const bool pow2 = (b_bits & (b_bits - 1)) == 0;
  switch (method) {
    case SSJ_BM_XOR:
      return launch_method<SSJ_BM_XOR>(pow2, st, sides, n_sides, seg_blocks, n_total, perm, rank,
                                       side_of, b_bits, out_words, out, fold, ctr);
    case SSJ_BM_SET:
      return launch_method<SSJ_BM_SET>(pow2, st, sides, n_sides, seg_blocks, n_total, perm, rank,
                                       side_of, b_bits, out_words, out, fold, ctr);
    case SSJ_BM_NEXT:
      return launch_method<SSJ_BM_NEXT>(pow2, st, sides, n_sides, seg_blocks, n_total, perm,
                                        rank, side_of, b_bits, out_words, out, fold, ctr);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_build_bitmaps_window(const SideDesc *sides, uint32_t n_sides,
                                       uint32_t seg_blocks, uint64_t n_total,
                                       const uint32_t *rank, const SizeWindow *win,
                                       uint32_t out_words, uint64_t *out, const FoldOut *fold,
                                       hipStream_t st) {
  if (n_total == 0 || seg_blocks == 0) return hipSuccess;
  if (!rank || !win || !out) return hipErrorInvalidValue;
  const FoldOut f = fold ? *fold : FoldOut{};
  switch (out_words) {
    case 16:
      hipLaunchKernelGGL(k_build_bitmaps_window<16>, dim3(seg_blocks), dim3(kBlock), 0, st, sides,
                         n_sides, rank, win, n_total, out, f);
      break;
    case 32:
      hipLaunchKernelGGL(k_build_bitmaps_window<32>, dim3(seg_blocks), dim3(kBlock), 0, st, sides,
                         n_sides, rank, win, n_total, out, f);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_check_sorted(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                               JoinCounters *ctr, hipStream_t st) {
  if (n == 0) return hipSuccess;
  dim3 grid((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL(k_check_sorted, grid, dim3(kBlock), 0, st, offsets, tokens, n, ctr);
  return hipGetLastError();
}

hipError_t launch_gather_bitmaps(const uint64_t *in, const uint32_t *perm, uint64_t n,
                                 uint32_t in_words, uint32_t out_words, uint64_t *out,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t total = n * out_words;
  dim3 grid((unsigned)((total + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_gather_bitmaps, grid, dim3(kBlock), 0, st, in, perm, n, in_words,
                     out_words, out);
  return hipGetLastError();
}

hipError_t launch_expand_signs(const uint64_t *bm, uint32_t words, uint64_t n, uint4 *planes,
                               hipStream_t st) {
  if (words == 0) return hipErrorInvalidValue;
  const uint64_t total = (n + kSignPad) * 2;
  hipLaunchKernelGGL(k_expand_signs, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, st, bm, words, n, planes);
  return hipGetLastError();
}

hipError_t launch_expand_signs_ranges(const uint64_t *bm, uint32_t words, uint64_t n,
                                      const PosRange *ranges, uint32_t n_ranges, uint64_t total,
                                      uint4 *planes, hipStream_t st) {
  if (words == 0 || n_ranges == 0) return hipErrorInvalidValue;
  const uint64_t threads = total * 2;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_signs_ranges, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, st, bm, words, n, ranges, n_ranges, total, planes);
  return hipGetLastError();
}

hipError_t launch_wide_ranges(const SideDesc *sides, uint32_t n_sides, const uint32_t *sstart,
                              uint32_t stride, uint32_t max_size, WideRange *ranges,
                              uint32_t *wide_lo, uint32_t *wide_slot, hipStream_t st) {
  if (n_sides == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wide_ranges, dim3(1), dim3(kBlock), 0, st, sides, n_sides, sstart, stride,
                     max_size, ranges, wide_lo, wide_slot);
  return hipGetLastError();
}

hipError_t launch_build_wide(const SideDesc *sides, const uint32_t *perm,
                             const WideRange *ranges, uint32_t n_ranges, uint64_t total,
                             uint64_t *out, hipStream_t st) {
  if (total == 0) return hipSuccess;
  if (n_ranges == 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((total + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL(k_build_wide, grid, dim3(kBlock), 0, st, sides, perm, ranges, n_ranges,
                     total, out);
  return hipGetLastError();
}

}  // namespace ssj
