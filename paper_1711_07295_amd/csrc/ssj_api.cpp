// C-ABI host layer of the library: argument checks, the size-ordered
// preparation of the collections, the tile plan of the length band, the
// filter/verify rounds over a bounded survivor queue, and the emission of
// the sorted result pairs.  Every step of a join runs in the library's own
// kernels; the host only plans, launches and copies.
//
// One call joins one or more tasks.  The sets of a call live in two spaces
// (rows and columns), each a list of sides (collections) laid out one after
// the other; a task joins one row side with one column side at its own
// threshold.  A self-join is one task whose row and column side coincide;
// a batch of self-joins is many such tasks in one space; a query against a
// resident index is one task per query batch, all against the index's side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "autotune_table.h"
#include "ssj.h"
#include "ssj_internal.h"

namespace ssj {
namespace {

// Survivor queue: a call starts with kInitialQueue entries (64 MiB of
// (row, column) pairs, and as many result keys) unless the caller fixes
// the capacity, and quadruples it after each round that filled it, up to
// kMaxQueue (4 GiB): memory follows what the band's survivors need.
constexpr uint64_t kInitialQueue = 1ull << 23;
constexpr uint64_t kMaxQueue = 1ull << 29;
constexpr uint32_t kDefaultTileCols = 2048;
// A width class with fewer than about kMinSlotTiles tiles of the default
// width gets narrower tiles, down to kMinTileCols columns; kMinTileColsValu
// for the vector-ALU kernel, whose classes hold the largest sets: on the
// sparse tail of the size distribution a tile crosses a size group every
// few columns, and the launch lasts as long as its slowest tile.  (The
// matrix-core kernel measured no gain below 64: it takes 32 columns a step.)
constexpr uint64_t kMinSlotTiles = 16384;
// A call of one task uses fewer, wider tiles: its blocks' column ranges are
// long, and each tile and each size group it crosses starts with dependent
// loads that three waves per SIMD do not hide (the 1,000,000-set join's
// b = 128 class: 0.185 ms at 4,096 tiles against 0.246 ms at 16,384).  The
// many short ranges of a batch's tasks balance the waves better with more
// tiles (its b = 64 class: 1.71 ms at 16,384 against 2.18 ms at 4,096).
constexpr uint64_t kMinSlotTilesOneTask = 4096;
// Host threads that plan the width classes of a call's tasks (16 tasks or
// more per thread), when the tasks' largest sizes sum to kPlanThreadSizes
// or more.
constexpr uint32_t kPlanThreads = 8;
constexpr uint64_t kPlanThreadSizes = 65536;
constexpr uint32_t kMinTileCols = 64;
constexpr uint32_t kMinTileColsValu = 32;
// A class of four or more words (b >= 256) and fewer band pairs than this
// runs on the vector ALUs: there the matrix-core launch has the larger fixed cost
// (about 0.12 ms against 0.07 ms for a class of 1.6e6 pairs), and its sign
// planes need not be built.  Narrower classes stay on the matrix cores at
// any size: a query of a few sets against a large index sweeps long column
// ranges, 32 columns a step there against a few on the vector ALUs.
constexpr uint64_t kMfmaMinBand = 1ull << 26;
constexpr uint32_t kMfmaMinBandWords = 4;
constexpr uint64_t kMaxTable = 1ull << 26;       // largest |r| + |s| handled

struct Fail {
  int code;
};

inline void check(hipError_t e) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) throw Fail{SSJ_E_NOMEM};
  throw Fail{SSJ_E_DEVICE};
}

// Host buffers of result pair lists.  A list of at least kPinnedMin bytes
// goes to page-locked memory, so that its copy from the device runs at the
// link's rate and touches no fresh pages; ssj_free_pairs keeps such buffers
// for later calls (at most kPinnedIdleMax bytes of them idle).  Smaller
// lists, and any a page-locked allocation fails for, use malloc.
class HostPairs {
 public:
  static HostPairs &get() {
    static HostPairs *h = new HostPairs;  // never destroyed: buffers may outlive exit handlers
    return *h;
  }
  ssj_pair *alloc(uint64_t n) {
    const size_t bytes = (size_t)n * sizeof(ssj_pair);
    if (bytes >= kPinnedMin) {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = idle_.lower_bound(bytes);
      if (it != idle_.end() && it->first <= 2 * bytes) {
        void *p = it->second;
        idle_bytes_ -= it->first;
        idle_.erase(it);
        return static_cast<ssj_pair *>(p);
      }
      size_t cap = kPinnedMin;
      while (cap < bytes) cap *= 2;
      void *p = nullptr;
      if (hipHostMalloc(&p, cap, hipHostMallocDefault) == hipSuccess && p) {
        cap_[p] = cap;
        return static_cast<ssj_pair *>(p);
      }
      (void)hipGetLastError();
    }
    return static_cast<ssj_pair *>(std::malloc(bytes));
  }
  void release(void *p) {
    if (!p) return;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = cap_.find(p);
      if (it != cap_.end()) {
        const size_t cap = it->second;
        if (idle_bytes_ + cap <= kPinnedIdleMax) {
          idle_.emplace(cap, p);
          idle_bytes_ += cap;
        } else {
          cap_.erase(it);
          (void)hipHostFree(p);
        }
        return;
      }
    }
    std::free(p);
  }

 private:
  static constexpr size_t kPinnedMin = size_t(1) << 20, kPinnedIdleMax = size_t(1) << 30;
  std::mutex mu_;
  std::multimap<size_t, void *> idle_;  // capacity -> idle buffer
  std::map<void *, size_t> cap_;        // every page-locked buffer -> capacity
  size_t idle_bytes_ = 0;
};

// Device memory chunks kept between calls, per device.  A call takes chunks
// at its start and gives them back only after its final stream
// synchronisation, so a chunk is never in use by two calls.  Chunk sizes are
// powers of two (at least 64 MiB), so a chunk fits any later request of up to
// its size.  The cache lives until the process ends.  An optional limit caps
// the bytes a device's chunks hold (cached or lent): a new chunk that would
// pass it first makes the cache free its idle chunks, and fails when that is
// not enough.  A failed hipMalloc also frees the idle chunks and tries once
// more.
class ChunkCache {
 public:
  static ChunkCache &get() {
    static ChunkCache c;
    return c;
  }
  void *take(int dev, uint64_t size) {
    std::lock_guard<std::mutex> lk(mu_);
    const int d = dev & 63;
    auto &v = free_[d];
    for (size_t k = 0; k < v.size(); ++k)
      if (v[k].size == size) {
        void *p = v[k].ptr;
        v[k] = v.back();
        v.pop_back();
        return p;
      }
    if (limit_ && held_[d] + size > limit_) release_idle(d);
    if (limit_ && held_[d] + size > limit_) return nullptr;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      release_idle(d);
      p = nullptr;
      e = hipMalloc(&p, size);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    held_[d] += size;
    return p;
  }
  void give(int dev, void *p, uint64_t size) {
    std::lock_guard<std::mutex> lk(mu_);
    const int d = dev & 63;
    free_[d].push_back({p, size});
    if (limit_ && held_[d] > limit_) release_idle(d);
  }
  // Sets the limit (0: none) and returns what the current device's chunks
  // hold; idle chunks beyond a new limit are freed.
  uint64_t limit(uint64_t bytes, int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    limit_ = bytes;
    const int d = dev & 63;
    if (limit_ && held_[d] > limit_) release_idle(d);
    return held_[d];
  }

 private:
  struct Chunk {
    void *ptr;
    uint64_t size;
  };
  // Frees the idle chunks of device d (the current device).  hipFree waits
  // for the device, so this happens only when memory runs short.
  void release_idle(int d) {
    for (auto &c : free_[d]) {
      (void)hipFree(c.ptr);
      held_[d] -= c.size;
    }
    free_[d].clear();
  }
  std::mutex mu_;
  std::vector<Chunk> free_[64];
  uint64_t held_[64] = {};
  uint64_t limit_ = 0;
};

// Bump allocator over device memory chunks.  A call's arena takes cached
// chunks and returns them when it ends, after synchronising its stream; an
// owned arena (a resident index) allocates its own and frees them when it is
// destroyed (hipFree waits for the device).  A fixed arena hands out one
// region the caller provides and never allocates: a request beyond the
// region fails with SSJ_E_UNSUPPORTED.
class Arena {
 public:
  explicit Arena(hipStream_t st, bool owned = false) : st_(st), owned_(owned) {
    if (hipGetDevice(&dev_) != hipSuccess) dev_ = 0;
  }
  Arena(hipStream_t st, void *region, uint64_t size)
      : st_(st), owned_(false), fixed_(true), next_(static_cast<char *>(region)), left_(size) {
    if (hipGetDevice(&dev_) != hipSuccess) dev_ = 0;
  }
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  ~Arena() {
    if (!owned_) (void)hipStreamSynchronize(st_);
    for (auto &c : chunks_) {
      if (owned_) (void)hipFree(c.first);
      else ChunkCache::get().give(dev_, c.first, c.second);
    }
    // an owned arena's work has finished by now: its owner synchronised
    // after the uploads, and hipFree waits for the device
    for (void *p : staged_) HostPairs::get().release(p);
  }
  // Host memory for an upload from this arena's stream: page-locked when
  // large (the copy then runs asynchronously, without a staged copy that
  // waits for the work queued before it), kept until the arena ends.
  template <class T>
  T *stage(uint64_t n) {
    const uint64_t bytes = std::max<uint64_t>(n, 1) * sizeof(T);
    void *p = HostPairs::get().alloc((bytes + sizeof(ssj_pair) - 1) / sizeof(ssj_pair));
    if (!p) throw std::bad_alloc();
    staged_.push_back(p);
    return static_cast<T *>(p);
  }
  template <class T>
  T *alloc(uint64_t n) {
    uint64_t bytes = (std::max<uint64_t>(n, 1) * sizeof(T) + 255) & ~255ull;
    if (bytes > left_) {
      if (fixed_) throw Fail{SSJ_E_UNSUPPORTED};
      uint64_t size = owned_ ? std::max<uint64_t>(bytes, kOwnedChunk) : kChunk;
      if (!owned_)
        while (size < bytes) size <<= 1;
      void *p = nullptr;
      if (owned_) {
        if (hipMalloc(&p, size) != hipSuccess) {
          (void)hipGetLastError();
          p = nullptr;
        }
      } else {
        p = ChunkCache::get().take(dev_, size);
      }
      if (!p) throw Fail{SSJ_E_NOMEM};
      chunks_.push_back({p, size});
      next_ = static_cast<char *>(p);
      left_ = size;
    }
    T *out = reinterpret_cast<T *>(next_);
    next_ += bytes;
    left_ -= bytes;
    return out;
  }
  int device() const { return dev_; }

 private:
  static constexpr uint64_t kChunk = 64ull << 20;
  static constexpr uint64_t kOwnedChunk = 16ull << 20;
  hipStream_t st_;
  bool owned_;
  bool fixed_ = false;
  int dev_ = 0;
  std::vector<std::pair<void *, uint64_t>> chunks_;
  std::vector<void *> staged_;  // host upload buffers (HostPairs)
  char *next_ = nullptr;
  uint64_t left_ = 0;
};

template <class T>
void d2h(T *dst, const T *src, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  check(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}
// The counters the host reads sit before the tile cursors: copy only those.
template <>
void d2h<JoinCounters>(JoinCounters *dst, const JoinCounters *src, uint64_t n, hipStream_t st) {
  if (n != 1) throw Fail{SSJ_E_DEVICE};
  check(hipMemcpyAsync(dst, src, offsetof(JoinCounters, tile_next), hipMemcpyDeviceToHost, st));
}
template <class T>
void h2d(T *dst, const T *src, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  check(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, st));
}
void sync(hipStream_t st) { check(hipStreamSynchronize(st)); }

// Device work whose inputs are the caller's tokens (bitmaps, sign planes,
// the filter and verification of a join's first round): launched at once,
// or recorded in order so that a prepared join can replay it from a HIP
// graph (work that depends only on the set sizes runs when it is planned).
class Launcher {
 public:
  explicit Launcher(bool record) : record_(record) {}
  bool recording() const { return record_; }
  void run(hipStream_t st, std::function<hipError_t(hipStream_t)> f) {
    if (record_) ops_.push_back(std::move(f));
    else check(f(st));
  }
  void replay(hipStream_t st) const {
    for (const auto &f : ops_) check(f(st));
  }

 private:
  bool record_;
  std::vector<std::function<hipError_t(hipStream_t)>> ops_;
};

// Runs f on st now, or records it when L records.
inline void go(Launcher *L, hipStream_t st, std::function<hipError_t(hipStream_t)> f) {
  if (L) L->run(st, std::move(f));
  else check(f(st));
}

int bits_for(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

void validate_sets(const ssj_sets *s) {
  if (!s) throw Fail{SSJ_E_INVALID};
  if (s->n_sets >= 0xFFFFFFFFull) throw Fail{SSJ_E_INVALID};
  if (s->n_sets > 0 && !s->offsets) throw Fail{SSJ_E_INVALID};
  if (s->n_tokens > 0 && !s->tokens) throw Fail{SSJ_E_INVALID};
  if (s->n_sets == 0 && s->n_tokens != 0) throw Fail{SSJ_E_INVALID};
}

// ------------------------------------------------------------------ spaces

// Sides laid out one after the other, validated and in size order per side.
struct Space {
  std::vector<SideDesc> h_sides;
  SideDesc *d_sides = nullptr;
  uint32_t n_sides = 0;
  uint64_t n = 0;                 // sets over all sides
  uint32_t max_size = 0;          // over all sides
  uint32_t stride = 2;            // group-start entries per side: max_size + 2
  uint32_t seg_blocks = 0;        // workgroups of the segmented bitmap build
  uint32_t *sizes = nullptr;      // size order, per side
  uint32_t *perm = nullptr;       // size-order position -> caller index in the side
  uint32_t *rank = nullptr;       // global caller position -> size-order position
  uint32_t *side_of = nullptr;    // side of every global position
  uint32_t *sstart = nullptr;     // [n_sides][stride]
  std::vector<uint32_t> sstart_h;
  std::vector<uint32_t> side_max; // largest size of each side
  JoinCounters *ctr = nullptr;    // preparation counters
  JoinCounters ctr_h{};
  // bitmaps in size order, one array per width
  uint32_t n_bm = 0;
  // a build of every set (which checks the token order) is enqueued
  bool checked = false;
  uint32_t bm_words[kMaxClasses] = {};
  uint64_t *bm[kMaxClasses] = {};
  // sign planes of the bitmaps (matrix-core filter), beside bm[k]
  uint4 *sg[kMaxClasses] = {};
  // wide bitmaps of the sets larger than kWideMin (verification)
  bool wide_built = false;
  uint64_t *bmw = nullptr;
  uint32_t *wide_lo = nullptr, *wide_slot = nullptr;  // per side

  const uint32_t *ss(uint32_t s) const { return sstart_h.data() + (size_t)s * stride; }
  const uint64_t *bitmaps(uint32_t words) const {
    for (uint32_t k = 0; k < n_bm; ++k)
      if (bm_words[k] == words) return bm[k];
    return nullptr;
  }
  const uint4 *signs(uint32_t words) const {
    for (uint32_t k = 0; k < n_bm; ++k)
      if (bm_words[k] == words) return sg[k];
    return nullptr;
  }
};

// Side table, sizes and offset checks of every side.  The caller
// synchronises before space_sort (ctr_h holds the largest size).
void space_begin(Space &sp, const ssj_sets *const *sides, uint32_t n_sides, Arena &ar,
                 hipStream_t st) {
  sp.n_sides = n_sides;
  sp.h_sides.resize(n_sides);
  uint64_t base = 0, blk = 0;
  for (uint32_t s = 0; s < n_sides; ++s) {
    validate_sets(sides[s]);
    SideDesc &d = sp.h_sides[s];
    d.offsets = sides[s]->offsets;
    d.tokens = sides[s]->tokens;
    d.n_tokens = sides[s]->n_tokens;
    d.base = base;
    d.n = (uint32_t)sides[s]->n_sets;
    d.blk0 = (uint32_t)blk;
    base += d.n;
    blk += bitmap_seg_blocks(d.n);
  }
  if (base >= 0xFFFFFFFFull || blk >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};
  sp.n = base;
  sp.seg_blocks = (uint32_t)blk;
  sp.d_sides = ar.alloc<SideDesc>(n_sides);
  h2d(sp.d_sides, sp.h_sides.data(), n_sides, st);
  sp.ctr = ar.alloc<JoinCounters>(1);
  check(launch_reset_all(sp.ctr, st));
  sp.sizes = ar.alloc<uint32_t>(sp.n);
  sp.side_of = ar.alloc<uint32_t>(sp.n);
  check(launch_set_sizes(sp.d_sides, n_sides, sp.n, sp.sizes, sp.side_of, sp.ctr, st));
  d2h(&sp.ctr_h, sp.ctr, 1, st);
}

// Stable sort by (side, size), group starts of every side (copied to the
// host; the caller synchronises before space_finish), and the inverse
// permutation when bitmaps are to be built.
// Arrays the space keeps come from `ar`, the sort's temporaries from `tmp_ar`.
void space_sort(Space &sp, bool need_rank, Arena &ar, Arena &tmp_ar, hipStream_t st) {
  if (sp.ctr_h.error & (kErrOffsets | kErrTooBig)) throw Fail{SSJ_E_INVALID};
  sp.max_size = sp.ctr_h.max_size;
  if ((uint64_t)sp.max_size * 2 + 2 > kMaxTable) throw Fail{SSJ_E_UNSUPPORTED};
  sp.stride = sp.max_size + 2;
  const int size_bits = std::max(1, bits_for(sp.max_size));
  const int side_bits = bits_for(sp.n_sides ? sp.n_sides - 1 : 0);
  if (size_bits + side_bits > 32) throw Fail{SSJ_E_UNSUPPORTED};
  const uint64_t n = sp.n;
  sp.perm = ar.alloc<uint32_t>(n);
  if (n) {
    unsigned long long *keys = tmp_ar.alloc<unsigned long long>(n);
    unsigned long long *tmp = tmp_ar.alloc<unsigned long long>(n);
    uint32_t *scr = tmp_ar.alloc<uint32_t>(radix_scratch_words(n));
    check(launch_make_keys(sp.d_sides, sp.sizes, sp.side_of, n, size_bits, keys, st));
    int shifts[4], ns = 0;
    for (int b = 0; b < size_bits + side_bits; b += 8) shifts[ns++] = 32 + b;
    unsigned long long *sorted = keys;
    check(radix_sort_u64(keys, tmp, n, shifts, ns, scr, st, &sorted));
    check(launch_unpack_keys(sorted, n, size_bits, sp.sizes, sp.perm, st));
  }
  sp.sstart = ar.alloc<uint32_t>((uint64_t)sp.n_sides * sp.stride);
  check(launch_group_starts(sp.d_sides, sp.sizes, sp.side_of, n, sp.max_size, sp.stride,
                            sp.n_sides, sp.sstart, st));
  if (need_rank) {
    sp.rank = ar.alloc<uint32_t>(n);
    check(launch_invert_perm(sp.d_sides, sp.perm, sp.side_of, n, sp.rank, st));
  }
  sp.sstart_h.assign((size_t)sp.n_sides * sp.stride, 0);
  d2h(sp.sstart_h.data(), sp.sstart, sp.sstart_h.size(), st);
}

// Largest size of every side, from its group starts.
void space_finish(Space &sp) {
  sp.side_max.assign(sp.n_sides, 0);
  for (uint32_t s = 0; s < sp.n_sides; ++s) {
    const uint32_t *t = sp.ss(s);
    const uint32_t n = sp.h_sides[s].n;
    uint32_t m = 0;
    for (uint32_t v = 1; v <= sp.max_size; ++v)
      if (t[v] < n) m = v;
    sp.side_max[s] = m;
  }
}

// Bitmap-Xor bitmaps of every set at `words` 64-bit words (nominal width
// `bits`), in size order.
void space_bitmaps(Space &sp, uint32_t words, uint32_t bits, Arena &ar, JoinCounters *ctr,
                   hipStream_t st, Launcher *L = nullptr) {
  if (sp.bitmaps(words)) return;
  if (sp.n_bm >= kMaxClasses) throw Fail{SSJ_E_DEVICE};
  uint64_t *out = ar.alloc<uint64_t>(sp.n * words);
  const SideDesc *sides = sp.d_sides;
  const uint32_t n_sides = sp.n_sides, seg = sp.seg_blocks;
  const uint64_t n = sp.n;
  const uint32_t *perm = sp.perm, *rank = sp.rank, *side_of = sp.side_of;
  go(L, st, [=](hipStream_t s) {
    return launch_build_bitmaps(sides, n_sides, seg, n, perm, rank, side_of, bits, SSJ_BM_XOR,
                                words, out, ctr, s);
  });
  sp.bm_words[sp.n_bm] = words;
  sp.bm[sp.n_bm] = out;
  ++sp.n_bm;
  sp.checked = true;
}

// Sign planes of the space's bitmaps at `words` words (built before): of
// every set, or only of the positions in `ranges` (the other planes stay
// unwritten, so only those positions may be read).
void space_signs(Space &sp, uint32_t words, Arena &ar, hipStream_t st, Launcher *L = nullptr,
                 const std::vector<PosRange> *ranges = nullptr) {
  for (uint32_t k = 0; k < sp.n_bm; ++k) {
    if (sp.bm_words[k] != words) continue;
    if (sp.sg[k]) return;
    uint4 *planes = ar.alloc<uint4>((sp.n + kSignPad) * words * 2);
    const uint64_t *bm = sp.bm[k];
    const uint64_t n = sp.n;
    if (ranges && !ranges->empty()) {
      const PosRange *d_ranges = nullptr;
      PosRange *up = ar.alloc<PosRange>(ranges->size());
      h2d(up, ranges->data(), ranges->size(), st);
      d_ranges = up;
      const uint32_t nr = (uint32_t)ranges->size();
      const uint64_t total = (uint64_t)ranges->back().first + kSignPad;
      go(L, st, [=](hipStream_t s) {
        return launch_expand_signs_ranges(bm, words, n, d_ranges, nr, total, planes, s);
      });
    } else {
      go(L, st, [=](hipStream_t s) { return launch_expand_signs(bm, words, n, planes, s); });
    }
    sp.sg[k] = planes;
    return;
  }
  throw Fail{SSJ_E_DEVICE};
}

// Wide bitmaps of every set larger than kWideMin: in size order they are a
// suffix of each side (from its group start at kWideMin + 1).  The host
// only sizes the array; the ranges are made on the device from the group
// starts, so that nothing is copied up (a copy from pageable memory could
// wait for the work already queued).
void space_wide(Space &sp, Arena &ar, hipStream_t st, Launcher *L = nullptr) {
  if (sp.wide_built) return;
  sp.wide_built = true;
  uint64_t total = 0;
  if ((uint64_t)kWideMin + 1 <= (uint64_t)sp.max_size)
    for (uint32_t s = 0; s < sp.n_sides; ++s) {
      const uint32_t n = sp.h_sides[s].n, first = std::min(sp.ss(s)[kWideMin + 1], n);
      total += n - first;
    }
  if (total == 0) return;
  if (total >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};
  sp.wide_lo = ar.alloc<uint32_t>(2 * (uint64_t)sp.n_sides);
  sp.wide_slot = sp.wide_lo + sp.n_sides;
  WideRange *d_ranges = ar.alloc<WideRange>(sp.n_sides);
  check(launch_wide_ranges(sp.d_sides, sp.n_sides, sp.sstart, sp.stride, sp.max_size, d_ranges,
                           sp.wide_lo, sp.wide_slot, st));
  sp.bmw = ar.alloc<uint64_t>(total * kWideWords);
  const SideDesc *sides = sp.d_sides;
  const uint32_t *perm = sp.perm, n_ranges = sp.n_sides;
  uint64_t *bmw = sp.bmw;
  go(L, st, [=](hipStream_t s) {
    return launch_build_wide(sides, perm, d_ranges, n_ranges, total, bmw, s);
  });
}

// Bitmap-Xor bitmaps at several widths.  Power-of-two widths of up to
// kMaxFoldWords words come from one pass over the tokens: the widest is
// built and the narrower ones are folded from it in the same kernel.
void space_bitmaps_multi(Space &sp, const uint32_t *words, const uint32_t *bits, uint32_t n,
                         Arena &ar, JoinCounters *ctr, hipStream_t st, Launcher *L = nullptr) {
  uint32_t need_w[kMaxClasses + 1], need_b[kMaxClasses + 1], m = 0, wmax = 0;
  for (uint32_t k = 0; k < n; ++k) {
    if (sp.bitmaps(words[k])) continue;
    const bool fold = sp.rank != nullptr && (words[k] & (words[k] - 1)) == 0 &&
                      words[k] <= kMaxFoldWords && bits[k] == 64 * words[k];
    if (!fold) {
      // wider than a fold allows: a pass of its own
      space_bitmaps(sp, words[k], bits[k], ar, ctr, st, L);
      continue;
    }
    need_w[m] = words[k];
    need_b[m] = bits[k];
    wmax = std::max(wmax, words[k]);
    ++m;
  }
  if (m == 0) return;
  if (m == 1 || sp.n_bm + m > kMaxClasses) {
    for (uint32_t k = 0; k < m; ++k) space_bitmaps(sp, need_w[k], need_b[k], ar, ctr, st, L);
    return;
  }
  FoldOut fold{};
  uint64_t *widest = ar.alloc<uint64_t>(sp.n * wmax);
  for (uint32_t k = 0; k < m; ++k) {
    uint64_t *dst = widest;
    if (need_w[k] != wmax) {
      dst = ar.alloc<uint64_t>(sp.n * need_w[k]);
      uint32_t f = 0;
      while ((wmax >> (f + 1)) != need_w[k]) ++f;
      fold.out[f] = dst;
    }
    sp.bm_words[sp.n_bm] = need_w[k];
    sp.bm[sp.n_bm] = dst;
    ++sp.n_bm;
  }
  const SideDesc *sides = sp.d_sides;
  const uint32_t n_sides = sp.n_sides, seg = sp.seg_blocks;
  const uint64_t nn = sp.n;
  const uint32_t *perm = sp.perm, *rank = sp.rank, *side_of = sp.side_of;
  go(L, st, [=](hipStream_t s) {
    FoldOut f = fold;
    return launch_build_bitmaps(sides, n_sides, seg, nn, perm, rank, side_of, 64 * wmax,
                                SSJ_BM_XOR, wmax, widest, ctr, s, &f);
  });
  sp.checked = true;
}

// Bitmap-Xor bitmaps at the power-of-two widths `words` (more than
// kCascadeWords, at most kMaxFoldWords words) of only the sets whose size
// lies in their side's window, in one pass: the widest is built and the
// others folded from it.  The arrays span the space; rows of the other sets
// stay unwritten, so only the sets inside the windows may be read.  Needs a
// build of every set enqueued before (it checks the token order).
void space_bitmaps_window(Space &sp, const uint32_t *words, uint32_t n,
                          const std::vector<SizeWindow> &win, Arena &ar, hipStream_t st,
                          Launcher *L) {
  if (!sp.checked || !sp.rank || win.size() != sp.n_sides || sp.n_bm + n > kMaxClasses)
    throw Fail{SSJ_E_DEVICE};
  uint32_t wmax = 0;
  for (uint32_t k = 0; k < n; ++k) wmax = std::max(wmax, words[k]);
  FoldOut fold{};
  uint64_t *widest = ar.alloc<uint64_t>(sp.n * wmax);
  for (uint32_t k = 0; k < n; ++k) {
    uint64_t *dst = widest;
    if (words[k] != wmax) {
      dst = ar.alloc<uint64_t>(sp.n * words[k]);
      uint32_t f = 0;
      while ((wmax >> (f + 1)) != words[k]) ++f;
      fold.out[f] = dst;
    }
    sp.bm_words[sp.n_bm] = words[k];
    sp.bm[sp.n_bm] = dst;
    ++sp.n_bm;
  }
  SizeWindow *d_win = ar.alloc<SizeWindow>(sp.n_sides);
  h2d(d_win, win.data(), sp.n_sides, st);
  const SideDesc *sides = sp.d_sides;
  const uint32_t n_sides = sp.n_sides, seg = sp.seg_blocks;
  const uint64_t nn = sp.n;
  const uint32_t *rank = sp.rank;
  go(L, st, [=](hipStream_t s) {
    FoldOut f = fold;
    return launch_build_bitmaps_window(sides, n_sides, seg, nn, rank, d_win, wmax, widest, &f,
                                       s);
  });
}

// The caller's bitmaps of a one-side space (caller order, bits/64 words),
// gathered into size order and padded to `words`.
void space_caller_bitmaps(Space &sp, const uint64_t *bm_caller, uint32_t words, uint32_t bits,
                          Arena &ar, JoinCounters *ctr, hipStream_t st) {
  uint64_t *out = ar.alloc<uint64_t>(sp.n * words);
  check(launch_gather_bitmaps(bm_caller, sp.perm, sp.n, bits / 64, words, out, st));
  check(launch_check_sorted(sp.h_sides[0].offsets, sp.h_sides[0].tokens, sp.n, ctr, st));
  sp.bm_words[0] = words;
  sp.bm[0] = out;
  sp.n_bm = 1;
  sp.checked = true;
}

// ------------------------------------------------------------- thresholds
inline uint64_t ceil_div(uint64_t x, uint64_t y) { return (x + y - 1) / y; }

// Least overlap o with sim >= p/q (Table 1, integer forms) for the
// functions where it depends on L = |r| + |s| only:
//   Jaccard  o / (L - o) >= p / q  <=>  (p + q) o >= p L
//   Dice     2 o / L >= p / q      <=>  2 q o >= p L
//   Overlap  o >= p / q            <=>  q o >= p
inline uint32_t omin_of_sum(int sim, uint64_t L, uint64_t p, uint64_t q) {
  switch (sim) {
    case SSJ_SIM_DICE: return (uint32_t)ceil_div(p * L, 2 * q);
    case SSJ_SIM_OVERLAP: return (uint32_t)ceil_div(p, q);
    default: return (uint32_t)ceil_div(p * L, p + q);
  }
}

// Least overlap for row size a and column size c, any function.
inline uint32_t omin_of(int sim, uint64_t a, uint64_t c, uint64_t p, uint64_t q) {
  if (sim == SSJ_SIM_COSINE) return cosine_omin((uint32_t)a, (uint32_t)c, (uint32_t)p, (uint32_t)q);
  return omin_of_sum(sim, a + c, p, q);
}

// Column sizes [lo, hi] that can reach the threshold with a row of size
// a >= 1 (Table 2: the best case o = min(|r|, |s|), solved for |s|):
//   Jaccard  p a / q <= c <= q a / p
//   Dice     p a / (2q - p) <= c <= (2q - p) a / p
//   Cosine   p^2 a / q^2 <= c <= q^2 a / p^2
//   Overlap  c >= p / q when a >= p / q; nothing otherwise
void size_band(int sim, uint64_t a, uint64_t p, uint64_t q, uint64_t &lo, uint64_t &hi) {
  typedef unsigned __int128 u128;
  auto clamp = [](u128 v) { return v > (u128)UINT64_MAX ? UINT64_MAX : (uint64_t)v; };
  switch (sim) {
    case SSJ_SIM_DICE:
      lo = ceil_div(p * a, 2 * q - p);
      hi = (2 * q - p) * a / p;
      break;
    case SSJ_SIM_COSINE: {
      const u128 pp = (u128)p * p, qq = (u128)q * q;
      lo = clamp((pp * a + qq - 1) / qq);
      hi = clamp(qq * a / pp);
      break;
    }
    case SSJ_SIM_OVERLAP: {
      const uint64_t o = ceil_div(p, q);
      if (a < o) {
        lo = UINT64_MAX;
        hi = 0;
      } else {
        lo = o;
        hi = UINT64_MAX;
      }
      break;
    }
    default:
      lo = ceil_div(p * a, q);
      hi = q * a / p;
      break;
  }
  lo = std::max<uint64_t>(lo, 1);
}

// P(X <= k) for X ~ Binomial(n, pi) with pi <= 1/2, summed in log space
// over the terms within 12 standard deviations of the mean.  By Chernoff's
// bound the lower tail beyond that holds less than exp(-36) of the mass
// (pi <= 1/2); the upper tail's share is also small next to what a cost
// model can use, so a k beyond either end gives 0 or 1.
double binomial_cdf(int n, double pi, int64_t k) {
  if (k < 0) return 0.0;
  if (k >= n) return 1.0;
  if (pi <= 0.0) return 1.0;
  if (pi >= 1.0) return 0.0;
  const double mean = n * pi, sd = std::sqrt(n * pi * (1.0 - pi));
  if ((double)k < mean - 12.0 * sd) return 0.0;
  if ((double)k > mean + 12.0 * sd) return 1.0;
  const int64_t i0 = std::max<int64_t>(0, (int64_t)std::floor(mean - 12.0 * sd));
  const double lp = std::log(pi), lq = std::log1p(-pi);
  double lc = std::lgamma(n + 1.0) - std::lgamma(i0 + 1.0) - std::lgamma((double)(n - i0) + 1.0);
  double acc = 0.0;
  for (int64_t i = i0; i <= k; ++i) {
    if (i > i0) lc += std::log((double)(n - i + 1)) - std::log((double)i);
    acc += std::exp(lc + i * lp + (n - i) * lq);
  }
  return std::min(acc, 1.0);
}

// Width classes for the automatic mode.  For a row of size a against columns
// of about its size (L = 2a), model the bits in which the bitmaps of two
// unrelated sets differ as Binomial(b, pi) with pi = (1 - (1 - 2/b)^L) / 2,
// the chance that a bit receives an odd number of the L tokens (the quantity
// Eq. 5 sums; Section 3.4).  A pair is a false survivor when that count is at
// most slack(L), with probability P.  The filter leaves its fast path for a
// step of s pairs (kPairsPerStep of the width's kernel) that keeps any pair,
// with probability 1 - (1 - P)^s, and every survivor costs queue writes and
// a verification.  So a band pair at width b is expected to cost
//   filter(b) + (1 - (1 - P)^s) * entry / s + P * survivor,
// with the costs measured on the GPU (calibrate.py writes them to
// autotune_table.h): the filter's time per band pair at each width, the time
// of a slow-path entry, the time a survivor adds, and the fixed cost of a
// width class's launch.  The survivor's time is a throughput figure, right
// when the survivors spread over the whole grid; the survivors of a size
// whose rows fill few tiles are staged by the few waves that own those
// tiles, one after the other, and the class waits for them.  So a survivor
// costs at least the time one wave takes to stage it at that width (measured
// too) divided by the tiles of its size (row tiles times column tiles of the
// width's tile shape, at most the grid's waves).  The widths b(a), b in {64, ..., 2048} and never decreasing with
// the size, are the ones that minimise the task's expected time: the sum over
// row sizes of band(a) times that cost, plus the launch cost of every width
// used, band(a) being the task's band pairs of rows of size a.  A dynamic
// program over the sizes finds them.
constexpr int kNumAuto = 6;
constexpr uint32_t kAutoWords[kNumAuto] = {1, 2, 4, 8, 16, 32};  // b = 64 .. 2048
// the width the verification's cascade test uses (built with the classes)
constexpr uint32_t kCascadeWords = 8;
static_assert(sizeof(kFilterNsPerPair) / sizeof(double) == kNumAuto, "one cost per width");
static_assert(kNumAuto <= (int)kMaxClasses, "every automatic width fits a slot");

struct WidthClass {
  uint32_t max_size;  // rows of size in (previous max_size, max_size]
  uint32_t words;
};

// Per row size a and automatic width: P, the chance of a false survivor,
// and the part of a band pair's cost that does not depend on the task
// (filter time and slow-path entries).
struct SizeOdds {
  std::array<double, kNumAuto> p{}, base{};
};

// SizeOdds of every size up to max_rows, per (function, threshold), kept
// and extended as larger sizes come up.
std::shared_ptr<const std::vector<SizeOdds>> false_survivor_odds(uint32_t max_rows, int sim,
                                                                 uint64_t p, uint64_t q) {
  static std::mutex mu;
  static std::map<std::pair<int, std::pair<uint64_t, uint64_t>>,
                  std::shared_ptr<const std::vector<SizeOdds>>>
      memo;
  std::lock_guard<std::mutex> lk(mu);
  std::shared_ptr<const std::vector<SizeOdds>> &slot = memo[{sim, {p, q}}];
  if (slot && slot->size() > max_rows) return slot;  // shared, never copied: many tasks read it
  // a longer table replaces the shorter one; tasks that hold the old one keep it
  auto grown = std::make_shared<std::vector<SizeOdds>>();
  if (slot) *grown = *slot;
  std::vector<SizeOdds> &v = *grown;
  if (v.empty()) v.push_back({});  // size 0: never pairs
  for (uint32_t a = (uint32_t)v.size(); a <= max_rows; ++a) {
    const uint64_t L = 2ull * a;
    const int64_t slack = (int64_t)L - 2 * (int64_t)omin_of(sim, a, a, p, q);
    SizeOdds o;
    for (int k = 0; k < kNumAuto; ++k) {
      const double b = 64.0 * kAutoWords[k];
      const double pi = 0.5 * (1.0 - std::pow(1.0 - 2.0 / b, (double)L));
      const double P = binomial_cdf((int)b, pi, slack), s = kPairsPerStep[k];
      const double step_hit = -std::expm1(s * std::log1p(-std::min(P, 1.0 - 1e-16)));
      o.p[k] = P;
      o.base[k] = kFilterNsPerPair[k] + step_hit * kSlowEntryNs / s;
    }
    v.push_back(o);
  }
  slot = grown;
  return slot;
}

// A task's rows of one size: their band pairs and their number.
struct SizeLoad {
  double band = 0, rows = 0;
};

// The width classes of a task whose rows of size a are load[a]
// (a = 0 .. load.size() - 1).  The dynamic program steps over the sizes that
// hold rows: a width change at an empty size costs what it costs at the next
// size with rows.
std::vector<WidthClass> choose_classes(const std::vector<SizeLoad> &load, int sim, uint64_t p,
                                       uint64_t q, double waves) {
  const uint32_t n = std::max<uint32_t>((uint32_t)load.size() - 1, 1);
  const auto odds_table = false_survivor_odds(n, sim, p, q);
  const std::vector<SizeOdds> &odds = *odds_table;
  // tile shape of each width's kernel (waves: the waves of a filter grid)
  double tile_rows[kNumAuto], tile_cols[kNumAuto];
  for (int k = 0; k < kNumAuto; ++k) {
    const uint32_t w = kAutoWords[k];
    tile_rows[k] = std::max<uint32_t>(1, filter_shape(filter_padded_words(w), true).rows);
    tile_cols[k] = kClassTileCols[k];
  }
  std::vector<uint32_t> sizes;
  for (uint32_t a = 1; a <= n; ++a)
    if (a < load.size() && load[a].rows > 0) sizes.push_back(a);
  if (sizes.empty()) sizes.push_back(n);
  // best[i][k]: least cost of the sizes up to sizes[i], sizes[i] at width k
  std::vector<std::array<double, kNumAuto>> best(sizes.size());
  std::vector<std::array<int8_t, kNumAuto>> from(sizes.size());
  for (size_t i = 0; i < sizes.size(); ++i) {
    const uint32_t a = sizes[i];
    const double w = a < load.size() ? load[a].band : 0.0;
    const double rows = a < load.size() ? load[a].rows : 0.0;
    const double cols = rows > 0 ? w / rows : 0.0;  // band columns of a row
    for (int k = 0; k < kNumAuto; ++k) {
      const double tiles = std::min(waves, std::max(1.0, rows / tile_rows[k]) *
                                               std::max(1.0, std::ceil(cols / tile_cols[k])));
      const double surv = std::max(kSurvivorNs, kSurvivorWaveNs[k] / tiles);
      const double here = w * (odds[a].base[k] + odds[a].p[k] * surv);
      if (i == 0) {
        best[i][k] = here + kClassLaunchNs[k];
        from[i][k] = (int8_t)k;
        continue;
      }
      double b = best[i - 1][k];
      int8_t f = (int8_t)k;
      for (int j = 0; j < k; ++j)
        if (best[i - 1][j] + kClassLaunchNs[k] < b) {
          b = best[i - 1][j] + kClassLaunchNs[k];
          f = (int8_t)j;
        }
      best[i][k] = here + b;
      from[i][k] = f;
    }
  }
  const size_t last = sizes.size() - 1;
  int k = 0;
  for (int j = 1; j < kNumAuto; ++j)
    if (best[last][j] < best[last][k]) k = j;
  std::vector<uint32_t> width(sizes.size());
  for (size_t i = sizes.size(); i-- > 0;) {
    width[i] = kAutoWords[k];
    k = from[i][k];
  }
  // a class ends at the last size with rows before the next width; the
  // last class covers every size up to n
  std::vector<WidthClass> cls;
  for (size_t i = 0; i < sizes.size(); ++i) {
    if (!cls.empty() && cls.back().words == width[i]) cls.back().max_size = sizes[i];
    else cls.push_back({sizes[i], width[i]});
  }
  cls.back().max_size = n;
  return cls;
}

// Band pairs of a task's rows of each size (Table 2's length band; a
// self-join counts each unordered pair once, same-size pairs included), and
// the rows of each size.
std::vector<SizeLoad> band_by_size(const Space &R, const Space &C, int sim, uint64_t p,
                                   uint64_t q, uint32_t row_side, uint32_t col_side, bool self) {
  const uint32_t a_max = R.side_max[row_side], c_max = C.side_max[col_side];
  const uint32_t *rs = R.ss(row_side), *cs = C.ss(col_side);
  std::vector<SizeLoad> w((size_t)a_max + 1);
  for (uint32_t a = 1; a <= a_max; ++a) {
    const double nr = (double)rs[a + 1] - (double)rs[a];
    if (nr <= 0) continue;
    w[a].rows = nr;
    uint64_t lo = 0, hi = 0;
    size_band(sim, a, p, q, lo, hi);
    hi = std::min<uint64_t>(hi, c_max);
    if (self) hi = std::min<uint64_t>(hi, a);
    if (lo > hi) continue;
    if (self && hi == a) {
      w[a].band = nr * ((double)cs[a] - (double)cs[lo]) + nr * (nr - 1) / 2;
    } else {
      w[a].band = nr * ((double)cs[hi + 1] - (double)cs[lo]);
    }
  }
  return w;
}

// ------------------------------------------------------------ cutoff point
// The cutoff point of Section 3.5 rests on E(b, n) of Section 3.4, the
// expected bound of two sets of n random tokens (Eqs. 4-6), here in
// closed form: Eq. 5's sum over odd k is the odd half of a binomial
// expansion, (1 - (1 - 2/b)^(2n)) / 2, so E = n - (b/4)(1 - (1 - 2/b)^(2n)).
// The overlap fraction o/n two n-sets need for sim >= p/q, as P/Q: Jaccard
// 2t/(1+t) = 2p/(p+q), Dice and Cosine t = p/q.  False for Overlap, which has
// none.
bool normalized_threshold(int sim, uint64_t p, uint64_t q, uint64_t &P, uint64_t &Q) {
  if (sim == SSJ_SIM_JACCARD) {
    P = 2 * p;
    Q = p + q;
    return true;
  }
  if (sim == SSJ_SIM_DICE || sim == SSJ_SIM_COSINE) {
    P = p;
    Q = q;
    return true;
  }
  return false;
}

// Whether E(b, n)/n <= P/Q.  The part of E/n that is rational is compared
// in integers, so that thresholds it meets exactly are decided exactly:
//   Xor   E/n - P/Q = [4n(Q-P) - bQ] / (4nQ) + (b/4n) r^(2n),  r = 1 - 2/b
//   Set   E/n - P/Q = (Q-P)/Q - (b/n) (s^n - s^(2n)),           s = 1 - 1/b
//   Next  E/n = n/b below saturation
bool bound_within(int method, uint64_t b, uint64_t n, uint64_t P, uint64_t Q) {
  if (P >= Q) return true;  // a normalized bound never exceeds 1
  switch (method) {
    case SSJ_BM_NEXT:
      return n <= b && n * Q <= P * b;
    case SSJ_BM_SET: {
      const double sn = std::pow(1.0 - 1.0 / (double)b, (double)n);
      return (double)(Q - P) / (double)Q <= (double)b / (double)n * (sn - sn * sn);
    }
    default: {
      const int64_t num = (int64_t)(4 * n * (Q - P)) - (int64_t)(b * Q);
      if (num >= 0) return false;  // the remaining term is positive
      const double r2n = std::pow(1.0 - 2.0 / (double)b, 2.0 * (double)n);
      return (double)b * (double)Q * r2n <= (double)(-num);
    }
  }
}

// Bitmap-Combined (Alg. 6, Section 3.5) for a normalized threshold P/Q:
// Bitmap-Next when P/Q <= 14/25 (0.56), Bitmap-Xor when P/Q >= 73/100,
// Bitmap-Set in between.
int combined_generator(uint64_t P, uint64_t Q) {
  if (25 * P <= 14 * Q) return SSJ_BM_NEXT;
  if (100 * P >= 73 * Q) return SSJ_BM_XOR;
  return SSJ_BM_SET;
}

// The largest n with E(b, n)/n <= tau (E/n grows with n), up to 2^20; the
// filter is applied to sets up to this size (Alg. 7).  UINT32_MAX: never
// cut off (Overlap).  Bitmap-Combined takes the curve of the generator it
// picks for tau.
uint32_t cutoff_point(int method, uint32_t b, int sim, uint64_t p, uint64_t q) {
  uint64_t P = 0, Q = 1;
  if (!normalized_threshold(sim, p, q, P, Q)) return 0xFFFFFFFFu;
  if (method == SSJ_BM_COMBINED) method = combined_generator(P, Q);
  auto ok = [&](uint64_t n) { return bound_within(method, b, n, P, Q); };
  if (!ok(1)) return 0;
  uint64_t lo = 1, hi = 1ull << 20;
  if (ok(hi)) return (uint32_t)hi;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) / 2;
    if (ok(mid)) lo = mid; else hi = mid;
  }
  return (uint32_t)lo;
}

// ------------------------------------------------------------------- plan

// One task of a call, as planned on the host (p/q reduced).
struct TaskIn {
  uint32_t row_side;
  uint32_t col_side;
  int sim;
  uint32_t p, q;
  bool self;
};

struct Plan {
  std::vector<uint32_t> tables;  // slack / omin / cmin / cmax of every task
  std::vector<TaskDesc> tasks;
  std::vector<RowBlock> blocks;
  uint32_t n_tiles = 0;
  uint64_t band_pairs = 0;
  uint64_t filter_ops = 0;       // sum over band pairs of b/16 + 1
  bool mfma = true;              // matrix-core filter where it exists (row block height)
  // per width slot: its tiles [tile_lo[k], tile_hi[k]), padded width, work,
  // and whether the matrix-core kernel runs it
  uint32_t n_slots = 0;
  bool slot_mfma[kMaxClasses] = {};
  uint32_t slot_words[kMaxClasses] = {};
  uint32_t slot_bits[kMaxClasses] = {};
  uint32_t slot_max_size[kMaxClasses] = {};
  uint32_t tile_lo[kMaxClasses] = {}, tile_hi[kMaxClasses] = {};
  uint32_t slot_tile_cols[kMaxClasses] = {};
  uint64_t ops[kMaxClasses] = {};
};

// Threshold tables for sizes up to a_max (rows) and c_max (columns),
// appended to pl.tables; their offsets and the function and threshold go
// into td.
void add_tables(Plan &pl, TaskDesc &td, uint64_t a_max, uint64_t c_max, int sim, uint64_t p,
                uint64_t q) {
  const uint64_t nL = sim == SSJ_SIM_COSINE ? 1 : a_max + c_max + 1, nA = a_max + 1;
  if (pl.tables.size() + 2 * nL + 2 * nA >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};
  // slack[L] = L - 2 omin(L); Cosine's depend on both sizes and are computed
  // where they are needed, its tables are one unused entry each
  td.slack_off = (uint32_t)pl.tables.size();
  for (uint64_t L = 0; L < nL; ++L)
    pl.tables.push_back(
        (uint32_t)(int32_t)((int64_t)L - 2 * (int64_t)omin_of_sum(sim, L, p, q)));
  td.omin_off = (uint32_t)pl.tables.size();
  for (uint64_t L = 0; L < nL; ++L) pl.tables.push_back(omin_of_sum(sim, L, p, q));
  // length filter; empty sets never pair: an empty row gets an empty range,
  // and cmin >= 1 otherwise
  td.cmin_off = (uint32_t)pl.tables.size();
  pl.tables.resize(pl.tables.size() + 2 * nA);
  td.cmax_off = td.cmin_off + (uint32_t)nA;
  for (uint64_t a = 0; a < nA; ++a) {
    uint64_t lo = UINT64_MAX, hi = 0;
    if (a) size_band(sim, a, p, q, lo, hi);
    pl.tables[td.cmin_off + a] = (uint32_t)std::min<uint64_t>(lo, 0xFFFFFFFFull);
    pl.tables[td.cmax_off + a] = (uint32_t)std::min<uint64_t>(hi, 0xFFFFFFFFull);
  }
  td.sim = (uint32_t)sim;
  td.p = (uint32_t)p;
  td.q = (uint32_t)q;
  td.pad = 0;
  (void)c_max;
}

// Row blocks and tiles of one task's length band for its rows of size in
// (lo, hi], which use `words`-word bitmaps of nominal width `bits`; blocks
// never straddle width classes.  With count_only, only the band pairs are
// added to band_out.
void plan_class(Plan &pl, const Space &R, const Space &C, const TaskIn &tk, uint32_t task_id,
                uint32_t lo, uint32_t hi, uint32_t words, uint32_t bits, uint32_t tile_cols,
                bool mfma, uint64_t &band_out, bool count_only = false) {
  const TaskDesc &td = pl.tasks[task_id];
  const uint32_t *rs = R.ss(tk.row_side), *cs = C.ss(tk.col_side);
  const uint64_t a_max = R.side_max[tk.row_side], c_max = C.side_max[tk.col_side];
  const uint32_t col_n = C.h_sides[tk.col_side].n;
  const uint32_t row_base = (uint32_t)R.h_sides[tk.row_side].base;
  const uint32_t col_base = (uint32_t)C.h_sides[tk.col_side].base;
  const uint32_t *cmin = pl.tables.data() + td.cmin_off;
  const uint32_t *cmax = pl.tables.data() + td.cmax_off;
  const FilterShape shape = filter_shape(words, mfma);
  auto col_lo = [&](uint64_t a) -> uint32_t {  // first column with size >= cmin[a]
    const uint64_t c = cmin[a];
    return c > c_max ? col_n : cs[c];
  };
  auto col_hi = [&](uint64_t a) -> uint32_t {  // first column with size > cmax[a]
    const uint64_t c = cmax[a];
    return c >= c_max ? col_n : cs[c + 1];
  };
  hi = (uint32_t)std::min<uint64_t>(hi, a_max);
  if (lo >= hi) return;
  // Sizes whose band is empty (Overlap: below ceil(p/q)) come first; the
  // class's row blocks start after them, so that every block's column range,
  // taken from its smallest size, is that of a size that pairs.
  auto empty_band = [&](uint64_t a) {
    return cmin[a] > cmax[a] || (tk.self && cmin[a] > a);
  };
  while (lo < hi && empty_band(lo + 1)) ++lo;
  if (lo >= hi) return;
  // band pairs of the class, exactly
  uint64_t band = 0;
  for (uint64_t a = lo + 1; a <= hi; ++a) {
    const uint64_t cnt = (uint64_t)rs[a + 1] - rs[a];
    if (!cnt || empty_band(a)) continue;
    if (tk.self) {
      band += cnt * ((uint64_t)rs[a] - col_lo(a)) + cnt * (cnt - 1) / 2;
    } else {
      const uint64_t l = col_lo(a), h = col_hi(a);
      if (h > l) band += cnt * (h - l);
    }
  }
  band_out += band;
  if (count_only) return;
  pl.band_pairs += band;
  pl.filter_ops += band * (bits / 16 + 1);

  const uint32_t rows_per_block = shape.rows;
  const uint32_t r_begin = rs[lo + 1], r_end = rs[hi + 1];
  uint64_t tiles = pl.n_tiles;
  uint32_t s_of = lo + 1;  // size of the current row, advanced monotonically
  auto size_at = [&](uint32_t row) {
    while (s_of + 1 <= hi && rs[s_of + 1] <= row) ++s_of;
    return s_of;
  };
  for (uint64_t r0 = r_begin; r0 < r_end; r0 += rows_per_block) {
    const uint32_t row0 = (uint32_t)r0;
    const uint32_t row_end = (uint32_t)std::min<uint64_t>(r0 + rows_per_block, r_end);
    const uint32_t a0 = size_at(row0);
    RowBlock rb{};
    rb.row0 = row_base + row0;
    rb.row_end = row_base + row_end;
    rb.tile_begin = (uint32_t)tiles;
    rb.task = task_id;
    rb.self = tk.self ? 1u : 0u;
    uint64_t nt;
    if (tk.self) {
      const uint32_t cb = std::min(col_lo(a0), row0);
      rb.col_begin = col_base + cb;
      rb.col_end = col_base + row_end;
      nt = ((uint64_t)row0 - cb + tile_cols - 1) / tile_cols + 1;
    } else {
      const uint32_t s_save = s_of;
      const uint32_t a1 = size_at(row_end - 1);  // the block's largest size
      s_of = s_save;
      const uint32_t cb = col_lo(a0);
      const uint32_t ce = std::max(col_hi(a1), cb);
      rb.col_begin = col_base + cb;
      rb.col_end = col_base + ce;
      nt = ((uint64_t)ce - cb + tile_cols - 1) / tile_cols;
    }
    tiles += nt;
    if (tiles >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};
    pl.blocks.push_back(rb);
  }
  pl.n_tiles = (uint32_t)tiles;
}

// Size of the set at size-order position pos (counted from the side's
// base) of side `side`: the largest v whose group starts at or before pos.
uint32_t size_at(const Space &X, uint32_t side, uint32_t pos) {
  const uint32_t *t = X.ss(side);
  uint32_t lo = 0, hi = X.max_size + 1;  // t[lo] <= pos < t[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (t[mid] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Positions [lo, hi) (counted from each side's base; lo > hi when none) of
// the sets that the row blocks of the width slots chosen by use(words) read,
// one hull per side of X: their rows when `rows` (X is the row space), their
// columns when `cols` (X is the column space).
template <class Use>
void block_hulls(const Plan &pl, const std::vector<TaskIn> &tasks, const Space &X, bool rows,
                 bool cols, const uint32_t *blk_lo, const uint32_t *blk_hi, Use use,
                 std::vector<uint32_t> &lo, std::vector<uint32_t> &hi) {
  lo.assign(X.n_sides, 0xFFFFFFFFu);
  hi.assign(X.n_sides, 0);
  auto add = [&](uint32_t side, uint32_t a, uint32_t b) {
    const uint32_t base = (uint32_t)X.h_sides[side].base;
    if (b <= a) return;
    lo[side] = std::min(lo[side], a - base);
    hi[side] = std::max(hi[side], b - base);
  };
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    if (!use(pl.slot_words[k])) continue;
    for (uint32_t b = blk_lo[k]; b < blk_hi[k]; ++b) {
      const RowBlock &rb = pl.blocks[b];
      const TaskIn &tk = tasks[rb.task];
      if (rows) add(tk.row_side, rb.row0, rb.row_end);
      if (cols) add(tk.col_side, rb.col_begin, rb.col_end);
    }
  }
}

// Size windows, one per side of X, of the sets that the row blocks of the
// width slots wider than kCascadeWords read (as block_hulls).
std::vector<SizeWindow> class_windows(const Plan &pl, const std::vector<TaskIn> &tasks,
                                      const Space &X, bool rows, bool cols,
                                      const uint32_t *blk_lo, const uint32_t *blk_hi) {
  std::vector<uint32_t> lo, hi;
  block_hulls(pl, tasks, X, rows, cols, blk_lo, blk_hi,
              [](uint32_t w) { return w > kCascadeWords; }, lo, hi);
  std::vector<SizeWindow> win(X.n_sides, SizeWindow{1, 0});
  for (uint32_t s = 0; s < X.n_sides; ++s)
    if (lo[s] < hi[s]) win[s] = SizeWindow{size_at(X, s, lo[s]), size_at(X, s, hi[s] - 1)};
  return win;
}

// Positions of X whose sign planes at `words` words the matrix-core filter
// reads: the hulls of the blocks of that width (as block_hulls), each
// extended by the kSignPad - 1 columns a step loads past its group's end,
// merged, and then the padding sets [n, n + kSignPad).
std::vector<PosRange> sign_ranges(const Plan &pl, const std::vector<TaskIn> &tasks,
                                  const Space &X, bool rows, bool cols, const uint32_t *blk_lo,
                                  const uint32_t *blk_hi, uint32_t words) {
  std::vector<uint32_t> lo, hi;
  block_hulls(pl, tasks, X, rows, cols, blk_lo, blk_hi,
              [words](uint32_t w) { return w == words; }, lo, hi);
  std::vector<std::pair<uint64_t, uint64_t>> iv;
  for (uint32_t s = 0; s < X.n_sides; ++s) {
    if (lo[s] >= hi[s]) continue;
    const uint64_t base = X.h_sides[s].base;
    iv.emplace_back(base + lo[s], std::min<uint64_t>(base + hi[s] + kSignPad - 1, X.n));
  }
  std::sort(iv.begin(), iv.end());
  std::vector<PosRange> out;
  uint64_t total = 0;
  for (size_t i = 0; i < iv.size();) {
    uint64_t a = iv[i].first, b = iv[i].second;
    for (++i; i < iv.size() && iv[i].first <= b; ++i) b = std::max(b, iv[i].second);
    out.push_back(PosRange{(uint32_t)a, (uint32_t)b, (uint32_t)total, 0});
    total += b - a;
  }
  out.push_back(PosRange{(uint32_t)X.n, (uint32_t)(X.n + kSignPad), (uint32_t)total, 0});
  return out;
}

struct Timer {
  hipEvent_t ev[2] = {nullptr, nullptr};
  Timer(const Timer &) = delete;
  Timer &operator=(const Timer &) = delete;
  Timer() {
    check(hipEventCreate(&ev[0]));
    check(hipEventCreate(&ev[1]));
  }
  ~Timer() {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
  }
  float ms() const {
    float v = 0;
    (void)hipEventElapsedTime(&v, ev[0], ev[1]);
    return v;
  }
};


// ------------------------------------------------------------------- join

struct JoinOut {
  ssj_pair *pairs = nullptr;            // host, HostPairs
  uint64_t count = 0;
  std::vector<uint64_t> task_start;     // [n_tasks + 1]
};

struct JoinConfig {
  uint32_t b_bits = 0;         // 0: width classes chosen per task
  uint32_t tile_cols = kDefaultTileCols;
  bool tile_cols_fixed = false;  // the caller chose tile_cols
  uint64_t cap = kInitialQueue;
  bool cap_fixed = false;       // the caller chose the queue capacity
  bool survivors_only = false;
  bool cutoff = false;         // rows past the cutoff point take prefix-filtered candidates
  bool cols_resident = false;  // the column space is an index's
  bool mfma = true;            // matrix-core filter at the widths it exists for
  bool mfma_always = false;    // ... for every width class, whatever its band pairs
};

// What a join keeps between its first round and its end: the plan, its
// device copies and its buffers.  A prepared join keeps them across
// executions; join_end works on copies of what a round changes.
struct JoinRun {
  Space *R = nullptr, *C = nullptr;
  std::vector<TaskIn> tasks;
  JoinConfig jc;
  bool automatic = false, any_cosine = false;
  uint32_t n_tasks = 0;
  Plan pl;
  JoinCounters *ctr = nullptr;
  const RowBlock *d_blocks = nullptr;
  const TaskDesc *d_tasks = nullptr;
  const uint32_t *d_side_task = nullptr, *d_tables = nullptr;
  uint32_t *d_tile_block = nullptr;
  uint64_t qcap = 0;
  uint32_t dense_chunk = 0;
  uint2 *queue = nullptr;
  Resume *res_a = nullptr, *res_b = nullptr;
  uint64_t res_cap = 0;
  unsigned long long *results = nullptr;
  int ib = 1, jb = 1, tb = 0;
  uint32_t w2 = 0;
  VerifySpace vrows{}, vcols{};
  FilterConfig cfg{};
  std::vector<PrefixRun> runs;    // rows past the cutoff
  std::vector<uint32_t> ilen;
  uint64_t n_probe = 0;
};

// Kernel timings of a join's rounds (events must not move).
struct RoundTimes {
  std::deque<Timer> filter, verify;
  std::vector<uint32_t> filter_slot;
  uint32_t launches = 0;
  hipEvent_t graph_ev[2] = {nullptr, nullptr};  // around a prepared join's graph
};

// One filter/verify round: a filter launch per width slot, then the
// verification of the queue.  Timed when tm is given (L then runs at once).
void launch_round(const JoinRun &jr, FilterConfig cfg, uint2 *queue, uint64_t qcap,
                  uint32_t dense_chunk, Resume *rin, Resume *rout, unsigned long long *results,
                  uint64_t res_cap, hipStream_t st, Launcher *L, RoundTimes *tm) {
  const Plan &pl = jr.pl;
  const Space &R = *jr.R, &C = *jr.C;
  cfg.cap = qcap;
  // one launch per width slot; after an overflow the later launches of
  // the round leave at once and resume in the next round
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    if (pl.tile_hi[k] == pl.tile_lo[k]) continue;
    cfg.tile_lo = pl.tile_lo[k];
    cfg.tile_hi = pl.tile_hi[k];
    cfg.tile_cols = pl.slot_tile_cols[k];
    cfg.cls = k;
    cfg.chunk = jr.automatic && pl.slot_words[k] < kCascadeWords ? kFilterStage : dense_chunk;
    const uint32_t w = pl.slot_words[k];
    const bool mf = pl.slot_mfma[k], cos = jr.any_cosine;
    const FilterArgs fa{R.bitmaps(w), C.bitmaps(w), mf ? R.signs(w) : nullptr,
                        mf ? C.signs(w) : nullptr, R.sizes, C.sizes, C.sstart, jr.d_tables,
                        jr.d_tasks, jr.d_blocks, jr.d_tile_block, queue, jr.ctr, rin, rout, cfg};
    if (tm) {
      tm->filter.emplace_back();
      tm->filter_slot.push_back(k);
      ++tm->launches;
      check(hipEventRecord(tm->filter.back().ev[0], st));
    }
    go(L, st, [=](hipStream_t s) { return launch_filter(w, cos, fa, s); });
    if (tm) check(hipEventRecord(tm->filter.back().ev[1], st));
  }
  if (tm) {
    tm->verify.emplace_back();
    check(hipEventRecord(tm->verify.back().ev[0], st));
  }
  const VerifySpace vr = jr.vrows, vc = jr.vcols;
  const uint32_t *side_task = jr.d_side_task, *tables = jr.d_tables, w2 = jr.w2;
  const TaskDesc *tasks = jr.d_tasks;
  const uint32_t n_tasks = jr.n_tasks;
  const int ib = jr.ib, jb = jr.jb;
  const uint32_t so = jr.jc.survivors_only ? 1u : 0u;
  JoinCounters *ctr = jr.ctr;
  go(L, st, [=](hipStream_t s) {
    return launch_verify(queue, queue + qcap, qcap, vr, vc, side_task, tasks, n_tasks, tables,
                         ib, jb, so, w2, results, res_cap, ctr, s);
  });
  if (tm) check(hipEventRecord(tm->verify.back().ev[1], st));
}

// Plans the tasks over prepared spaces R (rows) and C (columns; C may be
// R), whose caller bitmaps, if any, are already in place, and starts the
// first filter/verify round.  Device work that reads the tokens goes
// through L (nullptr: at once); work that depends only on the set sizes
// (the plan's upload, the tile list) runs at once.
void join_begin(Space &R, Space &C, const std::vector<TaskIn> &tasks, const JoinConfig &jc,
                Arena &ar, JoinCounters *ctr, hipStream_t st, Timer *t_prep, Launcher *L,
                RoundTimes *tm, JoinRun &jr) {
  jr.R = &R;
  jr.C = &C;
  jr.tasks = tasks;
  jr.jc = jc;
  jr.ctr = ctr;
  const bool automatic = jc.b_bits == 0;
  const uint32_t n_tasks = (uint32_t)tasks.size();
  Plan &pl = jr.pl;
  pl.mfma = jc.mfma;
  pl.tasks.resize(n_tasks);
  std::vector<std::vector<WidthClass>> classes(n_tasks);
  std::vector<uint64_t> task_band(n_tasks, 0);
  std::vector<uint32_t> side_task(R.n_sides, 0xFFFFFFFFu);
  const uint32_t wpad = automatic ? 0 : filter_padded_words(jc.b_bits / 64);
  if (!automatic && !wpad) throw Fail{SSJ_E_UNSUPPORTED};
  // Threshold tables depend on the function and threshold alone (entry L or
  // a holds the same value in any task): tasks that share them share one
  // copy, long enough for the largest sizes among those tasks.
  using TableKey = std::pair<int, std::pair<uint64_t, uint64_t>>;
  std::map<TableKey, std::pair<uint32_t, uint32_t>> table_sizes;  // largest a_max, c_max
  for (const TaskIn &tk : tasks) {
    auto &m = table_sizes[{tk.sim, {tk.p, tk.q}}];
    m.first = std::max(m.first, R.side_max[tk.row_side]);
    m.second = std::max(m.second, C.side_max[tk.col_side]);
  }
  std::map<TableKey, TaskDesc> shared_tables;
  for (const auto &e : table_sizes)
    add_tables(pl, shared_tables[e.first], e.second.first, e.second.second, e.first.first,
               e.first.second.first, e.first.second.second);
  for (uint32_t k = 0; k < n_tasks; ++k) {
    const TaskIn &tk = tasks[k];
    const uint32_t key_side = tk.row_side;
    if (side_task[key_side] != 0xFFFFFFFFu) throw Fail{SSJ_E_INVALID};
    side_task[key_side] = k;
    TaskDesc &td = pl.tasks[k];
    const uint32_t a_max = R.side_max[tk.row_side];
    td = shared_tables.at({tk.sim, {tk.p, tk.q}});
    td.row_side = tk.row_side;
    td.col_side = tk.col_side;
    td.col_base = (uint32_t)C.h_sides[tk.col_side].base;
    td.self = tk.self ? 1u : 0u;
    td.col_sstart_off = (uint64_t)tk.col_side * C.stride;
    if (!automatic) classes[k].push_back({a_max, wpad});
  }
  if (automatic) {
    // the tasks' width classes are independent: many tasks are planned on
    // several host threads, each taking the next task in turn
    const double waves = (double)filter_grid_blocks() * (kBlock / 64);
    auto plan_task = [&](uint32_t k) {
      const TaskIn &tk = tasks[k];
      classes[k] = choose_classes(
          band_by_size(R, C, tk.sim, tk.p, tk.q, tk.row_side, tk.col_side, tk.self), tk.sim,
          tk.p, tk.q, waves);
    };
    // threads only pay when the sizes to plan are many (a thread's start
    // costs about what a few thousand sizes do)
    uint64_t work = 0;
    for (uint32_t k = 0; k < n_tasks; ++k) work += R.side_max[tasks[k].row_side];
    const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
    const uint32_t n_threads =
        work < kPlanThreadSizes ? 1u : std::min<uint32_t>({kPlanThreads, hw, n_tasks / 16});
    if (n_threads <= 1) {
      for (uint32_t k = 0; k < n_tasks; ++k) plan_task(k);
    } else {
      std::atomic<uint32_t> next{0};
      std::exception_ptr failed;
      std::mutex fail_mu;
      auto worker = [&]() {
        try {
          for (uint32_t k; (k = next.fetch_add(1)) < n_tasks;) plan_task(k);
        } catch (...) {
          std::lock_guard<std::mutex> lk(fail_mu);
          if (!failed) failed = std::current_exception();
        }
      };
      std::vector<std::thread> pool;
      for (uint32_t t = 1; t < n_threads; ++t) pool.emplace_back(worker);
      worker();
      for (auto &th : pool) th.join();
      if (failed) std::rethrow_exception(failed);
    }
  }
  // The cutoff point (Section 3.5) of every task at its widest width: rows
  // of larger sets skip the bitmap filter and take prefix-filtered
  // candidates instead.
  std::vector<uint32_t> omega(n_tasks, 0xFFFFFFFFu);
  if (jc.cutoff) {
    for (uint32_t k = 0; k < n_tasks; ++k) {
      const TaskIn &tk = tasks[k];
      const uint32_t widest = automatic ? 64 * classes[k].back().words : jc.b_bits;
      omega[k] = cutoff_point(SSJ_BM_XOR, widest, tk.sim, tk.p, tk.q);
      if (omega[k] >= R.side_max[tk.row_side]) {
        omega[k] = 0xFFFFFFFFu;
        continue;
      }
      std::vector<WidthClass> cut;
      uint32_t prev = 0;
      for (const auto &c : classes[k]) {
        if (prev >= omega[k]) break;
        cut.push_back({std::min(c.max_size, omega[k]), c.words});
        prev = cut.back().max_size;
      }
      classes[k] = cut;
    }
  }
  bool any_cosine = false;
  for (const auto &tk : tasks) any_cosine |= tk.sim == SSJ_SIM_COSINE;
  // width slots: every width some task uses, narrowest first
  if (automatic) {
    for (uint32_t w : kAutoWords) {
      bool used = false;
      for (auto &cl : classes)
        for (auto &c : cl) used |= c.words == w;
      if (!used) continue;
      pl.slot_words[pl.n_slots] = w;
      pl.slot_bits[pl.n_slots] = 64 * w;
      ++pl.n_slots;
    }
  } else if (n_tasks) {
    pl.slot_words[0] = wpad;
    pl.slot_bits[0] = jc.b_bits;
    pl.n_slots = 1;
  }
  // band pairs of each slot, and its kernel: the matrix cores where the
  // width has a matrix-core shape, unless it is a small b = 256 class (see
  // kMfmaMinBand) and the caller did not ask for them
  uint64_t slot_band[kMaxClasses] = {};
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    for (uint32_t t = 0; t < n_tasks; ++t) {
      uint32_t prev = 0;
      for (auto &c : classes[t]) {
        if (c.words == pl.slot_words[k])
          plan_class(pl, R, C, tasks[t], t, prev, c.max_size, c.words, pl.slot_bits[k],
                     jc.tile_cols, false, slot_band[k], true);
        prev = c.max_size;
      }
    }
    pl.slot_mfma[k] = filter_shape(pl.slot_words[k], pl.mfma).mfma &&
                      (jc.mfma_always || pl.slot_words[k] < kMfmaMinBandWords ||
                       slot_band[k] >= kMfmaMinBand);
  }
  uint32_t blk_lo[kMaxClasses] = {}, blk_hi[kMaxClasses] = {};  // row blocks of each slot
  // tiles, slot by slot, task by task.  Unless the caller fixed the tile
  // width, a slot with little work gets narrower tiles, so that it is cut
  // into enough tiles to occupy every wave of the GPU.
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    uint32_t tile_cols = jc.tile_cols;
    if (!jc.tile_cols_fixed && automatic) {
      // the measured best tile width of the class's width
      for (int a = 0; a < kNumAuto; ++a)
        if (kAutoWords[a] == pl.slot_words[k]) tile_cols = kClassTileCols[a];
    }
    if (!jc.tile_cols_fixed) {
      const FilterShape shape = filter_shape(pl.slot_words[k], pl.slot_mfma[k]);
      const uint64_t min_tiles = n_tasks > 1 ? kMinSlotTiles : kMinSlotTilesOneTask;
      const uint64_t want = slot_band[k] / ((uint64_t)shape.rows * min_tiles);
      const uint32_t floor_cols = shape.mfma ? kMinTileCols : kMinTileColsValu;
      tile_cols = (uint32_t)std::max<uint64_t>(floor_cols, std::min<uint64_t>(tile_cols, want));
    }
    pl.slot_tile_cols[k] = tile_cols;
    pl.tile_lo[k] = pl.n_tiles;
    blk_lo[k] = (uint32_t)pl.blocks.size();
    const uint64_t ops0 = pl.filter_ops;
    for (uint32_t t = 0; t < n_tasks; ++t) {
      uint32_t prev = 0;
      for (auto &c : classes[t]) {
        if (c.words == pl.slot_words[k]) {
          plan_class(pl, R, C, tasks[t], t, prev, c.max_size, c.words, pl.slot_bits[k],
                     tile_cols, pl.slot_mfma[k], task_band[t]);
          pl.slot_max_size[k] = std::max(pl.slot_max_size[k], c.max_size);
        }
        prev = c.max_size;
      }
    }
    pl.tile_hi[k] = pl.n_tiles;
    blk_hi[k] = (uint32_t)pl.blocks.size();
    pl.ops[k] = pl.filter_ops - ops0;
  }

  // the widths to build: every class's, and in automatic mode the widest
  // automatic width for the cascade test of verification (same pass)
  uint32_t bw[kMaxClasses + 1], bb[kMaxClasses + 1], nbw = 0;
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    bw[nbw] = pl.slot_words[k];
    bb[nbw++] = pl.slot_bits[k];
  }
  bool have_cascade = false;
  for (uint32_t k = 0; k < nbw; ++k) have_cascade |= bw[k] == kCascadeWords;
  if (automatic && !jc.survivors_only && pl.n_slots > 0 && pl.slot_words[0] < kCascadeWords &&
      !have_cascade) {
    bw[nbw] = kCascadeWords;
    bb[nbw++] = 64 * kCascadeWords;
  }
  // a resident space (an index's) already holds every width it may need
  for (uint32_t k = 0; k < nbw; ++k) {
    if (jc.cols_resident && !C.bitmaps(bw[k])) throw Fail{SSJ_E_UNSUPPORTED};
  }
  // Widths up to the cascade width take one pass over every set of a space
  // (which also checks the token order).  In automatic mode the wider ones
  // then take a pass over only the sets their classes' blocks read: the
  // rows of those blocks and, on the column side, their columns.
  uint32_t sw[kMaxClasses + 1], sb[kMaxClasses + 1], ns = 0, lw[kMaxClasses + 1], nl = 0;
  for (uint32_t k = 0; k < nbw; ++k) {
    const bool window = automatic && bw[k] > kCascadeWords && bw[k] <= kMaxFoldWords &&
                        (bw[k] & (bw[k] - 1)) == 0 && bb[k] == 64 * bw[k];
    if (window) {
      lw[nl++] = bw[k];
    } else {
      sw[ns] = bw[k];
      sb[ns++] = bb[k];
    }
  }
  auto build = [&](Space &X, bool rows, bool cols) {
    space_bitmaps_multi(X, sw, sb, ns, ar, ctr, st, L);
    uint32_t need[kMaxClasses + 1], nn = 0;
    for (uint32_t k = 0; k < nl; ++k)
      if (!X.bitmaps(lw[k])) need[nn++] = lw[k];
    if (nn == 0) return;
    if (X.checked && X.rank) {
      space_bitmaps_window(X, need, nn, class_windows(pl, tasks, X, rows, cols, blk_lo, blk_hi),
                           ar, st, L);
    } else {
      uint32_t nb[kMaxClasses + 1];
      for (uint32_t k = 0; k < nn; ++k) nb[k] = 64 * need[k];
      space_bitmaps_multi(X, need, nb, nn, ar, ctr, st, L);
    }
  };
  build(R, true, &C == &R);
  if (!jc.cols_resident && &C != &R) build(C, false, true);
  // sign planes for the widths the matrix-core kernel runs (an index holds
  // its own)
  // of only the sets that the width's blocks read
  for (uint32_t k = 0; k < pl.n_slots; ++k) {
    const uint32_t w = pl.slot_words[k];
    if (!pl.slot_mfma[k]) continue;
    const std::vector<PosRange> rr = sign_ranges(pl, tasks, R, true, &C == &R, blk_lo, blk_hi, w);
    space_signs(R, w, ar, st, L, &rr);
    if (jc.cols_resident) {
      if (!C.signs(w)) throw Fail{SSJ_E_UNSUPPORTED};
    } else if (&C != &R) {
      const std::vector<PosRange> cr = sign_ranges(pl, tasks, C, false, true, blk_lo, blk_hi, w);
      space_signs(C, w, ar, st, L, &cr);
    }
  }
  if (pl.n_slots == 0) {
    // no bitmaps (every row past the cutoff): check the token order directly
    for (const auto &d : R.h_sides)
      go(L, st, [=](hipStream_t s) { return launch_check_sorted(d.offsets, d.tokens, d.n, ctr, s); });
    if (&C != &R && !jc.cols_resident)
      for (const auto &d : C.h_sides)
        go(L, st, [=](hipStream_t s) { return launch_check_sorted(d.offsets, d.tokens, d.n, ctr, s); });
  }

  // rows past the cutoff: their band pairs, probe runs and prefix lengths
  std::vector<PrefixRun> &runs = jr.runs;
  std::vector<uint32_t> &ilen = jr.ilen;  // [column side][size]: prefix length indexed (0: none)
  uint64_t &n_probe = jr.n_probe;
  for (uint32_t k = 0; k < n_tasks; ++k) {
    if (omega[k] == 0xFFFFFFFFu) continue;
    const TaskIn &tk = tasks[k];
    const uint32_t a_max = R.side_max[tk.row_side];
    uint64_t pb = 0;
    plan_class(pl, R, C, tk, k, omega[k], a_max, 1, 64, jc.tile_cols, false, pb, true);
    pl.band_pairs += pb;
    task_band[k] += pb;
    // probe prefix: |r| - omin(|r|, cmin(|r|)) + 1 tokens, the longest any
    // partner in the band can need (omin grows with the partner's size)
    const TaskDesc &td = pl.tasks[k];
    const uint32_t plen_off = (uint32_t)pl.tables.size();
    for (uint64_t a = 0; a <= a_max; ++a) {
      uint32_t len = 0;
      const uint32_t cmn = pl.tables[td.cmin_off + a], cmx = pl.tables[td.cmax_off + a];
      if (a > omega[k] && cmn <= cmx) {
        const int64_t o = omin_of(tk.sim, a, cmn, tk.p, tk.q);
        len = (uint32_t)std::min<int64_t>(std::max<int64_t>((int64_t)a - o + 1, 1), (int64_t)a);
      }
      pl.tables.push_back(len);
    }
    const uint32_t *rs = R.ss(tk.row_side);
    PrefixRun run{};
    run.row_begin = (uint32_t)R.h_sides[tk.row_side].base + rs[omega[k] + 1];
    run.row_end = (uint32_t)R.h_sides[tk.row_side].base + R.h_sides[tk.row_side].n;
    run.task = k;
    run.plen_off = plen_off;
    run.first = n_probe;
    if (run.row_end <= run.row_begin) continue;
    n_probe += run.row_end - run.row_begin;
    runs.push_back(run);
    // index prefix of a column of size c: c - omin(a*, c) + 1 tokens, a* the
    // smallest row size past the cutoff whose band holds c
    if (ilen.empty()) ilen.assign((size_t)C.n_sides * C.stride, 0);
    const uint32_t c_max = C.side_max[tk.col_side];
    for (uint64_t c = 1; c <= c_max; ++c) {
      uint64_t lo = 0, hi = 0;
      size_band(tk.sim, c, tk.p, tk.q, lo, hi);  // row sizes that pair with c (Table 2 is symmetric)
      uint64_t a_lo = std::max<uint64_t>(lo, (uint64_t)omega[k] + 1);
      if (tk.self) a_lo = std::max<uint64_t>(a_lo, c);
      if (a_lo > std::min<uint64_t>(hi, a_max)) continue;
      const int64_t o = omin_of(tk.sim, a_lo, c, tk.p, tk.q);
      const uint32_t len =
          (uint32_t)std::min<int64_t>(std::max<int64_t>((int64_t)c - o + 1, 1), (int64_t)c);
      uint32_t &slot = ilen[(size_t)tk.col_side * C.stride + c];
      slot = std::max(slot, len);
    }
  }
  if (pl.tables.size() >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};

  // blocks, tasks, the row sides' tasks and the tables go up in one copy
  constexpr uint64_t kBlockWords = sizeof(RowBlock) / 4, kTaskWords = sizeof(TaskDesc) / 4;
  static_assert(sizeof(RowBlock) % 8 == 0 && sizeof(TaskDesc) % 8 == 0, "8-byte layout");
  const uint64_t nB = pl.blocks.size(), nT = pl.tasks.size(), nS = side_task.size();
  const uint64_t n_packed = kBlockWords * nB + kTaskWords * nT + nS + pl.tables.size();
  uint32_t *hp = ar.stage<uint32_t>(n_packed);
  std::memcpy(hp, pl.blocks.data(), nB * sizeof(RowBlock));
  std::memcpy(hp + kBlockWords * nB, pl.tasks.data(), nT * sizeof(TaskDesc));
  std::memcpy(hp + kBlockWords * nB + kTaskWords * nT, side_task.data(), nS * 4);
  std::memcpy(hp + kBlockWords * nB + kTaskWords * nT + nS, pl.tables.data(),
              pl.tables.size() * 4);
  uint32_t *d_packed = ar.alloc<uint32_t>(n_packed);
  h2d(d_packed, hp, n_packed, st);
  const RowBlock *d_blocks = reinterpret_cast<const RowBlock *>(d_packed);
  const TaskDesc *d_tasks = reinterpret_cast<const TaskDesc *>(d_packed + kBlockWords * nB);
  const uint32_t *d_side_task = d_packed + kBlockWords * nB + kTaskWords * nT;
  const uint32_t *d_tables = d_side_task + nS;
  uint32_t *d_tile_block = ar.alloc<uint32_t>(pl.n_tiles);
  check(launch_expand_tiles(d_blocks, (uint32_t)nB, pl.n_tiles, d_tile_block, st));
  if (t_prep) check(hipEventRecord(t_prep->ev[1], st));

  // filter / verify rounds.  A wave reserves queue slots a chunk at a time
  // and writes staged runs (at most kFilterStage pairs) into its chunk; the
  // queue must hold at least one chunk, or a run could never be written and
  // its tile never resumed.  Chunks are small against the queue, so that
  // many waves hold one in a round.  The unused end of a chunk costs
  // verification a sentinel read per slot, a reservation costs an atomic on
  // one address.  The width classes below the cascade width keep false
  // survivors rare (their widths are chosen for it), so their waves take
  // kFilterStage slots at a time; the widest class (every size beyond the
  // others, where the bits saturate) and a fixed width can keep many pairs,
  // and their waves take up to 1024.
  static_assert(kFilterStage <= 4096, "the queue holds at least 4096 entries");
  uint64_t qcap = std::max<uint64_t>(4096, std::min<uint64_t>(jc.cap, pl.band_pairs + 1));
  uint32_t dense_chunk =
      (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(kFilterStage, qcap / 64));
  // the queue, then as many slots for the long pairs verification defers
  uint2 *queue = ar.alloc<uint2>(2 * qcap);
  const uint32_t max_waves = (uint32_t)filter_grid_blocks() * (kBlock / 64);
  Resume *res_a = ar.alloc<Resume>(max_waves), *res_b = ar.alloc<Resume>(max_waves);
  uint64_t res_cap = std::max<uint64_t>(qcap, 1024);
  unsigned long long *results = ar.alloc<unsigned long long>(res_cap);
  // result keys (task, i, j): i of the row side, j of the column side
  int ib = 1, jb = 1;
  for (const auto &d : R.h_sides) ib = std::max(ib, bits_for(d.n ? d.n - 1 : 0));
  for (const auto &d : C.h_sides) jb = std::max(jb, bits_for(d.n ? d.n - 1 : 0));
  const int tb = bits_for(n_tasks > 1 ? n_tasks - 1 : 0);
  if (tb + ib + jb > 64) throw Fail{SSJ_E_UNSUPPORTED};
  // cascade width: the widest bitmaps both spaces hold, when wider than the
  // narrowest class (a second test before every merge)
  uint32_t w2 = 0;
  for (uint32_t k = 0; k < R.n_bm; ++k)
    if (R.bm_words[k] > w2 && R.bm_words[k] <= kCascadeWords && C.bitmaps(R.bm_words[k]))
      w2 = R.bm_words[k];
  const bool cascade = automatic && !jc.survivors_only && pl.n_slots > 0 && w2 > pl.slot_words[0];
  // wide bitmaps for pairs of large sets (automatic mode, as the cascade);
  // an index holds its own
  if (cascade) {
    space_wide(R, ar, st, L);
    if (!jc.cols_resident) space_wide(C, ar, st, L);
  }
  const bool wide = cascade && R.bmw && C.bmw;
  const VerifySpace vrows{R.d_sides, R.side_of, R.perm, R.sizes, cascade ? R.bitmaps(w2) : nullptr,
                          (uint32_t)R.n, wide ? R.bmw : nullptr, R.wide_lo, R.wide_slot};
  const VerifySpace vcols{C.d_sides, C.side_of, C.perm, C.sizes, cascade ? C.bitmaps(w2) : nullptr,
                          (uint32_t)C.n, wide ? C.bmw : nullptr, C.wide_lo, C.wide_slot};
  if (!cascade) w2 = 0;


  jr.automatic = automatic;
  jr.any_cosine = any_cosine;
  jr.n_tasks = n_tasks;
  jr.d_blocks = d_blocks;
  jr.d_tasks = d_tasks;
  jr.d_side_task = d_side_task;
  jr.d_tables = d_tables;
  jr.d_tile_block = d_tile_block;
  jr.qcap = qcap;
  jr.dense_chunk = dense_chunk;
  jr.queue = queue;
  jr.res_a = res_a;
  jr.res_b = res_b;
  jr.res_cap = res_cap;
  jr.results = results;
  jr.ib = ib;
  jr.jb = jb;
  jr.tb = tb;
  jr.w2 = w2;
  jr.vrows = vrows;
  jr.vcols = vcols;
  FilterConfig &cfg = jr.cfg;
  cfg = FilterConfig{};
  cfg.n_rows = (uint32_t)R.n;
  cfg.n_cols = (uint32_t)C.n;
  cfg.n_tiles = pl.n_tiles;
  cfg.n_blocks = (uint32_t)nB;
  cfg.resume_cap = max_waves;
  cfg.cap = qcap;
  cfg.n_resume_in = 0;
  if (pl.n_tiles)
    launch_round(jr, cfg, queue, qcap, dense_chunk, res_a, res_b, results, res_cap, st, L, tm);
}

// Finishes a join whose first round join_begin (or a prepared join's graph)
// started: drains and resumes the filter while the queue fills, verifies
// the prefix-filtered candidates of rows past the cutoff, sorts the
// result keys and copies the pairs out.  Temporaries come from ar.
void join_end(const JoinRun &jr, Arena &ar, hipStream_t st, RoundTimes &tm, Timer *t_prep,
              JoinOut &jo, ssj_stats *stats) {
  const Space &R = *jr.R, &C = *jr.C;
  const Plan &pl = jr.pl;
  const JoinConfig &jc = jr.jc;
  const uint32_t n_tasks = jr.n_tasks;
  JoinCounters *ctr = jr.ctr;
  const TaskDesc *d_tasks = jr.d_tasks;
  const uint32_t *d_side_task = jr.d_side_task, *d_tables = jr.d_tables;
  const int ib = jr.ib, jb = jr.jb, tb = jr.tb;
  const uint32_t w2 = jr.w2;
  const VerifySpace &vrows = jr.vrows, &vcols = jr.vcols;
  const std::vector<PrefixRun> &runs = jr.runs;
  const std::vector<uint32_t> &ilen = jr.ilen;
  const uint64_t n_probe = jr.n_probe;
  // what a round may change: a prepared join's own buffers stay as planned
  uint64_t qcap = jr.qcap;
  uint32_t dense_chunk = jr.dense_chunk;
  uint2 *queue = jr.queue;
  Resume *res_a = jr.res_a, *res_b = jr.res_b;
  uint64_t res_cap = jr.res_cap;
  unsigned long long *results = jr.results;
  FilterConfig cfg = jr.cfg;
  float prefix_ms_index = 0, prefix_ms_verify = 0;
  uint64_t prefix_candidates = 0;
  uint64_t results_n = 0, queue_slots = 0;
  JoinCounters ctr_h{};
  if (pl.n_tiles) {
    for (;;) {
      d2h(&ctr_h, ctr, 1, st);
      sync(st);
      if (ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
      queue_slots += std::min<uint64_t>(ctr_h.queue_count, qcap);
      results_n = ctr_h.results;
      if (results_n > res_cap) throw Fail{SSJ_E_DEVICE};  // cannot happen: capacity grows first
      if (!ctr_h.overflow) break;
      // drain done; a queue the library sized itself grows for the next round
      if (!jc.cap_fixed && qcap < std::min<uint64_t>(kMaxQueue, pl.band_pairs + 1)) {
        qcap = std::min<uint64_t>(std::min<uint64_t>(kMaxQueue, pl.band_pairs + 1), 4 * qcap);
        queue = ar.alloc<uint2>(2 * qcap);
        dense_chunk =
            (uint32_t)std::min<uint64_t>(1024, std::max<uint64_t>(kFilterStage, qcap / 64));
      }
      // make room for another full queue of results, then resume
      if (results_n + qcap > res_cap) {
        const uint64_t ncap = std::max<uint64_t>(2 * res_cap, results_n + qcap);
        unsigned long long *nr = ar.alloc<unsigned long long>(ncap);
        check(launch_copy_u64(results, results_n, nr, st));
        results = nr;
        res_cap = ncap;
      }
      cfg.n_resume_in = ctr_h.n_resume;
      std::swap(res_a, res_b);
      check(launch_reset_round(ctr, st));
      launch_round(jr, cfg, queue, qcap, dense_chunk, res_a, res_b, results, res_cap, st, nullptr,
                   &tm);
    }
  } else {
    // nothing to filter; still report unsorted input
    d2h(&ctr_h, ctr, 1, st);
    sync(st);
    if (ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
  }

  // rows past the cutoff: index of column prefixes, probe, deduplicate,
  // verify, chunk by chunk so that each chunk's candidates fit one queue
  if (n_probe) {
    Timer t_index, t_pver;
    check(hipEventRecord(t_index.ev[0], st));
    uint32_t *d_ilen = ar.alloc<uint32_t>(ilen.size());
    h2d(d_ilen, ilen.data(), ilen.size(), st);
    uint32_t *len = ar.alloc<uint32_t>(C.n);
    unsigned long long *off = ar.alloc<unsigned long long>(C.n);
    unsigned long long *d_tot = ar.alloc<unsigned long long>(2);
    unsigned long long *scan_scr =
        ar.alloc<unsigned long long>(scan_scratch_words(std::max<uint64_t>(C.n, n_probe)));
    check(launch_index_len(C.sizes, C.side_of, d_ilen, C.stride, C.n, len, st));
    check(launch_scan_u32(len, C.n, off, d_tot, scan_scr, st));
    unsigned long long n_keys = 0;
    d2h(&n_keys, d_tot, 1, st);
    sync(st);
    unsigned long long *keys = ar.alloc<unsigned long long>(n_keys);
    unsigned long long *ktmp = ar.alloc<unsigned long long>(n_keys);
    uint32_t *kscr = ar.alloc<uint32_t>(radix_scratch_words(n_keys));
    check(launch_index_fill(C.d_sides, C.side_of, C.perm, len, off, C.n, keys, st));
    const int tok_shifts[4] = {32, 40, 48, 56};
    unsigned long long *sorted_keys = keys;
    if (n_keys) check(radix_sort_u64(keys, ktmp, n_keys, tok_shifts, 4, kscr, st, &sorted_keys));
    PrefixRun *d_runs = ar.alloc<PrefixRun>(runs.size());
    h2d(d_runs, runs.data(), runs.size(), st);
    const ProbeArgs pa{d_runs, (uint32_t)runs.size(), C.max_size, d_tasks, d_tables, R.sizes,
                       R.d_sides, R.side_of, R.perm, C.sstart, sorted_keys, n_keys};
    uint32_t *counts = ar.alloc<uint32_t>(n_probe);
    unsigned long long *row_off = ar.alloc<unsigned long long>(n_probe);
    check(launch_probe_count(pa, n_probe, counts, st));
    check(launch_scan_u32(counts, n_probe, row_off, d_tot + 1, scan_scr, st));
    std::vector<unsigned long long> off_h(n_probe + 1);
    d2h(off_h.data(), row_off, n_probe, st);
    d2h(&off_h[n_probe], d_tot + 1, 1, st);
    check(hipEventRecord(t_index.ev[1], st));
    sync(st);
    uint64_t biggest = 0;
    for (uint64_t x = 0; x < n_probe; ++x) {
      const uint64_t c = off_h[x + 1] - off_h[x];
      if (c >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};  // one row's candidates saturated
      biggest = std::max(biggest, c);
    }
    const uint64_t ccap = std::max<uint64_t>(qcap, biggest);
    unsigned long long *cand = ar.alloc<unsigned long long>(ccap);
    unsigned long long *ctmp = ar.alloc<unsigned long long>(ccap);
    uint32_t *cscr = ar.alloc<uint32_t>(radix_scratch_words(ccap));
    uint2 *pqueue = ccap > qcap ? ar.alloc<uint2>(2 * ccap) : queue;
    int cshifts[8], ncs = 0;
    const int bs = std::max(1, bits_for(C.n ? C.n - 1 : 0)), br = std::max(1, bits_for(R.n ? R.n - 1 : 0));
    for (int b = 0; b < bs; b += 8) cshifts[ncs++] = b;
    for (int b = 0; b < br; b += 8) cshifts[ncs++] = 32 + b;
    check(hipEventRecord(t_pver.ev[0], st));
    for (uint64_t x0 = 0; x0 < n_probe;) {
      uint64_t x1 = x0 + 1;
      while (x1 < n_probe && off_h[x1 + 1] - off_h[x0] <= ccap) ++x1;
      const uint64_t nc = off_h[x1] - off_h[x0];
      if (nc) {
        check(launch_reset_round(ctr, st));
        check(launch_probe_fill(pa, x0, x1, row_off, off_h[x0], cand, st));
        unsigned long long *sc = cand;
        check(radix_sort_u64(cand, ctmp, nc, cshifts, ncs, cscr, st, &sc));
        check(launch_unique_to_queue(sc, nc, pqueue, ctr, st));
        if (results_n + nc > res_cap) {
          const uint64_t ncap = std::max<uint64_t>(2 * res_cap, results_n + nc);
          unsigned long long *nr = ar.alloc<unsigned long long>(ncap);
          check(launch_copy_u64(results, results_n, nr, st));
          results = nr;
          res_cap = ncap;
        }
        check(launch_verify(pqueue, pqueue + ccap, ccap, vrows, vcols, d_side_task, d_tasks,
                            n_tasks, d_tables, ib, jb, jc.survivors_only ? 1u : 0u, w2, results,
                            res_cap, ctr, st));
        d2h(&ctr_h, ctr, 1, st);
        sync(st);
        if (ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
        results_n = ctr_h.results;
        if (results_n > res_cap) throw Fail{SSJ_E_DEVICE};
      }
      x0 = x1;
    }
    check(hipEventRecord(t_pver.ev[1], st));
    sync(st);
    prefix_ms_index = t_index.ms();
    prefix_ms_verify = t_pver.ms();
    prefix_candidates = off_h[n_probe];
  }

  // emit: sort the keys (task, i, j) on all their digits, split, copy out
  Timer t_emit;
  check(hipEventRecord(t_emit.ev[0], st));
  jo.task_start.assign(n_tasks + 1, 0);
  if (results_n) {
    unsigned long long *tmp = ar.alloc<unsigned long long>(results_n);
    uint32_t *scr = ar.alloc<uint32_t>(radix_scratch_words(results_n));
    int shifts[8], ns = 0;
    for (int b = 0; b < tb + ib + jb; b += 8) shifts[ns++] = b;
    unsigned long long *sorted = results;
    check(radix_sort_u64(results, tmp, results_n, shifts, ns, scr, st, &sorted));
    ssj_pair *dpairs = ar.alloc<ssj_pair>(results_n);
    uint64_t *dstart = ar.alloc<uint64_t>(n_tasks + 1);
    check(launch_split_results(sorted, results_n, ib, jb, n_tasks, dpairs, dstart, st));
    jo.pairs = HostPairs::get().alloc(results_n);
    if (!jo.pairs) throw Fail{SSJ_E_NOMEM};
    jo.count = results_n;
    d2h(jo.pairs, dpairs, results_n, st);
    d2h(jo.task_start.data(), dstart, n_tasks + 1, st);
  }
  check(hipEventRecord(t_emit.ev[1], st));
  sync(st);
  if (stats) {
    stats->band_pairs = pl.band_pairs;
    stats->survivors = ctr_h.survivors;
    stats->results = results_n;
    stats->filter_launches = tm.launches;
    stats->b_bits = jc.b_bits;
    stats->filter_ops = pl.filter_ops;
    stats->queue_slots = queue_slots;
    stats->n_classes = pl.n_slots;
    for (uint32_t k = 0; k < pl.n_slots; ++k) {
      stats->class_bits[k] = pl.slot_bits[k];
      stats->class_max_size[k] = pl.slot_max_size[k];
      stats->class_ops[k] = pl.ops[k];
      stats->class_tiles[k] = pl.tile_hi[k] - pl.tile_lo[k];
    }
    stats->ms_prepare = t_prep ? t_prep->ms() : 0.f;
    float gms = 0;
    if (tm.graph_ev[0]) (void)hipEventElapsedTime(&gms, tm.graph_ev[0], tm.graph_ev[1]);
    stats->ms_filter = gms;
    for (size_t k = 0; k < tm.filter.size(); ++k) {
      const float ms = tm.filter[k].ms();
      stats->ms_filter += ms;
      stats->class_ms[tm.filter_slot[k]] += ms;
    }
    for (auto &t : tm.verify) stats->ms_verify += t.ms();
    // prefix-filtered rows: index and probe count as filtering, the
    // deduplication and verification of their candidates as verification
    stats->ms_filter += prefix_ms_index;
    stats->ms_verify += prefix_ms_verify;
    (void)prefix_candidates;
    stats->ms_emit = t_emit.ms();
  }
}


// Plans and runs the tasks at once: join_begin, then join_end.
void run_join(Space &R, Space &C, const std::vector<TaskIn> &tasks, const JoinConfig &jc,
              Arena &ar, JoinCounters *ctr, hipStream_t st, Timer &t_prep, JoinOut &jo,
              ssj_stats *stats) {
  JoinRun jr;
  RoundTimes tm;
  join_begin(R, C, tasks, jc, ar, ctr, st, &t_prep, nullptr, &tm, jr);
  join_end(jr, ar, st, tm, &t_prep, jo, stats);
}

// Checks and reduces a threshold: 1 <= p <= q, except Overlap (o >= p/q),
// which takes any p >= 1.
void check_threshold(int sim, uint32_t &p, uint32_t &q) {
  if (sim < SSJ_SIM_JACCARD || sim > SSJ_SIM_OVERLAP) throw Fail{SSJ_E_INVALID};
  if (p == 0 || q == 0 || (p > q && sim != SSJ_SIM_OVERLAP)) throw Fail{SSJ_E_INVALID};
  const uint32_t g = std::gcd(p, q);
  p /= g;
  q /= g;
}

JoinConfig config_of(uint32_t b_bits, const ssj_options *opts) {
  if (b_bits != 0 && (b_bits < 64 || b_bits > 4096 || b_bits % 64)) throw Fail{SSJ_E_INVALID};
  JoinConfig jc;
  jc.b_bits = b_bits;
  if (opts && opts->tile_cols) {
    jc.tile_cols = opts->tile_cols;
    jc.tile_cols_fixed = true;
  }
  if (opts && opts->queue_capacity) {
    jc.cap = opts->queue_capacity;
    jc.cap_fixed = true;
  }
  jc.survivors_only = opts && (opts->flags & SSJ_FLAG_SURVIVORS_ONLY);
  jc.cutoff = opts && (opts->flags & SSJ_FLAG_CUTOFF);
  jc.mfma = !(opts && (opts->flags & SSJ_FLAG_VALU));
  jc.mfma_always = opts && (opts->flags & SSJ_FLAG_MFMA);
  if (!jc.mfma && jc.mfma_always) throw Fail{SSJ_E_INVALID};
  return jc;
}

void clear_out(ssj_pairs *out, ssj_stats *stats) {
  out->pairs = nullptr;
  out->count = 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
}

float ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ssj_self_join / ssj_rs_join: one task, each side in its own space (the
// self-join's row and column space are one).
// A point in a stream the host can wait for without waiting for the work
// enqueued after it.
struct Marker {
  hipEvent_t ev = nullptr;
  Marker() { check(hipEventCreateWithFlags(&ev, hipEventDisableTiming)); }
  ~Marker() {
    if (ev) (void)hipEventDestroy(ev);
  }
  Marker(const Marker &) = delete;
  Marker &operator=(const Marker &) = delete;
  void record(hipStream_t st) { check(hipEventRecord(ev, st)); }
  void wait() { check(hipEventSynchronize(ev)); }
};

// In automatic mode the bitmaps up to the cascade width (one build pass,
// the narrower widths folded from it) do not depend on the plan: they are
// enqueued before the host waits for the group starts, so that the device
// builds them while the host plans.
void early_bitmaps(Space &sp, const JoinConfig &jc, Arena &ar, JoinCounters *ctr,
                   hipStream_t st) {
  if (jc.b_bits != 0 || jc.survivors_only || !sp.rank) return;
  static constexpr uint32_t words[4] = {1, 2, 4, kCascadeWords}, bits[4] = {64, 128, 256, 512};
  static_assert(kCascadeWords == 8, "the cascade width is the widest of one fold pass");
  space_bitmaps_multi(sp, words, bits, 4, ar, ctr, st);
}

// The wide bitmaps of verification depend only on the sizes: in automatic
// mode they are enqueued once the group starts are on the host, so that the
// device builds them while the host plans (a plan with no cascade test
// leaves them unused).
void early_wide(Space &sp, const JoinConfig &jc, Arena &ar, hipStream_t st) {
  if (jc.b_bits != 0 || jc.survivors_only || !sp.rank) return;
  space_wide(sp, ar, st);
}

int join_one(const ssj_sets *R, const uint64_t *r_bm, const ssj_sets *S, const uint64_t *s_bm,
             bool self, uint32_t b_bits, int sim, uint32_t p, uint32_t q,
             const ssj_options *opts, ssj_pairs *out, ssj_stats *stats, void *hip_stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return SSJ_E_INVALID;
  clear_out(out, stats);
  JoinOut jo;
  try {
    const JoinConfig jc = config_of(b_bits, opts);
    if (b_bits == 0 && (r_bm || s_bm)) return SSJ_E_INVALID;
    check_threshold(sim, p, q);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Arena ar(st);
    Timer t_prep;
    check(hipEventRecord(t_prep.ev[0], st));
    JoinCounters *ctr = ar.alloc<JoinCounters>(1);
    check(launch_reset_all(ctr, st));
    Space A, B;
    space_begin(A, &R, 1, ar, st);
    if (!self) space_begin(B, &S, 1, ar, st);
    sync(st);
    space_sort(A, r_bm == nullptr, ar, ar, st);
    if (!self) space_sort(B, s_bm == nullptr, ar, ar, st);
    Marker sorted;
    sorted.record(st);
    early_bitmaps(A, jc, ar, ctr, st);
    if (!self) early_bitmaps(B, jc, ar, ctr, st);
    sorted.wait();
    space_finish(A);
    if (!self) space_finish(B);
    early_wide(A, jc, ar, st);
    if (!self) early_wide(B, jc, ar, st);
    Space &C = self ? A : B;
    if (r_bm) {
      const uint32_t w = filter_padded_words(b_bits / 64);
      if (!w) return SSJ_E_UNSUPPORTED;
      space_caller_bitmaps(A, r_bm, w, b_bits, ar, ctr, st);
      if (!self) space_caller_bitmaps(B, s_bm, w, b_bits, ar, ctr, st);
    }
    std::vector<TaskIn> tasks{{0, 0, sim, p, q, self}};
    run_join(A, C, tasks, jc, ar, ctr, st, t_prep, jo, stats);
  } catch (const Fail &f) {
    HostPairs::get().release(jo.pairs);
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    HostPairs::get().release(jo.pairs);
    return SSJ_E_NOMEM;
  }
  out->pairs = jo.pairs;
  out->count = jo.count;
  if (stats) stats->ms_total = ms_since(t_start);
  return SSJ_OK;
}

}  // namespace
}  // namespace ssj

// A resident collection for repeated R-S queries: a copy of the caller's CSR
// in the index's own device memory, prepared (sizes, size order, group
// starts) and with its bitmaps built once.
struct ssj_index {
  ssj::Arena ar;
  ssj::Space S;
  ssj_sets sets{};
  uint32_t b_bits = 0;
  int device = 0;
  explicit ssj_index(hipStream_t st) : ar(st, true) {}
};

// A prepared join: its plan and buffers in memory it owns, and the graph of
// its first round.  jr points into S, so a plan never moves.
struct ssj_plan {
  ssj::Arena ar;
  ssj::Space S;
  ssj::JoinRun jr;
  hipStream_t cap_stream = nullptr;  // capture happens on a stream of the plan's own
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::mutex mu;                     // executions take turns
  int device = 0;
  uint32_t n_tasks = 0;
  explicit ssj_plan(hipStream_t st) : ar(st, true) {}
  ssj_plan(const ssj_plan &) = delete;
  ssj_plan &operator=(const ssj_plan &) = delete;
  ~ssj_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace ssj {
namespace {

// Several tasks whose row sides are `rows` (one task per side) against the
// prepared space C (or against themselves when self).
int join_tasks(const ssj_sets *rows, uint32_t n, const uint32_t *p, const uint32_t *q,
               bool self, ssj_index *idx, uint32_t b_bits, int sim, const ssj_options *opts,
               ssj_pairs *out, uint64_t *starts, ssj_stats *stats, void *hip_stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return SSJ_E_INVALID;
  clear_out(out, stats);
  if (n && (!rows || !p || !q)) return SSJ_E_INVALID;
  JoinOut jo;
  try {
    const JoinConfig jc0 = config_of(b_bits, opts);
    JoinConfig jc = jc0;
    std::vector<TaskIn> tasks(n);
    std::vector<const ssj_sets *> sides(n);
    for (uint32_t k = 0; k < n; ++k) {
      uint32_t pk = p[k], qk = q[k];
      check_threshold(sim, pk, qk);
      tasks[k] = {k, self ? k : 0u, sim, pk, qk, self};
      sides[k] = rows + k;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (idx) {
      int dev = 0;
      check(hipGetDevice(&dev));
      if (dev != idx->device) return SSJ_E_INVALID;
      jc.b_bits = idx->b_bits;
      jc.cols_resident = true;
    }
    Arena ar(st);
    Timer t_prep;
    check(hipEventRecord(t_prep.ev[0], st));
    JoinCounters *ctr = ar.alloc<JoinCounters>(1);
    check(launch_reset_all(ctr, st));
    Space A;
    space_begin(A, sides.data(), n, ar, st);
    sync(st);
    space_sort(A, true, ar, ar, st);
    Marker sorted;
    sorted.record(st);
    early_bitmaps(A, jc, ar, ctr, st);
    sorted.wait();
    space_finish(A);
    early_wide(A, jc, ar, st);
    run_join(A, idx ? idx->S : A, tasks, jc, ar, ctr, st, t_prep, jo, stats);
  } catch (const Fail &f) {
    HostPairs::get().release(jo.pairs);
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    HostPairs::get().release(jo.pairs);
    return SSJ_E_NOMEM;
  }
  out->pairs = jo.pairs;
  out->count = jo.count;
  if (starts) {
    if (jo.task_start.size() == (size_t)n + 1) std::memcpy(starts, jo.task_start.data(), (n + 1) * 8);
    else std::memset(starts, 0, ((size_t)n + 1) * 8);
  }
  if (stats) stats->ms_total = ms_since(t_start);
  return SSJ_OK;
}

// Arguments of ssj_build_bitmaps: the generator to build (Bitmap-Combined
// resolved by Alg. 6 from the Jaccard threshold p/q), or a status < 0.
int bitmap_args(const ssj_sets *s, uint32_t b_bits, int method, uint32_t p, uint32_t q,
                const uint64_t *bitmaps_dev) {
  if (!s || s->n_sets >= 0xFFFFFFFFull || (s->n_sets > 0 && !s->offsets) ||
      (s->n_tokens > 0 && !s->tokens) || (s->n_sets == 0 && s->n_tokens != 0))
    return SSJ_E_INVALID;
  if (b_bits < 64 || b_bits > 4096 || b_bits % 64) return SSJ_E_INVALID;
  if (method < SSJ_BM_XOR || method > SSJ_BM_COMBINED) return SSJ_E_UNSUPPORTED;
  if (method == SSJ_BM_COMBINED) {
    // Alg. 6 by the normalized value 2t/(1+t) of the Jaccard threshold
    if (p == 0 || q == 0 || p > q) return SSJ_E_INVALID;
    const uint32_t g = std::gcd(p, q);
    uint64_t P = 0, Q = 1;
    normalized_threshold(SSJ_SIM_JACCARD, p / g, q / g, P, Q);
    method = combined_generator(P, Q);
  }
  if (s->n_sets > 0 && !bitmaps_dev) return SSJ_E_INVALID;
  return method;
}

// The bitmaps of one collection in caller order, `method` one of Xor, Set,
// Next.  The offsets are validated first (set sizes, side table and
// counters come from `ar`), the token order on the way.  No host memory is
// allocated.
int build_bitmaps(const ssj_sets *s, uint32_t b_bits, int method, uint64_t *out, hipStream_t st,
                  Arena &ar) {
  const uint64_t n = s->n_sets;
  if (n == 0) return SSJ_OK;
  SideDesc side{};
  side.offsets = s->offsets;
  side.tokens = s->tokens;
  side.n_tokens = s->n_tokens;
  side.base = 0;
  side.n = (uint32_t)n;
  side.blk0 = 0;
  SideDesc *d_side = ar.alloc<SideDesc>(1);
  JoinCounters *ctr = ar.alloc<JoinCounters>(1);
  uint32_t *sizes = ar.alloc<uint32_t>(n);
  uint32_t *side_of = ar.alloc<uint32_t>(n);
  h2d(d_side, &side, 1, st);
  check(launch_reset_all(ctr, st));
  check(launch_set_sizes(d_side, 1, n, sizes, side_of, ctr, st));
  JoinCounters ctr_h{};
  d2h(&ctr_h, ctr, 1, st);
  sync(st);
  if (ctr_h.error & (kErrOffsets | kErrTooBig)) return SSJ_E_INVALID;
  check(launch_build_bitmaps(d_side, 1, bitmap_seg_blocks(n), n, nullptr, nullptr, nullptr,
                             b_bits, method, b_bits / 64, out, ctr, st));
  d2h(&ctr_h, ctr, 1, st);
  sync(st);
  if (ctr_h.error & kErrUnsorted) return SSJ_E_UNSORTED;
  return SSJ_OK;
}

// Device memory of ssj_build_bitmaps_noalloc: side table, counters and the
// set sizes of one collection, in a fixed array of every device.  Host code
// reaches a device's copy only through the address hipGetSymbolAddress
// returns for it (kept per device in g_scratch).
constexpr uint64_t kScratchBytes = 32ull << 20;
constexpr int kScratchDevices = 64;
constexpr uint64_t round256(uint64_t b) { return (b + 255) & ~255ull; }
static_assert(round256(sizeof(SideDesc)) + round256(sizeof(JoinCounters)) +
                      2 * round256(4ull * SSJ_NOALLOC_MAX_SETS) <= kScratchBytes,
              "SSJ_NOALLOC_MAX_SETS sets fit the scratch array");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
  std::mutex mu;       // held for a whole call: calls on one device never overlap
  void *ptr = nullptr; // the device's copy of `scratch`
};
ScratchSlot g_scratch[kScratchDevices];

}  // namespace
}  // namespace ssj

extern "C" {

int ssj_abi_version(void) { return SSJ_ABI_VERSION; }

int ssj_memory_limit(uint64_t bytes, uint64_t *held) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return SSJ_E_DEVICE;
  }
  const uint64_t h = ssj::ChunkCache::get().limit(bytes, dev);
  if (held) *held = h;
  return SSJ_OK;
}

const char *ssj_status_string(int status) {
  switch (status) {
    case SSJ_OK: return "ok";
    case SSJ_E_INVALID: return "invalid argument";
    case SSJ_E_UNSORTED: return "a set is not strictly increasing";
    case SSJ_E_NOMEM: return "out of memory";
    case SSJ_E_DEVICE: return "device error";
    case SSJ_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int ssj_build_bitmaps(const ssj_sets *s, uint32_t b_bits, int method, uint32_t p, uint32_t q,
                      uint64_t *bitmaps_dev, void *hip_stream) {
  using namespace ssj;
  try {
    const int m = bitmap_args(s, b_bits, method, p, q, bitmaps_dev);
    if (m < 0) return m;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Arena ar(st);
    return build_bitmaps(s, b_bits, m, bitmaps_dev, st, ar);
  } catch (const Fail &f) {
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    return SSJ_E_NOMEM;
  }
}

int ssj_build_bitmaps_noalloc(const ssj_sets *s, uint32_t b_bits, int method, uint32_t p,
                              uint32_t q, uint64_t *bitmaps_dev, void *hip_stream) {
  using namespace ssj;
  const int m = bitmap_args(s, b_bits, method, p, q, bitmaps_dev);
  if (m < 0) return m;
  if (s->n_sets > SSJ_NOALLOC_MAX_SETS) return SSJ_E_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
    (void)hipGetLastError();
    return SSJ_E_DEVICE;
  }
  ScratchSlot &slot = g_scratch[dev];
  std::lock_guard<std::mutex> lk(slot.mu);  // one call at a time per device
  if (!slot.ptr) {
    // the device's copy of the array: its address is known only at run time
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return SSJ_E_DEVICE;
    }
    slot.ptr = ptr;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    Arena ar(st, slot.ptr, kScratchBytes);
    return build_bitmaps(s, b_bits, m, bitmaps_dev, st, ar);
  } catch (const Fail &f) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    return f.code;
  }
}

int ssj_self_join(const ssj_sets *s, const uint64_t *bitmaps_dev, uint32_t b_bits, int sim,
                  uint32_t p, uint32_t q, const ssj_options *opts, ssj_pairs *out,
                  ssj_stats *stats, void *hip_stream) {
  return ssj::join_one(s, bitmaps_dev, s, bitmaps_dev, true, b_bits, sim, p, q, opts, out, stats,
                       hip_stream);
}

int ssj_rs_join(const ssj_sets *r, const uint64_t *r_bitmaps_dev, const ssj_sets *s,
                const uint64_t *s_bitmaps_dev, uint32_t b_bits, int sim, uint32_t p, uint32_t q,
                const ssj_options *opts, ssj_pairs *out, ssj_stats *stats, void *hip_stream) {
  if ((r_bitmaps_dev == nullptr) != (s_bitmaps_dev == nullptr)) {
    if (out) {
      out->pairs = nullptr;
      out->count = 0;
    }
    return SSJ_E_INVALID;
  }
  return ssj::join_one(r, r_bitmaps_dev, s, s_bitmaps_dev, false, b_bits, sim, p, q, opts, out,
                       stats, hip_stream);
}

int ssj_self_join_batch(const ssj_sets *sets, uint32_t n_instances, const uint32_t *p,
                        const uint32_t *q, uint32_t b_bits, int sim, const ssj_options *opts,
                        ssj_pairs *out, uint64_t *starts, ssj_stats *stats, void *hip_stream) {
  return ssj::join_tasks(sets, n_instances, p, q, true, nullptr, b_bits, sim, opts, out, starts,
                         stats, hip_stream);
}

int ssj_index_create(const ssj_sets *s, uint32_t b_bits, ssj_index **out, void *hip_stream) {
  using namespace ssj;
  if (!out) return SSJ_E_INVALID;
  *out = nullptr;
  ssj_index *idx = nullptr;
  try {
    validate_sets(s);
    if (b_bits != 0 && (b_bits < 64 || b_bits > 4096 || b_bits % 64)) return SSJ_E_INVALID;
    const uint32_t wfix = b_bits ? filter_padded_words(b_bits / 64) : 0;
    if (b_bits && !wfix) return SSJ_E_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    idx = new ssj_index(st);
    check(hipGetDevice(&idx->device));
    idx->b_bits = b_bits;
    // the index's own copy of the collection
    uint64_t *offs = idx->ar.alloc<uint64_t>(s->n_sets + 1);
    uint32_t *toks = idx->ar.alloc<uint32_t>(s->n_tokens);
    if (s->n_sets)
      check(hipMemcpyAsync(offs, s->offsets, (s->n_sets + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (s->n_tokens)
      check(hipMemcpyAsync(toks, s->tokens, s->n_tokens * 4, hipMemcpyDeviceToDevice, st));
    idx->sets = ssj_sets{s->n_sets ? offs : nullptr, s->n_tokens ? toks : nullptr, s->n_sets,
                         s->n_tokens};
    const ssj_sets *side = &idx->sets;
    {
      Arena tmp(st);
      space_begin(idx->S, &side, 1, idx->ar, st);
      sync(st);
      space_sort(idx->S, true, idx->ar, tmp, st);
      sync(st);
      space_finish(idx->S);
      JoinCounters *ctr = idx->S.ctr;
      check(launch_reset_all(ctr, st));
      if (b_bits) {
        space_bitmaps(idx->S, wfix, b_bits, idx->ar, ctr, st);
      } else {
        uint32_t bits[kNumAuto];
        for (int k = 0; k < kNumAuto; ++k) bits[k] = 64 * kAutoWords[k];
        space_bitmaps_multi(idx->S, kAutoWords, bits, kNumAuto, idx->ar, ctr, st);
      }
      // sign planes of every width the matrix-core filter runs, and wide
      // bitmaps of its large sets for verification
      for (uint32_t k = 0; k < idx->S.n_bm; ++k)
        if (filter_shape(idx->S.bm_words[k], true).mfma)
          space_signs(idx->S, idx->S.bm_words[k], idx->ar, st);
      space_wide(idx->S, idx->ar, st);
      d2h(&idx->S.ctr_h, ctr, 1, st);
      sync(st);
      if (idx->S.ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
    }
  } catch (const Fail &f) {
    (void)hipGetLastError();
    delete idx;
    return f.code;
  } catch (const std::bad_alloc &) {
    delete idx;
    return SSJ_E_NOMEM;
  }
  *out = idx;
  return SSJ_OK;
}

int ssj_index_query(ssj_index *idx, const ssj_sets *batches, uint32_t n_batches,
                    const uint32_t *p, const uint32_t *q, int sim, const ssj_options *opts,
                    ssj_pairs *out, uint64_t *starts, ssj_stats *stats, void *hip_stream) {
  if (!idx) {
    if (out) {
      out->pairs = nullptr;
      out->count = 0;
    }
    return SSJ_E_INVALID;
  }
  return ssj::join_tasks(batches, n_batches, p, q, false, idx, idx->b_bits, sim, opts, out,
                         starts, stats, hip_stream);
}

void ssj_index_destroy(ssj_index *idx) { delete idx; }

int ssj_plan_self_join_batch(const ssj_sets *sets, uint32_t n_instances, const uint32_t *p,
                             const uint32_t *q, uint32_t b_bits, int sim,
                             const ssj_options *opts, ssj_plan **out, void *hip_stream) {
  using namespace ssj;
  if (!out) return SSJ_E_INVALID;
  *out = nullptr;
  if (n_instances == 0 || !sets || !p || !q) return SSJ_E_INVALID;
  ssj_plan *plan = nullptr;
  try {
    const JoinConfig jc = config_of(b_bits, opts);
    std::vector<TaskIn> tasks(n_instances);
    std::vector<const ssj_sets *> sides(n_instances);
    for (uint32_t k = 0; k < n_instances; ++k) {
      uint32_t pk = p[k], qk = q[k];
      check_threshold(sim, pk, qk);
      tasks[k] = {k, k, sim, pk, qk, true};
      sides[k] = sets + k;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    plan = new ssj_plan(st);
    check(hipGetDevice(&plan->device));
    plan->n_tasks = n_instances;
    check(hipEventCreate(&plan->ev[0]));
    check(hipEventCreate(&plan->ev[1]));
    JoinCounters *ctr = plan->ar.alloc<JoinCounters>(1);
    check(launch_reset_all(ctr, st));
    {
      Arena tmp(st);  // the size sort's temporaries
      space_begin(plan->S, sides.data(), n_instances, plan->ar, st);
      sync(st);
      space_sort(plan->S, true, plan->ar, tmp, st);
      sync(st);
      space_finish(plan->S);
    }
    // every execution starts from zeroed counters and cursors
    Launcher L(true);
    L.run(st, [=](hipStream_t s) { return launch_reset_all(ctr, s); });
    join_begin(plan->S, plan->S, tasks, jc, plan->ar, ctr, st, nullptr, &L, nullptr, plan->jr);
    sync(st);
    // the recorded work, captured on the plan's own stream (the legacy
    // default stream cannot be captured), at the default priority
    check(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    check(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      L.replay(plan->cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(plan->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    check(hipStreamEndCapture(plan->cap_stream, &plan->graph));
    check(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
  } catch (const Fail &f) {
    (void)hipGetLastError();
    delete plan;
    return f.code;
  } catch (const std::bad_alloc &) {
    delete plan;
    return SSJ_E_NOMEM;
  }
  *out = plan;
  return SSJ_OK;
}

int ssj_plan_execute(ssj_plan *plan, ssj_pairs *out, uint64_t *starts, ssj_stats *stats,
                     void *hip_stream) {
  using namespace ssj;
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return SSJ_E_INVALID;
  clear_out(out, stats);
  if (!plan) return SSJ_E_INVALID;
  std::lock_guard<std::mutex> lk(plan->mu);
  JoinOut jo;
  try {
    int dev = 0;
    check(hipGetDevice(&dev));
    if (dev != plan->device) return SSJ_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Arena tmp(st);  // drain rounds and the result sort
    RoundTimes tm;
    tm.graph_ev[0] = plan->ev[0];
    tm.graph_ev[1] = plan->ev[1];
    check(hipEventRecord(plan->ev[0], st));
    check(hipGraphLaunch(plan->exec, st));
    check(hipEventRecord(plan->ev[1], st));
    join_end(plan->jr, tmp, st, tm, nullptr, jo, stats);
  } catch (const Fail &f) {
    HostPairs::get().release(jo.pairs);
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    HostPairs::get().release(jo.pairs);
    return SSJ_E_NOMEM;
  }
  out->pairs = jo.pairs;
  out->count = jo.count;
  if (starts) {
    if (jo.task_start.size() == (size_t)plan->n_tasks + 1)
      std::memcpy(starts, jo.task_start.data(), ((size_t)plan->n_tasks + 1) * 8);
    else std::memset(starts, 0, ((size_t)plan->n_tasks + 1) * 8);
  }
  if (stats) stats->ms_total = ms_since(t_start);
  return SSJ_OK;
}

void ssj_plan_destroy(ssj_plan *plan) { delete plan; }

int ssj_cutoff(uint32_t b_bits, int method, int sim, uint32_t p, uint32_t q, uint32_t *out) {
  using namespace ssj;
  if (!out) return SSJ_E_INVALID;
  *out = 0;
  if (b_bits < 64 || b_bits > 4096 || b_bits % 64) return SSJ_E_INVALID;
  if (method < SSJ_BM_XOR || method > SSJ_BM_COMBINED) return SSJ_E_UNSUPPORTED;
  try {
    check_threshold(sim, p, q);
  } catch (const Fail &f) {
    return f.code;
  }
  *out = cutoff_point(method, b_bits, sim, p, q);
  return SSJ_OK;
}

void ssj_free_pairs(ssj_pairs *out) {
  if (!out) return;
  ssj::HostPairs::get().release(out->pairs);
  out->pairs = nullptr;
  out->count = 0;
}

}  // extern "C"
