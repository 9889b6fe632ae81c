// C-ABI host layer of the library: argument checks, the size-ordered
// preparation of each collection, the tile plan of the length band, the
// filter/verify rounds over a bounded survivor queue, and the emission of
// the sorted result pairs.  Every step of the join runs in the library's
// own kernels; the host only plans, launches and copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <numeric>
#include <vector>

#include "ssj.h"
#include "ssj_internal.h"

namespace ssj {
namespace {

constexpr uint64_t kDefaultQueue = 1ull << 27;   // 1 GiB of (row, column) pairs
constexpr uint32_t kDefaultTileCols = 2048;
constexpr uint64_t kMaxTable = 1ull << 26;       // largest |r| + |s| handled

struct Fail {
  int code;
};

inline void check(hipError_t e) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) throw Fail{SSJ_E_NOMEM};
  throw Fail{SSJ_E_DEVICE};
}

// Device memory chunks kept between calls, per device.  A call takes chunks
// at its start and gives them back only after its final stream
// synchronisation, so a chunk is never in use by two calls.  Chunk sizes are
// powers of two (at least 64 MiB), so a chunk fits any later request of up to
// its size.  The cache lives until the process ends.
class ChunkCache {
 public:
  static ChunkCache &get() {
    static ChunkCache c;
    return c;
  }
  void *take(int dev, uint64_t size) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto &v = free_[dev & 63];
      for (size_t k = 0; k < v.size(); ++k)
        if (v[k].size == size) {
          void *p = v[k].ptr;
          v[k] = v.back();
          v.pop_back();
          return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void give(int dev, void *p, uint64_t size) {
    std::lock_guard<std::mutex> lk(mu_);
    free_[dev & 63].push_back({p, size});
  }

 private:
  struct Chunk {
    void *ptr;
    uint64_t size;
  };
  std::mutex mu_;
  std::vector<Chunk> free_[64];
};

// Device memory of one call, carved from cached chunks.  The destructor
// returns the chunks; every exit path synchronises the stream first.
class Arena {
 public:
  explicit Arena(hipStream_t st) : st_(st) {
    if (hipGetDevice(&dev_) != hipSuccess) dev_ = 0;
  }
  ~Arena() {
    (void)hipStreamSynchronize(st_);
    for (auto &c : chunks_) ChunkCache::get().give(dev_, c.first, c.second);
  }
  template <class T>
  T *alloc(uint64_t n) {
    uint64_t bytes = (std::max<uint64_t>(n, 1) * sizeof(T) + 255) & ~255ull;
    if (bytes > left_) {
      uint64_t size = kChunk;
      while (size < bytes) size <<= 1;
      void *p = ChunkCache::get().take(dev_, size);
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

 private:
  static constexpr uint64_t kChunk = 64ull << 20;
  hipStream_t st_;
  int dev_ = 0;
  std::vector<std::pair<void *, uint64_t>> chunks_;
  char *next_ = nullptr;
  uint64_t left_ = 0;
};

template <class T>
void d2h(T *dst, const T *src, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  check(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, st));
}
template <class T>
void h2d(T *dst, const T *src, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  check(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, st));
}
void sync(hipStream_t st) { check(hipStreamSynchronize(st)); }

int bits_for(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// One collection, validated and in size order.
struct Side {
  const ssj_sets *in = nullptr;
  uint64_t n = 0;
  uint32_t max_size = 0;
  uint32_t *sizes = nullptr;   // size order
  uint32_t *perm = nullptr;    // size order -> caller index
  uint32_t *rank = nullptr;    // caller index -> size order
  uint32_t *sstart = nullptr;  // [max_size + 2]
  std::vector<uint32_t> sstart_h;
  uint64_t *bm = nullptr;      // size-order bitmaps of every width, one after the other
  uint32_t first_nonempty() const { return sstart_h.size() > 1 ? sstart_h[1] : (uint32_t)n; }
  uint64_t count_of(uint32_t s) const { return (uint64_t)sstart_h[s + 1] - sstart_h[s]; }
};

void validate_sets(const ssj_sets *s) {
  if (!s) throw Fail{SSJ_E_INVALID};
  if (s->n_sets >= 0xFFFFFFFFull) throw Fail{SSJ_E_INVALID};
  if (s->n_sets > 0 && !s->offsets) throw Fail{SSJ_E_INVALID};
  if (s->n_tokens > 0 && !s->tokens) throw Fail{SSJ_E_INVALID};
}

// Sizes and offset check (one sync for the largest size), stable size sort,
// group starts (copied to the host; the caller synchronises).
void order(Side &sd, const ssj_sets *s, Arena &ar, hipStream_t st) {
  sd.in = s;
  sd.n = s->n_sets;
  const uint64_t n = sd.n;
  JoinCounters *ctr = ar.alloc<JoinCounters>(1);
  JoinCounters ctr_h;
  check(launch_reset_all(ctr, st));
  unsigned long long *keys = ar.alloc<unsigned long long>(n);
  check(launch_set_sizes(s->offsets, n, s->n_tokens, keys, ctr, st));
  d2h(&ctr_h, ctr, 1, st);
  sync(st);
  if (ctr_h.error & (kErrOffsets | kErrTooBig)) throw Fail{SSJ_E_INVALID};
  if (n == 0 && s->n_tokens != 0) throw Fail{SSJ_E_INVALID};
  sd.max_size = ctr_h.max_size;
  if ((uint64_t)sd.max_size * 2 + 2 > kMaxTable) throw Fail{SSJ_E_UNSUPPORTED};

  // stable sort by size: keys (size << 32 | index), digits of the size only
  unsigned long long *tmp = ar.alloc<unsigned long long>(n);
  uint32_t *scr = ar.alloc<uint32_t>(radix_scratch_words(n));
  int shifts[4], ns = 0;
  for (int b = 0; b < bits_for(sd.max_size); b += 8) shifts[ns++] = 32 + b;
  unsigned long long *sorted = keys;
  check(radix_sort_u64(keys, tmp, n, shifts, ns, scr, st, &sorted));
  sd.sizes = ar.alloc<uint32_t>(n);
  sd.perm = ar.alloc<uint32_t>(n);
  check(launch_unpack_keys(sorted, n, sd.sizes, sd.perm, st));
  sd.sstart = ar.alloc<uint32_t>((uint64_t)sd.max_size + 2);
  check(launch_group_starts(sd.sizes, n, sd.max_size, sd.sstart, st));
  sd.sstart_h.assign((size_t)sd.max_size + 2, 0);
  d2h(sd.sstart_h.data(), sd.sstart, sd.sstart_h.size(), st);
}

// The bitmap widths of a join.  Each slot k holds the bitmaps of all sets in
// size order at `words[k]` 64-bit words (b = 64 * words[k] bits, or the
// caller's b padded to words[k]) at word offset off[k] of Side::bm.
struct Widths {
  uint32_t n = 0;
  uint32_t words[4] = {0, 0, 0, 0};
  uint32_t bits[4] = {0, 0, 0, 0};     // the width b the bitmaps are built for
  uint64_t off[4] = {0, 0, 0, 0};
  uint32_t slot_of(uint32_t w) const {
    for (uint32_t k = 0; k < n; ++k)
      if (words[k] == w) return k;
    return 0;
  }
};

// Bitmap-Xor bitmaps of every slot (or the caller's, gathered and padded).
// Token-order violations are reported in ctr->error.
void build_bitmaps(Side &sd, const uint64_t *bm_caller, const Widths &wd, Arena &ar,
                   JoinCounters *ctr, hipStream_t st) {
  const uint64_t n = sd.n;
  uint64_t total = 0;
  for (uint32_t k = 0; k < wd.n; ++k) total = std::max(total, wd.off[k] + n * wd.words[k]);
  sd.bm = ar.alloc<uint64_t>(total);
  if (bm_caller) {  // one slot, the caller's width
    check(launch_gather_bitmaps(bm_caller, sd.perm, n, wd.bits[0] / 64, wd.words[0],
                                sd.bm + wd.off[0], st));
    check(launch_check_sorted(sd.in->offsets, sd.in->tokens, n, ctr, st));
    return;
  }
  sd.rank = ar.alloc<uint32_t>(n);
  check(launch_invert_perm(sd.perm, n, sd.rank, st));
  for (uint32_t k = 0; k < wd.n; ++k)
    check(launch_build_bitmaps(sd.in->offsets, sd.in->tokens, sd.perm, sd.rank, n, wd.bits[k],
                               SSJ_BM_XOR, wd.words[k], sd.bm + wd.off[k], ctr, st));
}

// Least overlap o with sim >= p/q for sizes summing to L (Jaccard, Table 1):
// o / (L - o) >= p / q  <=>  (p + q) o >= p L.
inline uint32_t jaccard_omin(uint64_t L, uint64_t p, uint64_t q) {
  return (uint32_t)((p * L + (p + q) - 1) / (p + q));
}

// P(X <= k) for X ~ Binomial(n, pi), summed in log space.
double binomial_cdf(int n, double pi, int64_t k) {
  if (k < 0) return 0.0;
  if (k >= n) return 1.0;
  if (pi <= 0.0) return 1.0;
  if (pi >= 1.0) return 0.0;
  const double lp = std::log(pi), lq = std::log1p(-pi);
  double acc = 0.0, lc = 0.0;  // log C(n, i)
  for (int64_t i = 0; i <= k; ++i) {
    if (i > 0) lc += std::log((double)(n - i + 1)) - std::log((double)i);
    acc += std::exp(lc + i * lp + (n - i) * lq);
  }
  return std::min(acc, 1.0);
}

// Width classes for the automatic mode.  For a row of size a against columns
// of about its size (L = 2a), model the bits in which the bitmaps of two
// unrelated sets differ as Binomial(b, pi) with pi = (1 - (1 - 2/b)^L) / 2,
// the chance that a bit receives an odd number of the L tokens (the quantity
// Eq. 5 sums; Section 3.4).  A pair is a false survivor when that count is at
// most slack(L).  Per row size the width minimising
//   (b/16 + 1)  +  P(false survivor) * kSurvivorCost
// lane-ops per band pair is chosen, b in {64, 128, 256, 512}; widths never
// decrease with the size.  kSurvivorCost prices a survivor (queue slot,
// slow path, verification) in filter lane-ops.
constexpr double kSurvivorCost = 3000.0;
constexpr uint32_t kAutoWords[4] = {1, 2, 4, 8};  // b = 64, 128, 256, 512

struct WidthClass {
  uint32_t max_size;  // rows of size in (previous max_size, max_size]
  uint32_t words;
};

std::vector<WidthClass> choose_classes(uint32_t max_rows, uint64_t p, uint64_t q) {
  std::vector<WidthClass> cls;
  uint32_t cur = 1;
  for (uint32_t a = 1; a <= max_rows; ++a) {
    const uint64_t L = 2ull * a;
    const int64_t slack = (int64_t)L - 2 * (int64_t)jaccard_omin(L, p, q);
    uint32_t best = cur;
    double best_cost = 1e300;
    for (uint32_t w : kAutoWords) {
      if (w < cur) continue;
      const double b = 64.0 * w;
      const double pi = 0.5 * (1.0 - std::pow(1.0 - 2.0 / b, (double)L));
      const double cost = (b / 16 + 1) + binomial_cdf((int)b, pi, slack) * kSurvivorCost;
      if (cost < best_cost) {
        best_cost = cost;
        best = w;
      }
    }
    cur = best;
    if (!cls.empty() && cls.back().words == cur) cls.back().max_size = a;
    else cls.push_back({a, cur});
  }
  if (cls.empty()) cls.push_back({max_rows, kAutoWords[0]});
  cls.back().max_size = max_rows;
  return cls;
}

struct Plan {
  std::vector<int32_t> slack;   // [maxA + maxB + 1]
  std::vector<uint32_t> omin;   // [maxA + maxB + 1]
  std::vector<uint32_t> cmin, cmax;  // [maxA + 1]
  std::vector<RowBlock> blocks;
  uint32_t n_tiles = 0;
  uint64_t band_pairs = 0;
  uint64_t filter_ops = 0;      // sum over band pairs of b/16 + 1
  uint32_t max_batch = 0;       // largest queue reservation of the kernels used
  // per width class: its tiles [tile_lo[k], tile_hi[k]) and padded width
  uint32_t n_classes = 0;
  uint32_t tile_lo[kMaxClasses] = {0, 0, 0, 0}, tile_hi[kMaxClasses] = {0, 0, 0, 0};
  uint32_t words[kMaxClasses] = {0, 0, 0, 0};
  uint64_t ops[kMaxClasses] = {0, 0, 0, 0};
};

void make_tables(Plan &pl, const Side &A, const Side &B, uint64_t p, uint64_t q) {
  const uint64_t maxA = A.max_size, maxB = B.max_size;
  pl.slack.resize(maxA + maxB + 1);
  pl.omin.resize(maxA + maxB + 1);
  for (uint64_t L = 0; L <= maxA + maxB; ++L) {
    uint32_t o = jaccard_omin(L, p, q);
    pl.omin[L] = o;
    pl.slack[L] = (int32_t)((int64_t)L - 2 * (int64_t)o);
  }
  // Length filter (Table 2, Jaccard): t |r| <= |s| <= |r| / t.  Empty sets
  // never pair: an empty row gets an empty range, and cmin >= 1 otherwise.
  pl.cmin.resize(maxA + 1);
  pl.cmax.resize(maxA + 1);
  for (uint64_t a = 0; a <= maxA; ++a) {
    if (a == 0) {
      pl.cmin[a] = 0xFFFFFFFFu;
      pl.cmax[a] = 0;
      continue;
    }
    uint64_t lo = (p * a + q - 1) / q;   // ceil(p a / q)
    uint64_t hi = (q * a) / p;           // floor(q a / p)
    if (lo < 1) lo = 1;
    pl.cmin[a] = (uint32_t)std::min<uint64_t>(lo, 0xFFFFFFFFull);
    pl.cmax[a] = (uint32_t)std::min<uint64_t>(hi, 0xFFFFFFFFull);
  }
}

// Row blocks and tiles of the length band.  Rows of size in (lo, hi] use
// `words`-word bitmaps of nominal width `bits`; blocks never straddle classes.
void plan_class(Plan &pl, const Side &A, const Side &B, bool self, uint32_t lo, uint32_t hi,
                uint32_t words, uint32_t bits, uint32_t tile_cols) {
  const uint64_t maxA = A.max_size, maxB = B.max_size;
  const FilterShape shape = filter_shape(words);
  pl.max_batch = std::max(pl.max_batch, shape.batch);
  auto col_lo = [&](uint64_t a) -> uint32_t {  // first column with size >= cmin[a]
    uint64_t c = pl.cmin[a];
    return c > maxB ? (uint32_t)B.n : B.sstart_h[c];
  };
  auto col_hi = [&](uint64_t a) -> uint32_t {  // first column with size > cmax[a]
    uint64_t c = pl.cmax[a];
    return c >= maxB ? (uint32_t)B.n : B.sstart_h[c + 1];
  };
  hi = (uint32_t)std::min<uint64_t>(hi, maxA);
  if (lo >= hi) return;
  // band pairs of the class, exactly
  uint64_t band = 0;
  for (uint64_t a = lo + 1; a <= hi; ++a) {
    uint64_t cnt = A.count_of((uint32_t)a);
    if (!cnt) continue;
    if (self) {
      band += cnt * ((uint64_t)A.sstart_h[a] - col_lo(a)) + cnt * (cnt - 1) / 2;
    } else {
      uint64_t l = col_lo(a), h = col_hi(a);
      if (h > l) band += cnt * (h - l);
    }
  }
  pl.band_pairs += band;
  pl.filter_ops += band * (bits / 16 + 1);

  const uint32_t rows_per_block = shape.rows;
  const uint32_t r_begin = A.sstart_h[lo + 1], r_end = A.sstart_h[hi + 1];
  uint64_t tiles = pl.n_tiles;
  uint32_t s_of = lo + 1;  // size of the current row, advanced monotonically
  auto size_at = [&](uint32_t row) {
    while (s_of + 1 <= hi && A.sstart_h[s_of + 1] <= row) ++s_of;
    return s_of;
  };
  for (uint64_t r0 = r_begin; r0 < r_end; r0 += rows_per_block) {
    const uint32_t row0 = (uint32_t)r0;
    const uint32_t row_end = (uint32_t)std::min<uint64_t>(r0 + rows_per_block, r_end);
    const uint32_t a0 = size_at(row0);
    RowBlock rb{};
    rb.row0 = row0;
    rb.row_end = row_end;
    rb.words = words;
    rb.tile_begin = (uint32_t)tiles;
    uint64_t nt;
    if (self) {
      rb.col_begin = std::min(col_lo(a0), row0);
      rb.col_end = row_end;
      nt = ((uint64_t)row0 - rb.col_begin + tile_cols - 1) / tile_cols + 1;
    } else {
      const uint32_t s_save = s_of;
      const uint32_t a1 = size_at(row_end - 1);  // the block's largest size
      s_of = s_save;
      rb.col_begin = col_lo(a0);
      rb.col_end = std::max(col_hi(a1), rb.col_begin);
      nt = ((uint64_t)rb.col_end - rb.col_begin + tile_cols - 1) / tile_cols;
    }
    tiles += nt;
    if (tiles >= 0xFFFFFFFFull) throw Fail{SSJ_E_UNSUPPORTED};
    pl.blocks.push_back(rb);
  }
  pl.n_tiles = (uint32_t)tiles;
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

int join(const ssj_sets *R, const uint64_t *r_bm, const ssj_sets *S, const uint64_t *s_bm,
         bool self, uint32_t b_bits, int sim, uint32_t p, uint32_t q, const ssj_options *opts,
         ssj_pairs *out, ssj_stats *stats, void *hip_stream) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return SSJ_E_INVALID;
  out->pairs = nullptr;
  out->count = 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  try {
    validate_sets(R);
    if (!self) validate_sets(S);
    const bool automatic = b_bits == 0;
    if (!automatic && (b_bits < 64 || b_bits > 4096 || b_bits % 64)) return SSJ_E_INVALID;
    if (automatic && (r_bm || s_bm)) return SSJ_E_INVALID;
    if (sim < SSJ_SIM_JACCARD || sim > SSJ_SIM_OVERLAP) return SSJ_E_INVALID;
    if (p == 0 || q == 0 || p > q) return SSJ_E_INVALID;
    if (sim != SSJ_SIM_JACCARD) return SSJ_E_UNSUPPORTED;
    const uint32_t g = std::gcd(p, q);
    p /= g;
    q /= g;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const uint32_t tile_cols = opts && opts->tile_cols ? opts->tile_cols : kDefaultTileCols;
    const uint64_t cap = opts && opts->queue_capacity ? opts->queue_capacity : kDefaultQueue;
    const bool survivors_only = opts && (opts->flags & SSJ_FLAG_SURVIVORS_ONLY);

    Arena ar(st);
    Timer t_prep, t_emit;
    check(hipEventRecord(t_prep.ev[0], st));
    JoinCounters *ctr = ar.alloc<JoinCounters>(1);
    JoinCounters ctr_h;
    check(launch_reset_all(ctr, st));

    Side A, B;
    order(A, R, ar, st);
    if (!self) order(B, S, ar, st);
    sync(st);  // group starts on the host
    const Side &Bc = self ? A : B;

    // bitmap widths: one fixed width, or classes of row sizes
    Widths wd;
    std::vector<WidthClass> classes;
    if (automatic) {
      classes = choose_classes(std::max<uint32_t>(A.max_size, 1), p, q);
      for (uint32_t w : kAutoWords) {
        bool used = false;
        for (auto &c : classes) used |= c.words == w;
        if (!used) continue;
        wd.words[wd.n] = w;
        wd.bits[wd.n] = 64 * w;
        ++wd.n;
      }
    } else {
      const uint32_t wpad = filter_padded_words(b_bits / 64);
      if (!wpad) return SSJ_E_UNSUPPORTED;
      wd.n = 1;
      wd.words[0] = wpad;
      wd.bits[0] = b_bits;
      classes.push_back({A.max_size, wpad});
    }
    if (classes.size() > kMaxClasses) throw Fail{SSJ_E_DEVICE};
    uint64_t o_a = 0, o_b = 0;
    for (uint32_t k = 0; k < wd.n; ++k) {
      wd.off[k] = o_a;
      o_a += A.n * wd.words[k];
    }
    Widths wd_b = wd;
    for (uint32_t k = 0; k < wd.n; ++k) {
      wd_b.off[k] = o_b;
      o_b += Bc.n * wd.words[k];
    }
    build_bitmaps(A, r_bm, wd, ar, ctr, st);
    if (!self) build_bitmaps(B, s_bm, wd_b, ar, ctr, st);

    Plan pl;
    make_tables(pl, A, Bc, p, q);
    uint32_t prev = 0;
    for (auto &c : classes) {
      const uint32_t bits = automatic ? 64 * c.words : b_bits;
      const uint32_t k = pl.n_classes++;
      pl.tile_lo[k] = pl.n_tiles;
      pl.words[k] = c.words;
      const uint64_t ops0 = pl.filter_ops;
      plan_class(pl, A, Bc, self, prev, c.max_size, c.words, bits, tile_cols);
      pl.tile_hi[k] = pl.n_tiles;
      pl.ops[k] = pl.filter_ops - ops0;
      prev = c.max_size;
    }

    // the plan's tables go up in one copy: blocks, slack, omin, cmin, cmax
    const uint64_t nL = pl.slack.size(), nA = pl.cmin.size(), nB = pl.blocks.size();
    constexpr uint64_t kBlockWords = sizeof(RowBlock) / 4;
    std::vector<uint32_t> packed(kBlockWords * nB + 2 * nL + 2 * nA);
    std::memcpy(packed.data(), pl.blocks.data(), nB * sizeof(RowBlock));
    uint32_t *tab = packed.data() + kBlockWords * nB;
    std::memcpy(tab, pl.slack.data(), nL * 4);
    std::memcpy(tab + nL, pl.omin.data(), nL * 4);
    std::memcpy(tab + 2 * nL, pl.cmin.data(), nA * 4);
    std::memcpy(tab + 2 * nL + nA, pl.cmax.data(), nA * 4);
    uint32_t *d_packed = ar.alloc<uint32_t>(packed.size());
    h2d(d_packed, packed.data(), packed.size(), st);
    RowBlock *d_blocks = reinterpret_cast<RowBlock *>(d_packed);
    uint32_t *d_tab = d_packed + kBlockWords * nB;
    int32_t *d_slack = reinterpret_cast<int32_t *>(d_tab);
    uint32_t *d_omin = d_tab + nL;
    uint32_t *d_cmin = d_tab + 2 * nL;
    uint32_t *d_cmax = d_tab + 2 * nL + nA;
    uint32_t *d_tile_block = ar.alloc<uint32_t>(pl.n_tiles);
    check(launch_expand_tiles(d_blocks, (uint32_t)nB, pl.n_tiles, d_tile_block, st));
    check(hipEventRecord(t_prep.ev[1], st));

    // filter / verify rounds.  A queue reservation covers one step of U
    // columns for all of a wave's rows; the queue must hold the largest such
    // batch, or a full step could never be written and its tile never resumed.
    const uint64_t qcap = std::max<uint64_t>(std::max<uint64_t>(pl.max_batch, 4096),
                                             std::min<uint64_t>(cap, pl.band_pairs + 1));
    uint2 *queue = ar.alloc<uint2>(qcap);
    const uint32_t max_waves = (uint32_t)filter_grid_blocks() * (kBlock / 64);
    Resume *res_a = ar.alloc<Resume>(max_waves), *res_b = ar.alloc<Resume>(max_waves);
    uint64_t res_cap = std::max<uint64_t>(qcap, 1024);
    unsigned long long *results = ar.alloc<unsigned long long>(res_cap);

    std::deque<Timer> t_filter, t_verify;  // events must not move
    std::vector<uint32_t> t_filter_cls;
    uint32_t n_resume_in = 0;
    uint64_t results_n = 0;
    FilterConfig cfg{};
    cfg.n_rows = (uint32_t)A.n;
    cfg.n_cols = (uint32_t)Bc.n;
    cfg.n_tiles = pl.n_tiles;
    cfg.tile_cols = tile_cols;
    cfg.self = self ? 1u : 0u;
    cfg.n_blocks = (uint32_t)nB;
    cfg.resume_cap = max_waves;
    cfg.cap = qcap;
    for (;;) {
      if (pl.n_tiles == 0) break;
      cfg.n_resume_in = n_resume_in;
      // one launch per width class; after an overflow the later launches of
      // the round leave at once and resume in the next round
      for (uint32_t k = 0; k < pl.n_classes; ++k) {
        if (pl.tile_hi[k] == pl.tile_lo[k]) continue;
        cfg.tile_lo = pl.tile_lo[k];
        cfg.tile_hi = pl.tile_hi[k];
        cfg.cls = k;
        const uint32_t slot = wd.slot_of(pl.words[k]);
        FilterArgs fa{A.bm + wd.off[slot], Bc.bm + wd_b.off[slot], A.sizes, Bc.sizes,
                      Bc.sstart, d_slack, d_cmin, d_cmax, d_blocks, d_tile_block, queue, ctr,
                      res_a, res_b, cfg};
        t_filter.emplace_back();
        t_filter_cls.push_back(k);
        check(hipEventRecord(t_filter.back().ev[0], st));
        check(launch_filter(pl.words[k], fa, st));
        check(hipEventRecord(t_filter.back().ev[1], st));
      }
      t_verify.emplace_back();
      check(hipEventRecord(t_verify.back().ev[0], st));
      check(launch_verify(queue, qcap, R->offsets, R->tokens, A.perm,
                          self ? R->offsets : S->offsets, self ? R->tokens : S->tokens, Bc.perm,
                          d_omin, (uint32_t)A.n, (uint32_t)Bc.n, self ? 1u : 0u,
                          survivors_only ? 1u : 0u, results, res_cap, ctr, st));
      check(hipEventRecord(t_verify.back().ev[1], st));
      d2h(&ctr_h, ctr, 1, st);
      sync(st);
      if (ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
      if (ctr_h.error & kErrPlan) throw Fail{SSJ_E_DEVICE};
      results_n = ctr_h.results;
      if (results_n > res_cap) throw Fail{SSJ_E_DEVICE};  // cannot happen: capacity grows first
      if (!ctr_h.overflow) break;
      // drain done; make room for another full queue of results, then resume
      if (results_n + qcap > res_cap) {
        uint64_t ncap = std::max<uint64_t>(2 * res_cap, results_n + qcap);
        unsigned long long *nr = ar.alloc<unsigned long long>(ncap);
        check(launch_copy_u64(results, results_n, nr, st));
        results = nr;
        res_cap = ncap;
      }
      n_resume_in = ctr_h.n_resume;
      std::swap(res_a, res_b);
      check(launch_reset_round(ctr, st));
    }
    if (pl.n_tiles == 0) {
      // nothing to filter; still report unsorted input
      d2h(&ctr_h, ctr, 1, st);
      sync(st);
      if (ctr_h.error & kErrUnsorted) throw Fail{SSJ_E_UNSORTED};
    }

    // emit: sort keys (i << 32 | j) by j's digits then i's, copy out
    check(hipEventRecord(t_emit.ev[0], st));
    ssj_pair *host = nullptr;
    if (results_n) {
      unsigned long long *tmp = ar.alloc<unsigned long long>(results_n);
      uint32_t *scr = ar.alloc<uint32_t>(radix_scratch_words(results_n));
      int shifts[8], ns = 0;
      const uint64_t ni = self ? A.n : A.n, nj = self ? A.n : Bc.n;
      const int bi = bits_for(ni ? ni - 1 : 0), bj = bits_for(nj ? nj - 1 : 0);
      for (int b = 0; b < bj; b += 8) shifts[ns++] = b;
      for (int b = 0; b < bi; b += 8) shifts[ns++] = 32 + b;
      unsigned long long *sorted = results;
      check(radix_sort_u64(results, tmp, results_n, shifts, ns, scr, st, &sorted));
      ssj_pair *dpairs = ar.alloc<ssj_pair>(results_n);
      check(launch_keys_to_pairs(sorted, results_n, dpairs, st));
      host = static_cast<ssj_pair *>(std::malloc(results_n * sizeof(ssj_pair)));
      if (!host) throw Fail{SSJ_E_NOMEM};
      hipError_t e = hipMemcpyAsync(host, dpairs, results_n * sizeof(ssj_pair),
                                    hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        std::free(host);
        check(e);
      }
    }
    check(hipEventRecord(t_emit.ev[1], st));
    sync(st);
    out->pairs = host;
    out->count = results_n;
    if (stats) {
      stats->band_pairs = pl.band_pairs;
      stats->survivors = ctr_h.survivors;
      stats->results = results_n;
      stats->filter_launches = (uint32_t)t_filter.size();
      stats->b_bits = automatic ? 0 : b_bits;
      stats->filter_ops = pl.filter_ops;
      stats->n_classes = (uint32_t)std::min<size_t>(classes.size(), 4);
      prev = 0;
      for (uint32_t k = 0; k < stats->n_classes; ++k) {
        stats->class_bits[k] = automatic ? 64 * classes[k].words : b_bits;
        stats->class_max_size[k] = classes[k].max_size;
      }
      stats->ms_prepare = t_prep.ms();
      for (size_t k = 0; k < t_filter.size(); ++k) {
        const float ms = t_filter[k].ms();
        stats->ms_filter += ms;
        stats->class_ms[t_filter_cls[k]] += ms;
      }
      for (uint32_t k = 0; k < stats->n_classes; ++k) stats->class_ops[k] = pl.ops[k];
      for (auto &t : t_verify) stats->ms_verify += t.ms();
      stats->ms_emit = t_emit.ms();
    }
  } catch (const Fail &f) {
    std::free(out->pairs);
    out->pairs = nullptr;
    out->count = 0;
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    return SSJ_E_NOMEM;
  }
  if (stats) {
    stats->ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                               t_start)
                          .count();
  }
  return SSJ_OK;
}

}  // namespace
}  // namespace ssj

extern "C" {

int ssj_abi_version(void) { return SSJ_ABI_VERSION; }

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

int ssj_build_bitmaps(const ssj_sets *s, uint32_t b_bits, int method, uint64_t *bitmaps_dev,
                      void *hip_stream) {
  using namespace ssj;
  try {
    validate_sets(s);
    if (b_bits < 64 || b_bits > 4096 || b_bits % 64) return SSJ_E_INVALID;
    if (method < SSJ_BM_XOR || method > SSJ_BM_NEXT) return SSJ_E_UNSUPPORTED;
    if (s->n_sets > 0 && !bitmaps_dev) return SSJ_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Arena ar(st);
    JoinCounters *ctr = ar.alloc<JoinCounters>(1);
    JoinCounters ctr_h;
    check(launch_reset_all(ctr, st));
    unsigned long long *keys = ar.alloc<unsigned long long>(s->n_sets);
    check(launch_set_sizes(s->offsets, s->n_sets, s->n_tokens, keys, ctr, st));
    d2h(&ctr_h, ctr, 1, st);
    sync(st);
    if (ctr_h.error & (kErrOffsets | kErrTooBig)) return SSJ_E_INVALID;
    if (s->n_sets == 0) return s->n_tokens ? SSJ_E_INVALID : SSJ_OK;
    check(launch_build_bitmaps(s->offsets, s->tokens, nullptr, nullptr, s->n_sets, b_bits, method,
                               b_bits / 64, bitmaps_dev, ctr, st));
    d2h(&ctr_h, ctr, 1, st);
    sync(st);
    if (ctr_h.error & kErrUnsorted) return SSJ_E_UNSORTED;
  } catch (const Fail &f) {
    (void)hipGetLastError();
    return f.code;
  } catch (const std::bad_alloc &) {
    return SSJ_E_NOMEM;
  }
  return SSJ_OK;
}

int ssj_self_join(const ssj_sets *s, const uint64_t *bitmaps_dev, uint32_t b_bits, int sim,
                  uint32_t p, uint32_t q, const ssj_options *opts, ssj_pairs *out,
                  ssj_stats *stats, void *hip_stream) {
  return ssj::join(s, bitmaps_dev, s, bitmaps_dev, true, b_bits, sim, p, q, opts, out, stats,
                   hip_stream);
}

int ssj_rs_join(const ssj_sets *r, const uint64_t *r_bitmaps_dev, const ssj_sets *s,
                const uint64_t *s_bitmaps_dev, uint32_t b_bits, int sim, uint32_t p, uint32_t q,
                const ssj_options *opts, ssj_pairs *out, ssj_stats *stats, void *hip_stream) {
  if ((r_bitmaps_dev == nullptr) != (s_bitmaps_dev == nullptr)) return SSJ_E_INVALID;
  return ssj::join(r, r_bitmaps_dev, s, s_bitmaps_dev, false, b_bits, sim, p, q, opts, out, stats,
                   hip_stream);
}

void ssj_free_pairs(ssj_pairs *out) {
  if (!out) return;
  std::free(out->pairs);
  out->pairs = nullptr;
  out->count = 0;
}

}  // extern "C"
