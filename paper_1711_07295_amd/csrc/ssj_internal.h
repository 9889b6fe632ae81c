// Internal declarations of the HIP library: device data layouts, kernel
// launchers and the host helpers they share.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssj.h"

namespace ssj {

// Sentinel queue entry: a reserved slot that holds no survivor.
constexpr uint32_t kSentinel = 0xFFFFFFFFu;

// Widest bitmap in 64-bit words (b = 4096 bits).
constexpr uint32_t kMaxWords = 64;

// Threads per workgroup for every kernel of the library (4 wave64s).
constexpr int kBlock = 256;

// Partitions of a tile range (one per XCD of the MI355X).
constexpr uint32_t kXcds = 8;   // XCDs of an MI355X (workgroups go to them round-robin)
constexpr uint32_t kParts = 64; // tile cursors per width class, kParts / kXcds per XCD
// Width classes of one join (one filter launch each).
constexpr uint32_t kMaxClasses = 6;

// Counters of one filter/verify round, in device memory.
struct JoinCounters {
  unsigned long long queue_count;   // slots reserved in the survivor queue
  unsigned long long survivors;     // real survivors seen by verification
  unsigned long long results;       // pairs written to the result buffer
  unsigned long long long_count;    // long pairs deferred by this round's verification
  uint32_t overflow;                // the queue filled during this filter launch
  uint32_t n_resume;                // resume entries written this launch
  uint32_t error;                   // validation error bits (kErr*)
  uint32_t max_size;                // largest set size seen
  // Tile cursors: each width class's tile range is cut into kXcds
  // contiguous regions, one per XCD, and each region's tiles are dealt to
  // kParts / kXcds sub-cursors; a cursor counts the tiles it has handed
  // out.  Each sits in its own 128-byte line.  The host reads only the
  // fields above.
  alignas(128) uint32_t tile_next[kMaxClasses][kParts][32];
};

constexpr uint32_t kErrOffsets = 1u;   // malformed offsets
constexpr uint32_t kErrUnsorted = 2u;  // a set is not strictly increasing
constexpr uint32_t kErrTooBig = 4u;    // a set has 2^32 or more tokens

// One collection of a space (device copy).  A space lays its sides out one
// after the other: the side owns global indices [base, base + n).
struct SideDesc {
  const uint64_t *offsets;  // caller CSR
  const uint32_t *tokens;
  uint64_t n_tokens;
  uint64_t base;
  uint32_t n;
  uint32_t blk0;            // first workgroup of the side in the bitmap build
};

// One join task: the rows of one side of the row space against the columns
// of one side of the column space, with its own similarity function and
// threshold p/q.  Its tables sit in one uint32 array at the given offsets:
// slack[L] and omin[L] for L in [0, a_max + c_max] (functions whose least
// overlap depends on |r| + |s| only; Cosine computes it per size pair),
// cmin[a] and cmax[a] for a in [0, a_max].
struct TaskDesc {
  uint32_t slack_off;
  uint32_t omin_off;
  uint32_t cmin_off;
  uint32_t cmax_off;
  uint32_t row_side;
  uint32_t col_side;
  uint32_t col_base;        // global index of the column side's first set
  uint32_t self;            // 1: rows and columns are one side (j < i only)
  uint64_t col_sstart_off;  // the column side's group-start table
  uint32_t sim;             // ssj_sim
  uint32_t p, q;
  uint32_t pad;
};

// Least overlap o with Cosine o / sqrt(a c) >= p / q (Table 1), exactly:
// the smallest o with q^2 o^2 >= p^2 a c, in 128-bit integers.  A double
// estimate is corrected by at most a few steps either way.
__host__ __device__ inline uint32_t cosine_omin(uint32_t a, uint32_t c, uint32_t p, uint32_t q) {
  const unsigned __int128 rhs = (unsigned __int128)((uint64_t)p * p) * ((uint64_t)a * c);
  auto reaches = [&](uint64_t o) {
    const uint64_t x = (uint64_t)q * o;
    return (unsigned __int128)x * x >= rhs;
  };
  const double est = (double)p / (double)q * sqrt((double)a * (double)c);
  uint64_t o = est > 0.0 ? (uint64_t)est : 0u;
  while (o > 0 && reaches(o - 1)) --o;
  while (!reaches(o)) ++o;
  return (uint32_t)o;
}

// slack = |r| + |s| - 2 omin of a Cosine task (negative: never similar)
__host__ __device__ inline int32_t cosine_slack(uint32_t a, uint32_t c, uint32_t p, uint32_t q) {
  return (int32_t)((int64_t)a + c - 2 * (int64_t)cosine_omin(a, c, p, q));
}

// One row block of the filter's tile plan: up to 64*R consecutive rows
// [row0, row_end) of one row side, all of one bitmap width, and the column
// range (global column indices) they are compared with.
// Self-join: columns [col_begin, row0) in interior tiles of tile_cols
// columns, then one diagonal tile [row0, col_end) where only j < i counts.
// R-S join: columns [col_begin, col_end) in tiles of tile_cols columns.
struct RowBlock {
  uint32_t row0;
  uint32_t row_end;
  uint32_t col_begin;
  uint32_t col_end;
  uint32_t tile_begin;
  uint32_t task;
  uint32_t self;
  uint32_t pad;
};

// A tile to resume after a queue drain: tile index, first column, and
//  - vector-ALU kernel: the first slab of rows (rows r*64 .. r*64+63 of the
//    block) of that column still to be written;
//  - matrix-core kernel: `col` starts a step of 32 columns and `slab` counts
//    the kept pairs of that step already written (in the step's fixed
//    emission order).
struct Resume {
  uint32_t tile;
  uint32_t col;
  uint32_t slab;
  uint32_t pad;
};

// Filter launch arguments that are not hot pointers.
struct FilterConfig {
  uint32_t n_rows;        // rows in the row space
  uint32_t n_cols;        // columns in the column space
  uint32_t n_tiles;
  uint32_t tile_cols;
  uint32_t n_resume_in;
  uint32_t n_blocks;
  uint32_t resume_cap;    // entries of the resume buffers
  uint32_t cls;           // width class (selects the tile cursors)
  unsigned long long cap; // survivor queue capacity (entries)
  uint32_t tile_lo;       // this launch's tile range [tile_lo, tile_hi)
  uint32_t tile_hi;
  uint32_t chunk;         // queue slots a wave reserves at a time (kFilterStage..cap)
  uint32_t pad;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipSuccess or the launch error.

// Side of global index g: the last side whose base is <= g (an empty side
// shares its base with the next side and comes before it).
__device__ __forceinline__ uint32_t side_of_index(const SideDesc *__restrict__ sides,
                                                  uint32_t n_sides, uint64_t g) {
  uint32_t lo = 0, hi = n_sides;  // sides[lo].base <= g < sides[hi].base
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sides[mid].base <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// sizes[g], side_of[g] of every set of every side; offsets validated;
// largest size in ctr->max_size.
hipError_t launch_set_sizes(const SideDesc *sides, uint32_t n_sides, uint64_t n_total,
                            uint32_t *sizes, uint32_t *side_of, JoinCounters *ctr,
                            hipStream_t st);
// keys (side, size, caller index) for the size sort
hipError_t launch_make_keys(const SideDesc *sides, const uint32_t *sizes, const uint32_t *side_of,
                            uint64_t n_total, int size_bits, unsigned long long *keys,
                            hipStream_t st);
// sorted keys -> sizes and perm (size order -> caller index within the side)
hipError_t launch_unpack_keys(const unsigned long long *keys, uint64_t n, int size_bits,
                              uint32_t *sizes, uint32_t *perm, hipStream_t st);
// per side s: sstart[s * stride + v] = first position of the side (from its
// base) with size >= v, v in [0, max_size + 1]
hipError_t launch_group_starts(const SideDesc *sides, const uint32_t *sizes,
                               const uint32_t *side_of, uint64_t n_total, uint32_t max_size,
                               uint32_t stride, uint32_t n_sides, uint32_t *sstart,
                               hipStream_t st);
// rank[base_s + perm[g]] = g
hipError_t launch_invert_perm(const SideDesc *sides, const uint32_t *perm,
                              const uint32_t *side_of, uint64_t n_total, uint32_t *rank,
                              hipStream_t st);

// Stable LSD radix sort of 64-bit keys on the digits given by `shifts`
// (8 bits each, least significant first).  Result in *keys (ping-pong with
// `tmp`); `scratch` must hold radix_scratch_words(n) uint32.
uint64_t radix_scratch_words(uint64_t n);
hipError_t radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n,
                          const int *shifts, int n_shifts, uint32_t *scratch, hipStream_t st,
                          unsigned long long **result);

// Bitmaps (Alg. 3/4/5, h(t) = t mod b) of every set of every side, `out_words`
// 64-bit words each (>= b/64; extra words zero).  Without perm/rank the
// output is in caller order (row base_s + k for caller set k); with them, in
// size order (row g for the set perm[g] of side side_of[g]).  The strict
// token order of every set is checked on the way.
// fold (optional): also write the widths out_words/2, /4, ..., /32 (out[k]
// for out_words >> (k+1) words; NULL entries skipped) from the same pass;
// needs a power-of-two width of at most kMaxFoldWords words, Xor or Set, and
// the segmented build (caller order, or size order through rank).
constexpr uint32_t kMaxFoldWords = 32;
struct FoldOut {
  uint64_t *out[5];
};
hipError_t launch_build_bitmaps(const SideDesc *sides, uint32_t n_sides, uint32_t seg_blocks,
                                uint64_t n_total, const uint32_t *perm, const uint32_t *rank,
                                const uint32_t *side_of, uint32_t b_bits, int method,
                                uint32_t out_words, uint64_t *out, JoinCounters *ctr,
                                hipStream_t st, const FoldOut *fold = nullptr);
// Sizes [lo, hi] of the sets of one side that a windowed build covers
// (none when lo > hi).
struct SizeWindow {
  uint32_t lo, hi;
};
// Bitmap-Xor bitmaps at out_words = 16 or 32 words (b = 64 out_words) of
// the sets whose size lies in their side's window win[s], in size order
// (row rank[g]), and the widths of `fold` (optional, as above) from the same
// pass.  Rows of the other sets are left as they are.  The token order is
// not checked: a full build of every set checks it.
hipError_t launch_build_bitmaps_window(const SideDesc *sides, uint32_t n_sides,
                                       uint32_t seg_blocks, uint64_t n_total,
                                       const uint32_t *rank, const SizeWindow *win,
                                       uint32_t out_words, uint64_t *out, const FoldOut *fold,
                                       hipStream_t st);
// workgroups the segmented build uses for a side of n sets
uint32_t bitmap_seg_blocks(uint64_t n);

// Token-order check only (when the caller brings bitmaps); one side.
hipError_t launch_check_sorted(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                               JoinCounters *ctr, hipStream_t st);

// out[x] = in[perm[x]] with `in_words` words widened to `out_words` (one side).
hipError_t launch_gather_bitmaps(const uint64_t *in, const uint32_t *perm, uint64_t n,
                                 uint32_t in_words, uint32_t out_words, uint64_t *out,
                                 hipStream_t st);

// Sign planes of bitmaps for the matrix-core filter: bit k of a set's
// bitmap becomes the fp4 (e2m1) value +1 (0x2) when set and -1 (0xA) when
// clear.  64-bit block kb of set s is stored as two uint4 halves at
// planes[(kb * (n + kSignPad) + s) * 2 + h]; half h holds bits 32h..32h+31
// of the block, bit 8e+m of a half in nibble m of its dword e.  Sets n ..
// n + kSignPad - 1 are all zero: lanes with no row load set n, and a step's
// column loads (at most 95 columns past a column below n) stay inside the
// plane without a bounds test.  `bm`: n sets of `words` words, in the
// order the planes take; planes: (n + kSignPad) * words * 2 entries.
constexpr uint32_t kSignPad = 96;
hipError_t launch_expand_signs(const uint64_t *bm, uint32_t words, uint64_t n, uint4 *planes,
                               hipStream_t st);

// Positions [lo, hi) of a size-ordered space, at elements [first, first +
// hi - lo) of the concatenation of a list of such ranges.
struct PosRange {
  uint32_t lo, hi, first, pad;
};
// Sign planes (layout as above) of only the positions in `ranges` (sorted
// by position and by first, disjoint, `total` positions in all); positions
// from n on are written as zeros, so the list holds [n, n + kSignPad).
hipError_t launch_expand_signs_ranges(const uint64_t *bm, uint32_t words, uint64_t n,
                                      const PosRange *ranges, uint32_t n_ranges, uint64_t total,
                                      uint4 *planes, hipStream_t st);

// Wide bitmaps for verification: Bitmap-Xor at 64 * kWideWords bits of the
// sets larger than kWideMin (where the widest automatic width no longer
// prunes: its bits saturate).  In size order those sets are a suffix of each
// side; WideRange r maps global positions [lo, hi) of side `side` to slots
// slot + (g - lo) of the wide array.
constexpr uint32_t kWideWords = 64;
constexpr uint32_t kWideMin = 256;
struct WideRange {
  uint32_t lo, hi, slot, side;
};
// The wide range of every side (ranges[s], empty when the side has no set
// larger than kWideMin) and the per-side lookup of verification (wide_lo:
// first global position with a wide bitmap, ~0u for none; wide_slot: its
// slot), from the group starts sstart[s * stride + v] on the device; the
// slots follow the sides' order.
hipError_t launch_wide_ranges(const SideDesc *sides, uint32_t n_sides, const uint32_t *sstart,
                              uint32_t stride, uint32_t max_size, WideRange *ranges,
                              uint32_t *wide_lo, uint32_t *wide_slot, hipStream_t st);
// out[slot * kWideWords ...] for every slot in [0, total); ranges sorted by
// slot (empty ones allowed), n_ranges >= 1 when total > 0.  perm: size-order position -> caller
// index within its side.
hipError_t launch_build_wide(const SideDesc *sides, const uint32_t *perm,
                             const WideRange *ranges, uint32_t n_ranges, uint64_t total,
                             uint64_t *out, hipStream_t st);

// tile_block[t] = row block of tile t
hipError_t launch_expand_tiles(const RowBlock *blocks, uint32_t n_blocks, uint32_t n_tiles,
                               uint32_t *tile_block, hipStream_t st);

// Kept pairs a wave stages in LDS before one queue reservation: the
// largest reservation a filter launch makes.
constexpr uint32_t kFilterStage = 256;

// Filter geometry for a padded width.
struct FilterShape {
  uint32_t words;      // padded 64-bit words per bitmap
  uint32_t rows;       // rows per wave: 64 * R (vector ALU) or 32 * RT (matrix cores)
  bool mfma;           // the matrix-core kernel (sign planes) runs this width
};
// Padded word count the filter is instantiated for (>= words), 0 if none.
uint32_t filter_padded_words(uint32_t words);
// mfma: prefer the matrix-core kernel where it exists for the width
FilterShape filter_shape(uint32_t padded_words, bool mfma);
int filter_grid_blocks();

struct FilterArgs {
  const uint64_t *bm_rows;
  const uint64_t *bm_cols;
  const uint4 *sg_rows;         // sign planes (matrix-core kernel), else null
  const uint4 *sg_cols;
  const uint32_t *size_rows;
  const uint32_t *size_cols;
  const uint32_t *sstart_cols;  // group-start tables of the column space
  const uint32_t *tables;       // slack / omin / cmin / cmax of every task
  const TaskDesc *tasks;
  const RowBlock *blocks;
  const uint32_t *tile_block;
  uint2 *queue;
  JoinCounters *ctr;
  const Resume *resume_in;
  Resume *resume_out;
  FilterConfig cfg;
};

// One launch for the width padded_words (from filter_padded_words); cosine:
// some task of the launch uses Cosine (a kernel variant that computes its
// thresholds per size pair).  With sign planes given, the matrix-core kernel
// runs (filter_shape(padded_words, true).mfma must hold); else the vector-ALU
// kernel.  The Resume entries the two write are not interchangeable.
hipError_t launch_filter(uint32_t padded_words, bool cosine, const FilterArgs &args,
                         hipStream_t st);

// Where verification finds a task's sets and threshold.
struct VerifySpace {
  const SideDesc *sides;
  const uint32_t *side_of;
  const uint32_t *perm;
  const uint32_t *sizes;   // set sizes in size order
  const uint64_t *bm2;     // size-order bitmaps at the cascade width (an even
                           // number of words per set), or NULL
  uint32_t n;              // sets in the space
  const uint64_t *bmw;     // wide bitmaps (kWideWords words per slot), or NULL
  const uint32_t *wide_lo; // per side: first position with a wide bitmap (~0u: none)
  const uint32_t *wide_slot; // per side: the slot of that position
};

// Verification of the queued survivors (sorted merge, Table 1 predicate)
// into 64-bit result keys (task << (ib + jb)) | (i << jb) | j of caller
// indices (self-join pairs as (min, max)).  side_task[s]: the task of row
// side s.
// w2: words of the cascade bitmaps, 2, 4 or 8 (rows.bm2 and cols.bm2 both
// set, or both NULL for no second test); rows.bmw and cols.bmw likewise for
// the wide test.  n_tasks: tasks of the call (>= 1); the column of an entry
// lies in its task's column side.
// longq (optional, cap entries, ctr->long_count zero): the pairs of long
// sets that pass the bitmap tests are merged there by whole waves, in a
// second launch on the same stream.
hipError_t launch_verify(const uint2 *queue, uint2 *longq, unsigned long long cap,
                         VerifySpace rows, VerifySpace cols, const uint32_t *side_task,
                         const TaskDesc *tasks, uint32_t n_tasks, const uint32_t *tables, int ib,
                         int jb, uint32_t survivors_only, uint32_t w2,
                         unsigned long long *results, unsigned long long results_cap,
                         JoinCounters *ctr, hipStream_t st);

// Sorted result keys -> ssj_pair {i, j}; task_start[k] = first result of
// task k (k in [0, n_tasks]).
hipError_t launch_split_results(const unsigned long long *keys, uint64_t n, int ib, int jb,
                                uint32_t n_tasks, ssj_pair *out, uint64_t *task_start,
                                hipStream_t st);

// ------------------------------------------------ prefix-filter candidates
// Rows [row_begin, row_end) (global row indices) of one task, past its
// cutoff point; `first` counts the rows of earlier runs, so that run k's
// rows are probe positions [first, first + row_end - row_begin).
struct PrefixRun {
  uint32_t row_begin;
  uint32_t row_end;
  uint32_t task;
  uint32_t plen_off;  // the task's probe prefix-length table (by row size)
  uint64_t first;
};

struct ProbeArgs {
  const PrefixRun *runs;
  uint32_t n_runs;
  uint32_t col_max_size;            // largest set size of the column space
  const TaskDesc *tasks;
  const uint32_t *tables;
  const uint32_t *size_rows;
  const SideDesc *row_sides;
  const uint32_t *side_of_rows;
  const uint32_t *perm_rows;
  const uint32_t *sstart_cols;
  const unsigned long long *keys;   // sorted index entries (token << 32 | column)
  uint64_t n_keys;
};

// Exclusive scan of n uint32 into uint64 offsets; *total = the sum (device).
// scratch: scan_scratch_words(n) uint64.
uint64_t scan_scratch_words(uint64_t n);
hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, unsigned long long *out,
                           unsigned long long *total, unsigned long long *scratch,
                           hipStream_t st);
// len[g] = ilen[side_of[g] * stride + sizes[g]]: prefix length of column g
hipError_t launch_index_len(const uint32_t *sizes, const uint32_t *side_of, const uint32_t *ilen,
                            uint32_t stride, uint64_t n, uint32_t *len, hipStream_t st);
// keys[off[g] + k] = token_k << 32 | g for the first len[g] tokens of column g
hipError_t launch_index_fill(const SideDesc *sides, const uint32_t *side_of, const uint32_t *perm,
                             const uint32_t *len, const unsigned long long *off, uint64_t n,
                             unsigned long long *keys, hipStream_t st);
// counts[x]: candidates (duplicates included) of probe row x, saturated at
// 2^32 - 1
hipError_t launch_probe_count(const ProbeArgs &a, uint64_t n_rows, uint32_t *counts,
                              hipStream_t st);
// candidate keys row << 32 | column of probe rows [x0, x1) at
// out[row_off[x] - base ...]
hipError_t launch_probe_fill(const ProbeArgs &a, uint64_t x0, uint64_t x1,
                             const unsigned long long *row_off, unsigned long long base,
                             unsigned long long *out, hipStream_t st);
// sorted candidate keys -> distinct queue entries (appended at queue_count)
hipError_t launch_unique_to_queue(const unsigned long long *keys, uint64_t n, uint2 *queue,
                                  JoinCounters *ctr, hipStream_t st);

// reset the per-round counters of the queue (not the tile cursors)
hipError_t launch_reset_round(JoinCounters *ctr, hipStream_t st);
// zero a whole JoinCounters
hipError_t launch_reset_all(JoinCounters *ctr, hipStream_t st);

// copy n 64-bit words
hipError_t launch_copy_u64(const unsigned long long *in, uint64_t n, unsigned long long *out,
                           hipStream_t st);

}  // namespace ssj
