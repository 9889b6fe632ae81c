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

// Counters of one filter/verify round, in device memory.
struct JoinCounters {
  unsigned long long queue_count;   // slots reserved in the survivor queue
  unsigned long long survivors;     // real survivors seen by verification
  unsigned long long results;       // pairs written to the result buffer
  uint32_t overflow;                // the queue filled during this filter launch
  uint32_t n_resume;                // resume entries written this launch
  uint32_t error;                   // validation error bits (kErr*)
  uint32_t max_size;                // largest set size seen
  // Tile cursors: each width class's tile range is cut into kParts
  // contiguous partitions, one per XCD; each cursor counts the tiles handed
  // out from its partition.  Each sits in its own 128-byte line.
  alignas(128) uint32_t tile_next[4][8][32];
};

// Partitions of a tile range (one per XCD of the MI355X).
constexpr uint32_t kParts = 8;
// Width classes of one join (one filter launch each).
constexpr uint32_t kMaxClasses = 4;

constexpr uint32_t kErrOffsets = 1u;   // malformed offsets
constexpr uint32_t kErrUnsorted = 2u;  // a set is not strictly increasing
constexpr uint32_t kErrTooBig = 4u;    // a set has 2^32 or more tokens
constexpr uint32_t kErrPlan = 8u;      // a row block with no filter path (internal error)

// One row block of the filter's tile plan: up to 64*R consecutive rows
// [row0, row_end) of the size-ordered row collection, all of one bitmap
// width (`words` 64-bit words), and the column range they are compared with.
// Self-join: columns [col_begin, row0) in interior tiles of tile_cols
// columns, then one diagonal tile [row0, col_end) where only j < i counts.
// R-S join: columns [col_begin, col_end) in tiles of tile_cols columns.
struct RowBlock {
  uint32_t row0;
  uint32_t row_end;
  uint32_t col_begin;
  uint32_t col_end;
  uint32_t tile_begin;
  uint32_t words;
  uint32_t pad[2];
};

// A tile to resume after a queue drain: tile index, first column, and the
// first slab of rows (rows r*64 .. r*64+63 of the block) of that column
// still to be written.
struct Resume {
  uint32_t tile;
  uint32_t col;
  uint32_t slab;
  uint32_t pad;
};

// Filter launch arguments that are not hot pointers.
struct FilterConfig {
  uint32_t n_rows;        // rows (size order), all sets
  uint32_t n_cols;        // columns (size order), all sets
  uint32_t n_tiles;
  uint32_t tile_cols;
  uint32_t self;          // 1: self-join (triangle j < i in diagonal tiles)
  uint32_t n_resume_in;
  uint32_t n_blocks;
  uint32_t resume_cap;    // entries of the resume buffers
  unsigned long long cap; // survivor queue capacity (entries)
  uint32_t tile_lo;       // this launch's tile range [tile_lo, tile_hi)
  uint32_t tile_hi;
  uint32_t cls;           // width class (selects the tile cursors)
  uint32_t pad;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipSuccess or the launch error.

// sizes[k] = offsets[k+1] - offsets[k]; validates offsets; keys[k] =
// (size << 32) | k for the size sort; tracks the largest size.
hipError_t launch_set_sizes(const uint64_t *offsets, uint64_t n, uint64_t n_tokens,
                            unsigned long long *keys, JoinCounters *ctr, hipStream_t st);

// Stable LSD radix sort of 64-bit keys on the digits given by `shifts`
// (8 bits each, least significant first).  Result in *keys (ping-pong with
// `tmp`); `scratch` must hold radix_scratch_words(n) uint32.
uint64_t radix_scratch_words(uint64_t n);
hipError_t radix_sort_u64(unsigned long long *keys, unsigned long long *tmp, uint64_t n,
                          const int *shifts, int n_shifts, uint32_t *scratch, hipStream_t st,
                          unsigned long long **result);

// sorted keys -> sizes (size order) and perm (size order -> caller index)
hipError_t launch_unpack_keys(const unsigned long long *keys, uint64_t n, uint32_t *sizes,
                              uint32_t *perm, hipStream_t st);

// sstart[s] = first size-order position whose size is >= s, s in [0, max+1]
hipError_t launch_group_starts(const uint32_t *sizes, uint64_t n, uint32_t max_size,
                               uint32_t *sstart, hipStream_t st);

// Bitmaps (Alg. 3/4/5, h(t) = t mod b).  Output row x (x < n) is input set
// perm ? perm[x] : x, written with `out_words` words (>= b/64; the extra
// words are zero); rank is the inverse of perm (both or neither given).
// Also checks that every set is strictly increasing.
hipError_t launch_build_bitmaps(const uint64_t *offsets, const uint32_t *tokens,
                                const uint32_t *perm, const uint32_t *rank, uint64_t n,
                                uint32_t b_bits, int method,
                                uint32_t out_words, uint64_t *out, JoinCounters *ctr,
                                hipStream_t st);

// rank[perm[x]] = x
hipError_t launch_invert_perm(const uint32_t *perm, uint64_t n, uint32_t *rank, hipStream_t st);

// Token-order check only (when the caller brings bitmaps).
hipError_t launch_check_sorted(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                               JoinCounters *ctr, hipStream_t st);

// out[x] = in[perm[x]] with `in_words` words widened to `out_words`.
hipError_t launch_gather_bitmaps(const uint64_t *in, const uint32_t *perm, uint64_t n,
                                 uint32_t in_words, uint32_t out_words, uint64_t *out,
                                 hipStream_t st);

// tile_block[t] = row block of tile t
hipError_t launch_expand_tiles(const RowBlock *blocks, uint32_t n_blocks, uint32_t n_tiles,
                               uint32_t *tile_block, hipStream_t st);

// Filter geometry for a padded width.
struct FilterShape {
  uint32_t words;      // padded 64-bit words per bitmap
  uint32_t rows;       // rows per wave = 64 * R
  uint32_t batch;      // most pairs one queue reservation can hold = 64 * R * U
};
// Padded word count the filter is instantiated for (>= words), 0 if none.
uint32_t filter_padded_words(uint32_t words);
FilterShape filter_shape(uint32_t padded_words);
int filter_grid_blocks();

struct FilterArgs {
  const uint64_t *bm_rows;
  const uint64_t *bm_cols;
  const uint32_t *size_rows;
  const uint32_t *size_cols;
  const uint32_t *sstart_cols;
  const int32_t *slack;
  const uint32_t *cmin;
  const uint32_t *cmax;
  const RowBlock *blocks;
  const uint32_t *tile_block;
  uint2 *queue;
  JoinCounters *ctr;
  const Resume *resume_in;
  Resume *resume_out;
  FilterConfig cfg;
};

// One launch for the width padded_words (from filter_padded_words).
hipError_t launch_filter(uint32_t padded_words, const FilterArgs &args, hipStream_t st);

// Verification of the queued survivors (sorted merge, Table 1 predicate)
// into 64-bit result keys (caller indices; self-join keys are (min, max)).
hipError_t launch_verify(const uint2 *queue, unsigned long long cap, const uint64_t *off_rows,
                         const uint32_t *tok_rows, const uint32_t *perm_rows,
                         const uint64_t *off_cols, const uint32_t *tok_cols,
                         const uint32_t *perm_cols, const uint32_t *omin, uint32_t n_rows,
                         uint32_t n_cols, uint32_t self,
                         uint32_t survivors_only, unsigned long long *results,
                         unsigned long long results_cap, JoinCounters *ctr, hipStream_t st);

// reset the per-round counters of the queue (not the tile cursor)
hipError_t launch_reset_round(JoinCounters *ctr, hipStream_t st);
// zero a whole JoinCounters
hipError_t launch_reset_all(JoinCounters *ctr, hipStream_t st);

// keys (i << 32 | j) -> ssj_pair {i, j}
hipError_t launch_keys_to_pairs(const unsigned long long *keys, uint64_t n, ssj_pair *out,
                                hipStream_t st);

// copy n 64-bit words
hipError_t launch_copy_u64(const unsigned long long *in, uint64_t n, unsigned long long *out,
                           hipStream_t st);

}  // namespace ssj
