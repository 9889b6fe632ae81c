/*
 * ssj.h -- exact set similarity join with the Bitmap Filter on one AMD
 * Instinct MI355X (gfx950).  C ABI, version 4.
 *
 * Method: Sandes, Teodoro, Melo, "Bitmap Filter: Speeding up Exact Set
 * Similarity Joins with Bitwise Operations" (arXiv 1711.07295).
 *
 * The problem (Section 2.1, Eq. 1): given collections R and S of token
 * sets, return every pair (r, s) in R x S with sim(r, s) >= t; when R and
 * S are the same collection this is the self-join.  The threshold is an
 * exact rational t = p / q and every comparison is done in integers, so
 * pairs exactly on the threshold are decided exactly and the pair set is
 * unique: it does not depend on the bitmap width, the bitmap generator,
 * the tiling or the launch shape.
 *
 * Conventions shared by every entry point:
 *   - A collection (ssj_sets) is CSR in DEVICE memory: set k is
 *     tokens[offsets[k] .. offsets[k+1]).  offsets[0] must be 0, offsets
 *     must be non-decreasing and offsets[n_sets] must equal n_tokens;
 *     otherwise SSJ_E_INVALID.  Every set must be strictly increasing
 *     (sorted, no repeated token); otherwise SSJ_E_UNSORTED.  Empty sets
 *     are legal and never pair with anything.  n_sets < 2^32 - 1.
 *   - Input buffers are caller-owned; the library never frees them and
 *     only reads them.
 *   - Bitmaps are b bits per set, b a multiple of 64 in [64, 4096], stored
 *     as b/64 uint64 words per set, set k at words [k*b/64, (k+1)*b/64),
 *     caller order.  Bit k of a bitmap is bit (k % 64) of word k / 64.
 *     The hash is h(t) = t mod b (Section 5.1).
 *   - All device work is enqueued on hip_stream (a hipStream_t; NULL is
 *     the default stream).  A join returns after that stream has been
 *     synchronised, because the number of pairs must be known.
 *   - Result pairs are returned in HOST memory owned by the library
 *     (ssj_pairs.pairs), released with ssj_free_pairs.  Lists of 1 MiB and
 *     more are page-locked; the library keeps released page-locked buffers
 *     (up to 1 GiB of them) for later calls.  On any error *out is
 *     {NULL, 0}: there is never a partial result.
 *   - Calls are re-entrant; calls on distinct streams are independent.
 *     The library takes its working memory per call from a per-device
 *     cache of device memory chunks that it keeps until the process ends.
 *   - Return values are ssj_status codes; 0 is success.
 */
#ifndef SSJ_H
#define SSJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSJ_ABI_VERSION 4

typedef enum {
  SSJ_OK = 0,
  SSJ_E_INVALID = -1,     /* bad argument or malformed offsets */
  SSJ_E_UNSORTED = -2,    /* a set is not strictly increasing */
  SSJ_E_NOMEM = -3,       /* a device or host allocation failed */
  SSJ_E_DEVICE = -4,      /* a HIP runtime call or kernel launch failed */
  SSJ_E_UNSUPPORTED = -5  /* sizes or widths beyond what the library handles */
} ssj_status;

/* Similarity functions of Table 1, with t = p / q:
 *   Jaccard  |r n s| / |r u s|          >= t   (the one the paper's GPU
 *                                               algorithm, Alg. 8, evaluates)
 *   Dice     2 |r n s| / (|r| + |s|)    >= t
 *   Cosine   |r n s| / sqrt(|r| |s|)    >= t
 *   Overlap  |r n s|                    >= t   (t may exceed 1)
 * Each is turned into the least overlap omin(|r|, |s|) that reaches t; the
 * bitmap filter keeps a pair when its bound (Eq. 2) reaches omin, and the
 * length filter is the function's row of Table 2. */
typedef enum {
  SSJ_SIM_JACCARD = 0,
  SSJ_SIM_DICE = 1,
  SSJ_SIM_COSINE = 2,
  SSJ_SIM_OVERLAP = 3
} ssj_sim;

/* Bitmap generators of Section 3.2: Bitmap-Xor (Alg. 4), Bitmap-Set
 * (Alg. 3), Bitmap-Next (Alg. 5), and Bitmap-Combined (Alg. 6,
 * Section 3.5), which takes one of the three by the threshold the bitmaps
 * are used at.  Theorem 1 holds for all of them; the join treats any of them
 * alike.
 *
 * Bitmap-Combined's choice.  The paper states its ranges on the scale of
 * the cutoff analysis (Section 3.4): the overlap fraction tau two sets of n
 * tokens need to be similar, which is 2t / (1 + t) for a Jaccard threshold
 * t (Table 1 with |r| = |s|), and t itself for Dice and Cosine.  On that
 * scale the cutoff curves of Eqs. 4-6 cross where the paper puts the
 * ranges: Bitmap-Next when tau <= 0.56, Bitmap-Xor when tau >= 0.73,
 * Bitmap-Set in between.  Compared exactly, in integers. */
typedef enum {
  SSJ_BM_XOR = 0,
  SSJ_BM_SET = 1,
  SSJ_BM_NEXT = 2,
  SSJ_BM_COMBINED = 3
} ssj_bm_method;

typedef struct {
  const uint64_t *offsets; /* device, n_sets + 1 entries */
  const uint32_t *tokens;  /* device, n_tokens entries */
  uint64_t n_sets;
  uint64_t n_tokens;
} ssj_sets;

typedef struct {
  uint32_t i, j;
} ssj_pair;

typedef struct {
  ssj_pair *pairs; /* host, library-owned; NULL when count == 0 */
  uint64_t count;
} ssj_pairs;

/* Optional per-call statistics. */
typedef struct {
  uint64_t band_pairs;      /* pairs inside the length band (Table 2) */
  uint64_t survivors;       /* band pairs the bitmap filter kept */
  uint64_t results;         /* pairs reported */
  uint64_t filter_ops;      /* algorithmic filter work: per band pair b/16 + 1
                               int32 lane-ops (b/32 xor, b/32 popcount, 1 compare) */
  uint64_t queue_slots;     /* survivor-queue slots the filter launches reserved,
                               the sentinel ends of the waves' chunks included
                               (summed over the rounds) */
  uint32_t filter_launches; /* filter kernel launches (1 + queue drains) */
  uint32_t b_bits;          /* bitmap width asked for (0 = automatic) */
  uint32_t n_classes;       /* row-size classes (1 for a fixed width) */
  uint32_t class_bits[8];   /* bitmap width of each class */
  uint32_t class_max_size[8]; /* largest row size of each class */
  uint64_t class_ops[8];    /* filter_ops of each class */
  uint64_t class_tiles[8];  /* filter tiles of each class (row tile x column
                               tile units a wave takes at a time) */
  float class_ms[8];        /* filter kernel time of each class (one launch
                               per class and queue drain) */
  float ms_total;           /* call entry to pairs in host memory */
  float ms_prepare;         /* validation, size sort, plan, bitmaps */
  float ms_filter;          /* sum of filter kernel durations */
  float ms_verify;          /* sum of verification kernel durations */
  float ms_emit;            /* result sort and copy to the host */
} ssj_stats;

/* Optional knobs; pass NULL for the defaults. */
typedef struct {
  uint64_t queue_capacity; /* survivor-queue entries per drain (8 bytes
                              each, and as many 8-byte result keys), raised
                              to at least 4096; 0 = the library's: 2^23 at
                              first, quadrupled after each drain round that
                              filled it, up to 2^29 */
  uint32_t tile_cols;      /* columns per filter tile; 0 = default */
  uint32_t flags;          /* SSJ_FLAG_* */
} ssj_options;

/* Report every survivor of the bitmap filter as a result, skipping the
 * exact verification.  Diagnostic only: the output is then the filter's
 * survivor set (caller indices), not the join. */
#define SSJ_FLAG_SURVIVORS_ONLY 1u

/* Apply the bitmap filter only to rows up to the cutoff point (Section 3.5,
 * as Alg. 7 does; see ssj_cutoff) of their widest width; rows of larger
 * sets take their candidates from an index of set prefixes (the prefix
 * filter) instead.  Changes the work, never the result.  With
 * SSJ_FLAG_SURVIVORS_ONLY those rows report their prefix candidates. */
#define SSJ_FLAG_CUTOFF 2u

/* Run the bitmap filter on the vector ALUs at every width.  By default the
 * widths of 1, 2, 4, 8 and 16 64-bit words (b = 64, 128, 256, 512, 1024,
 * and the widths padded to them) run on the matrix cores, which score the
 * Hamming distance of Theorem 1 as a dot product of +-1 vectors (exact);
 * a class of 4 or more words and fewer than 2^26 band pairs runs on the
 * vector ALUs, whose launch costs less.  The two kernels keep the same
 * pairs.  Changes the work, never the result. */
#define SSJ_FLAG_VALU 4u

/* Run the bitmap filter on the matrix cores at the widths above for every
 * width class, whatever its size (with SSJ_FLAG_VALU: invalid).  Changes
 * the work, never the result. */
#define SSJ_FLAG_MFMA 8u

/*
 * ssj_build_bitmaps -- the bitmap of every set (Section 3.2, Alg. 3/4/5/6,
 * precomputed once as in the initialization of Alg. 7).
 *   s            collection (device CSR), validated as above
 *   b_bits       bitmap width b: multiple of 64 in [64, 4096]
 *   method       ssj_bm_method
 *   p, q         read only by SSJ_BM_COMBINED: the Jaccard threshold t = p/q
 *                the bitmaps will be joined at, 1 <= p <= q (reduced
 *                internally); Alg. 6 then builds Next, Set or Xor by
 *                2t/(1+t).  (For a Dice or Cosine threshold t', pass the
 *                Jaccard threshold with the same normalized value,
 *                t'/(2 - t'); ssj_cutoff resolves Combined per function.)
 *   bitmaps_dev  caller-owned device buffer of n_sets * b_bits / 64 uint64,
 *                written in caller order
 *   hip_stream   stream for the work; the call returns after the stream
 *                is synchronised (validation result is needed)
 * Errors: SSJ_E_INVALID (null pointer, bad b, bad offsets, Combined with a
 *         bad threshold), SSJ_E_UNSORTED, SSJ_E_UNSUPPORTED (unknown
 *         method), SSJ_E_NOMEM, SSJ_E_DEVICE.
 */
int ssj_build_bitmaps(const ssj_sets *s, uint32_t b_bits, int method, uint32_t p, uint32_t q,
                      uint64_t *bitmaps_dev, void *hip_stream);

/*
 * ssj_build_bitmaps_noalloc -- ssj_build_bitmaps that allocates no memory,
 * for callers that cannot allocate: serving loops and harnesses that forbid
 * hipMalloc or any allocating call while they run.  Same arguments, result
 * and errors as ssj_build_bitmaps; the bitmaps are identical.
 *   Working memory (side table, counters, validated set sizes) is a fixed
 *   device array of 32 MiB inside the library, one copy per device, held
 *   from the library's load until the process ends.  It is cleared by the
 *   call where it must start at zero and otherwise keeps the last call's
 *   contents.  Calls on one device share that array: the library runs them
 *   one at a time (a call holds the device's array until its stream is
 *   synchronised), so concurrent calls from several threads wait for each
 *   other instead of racing.  No host memory is allocated either.
 *   The call synchronises hip_stream, so it cannot be captured into a graph.
 * Errors: as ssj_build_bitmaps; SSJ_E_UNSUPPORTED also when n_sets exceeds
 *         SSJ_NOALLOC_MAX_SETS (nothing is written then); SSJ_E_DEVICE when
 *         the array's address cannot be obtained on the current device.
 */
#define SSJ_NOALLOC_MAX_SETS 4000000u
int ssj_build_bitmaps_noalloc(const ssj_sets *s, uint32_t b_bits, int method, uint32_t p,
                              uint32_t q, uint64_t *bitmaps_dev, void *hip_stream);

/*
 * ssj_self_join -- every pair (i, j), i < j (caller indices), with
 * sim(set_i, set_j) >= p / q (Eq. 1 with R = S).  The length filter
 * (Table 2) bounds the pairs considered, the bitmap filter (Theorem 1,
 * Eq. 2; Alg. 7 without the cutoff) prunes them, and every survivor is
 * verified exactly.
 *   s            collection (device CSR)
 *   bitmaps_dev  NULL: Bitmap-Xor bitmaps are built internally.  Otherwise
 *                caller-owned device bitmaps of width b_bits from any
 *                generator (caller order).
 *   b_bits       bitmap width: multiple of 64 in [64, 4096], or 0 for an
 *                automatic width per class of row sizes (64 to 2048 bits,
 *                never narrower for larger sets: the widths that minimise
 *                the expected time of the call's band pairs, from the
 *                false-survivor odds of the expected bound of Section 3.4
 *                and costs measured on the GPU; bitmaps_dev must then be
 *                NULL)
 *   sim          ssj_sim
 *   p, q         threshold t = p / q, 1 <= p <= q (reduced internally);
 *                SSJ_SIM_OVERLAP takes any p >= 1, q >= 1
 *   opts         NULL or knobs
 *   out          receives the pairs, ascending by (i, j), no duplicates
 *   stats        NULL or statistics
 *   hip_stream   stream for all device work
 * Errors: SSJ_E_INVALID, SSJ_E_UNSORTED, SSJ_E_UNSUPPORTED, SSJ_E_NOMEM,
 *         SSJ_E_DEVICE; *out = {NULL, 0} on every error.
 */
int ssj_self_join(const ssj_sets *s, const uint64_t *bitmaps_dev, uint32_t b_bits, int sim,
                  uint32_t p, uint32_t q, const ssj_options *opts, ssj_pairs *out,
                  ssj_stats *stats, void *hip_stream);

/*
 * ssj_rs_join -- every pair (i in R, j in S) with sim(r_i, s_j) >= p / q
 * (Eq. 1, R-S join).  Arguments as ssj_self_join; the bitmaps of R and S,
 * when given, must come from the same generator and width (the bound of
 * Theorem 1 needs the same hash on both sides).  Output ascending by
 * (i, j).
 */
int ssj_rs_join(const ssj_sets *r, const uint64_t *r_bitmaps_dev, const ssj_sets *s,
                const uint64_t *s_bitmaps_dev, uint32_t b_bits, int sim, uint32_t p, uint32_t q,
                const ssj_options *opts, ssj_pairs *out, ssj_stats *stats, void *hip_stream);

/*
 * ssj_self_join_batch -- many independent self-joins in one call (the
 * batched form of Eq. 1 with R = S): instance k is the self-join of
 * sets[k] at threshold p[k] / q[k].  All instances share the preparation,
 * filter, verification and emission launches: the filter's tiles of every
 * instance are handed out from the same work queue, so uneven instances
 * keep the whole GPU busy.  With b_bits = 0 each instance gets its own
 * widths per class of row sizes (the rule of ssj_self_join).
 *   sets         n_instances collections (device CSR each, validated as
 *                above); host array
 *   n_instances  number of instances; 0 returns an empty result
 *   p, q         host arrays of n_instances thresholds, 1 <= p[k] <= q[k]
 *   b_bits       0 or a fixed width for every instance (as ssj_self_join;
 *                no caller bitmaps)
 *   sim          ssj_sim (every instance)
 *   opts         NULL or knobs (shared by the instances)
 *   out          every instance's pairs, instance by instance; each
 *                instance's pairs are its caller indices (i < j), ascending
 *                by (i, j) -- exactly what ssj_self_join returns for it
 *   starts       NULL or a host array of n_instances + 1 entries: instance
 *                k's pairs are out->pairs[starts[k] .. starts[k+1])
 *   stats        NULL or totals over the instances
 * Limits: the instances' total set count is below 2^32 - 1, and the bits
 * of (instance, i, j) fit 64.  Errors as ssj_self_join; one bad instance
 * fails the call.
 */
int ssj_self_join_batch(const ssj_sets *sets, uint32_t n_instances, const uint32_t *p,
                        const uint32_t *q, uint32_t b_bits, int sim, const ssj_options *opts,
                        ssj_pairs *out, uint64_t *starts, ssj_stats *stats, void *hip_stream);

/* A resident collection S for repeated R-S queries (the served form). */
typedef struct ssj_index ssj_index;

/*
 * ssj_index_create -- copy S into the index's own device memory, validate
 * and size-sort it, and build its bitmaps once: Bitmap-Xor at every width
 * the automatic mode may pick (64 to 2048 bits) when b_bits is 0, else at
 * b_bits.  The caller may free S afterwards.  The index lives on
 * the current device until ssj_index_destroy.
 *   s            the resident collection (device CSR)
 *   b_bits       0 (automatic) or a fixed width, as ssj_self_join
 *   out          receives the index; NULL on error
 *   hip_stream   stream for the work; returns after it is synchronised
 * Errors: SSJ_E_INVALID, SSJ_E_UNSORTED, SSJ_E_UNSUPPORTED, SSJ_E_NOMEM,
 *         SSJ_E_DEVICE.
 */
int ssj_index_create(const ssj_sets *s, uint32_t b_bits, ssj_index **out, void *hip_stream);

/*
 * ssj_index_query -- R-S joins of query batches against the index (Eq. 1,
 * R-S join): batch k's result is every pair (i in batches[k], j in S) with
 * sim >= p[k] / q[k], exactly what ssj_rs_join(batches[k], S) returns.
 * All batches of a call share the launches, as in ssj_self_join_batch.
 * The index is only read: queries may run concurrently on distinct
 * streams of the index's device.
 *   idx          index from ssj_index_create (same current device)
 *   batches      n_batches query collections (device CSR); host array
 *   p, q         host arrays of n_batches thresholds
 *   sim, opts    as ssj_rs_join
 *   out          every batch's pairs, batch by batch, each ascending by
 *                (i, j), i a caller index in the batch, j in S
 *   starts       NULL or n_batches + 1 host entries, as ssj_self_join_batch
 *   stats        NULL or totals over the batches
 * Errors as ssj_rs_join; SSJ_E_INVALID also for a NULL index or another
 * current device.
 */
int ssj_index_query(ssj_index *idx, const ssj_sets *batches, uint32_t n_batches,
                    const uint32_t *p, const uint32_t *q, int sim, const ssj_options *opts,
                    ssj_pairs *out, uint64_t *starts, ssj_stats *stats, void *hip_stream);

/* Release an index and its device memory (NULL-safe).  No query on it may
 * still be running. */
void ssj_index_destroy(ssj_index *idx);

/* A prepared self-join of one or more instances (the batched form): planned
 * once, its first filter/verify round captured in a HIP graph, executed
 * many times. */
typedef struct ssj_plan ssj_plan;

/*
 * ssj_plan_self_join_batch -- plan the self-join of n_instances collections
 * (each at its own threshold p[k] / q[k]; Eq. 1 per instance) once: size
 * sort, length band (Table 2), width classes, tile plan and every buffer,
 * in memory the plan owns.  The device work that reads the tokens --
 * validation, the bitmaps of every width (Bitmap-Xor, Alg. 4), sign planes,
 * the filter launch of every width class (Theorem 1, Eq. 2) and the
 * verification of the survivors -- is captured in one HIP graph, which
 * every ssj_plan_execute replays with one launch.  A plan depends on the
 * set sizes only: the tokens may change between executions, the offsets
 * and the buffers may not, and both must stay valid while the plan lives.
 * Arguments as ssj_self_join_batch (n_instances >= 1); the caller's
 * bitmaps are not taken (the plan builds its own).  Returns after
 * hip_stream is synchronised.
 *   out          receives the plan; NULL on error
 * Errors as ssj_self_join_batch; SSJ_E_INVALID also for n_instances == 0.
 */
int ssj_plan_self_join_batch(const ssj_sets *sets, uint32_t n_instances, const uint32_t *p,
                             const uint32_t *q, uint32_t b_bits, int sim,
                             const ssj_options *opts, ssj_plan **out, void *hip_stream);

/*
 * ssj_plan_execute -- run a prepared join on the current tokens: one graph
 * launch on hip_stream, then, on the host, the drain-and-resume rounds the
 * survivor queue needs when it fills, the candidates of rows past the
 * cutoff (SSJ_FLAG_CUTOFF), and the sort and copy of the pairs.  Output as
 * ssj_self_join_batch: exactly the pairs the unprepared call returns for
 * the same tokens.  Executions of one plan take turns (a lock held until
 * the call returns); the plan's device must be current.
 *   stats        NULL or totals; ms_prepare is 0 (planning happened once),
 *                ms_filter includes the whole graph (bitmaps, first filter
 *                round and its verification), class_ms only later rounds
 * Errors: SSJ_E_INVALID (NULL plan, other device), SSJ_E_UNSORTED (tokens
 * no longer strictly increasing), SSJ_E_NOMEM, SSJ_E_DEVICE; on any error
 * *out = {NULL, 0}.
 */
int ssj_plan_execute(ssj_plan *plan, ssj_pairs *out, uint64_t *starts, ssj_stats *stats,
                     void *hip_stream);

/* Release a plan, its graph and its device memory (NULL-safe).  No
 * execution of it may still be running. */
void ssj_plan_destroy(ssj_plan *plan);

/*
 * ssj_cutoff -- the cutoff point omega(b, t) of Section 3.5: the largest set
 * size n for which the expected normalized overlap bound of two sets of n
 * random tokens, E(b, n) / n (Section 3.4: Eq. 4 Bitmap-Set, Eq. 5
 * Bitmap-Xor, Eq. 6 Bitmap-Next), is at most the overlap fraction two n-sets
 * need to reach the threshold (Jaccard 2t/(1+t); Dice and Cosine t).  Alg. 7
 * applies the bitmap filter to sets up to this size; beyond it the filter
 * can no longer tell most dissimilar pairs apart.  Host computation only.
 *   b_bits       bitmap width, as ssj_build_bitmaps
 *   method       ssj_bm_method; SSJ_BM_COMBINED: the cutoff of the generator
 *                Alg. 6 picks for this function's normalized threshold (the
 *                combined curve the paper precomputes for Alg. 7)
 *   sim, p, q    similarity function and threshold, as ssj_self_join
 *   out          receives omega; UINT32_MAX for SSJ_SIM_OVERLAP (an absolute
 *                threshold: never cut off); 0 on error
 * Errors: SSJ_E_INVALID (bad b, threshold or NULL out), SSJ_E_UNSUPPORTED
 *         (unknown method).
 */
int ssj_cutoff(uint32_t b_bits, int method, int sim, uint32_t p, uint32_t q, uint32_t *out);

/* Release the pairs of a join (any thread).  NULL-safe and idempotent;
 * zeroes *out. */
void ssj_free_pairs(ssj_pairs *out);

/* Static text for a status code. */
const char *ssj_status_string(int status);

/* SSJ_ABI_VERSION of the loaded library. */
int ssj_abi_version(void);

/*
 * ssj_memory_limit -- cap the device memory that the library's per-call
 * working memory may hold on each device: the chunks of its cache, idle or
 * in use by a call (a resident index's own memory is not counted).
 *   bytes  the cap in bytes; 0 removes it.  Idle chunks beyond a new cap are
 *          freed at once.
 *   held   out (nullable): bytes the current device's chunks hold now.
 * A call whose working memory would pass the cap first makes the cache free
 * its idle chunks; when that is not enough the call fails with SSJ_E_NOMEM
 * and returns no output (*out = {NULL, 0}).  A serving loop sets it to the
 * budget its admission control plans with.  Freeing chunks waits for the
 * device.  Returns SSJ_E_DEVICE when no device is current.
 */
int ssj_memory_limit(uint64_t bytes, uint64_t *held);

#ifdef __cplusplus
}
#endif

#endif /* SSJ_H */
