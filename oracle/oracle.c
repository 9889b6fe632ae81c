/*
 * CPU oracle for the exact set similarity join -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library; the GPU
 * library never calls it and shares no code with it.
 *
 * Everything is integer arithmetic.  A similarity threshold is an exact
 * rational t = p/q.  Collections are CSR: set k is
 * tokens[offsets[k] .. offsets[k+1]), strictly increasing uint32.
 *
 * Paper: Sandes, Teodoro, Melo, "Bitmap Filter: Speeding up Exact Set
 * Similarity Joins with Bitwise Operations" (arXiv 1711.07295).
 *
 * Readings of the paper taken here (the paper is silent or loose):
 *   - sim >= t is inclusive (Section 2.1, Eq. 1);
 *   - every real-valued threshold comparison becomes an integer
 *     cross-multiplication, so pairs exactly on t are decided exactly;
 *   - a pair in which either set is empty is never similar (Jaccard of
 *     two empty sets is 0/0; with one empty set every function is 0);
 *   - the hash is h(t) = t mod b (Section 5.1), bit k lives in word
 *     k / 64 at bit k % 64 (least significant first).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { SIM_JACCARD = 0, SIM_DICE = 1, SIM_COSINE = 2, SIM_OVERLAP = 3 };
enum { BM_XOR = 0, BM_SET = 1, BM_NEXT = 2, BM_COMBINED = 3 };

/* ------------------------------------------------------------------ */
/* Overlap and union of two sorted sets by one two-pointer pass; both are
 * counted, not derived (Section 2.1, Table 1: |r n s| and |r u s|). */
void oracle_merge_count(const uint32_t *r, uint64_t nr, const uint32_t *s, uint64_t ns,
                        uint64_t *o_out, uint64_t *u_out) {
  uint64_t a = 0, b = 0, o = 0, u = 0;
  while (a < nr && b < ns) {
    if (r[a] == s[b]) { ++o; ++u; ++a; ++b; }
    else if (r[a] < s[b]) { ++u; ++a; }
    else { ++u; ++b; }
  }
  u += (nr - a) + (ns - b);
  *o_out = o;
  *u_out = u;
}

/* sim(r, s) >= p/q for the four functions of Table 1, by cross-multiplying:
 *   Overlap  |r n s|                    >= p/q  <=>  q*o >= p
 *   Jaccard  |r n s| / |r u s|          >= p/q  <=>  q*o >= p*u
 *   Cosine   |r n s| / sqrt(|r| |s|)    >= p/q  <=>  q^2 o^2 >= p^2 |r||s|
 *   Dice     2 |r n s| / (|r| + |s|)    >= p/q  <=>  2 q o >= p (|r|+|s|)
 * A pair with an empty set is never similar. */
int oracle_similar(int sim, uint64_t o, uint64_t u, uint64_t nr, uint64_t ns, uint64_t p, uint64_t q) {
  if (nr == 0 || ns == 0) return 0;
  switch (sim) {
    case SIM_JACCARD: return q * o >= p * u;
    case SIM_DICE: return 2 * q * o >= p * (nr + ns);
    case SIM_COSINE: {
      unsigned __int128 lhs = (unsigned __int128)(q * o) * (q * o);
      unsigned __int128 rhs = (unsigned __int128)(p * p) * ((unsigned __int128)nr * ns);
      return lhs >= rhs;
    }
    case SIM_OVERLAP: return q * o >= p;
    default: return 0;
  }
}

/* Length filter (Section 2.3.2, Table 2): the size bounds outside of which
 * sim(r, s) < t for sure.  Returns 1 when |s| may still pair with |r|.
 *   Overlap  |s| >= tau
 *   Jaccard  |r| t <= |s| <= |r| / t
 *   Cosine   |r| t^2 <= |s| <= |r| / t^2
 *   Dice     |r| t/(2-t) <= |s| <= |r| (2-t)/t                          */
int oracle_length_ok(int sim, uint64_t nr, uint64_t ns, uint64_t p, uint64_t q) {
  uint64_t lo = nr < ns ? nr : ns, hi = nr < ns ? ns : nr;
  switch (sim) {
    case SIM_JACCARD: return q * lo >= p * hi;
    case SIM_COSINE: return q * q * lo >= p * p * hi;
    case SIM_DICE: return (2 * q - p) * lo >= p * hi;
    case SIM_OVERLAP: return q * lo >= p;
    default: return 1;
  }
}

/* ------------------------------------------------------------------ */
/* growable pair buffer: pairs are (i, j) packed as (i << 32) | j */
typedef struct { uint64_t *v; uint64_t n, cap; } pairbuf;

static int pb_push(pairbuf *b, uint64_t key) {
  if (b->n == b->cap) {
    uint64_t nc = b->cap ? 2 * b->cap : 1024;
    uint64_t *nv = (uint64_t *)realloc(b->v, nc * sizeof(uint64_t));
    if (!nv) return -1;
    b->v = nv;
    b->cap = nc;
  }
  b->v[b->n++] = key;
  return 0;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

typedef struct {
  /* inputs */
  const uint64_t *ro; const uint32_t *rt; uint64_t nr_sets;
  const uint64_t *so; const uint32_t *st; uint64_t ns_sets;
  int self, banded, sim;
  uint64_t p, q;
  const uint64_t *rows; uint64_t n_rows; /* optional: only these rows of R */
  const uint32_t *order; /* banded self-join: positions sorted by (size, index) */
  /* shared scheduling */
  uint64_t next;
  uint64_t chunk;
  /* per-thread results */
  pairbuf *bufs;
  uint64_t *evaluated;
  int failed;
} join_job;

typedef struct { join_job *job; int tid; } join_arg;

static inline uint64_t set_len(const uint64_t *off, uint64_t k) { return off[k + 1] - off[k]; }

static int test_pair(join_job *J, uint64_t i, uint64_t j, pairbuf *out, uint64_t *evaluated) {
  uint64_t ni = set_len(J->ro, i), nj = set_len(J->so, j);
  if (J->banded && !oracle_length_ok(J->sim, ni, nj, J->p, J->q)) return 0;
  ++*evaluated;
  uint64_t o, u;
  oracle_merge_count(J->rt + J->ro[i], ni, J->st + J->so[j], nj, &o, &u);
  if (u == 0) return 0;
  if (oracle_similar(J->sim, o, u, ni, nj, J->p, J->q)) {
    uint64_t a = i, b = j;
    if (J->self && a > b) { uint64_t t = a; a = b; b = t; }
    return pb_push(out, (a << 32) | b);
  }
  return 0;
}

/* Naive algorithm (Alg. 1): verify every pair of R x S.  For a self-join
 * every unordered pair {i, j}, i != j, once.  With `banded`, pairs the
 * length filter rules out are skipped (same result, Table 2). */
static void *join_worker(void *vp) {
  join_arg *a = (join_arg *)vp;
  join_job *J = a->job;
  pairbuf *out = &J->bufs[a->tid];
  uint64_t ev = 0;
  uint64_t n_units = J->rows ? J->n_rows : J->nr_sets;
  for (;;) {
    uint64_t u0 = __atomic_fetch_add(&J->next, J->chunk, __ATOMIC_RELAXED);
    if (u0 >= n_units) break;
    uint64_t u1 = u0 + J->chunk < n_units ? u0 + J->chunk : n_units;
    for (uint64_t unit = u0; unit < u1; ++unit) {
      if (J->order) {
        /* banded self-join over size order: position x pairs with earlier
         * positions y < x while the length filter still holds; sizes are
         * non-increasing going back, so the first failure ends the row. */
        uint64_t x = J->rows ? J->rows[unit] : unit;
        uint64_t i = J->order[x];
        uint64_t ni = set_len(J->ro, i);
        for (uint64_t y = x; y-- > 0;) {
          uint64_t j = J->order[y];
          uint64_t nj = set_len(J->ro, j);
          if (!oracle_length_ok(J->sim, ni, nj, J->p, J->q)) break;
          if (test_pair(J, i, j, out, &ev)) { J->failed = 1; return NULL; }
        }
      } else {
        uint64_t i = J->rows ? J->rows[unit] : unit;
        uint64_t j0 = J->self && !J->rows ? i + 1 : 0;
        for (uint64_t j = j0; j < J->ns_sets; ++j) {
          if (J->self && j == i) continue;
          if (test_pair(J, i, j, out, &ev)) { J->failed = 1; return NULL; }
        }
      }
    }
  }
  J->evaluated[a->tid] = ev;
  return NULL;
}

static int64_t run_join(join_job *J, int nthreads, uint64_t **pairs_out, uint64_t *evaluated_out) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  J->bufs = (pairbuf *)calloc((size_t)nthreads, sizeof(pairbuf));
  J->evaluated = (uint64_t *)calloc((size_t)nthreads, sizeof(uint64_t));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
  join_arg *args = (join_arg *)malloc(sizeof(join_arg) * nthreads);
  if (!J->bufs || !J->evaluated || !th || !args) return -1;
  if (J->chunk == 0) J->chunk = 16;
  for (int t = 0; t < nthreads; ++t) {
    args[t].job = J;
    args[t].tid = t;
    pthread_create(&th[t], NULL, join_worker, &args[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  uint64_t total = 0, ev = 0;
  for (int t = 0; t < nthreads; ++t) { total += J->bufs[t].n; ev += J->evaluated[t]; }
  uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
  int64_t rc = J->failed || !all ? -1 : (int64_t)total;
  if (all) {
    uint64_t at = 0;
    for (int t = 0; t < nthreads; ++t) {
      if (J->bufs[t].n) memcpy(all + at, J->bufs[t].v, J->bufs[t].n * sizeof(uint64_t));
      at += J->bufs[t].n;
    }
    qsort(all, total, sizeof(uint64_t), cmp_u64);
    /* a sampled-rows self-join may see a pair from both ends: keep one */
    uint64_t w = 0;
    for (uint64_t k = 0; k < total; ++k)
      if (w == 0 || all[w - 1] != all[k]) all[w++] = all[k];
    if (rc >= 0) rc = (int64_t)w;
  }
  for (int t = 0; t < nthreads; ++t) free(J->bufs[t].v);
  free(J->bufs); free(J->evaluated); free(th); free(args);
  if (rc < 0) { free(all); *pairs_out = NULL; return -1; }
  *pairs_out = all;
  if (evaluated_out) *evaluated_out = ev;
  return rc;
}

/* Self-join R ~join R (Eq. 1 with S = R) by the naive algorithm (Alg. 1).
 * Returns the number of pairs, or -1; *pairs_out (malloc'd, free with
 * oracle_free) holds (i << 32 | j), i < j, ascending. */
int64_t oracle_self_join(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                         int sim, uint64_t p, uint64_t q, int nthreads, uint64_t **pairs_out) {
  join_job J;
  memset(&J, 0, sizeof(J));
  J.ro = J.so = offsets; J.rt = J.st = tokens; J.nr_sets = J.ns_sets = n;
  J.self = 1; J.sim = sim; J.p = p; J.q = q;
  return run_join(&J, nthreads, pairs_out, NULL);
}

/* R-S join (Eq. 1) by the naive algorithm (Alg. 1): all (i in R, j in S). */
int64_t oracle_rs_join(const uint64_t *r_off, const uint32_t *r_tok, uint64_t nr,
                       const uint64_t *s_off, const uint32_t *s_tok, uint64_t ns,
                       int sim, uint64_t p, uint64_t q, int nthreads, uint64_t **pairs_out) {
  join_job J;
  memset(&J, 0, sizeof(J));
  J.ro = r_off; J.rt = r_tok; J.nr_sets = nr;
  J.so = s_off; J.st = s_tok; J.ns_sets = ns;
  J.sim = sim; J.p = p; J.q = q;
  return run_join(&J, nthreads, pairs_out, NULL);
}

/* Every pair that involves one of the given sets: for each listed i, all
 * j != i of the same collection with sim >= t (plain definition, Alg. 1
 * restricted to rows).  Output (min, max), ascending, unique. */
int64_t oracle_self_join_rows(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                              const uint64_t *rows, uint64_t n_rows,
                              int sim, uint64_t p, uint64_t q, int nthreads, uint64_t **pairs_out) {
  join_job J;
  memset(&J, 0, sizeof(J));
  J.ro = J.so = offsets; J.rt = J.st = tokens; J.nr_sets = J.ns_sets = n;
  J.self = 1; J.sim = sim; J.p = p; J.q = q;
  J.rows = rows; J.n_rows = n_rows; J.chunk = 1;
  return run_join(&J, nthreads, pairs_out, NULL);
}

static const uint64_t *g_sort_off; /* qsort has no context argument */
static int cmp_size_index(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  uint64_t nx = set_len(g_sort_off, x), ny = set_len(g_sort_off, y);
  if (nx != ny) return (nx > ny) - (nx < ny);
  return (x > y) - (x < y);
}
static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

/* Size order used by the banded oracle: positions sorted by (size, index). */
int oracle_size_order(const uint64_t *offsets, uint64_t n, uint32_t *order_out) {
  for (uint64_t k = 0; k < n; ++k) order_out[k] = (uint32_t)k;
  pthread_mutex_lock(&g_sort_lock);
  g_sort_off = offsets;
  qsort(order_out, n, sizeof(uint32_t), cmp_size_index);
  pthread_mutex_unlock(&g_sort_lock);
  return 0;
}

/* Banded self-join: the same definition as oracle_self_join, but pairs the
 * length filter (Section 2.3.2, Table 2) rules out are never merged.  The
 * collection is walked in size order; a row scans back while the length
 * bound holds.  `rows` (size-order positions, may be NULL = all) limits
 * the rows processed; *evaluated_out receives the pairs merged.  Pairs are
 * caller indices (min, max), ascending. */
int64_t oracle_self_join_banded(const uint64_t *offsets, const uint32_t *tokens, uint64_t n,
                                const uint32_t *order, const uint64_t *rows, uint64_t n_rows,
                                int sim, uint64_t p, uint64_t q, int nthreads,
                                uint64_t **pairs_out, uint64_t *evaluated_out) {
  join_job J;
  memset(&J, 0, sizeof(J));
  J.ro = J.so = offsets; J.rt = J.st = tokens; J.nr_sets = J.ns_sets = n;
  J.self = 1; J.banded = 1; J.sim = sim; J.p = p; J.q = q;
  J.order = order; J.rows = rows; J.n_rows = n_rows; J.chunk = rows ? 1 : 64;
  return run_join(&J, nthreads, pairs_out, evaluated_out);
}

/* Number of unordered pairs {i, j} of one collection that pass the length
 * filter (Table 2), both sets non-empty: the pairs the paper's GPU
 * algorithm (Alg. 8) hands to the bitmap filter.  Direct double loop over
 * the size histogram. */
uint64_t oracle_band_pairs(const uint64_t *hist, uint64_t max_size, int sim, uint64_t p, uint64_t q) {
  uint64_t total = 0;
  for (uint64_t a = 1; a <= max_size; ++a) {
    if (!hist[a]) continue;
    total += hist[a] * (hist[a] - 1) / 2 * (uint64_t)oracle_length_ok(sim, a, a, p, q);
    for (uint64_t c = 1; c < a; ++c)
      if (hist[c] && oracle_length_ok(sim, a, c, p, q)) total += hist[a] * hist[c];
  }
  return total;
}

/* ------------------------------------------------------------------ */
/* Bitmap-Combined (Alg. 6, Section 3.5): Bitmap-Next when tau <= 0.56,
 * Bitmap-Xor when tau >= 0.73, Bitmap-Set in between.  tau is on the scale of
 * the cutoff analysis (Section 3.4): the overlap fraction two sets of n tokens
 * need, which for a Jaccard threshold t = p/q is 2t / (1 + t) = 2p / (p + q)
 * (Table 1 with |r| = |s| = n).  Decided in integers:
 *   2p/(p+q) <= 56/100  <=>  200 p <= 56 (p + q)
 *   2p/(p+q) >= 73/100  <=>  200 p >= 73 (p + q)                        */
int oracle_combined_method(uint64_t p, uint64_t q) {
  if (200 * p <= 56 * (p + q)) return BM_NEXT;
  if (200 * p >= 73 * (p + q)) return BM_XOR;
  return BM_SET;
}

/* ------------------------------------------------------------------ */
/* Bitmap generation (Section 3.2) with h(t) = t mod b.
 *   Bitmap-Set (Alg. 3): set bit h(t) for every token.
 *   Bitmap-Xor (Alg. 4): flip bit h(t) for every token.
 *   Bitmap-Next (Alg. 5): all ones when n >= b, otherwise set bit h(t), or
 *   the next unset bit after it, cyclically.
 * out: n * (b / 64) words; set k's bitmap is out[k*W .. k*W+W). */
static inline int bit_get(const uint64_t *w, uint64_t k) { return (int)((w[k >> 6] >> (k & 63)) & 1u); }
static inline void bit_put(uint64_t *w, uint64_t k, int v) {
  if (v) w[k >> 6] |= 1ull << (k & 63); else w[k >> 6] &= ~(1ull << (k & 63));
}

int oracle_bitmap_one(const uint32_t *s, uint64_t n, int method, uint32_t b, uint64_t *out) {
  if (b == 0 || b % 64) return -1;
  uint32_t W = b / 64;
  memset(out, 0, sizeof(uint64_t) * W);
  if (method == BM_NEXT && n >= b) {
    for (uint32_t w = 0; w < W; ++w) out[w] = ~0ull;
    return 0;
  }
  for (uint64_t k = 0; k < n; ++k) {
    uint64_t i = s[k] % b;
    switch (method) {
      case BM_SET: bit_put(out, i, 1); break;
      case BM_XOR: bit_put(out, i, bit_get(out, i) ^ 1); break;
      case BM_NEXT:
        while (bit_get(out, i)) i = (i + 1) % b;
        bit_put(out, i, 1);
        break;
      default: return -1;
    }
  }
  return 0;
}

int oracle_bitmaps(const uint64_t *offsets, const uint32_t *tokens, uint64_t n, int method,
                   uint32_t b, uint64_t *out) {
  if (b == 0 || b % 64) return -1;
  uint32_t W = b / 64;
  for (uint64_t k = 0; k < n; ++k) {
    int rc = oracle_bitmap_one(tokens + offsets[k], set_len(offsets, k), method, b, out + k * W);
    if (rc) return rc;
  }
  return 0;
}

static uint64_t popcount_words(const uint64_t *x, const uint64_t *y, uint32_t W) {
  uint64_t h = 0;
  for (uint32_t w = 0; w < W; ++w) h += (uint64_t)__builtin_popcountll(x[w] ^ y[w]);
  return h;
}

/* Overlap upper bound of Theorem 1 (Eq. 2):
 *   |r n s| <= floor((|r| + |s| - popcount(b_r xor b_s)) / 2).  */
uint64_t oracle_overlap_ub(uint64_t nr, uint64_t ns, uint64_t hamming) {
  return (nr + ns - hamming) / 2;
}

/* Bitmap filter decision for a Jaccard threshold (Alg. 7, without the
 * cutoff, as the GPU algorithm runs it): the pair is pruned when the upper
 * bound is below the equivalent overlap threshold of Table 1,
 *   UB < t/(1+t) (|r|+|s|)  <=>  (p+q) UB < p (|r|+|s|)   for t = p/q.
 * Returns 1 when the pair survives (is not pruned). */
int oracle_bitmap_survives(uint64_t nr, uint64_t ns, uint64_t hamming, uint64_t p, uint64_t q) {
  uint64_t ub = oracle_overlap_ub(nr, ns, hamming);
  return !((p + q) * ub < p * (nr + ns));
}

/* Alg. 7's decision for any function of Table 1: the pair is pruned when
 * the upper bound of Eq. 2 is below the overlap the threshold t = p/q
 * requires (Table 1's overlap column):
 *   Jaccard  UB < t/(1+t) (|r|+|s|)   <=>  (p+q) UB < p (|r|+|s|)
 *   Dice     UB < t/2 (|r|+|s|)       <=>  2q UB < p (|r|+|s|)
 *   Cosine   UB < t sqrt(|r| |s|)     <=>  q^2 UB^2 < p^2 |r| |s|   (UB >= 0)
 *   Overlap  UB < t                   <=>  q UB < p
 * Returns 1 when the pair survives. */
int oracle_bitmap_survives_sim(int sim, uint64_t nr, uint64_t ns, uint64_t hamming, uint64_t p,
                               uint64_t q) {
  uint64_t ub = oracle_overlap_ub(nr, ns, hamming);
  switch (sim) {
    case SIM_JACCARD: return !((p + q) * ub < p * (nr + ns));
    case SIM_DICE: return !(2 * q * ub < p * (nr + ns));
    case SIM_COSINE: {
      unsigned __int128 lhs = (unsigned __int128)(q * ub) * (q * ub);
      unsigned __int128 rhs = (unsigned __int128)(p * p) * ((unsigned __int128)nr * ns);
      return !(lhs < rhs);
    }
    case SIM_OVERLAP: return !(q * ub < p);
    default: return 1;
  }
}

typedef struct {
  const uint64_t *off; const uint64_t *bm; uint32_t W;
  const uint32_t *order; uint64_t n; uint64_t p, q; int sim;
  uint64_t next;
  uint64_t *surv;   /* per thread */
  uint64_t *band;   /* per thread */
  pairbuf *bufs;    /* optional lists */
  int list;
} surv_job;
typedef struct { surv_job *job; int tid; } surv_arg;

static void *surv_worker(void *vp) {
  surv_arg *a = (surv_arg *)vp;
  surv_job *J = a->job;
  uint64_t sv = 0, bd = 0;
  for (;;) {
    uint64_t x0 = __atomic_fetch_add(&J->next, 64, __ATOMIC_RELAXED);
    if (x0 >= J->n) break;
    uint64_t x1 = x0 + 64 < J->n ? x0 + 64 : J->n;
    for (uint64_t x = x0; x < x1; ++x) {
      uint64_t i = J->order[x], ni = set_len(J->off, i);
      if (ni == 0) continue;
      for (uint64_t y = x; y-- > 0;) {
        uint64_t j = J->order[y], nj = set_len(J->off, j);
        if (nj == 0 || !oracle_length_ok(J->sim, ni, nj, J->p, J->q)) break;
        ++bd;
        uint64_t h = popcount_words(J->bm + i * J->W, J->bm + j * J->W, J->W);
        if (oracle_bitmap_survives_sim(J->sim, ni, nj, h, J->p, J->q)) {
          ++sv;
          if (J->list) {
            uint64_t lo = i < j ? i : j, hi = i < j ? j : i;
            pb_push(&J->bufs[a->tid], (lo << 32) | hi);
          }
        }
      }
    }
  }
  J->surv[a->tid] = sv;
  J->band[a->tid] = bd;
  return NULL;
}

/* Survivors of the bitmap filter over the length band of a self-join with
 * any function of Table 1 (Alg. 8: length filter of Table 2, then the bitmap
 * filter of Alg. 7 on every band pair).  Bitmaps are given (from
 * oracle_bitmaps).  Returns the survivor count; *band_out gets the band size;
 * when pairs_out is non-NULL the survivors are listed as caller
 * (min << 32 | max), ascending. */
int64_t oracle_survivors(const uint64_t *offsets, uint64_t n, const uint64_t *bitmaps, uint32_t b,
                         const uint32_t *order, int sim, uint64_t p, uint64_t q, int nthreads,
                         uint64_t *band_out, uint64_t **pairs_out) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  surv_job J;
  memset(&J, 0, sizeof(J));
  J.off = offsets; J.bm = bitmaps; J.W = b / 64; J.order = order; J.n = n; J.p = p; J.q = q;
  J.sim = sim;
  J.list = pairs_out != NULL;
  J.surv = (uint64_t *)calloc(nthreads, sizeof(uint64_t));
  J.band = (uint64_t *)calloc(nthreads, sizeof(uint64_t));
  J.bufs = (pairbuf *)calloc(nthreads, sizeof(pairbuf));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
  surv_arg *args = (surv_arg *)malloc(sizeof(surv_arg) * nthreads);
  if (!J.surv || !J.band || !J.bufs || !th || !args) return -1;
  for (int t = 0; t < nthreads; ++t) {
    args[t].job = &J; args[t].tid = t;
    pthread_create(&th[t], NULL, surv_worker, &args[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  uint64_t sv = 0, bd = 0, nl = 0;
  for (int t = 0; t < nthreads; ++t) { sv += J.surv[t]; bd += J.band[t]; nl += J.bufs[t].n; }
  if (band_out) *band_out = bd;
  int64_t rc = (int64_t)sv;
  if (pairs_out) {
    uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * (nl ? nl : 1));
    if (!all) rc = -1;
    else {
      uint64_t at = 0;
      for (int t = 0; t < nthreads; ++t) {
        if (J.bufs[t].n) memcpy(all + at, J.bufs[t].v, J.bufs[t].n * sizeof(uint64_t));
        at += J.bufs[t].n;
      }
      qsort(all, nl, sizeof(uint64_t), cmp_u64);
      *pairs_out = all;
    }
  }
  for (int t = 0; t < nthreads; ++t) free(J.bufs[t].v);
  free(J.surv); free(J.band); free(J.bufs); free(th); free(args);
  return rc;
}

/* For each listed pair (i, j) of collections R and S: 1 when sim >= p/q
 * (Table 1 by merge), else 0.  Used to re-verify pairs reported at sizes the
 * full oracle cannot enumerate. */
void oracle_check_pairs(const uint64_t *r_off, const uint32_t *r_tok, const uint64_t *s_off,
                        const uint32_t *s_tok, const uint32_t *pairs, uint64_t n_pairs, int sim,
                        uint64_t p, uint64_t q, uint8_t *ok_out) {
  for (uint64_t k = 0; k < n_pairs; ++k) {
    uint64_t i = pairs[2 * k], j = pairs[2 * k + 1];
    uint64_t ni = set_len(r_off, i), nj = set_len(s_off, j), o, u;
    oracle_merge_count(r_tok + r_off[i], ni, s_tok + s_off[j], nj, &o, &u);
    ok_out[k] = (uint8_t)(u != 0 && oracle_similar(sim, o, u, ni, nj, p, q));
  }
}

void oracle_free(void *p) { free(p); }
