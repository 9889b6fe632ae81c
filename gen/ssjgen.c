/*
 * ssjgen -- seeded synthetic token-set collections for the set similarity
 * join.  This module only draws input data; it holds none of the join's
 * arithmetic (no similarity, no bitmap, no bound).  Both the CPU oracle
 * and the GPU library consume what it writes.
 *
 * A collection is written in CSR form: offsets[N+1] (uint64) and
 * tokens[T] (uint32), set k being tokens[offsets[k] .. offsets[k+1]).
 * Every set is strictly increasing.
 *
 * Recipe (mirrors the shape of the paper's collections, Section 5 and
 * Table 4: size-sorted sets over a token universe whose occurrence
 * histogram is Zipf-like, with tokens ordered by global frequency):
 *   - random numbers: splitmix64 seeds xoshiro256** (Blackman & Vigna);
 *     each set owns its own stream, derived from (seed, purpose, index),
 *     so the output does not depend on the thread count;
 *   - token ranks r in 1..U drawn from Zipf(s): P(r) ~ r^-s, by inverse
 *     CDF over a double table and binary search; token id = r - 1;
 *     s = 0 gives the uniform distribution;
 *   - set size: uniform on [lo, hi], log-normal
 *     clip(round(exp(ln(median) + sigma * Z)), lo, hi) with Z by
 *     Box-Muller, or Poisson(mean) clipped to [lo, hi];
 *   - a set of size n draws tokens until it holds n distinct ones;
 *   - planted near-duplicate clusters: round(f * N) sets are grouped in
 *     clusters of uniform size [cl_lo, cl_hi] (the last one truncated);
 *     each cluster is a base set plus copies in which round(swap * n)
 *     distinct positions are replaced by fresh tokens not in the copy;
 *   - relabel: tokens are renumbered by ascending global frequency
 *     (rarest = 0, ties by original id, unused ids dropped), then every
 *     set is sorted ascending;
 *   - finally the collection order is shuffled (Fisher-Yates).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SSJGEN_SIZE_UNIFORM 0
#define SSJGEN_SIZE_LOGNORMAL 1
#define SSJGEN_SIZE_POISSON 2

typedef struct {
  uint64_t n_sets;
  uint32_t universe;
  double zipf_s;
  int32_t size_dist;
  double size_a; /* lognormal: median; poisson: mean */
  double size_b; /* lognormal: sigma */
  uint32_t size_lo, size_hi;
  double planted_frac;
  uint32_t cluster_lo, cluster_hi;
  double swap_frac;
  int32_t relabel;
  int32_t shuffle;
  uint64_t seed;
  int32_t n_threads;
} ssjgen_cfg;

typedef struct {
  uint64_t n_sets;
  uint64_t n_tokens;
  uint64_t *offsets;
  uint32_t *tokens;
  uint32_t n_distinct; /* distinct token ids after relabel */
} ssjgen_out;

/* ---------------------------------------------------------------- rng */
static inline uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } rng_t;

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t *r) {
  uint64_t *s = r->s;
  uint64_t result = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

/* Stream for (seed, purpose, index): a splitmix64 chain over the three. */
static void rng_stream(rng_t *r, uint64_t seed, uint64_t purpose, uint64_t index) {
  uint64_t x = seed;
  uint64_t a = splitmix64(&x) ^ (purpose * 0xD1B54A32D192ED03ull);
  x = a;
  uint64_t b = splitmix64(&x) ^ (index * 0x8CB92BA72F3D8DD7ull);
  x = b;
  for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

/* uniform double in [0, 1) */
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [lo, hi] (multiply-shift on the top 32 bits) */
static inline uint32_t rng_range(rng_t *r, uint32_t lo, uint32_t hi) {
  uint64_t span = (uint64_t)hi - lo + 1;
  return lo + (uint32_t)(((rng_next(r) >> 32) * span) >> 32);
}

static double rng_normal(rng_t *r) {
  double u1 = 1.0 - rng_u01(r); /* (0, 1] */
  double u2 = rng_u01(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static uint32_t rng_poisson(rng_t *r, double mean) {
  /* Knuth's product method; fine for the small means used here. */
  double l = exp(-mean), p = 1.0;
  uint32_t k = 0;
  do {
    ++k;
    p *= rng_u01(r);
  } while (p > l);
  return k - 1;
}

/* ------------------------------------------------------------ context */
typedef struct {
  const ssjgen_cfg *cfg;
  double *cdf; /* cumulative Zipf weights, cdf[U-1] = total */
  uint32_t universe;
} gen_ctx;

static uint32_t draw_token(const gen_ctx *g, rng_t *r) {
  if (g->cdf == NULL) return rng_range(r, 0, g->universe - 1);
  double u = rng_u01(r) * g->cdf[g->universe - 1];
  uint32_t lo = 0, hi = g->universe - 1; /* first index with cdf > u */
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (g->cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

static uint32_t draw_size(const gen_ctx *g, rng_t *r) {
  const ssjgen_cfg *c = g->cfg;
  double v;
  switch (c->size_dist) {
    case SSJGEN_SIZE_LOGNORMAL:
      v = round(exp(log(c->size_a) + c->size_b * rng_normal(r)));
      break;
    case SSJGEN_SIZE_POISSON:
      v = (double)rng_poisson(r, c->size_a);
      break;
    default:
      v = (double)rng_range(r, c->size_lo, c->size_hi);
      break;
  }
  if (v < c->size_lo) v = c->size_lo;
  if (v > c->size_hi) v = c->size_hi;
  uint32_t n = (uint32_t)v;
  if (n > g->universe) n = g->universe;
  return n;
}

/* Small open-addressing membership set used while drawing distinct tokens. */
typedef struct { uint32_t *slot; uint32_t mask; } tokset;

static void tokset_init(tokset *h, uint32_t *buf, uint32_t cap_pow2) {
  h->slot = buf;
  h->mask = cap_pow2 - 1;
  memset(buf, 0xff, sizeof(uint32_t) * cap_pow2);
}
static inline uint32_t tokhash(uint32_t t) { return t * 0x9E3779B1u; }
/* returns 1 if inserted, 0 if already present */
static int tokset_insert(tokset *h, uint32_t t) {
  uint32_t i = tokhash(t) & h->mask;
  while (h->slot[i] != 0xffffffffu) {
    if (h->slot[i] == t) return 0;
    i = (i + 1) & h->mask;
  }
  h->slot[i] = t;
  return 1;
}
static int tokset_has(const tokset *h, uint32_t t) {
  uint32_t i = tokhash(t) & h->mask;
  while (h->slot[i] != 0xffffffffu) {
    if (h->slot[i] == t) return 1;
    i = (i + 1) & h->mask;
  }
  return 0;
}
static void tokset_erase_rebuild(tokset *h, const uint32_t *toks, uint32_t n) {
  memset(h->slot, 0xff, sizeof(uint32_t) * (h->mask + 1));
  for (uint32_t k = 0; k < n; ++k) tokset_insert(h, toks[k]);
}

static uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 16;
  while (p < x) p <<= 1;
  return p;
}

static void draw_distinct(const gen_ctx *g, rng_t *r, uint32_t *out, uint32_t n, tokset *h) {
  uint32_t k = 0;
  while (k < n) {
    uint32_t t = draw_token(g, r);
    if (tokset_insert(h, t)) out[k++] = t;
  }
}

/* --------------------------------------------------------- the layout */
/* Set k of the pre-shuffle collection is either the m-th member of a
 * planted cluster or a background set.  Cluster c covers pre-shuffle
 * sets [cl_start[c], cl_start[c+1]); background sets follow. */
typedef struct {
  gen_ctx g;
  uint64_t n_planted, n_clusters;
  uint64_t *cl_start; /* n_clusters + 1 */
  uint64_t *offsets;  /* pre-shuffle */
  uint32_t *tokens;
  uint32_t *sizes;
  uint32_t *relabel; /* universe */
  uint32_t *freq;    /* universe */
  uint64_t *perm;
  uint64_t *offsets2;
  uint32_t *tokens2;
  int nthreads;
} job_t;

enum { P_SIZE = 1, P_TOKENS = 2, P_CLUSTER = 3, P_SHUFFLE = 4, P_LAYOUT = 5 };

typedef struct { job_t *job; int tid; int phase; } worker_arg;

static void phase_sizes(job_t *j, uint64_t lo, uint64_t hi) {
  const ssjgen_cfg *c = j->g.cfg;
  for (uint64_t cl = lo; cl < hi; ++cl) {
    if (cl < j->n_clusters) {
      rng_t r;
      rng_stream(&r, c->seed, P_CLUSTER, cl);
      uint32_t n = draw_size(&j->g, &r);
      for (uint64_t k = j->cl_start[cl]; k < j->cl_start[cl + 1]; ++k) j->sizes[k] = n;
    }
  }
}

static void phase_bg_sizes(job_t *j, uint64_t lo, uint64_t hi) {
  const ssjgen_cfg *c = j->g.cfg;
  for (uint64_t k = lo; k < hi; ++k) {
    if (k < j->n_planted) continue;
    rng_t r;
    rng_stream(&r, c->seed, P_SIZE, k);
    j->sizes[k] = draw_size(&j->g, &r);
  }
}

static void phase_tokens(job_t *j, uint64_t lo, uint64_t hi, uint32_t *scratch, uint32_t scratch_cap) {
  const ssjgen_cfg *c = j->g.cfg;
  /* units: clusters first (index < n_clusters), then background sets */
  for (uint64_t u = lo; u < hi; ++u) {
    if (u < j->n_clusters) {
      uint64_t k0 = j->cl_start[u], k1 = j->cl_start[u + 1];
      uint32_t n = j->sizes[k0];
      rng_t r;
      rng_stream(&r, c->seed, P_CLUSTER, u);
      (void)draw_size(&j->g, &r); /* same stream as the size draw */
      uint32_t cap = pow2_at_least(4 * n + 4);
      if (cap > scratch_cap) cap = scratch_cap; /* scratch_cap >= 4*max+4 */
      tokset h;
      tokset_init(&h, scratch, cap);
      uint32_t *base = j->tokens + j->offsets[k0];
      draw_distinct(&j->g, &r, base, n, &h);
      uint32_t nswap = (uint32_t)round(c->swap_frac * (double)n);
      uint32_t *pos = scratch + cap; /* positions for partial Fisher-Yates */
      for (uint64_t k = k0 + 1; k < k1; ++k) {
        uint32_t *cp = j->tokens + j->offsets[k];
        memcpy(cp, base, sizeof(uint32_t) * n);
        if (nswap == 0) continue;
        tokset_erase_rebuild(&h, cp, n);
        for (uint32_t x = 0; x < n; ++x) pos[x] = x;
        for (uint32_t s = 0; s < nswap && s < n; ++s) {
          uint32_t pick = rng_range(&r, s, n - 1);
          uint32_t tmp = pos[s]; pos[s] = pos[pick]; pos[pick] = tmp;
          uint32_t t;
          if (n >= j->g.universe) break; /* no fresh token exists */
          do { t = draw_token(&j->g, &r); } while (tokset_has(&h, t));
          tokset_insert(&h, t);
          cp[pos[s]] = t;
        }
      }
    } else {
      uint64_t k = j->n_planted + (u - j->n_clusters);
      uint32_t n = j->sizes[k];
      rng_t r;
      rng_stream(&r, c->seed, P_TOKENS, k);
      uint32_t cap = pow2_at_least(2 * n + 2);
      tokset h;
      tokset_init(&h, scratch, cap);
      draw_distinct(&j->g, &r, j->tokens + j->offsets[k], n, &h);
    }
  }
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

static void sort_small(uint32_t *a, uint32_t n) {
  if (n > 32) { qsort(a, n, sizeof(uint32_t), cmp_u32); return; }
  for (uint32_t i = 1; i < n; ++i) {
    uint32_t v = a[i], k = i;
    while (k > 0 && a[k - 1] > v) { a[k] = a[k - 1]; --k; }
    a[k] = v;
  }
}

typedef struct { job_t *job; uint64_t lo, hi; int phase; } range_arg;

static void *range_worker(void *p) {
  range_arg *a = (range_arg *)p;
  job_t *j = a->job;
  const ssjgen_cfg *c = j->g.cfg;
  if (a->phase == 0) {
    phase_sizes(j, a->lo, a->hi);
  } else if (a->phase == 1) {
    phase_bg_sizes(j, a->lo, a->hi);
  } else if (a->phase == 2) {
    uint32_t cap = pow2_at_least(4 * c->size_hi + 4);
    uint32_t *scratch = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)cap + c->size_hi + 8));
    phase_tokens(j, a->lo, a->hi, scratch, cap);
    free(scratch);
  } else if (a->phase == 3) { /* frequency count */
    for (uint64_t t = j->offsets[a->lo]; t < j->offsets[a->hi]; ++t)
      __atomic_fetch_add(&j->freq[j->tokens[t]], 1u, __ATOMIC_RELAXED);
  } else if (a->phase == 4) { /* relabel + sort each set */
    for (uint64_t k = a->lo; k < a->hi; ++k) {
      uint32_t *s = j->tokens + j->offsets[k];
      uint32_t n = (uint32_t)(j->offsets[k + 1] - j->offsets[k]);
      if (j->relabel)
        for (uint32_t x = 0; x < n; ++x) s[x] = j->relabel[s[x]];
      sort_small(s, n);
    }
  } else if (a->phase == 5) { /* gather into shuffled order */
    for (uint64_t k = a->lo; k < a->hi; ++k) {
      uint64_t src = j->perm[k];
      uint64_t n = j->offsets[src + 1] - j->offsets[src];
      memcpy(j->tokens2 + j->offsets2[k], j->tokens + j->offsets[src], sizeof(uint32_t) * n);
    }
  }
  return NULL;
}

static void run_parallel(job_t *j, uint64_t n_units, int phase) {
  int nt = j->nthreads;
  if ((uint64_t)nt > n_units) nt = n_units ? (int)n_units : 1;
  pthread_t th[64];
  range_arg args[64];
  for (int t = 0; t < nt; ++t) {
    args[t].job = j;
    args[t].lo = n_units * t / nt;
    args[t].hi = n_units * (t + 1) / nt;
    args[t].phase = phase;
    pthread_create(&th[t], NULL, range_worker, &args[t]);
  }
  for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
}

typedef struct { uint32_t freq, id; } freq_id;
static int cmp_freq_id(const void *a, const void *b) {
  const freq_id *x = (const freq_id *)a, *y = (const freq_id *)b;
  if (x->freq != y->freq) return (x->freq > y->freq) - (x->freq < y->freq);
  return (x->id > y->id) - (x->id < y->id);
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int ssjgen_generate(const ssjgen_cfg *cfg, ssjgen_out *out) {
  memset(out, 0, sizeof(*out));
  if (!cfg || cfg->universe == 0 || cfg->size_lo > cfg->size_hi) return -1;
  if (cfg->planted_frac < 0 || cfg->planted_frac > 1) return -1;
  if (cfg->planted_frac > 0 && (cfg->cluster_lo < 1 || cfg->cluster_lo > cfg->cluster_hi)) return -1;
  job_t j;
  memset(&j, 0, sizeof(j));
  j.g.cfg = cfg;
  j.g.universe = cfg->universe;
  j.nthreads = cfg->n_threads > 0 ? cfg->n_threads : 8;
  if (j.nthreads > 64) j.nthreads = 64;
  uint64_t N = cfg->n_sets;
  int rc = -2;

  if (cfg->zipf_s != 0.0) {
    j.g.cdf = (double *)malloc(sizeof(double) * cfg->universe);
    if (!j.g.cdf) goto fail;
    double acc = 0.0;
    for (uint32_t r = 0; r < cfg->universe; ++r) {
      acc += pow((double)(r + 1), -cfg->zipf_s);
      j.g.cdf[r] = acc;
    }
  }

  /* cluster layout, from its own sequential stream */
  j.n_planted = (uint64_t)llround(cfg->planted_frac * (double)N);
  {
    rng_t r;
    rng_stream(&r, cfg->seed, P_LAYOUT, 0);
    uint64_t cap = j.n_planted + 2, nc = 0, at = 0;
    j.cl_start = (uint64_t *)malloc(sizeof(uint64_t) * (cap + 1));
    if (!j.cl_start) goto fail;
    j.cl_start[0] = 0;
    while (at < j.n_planted) {
      uint64_t k = rng_range(&r, cfg->cluster_lo, cfg->cluster_hi);
      if (k > j.n_planted - at) k = j.n_planted - at;
      at += k;
      j.cl_start[++nc] = at;
    }
    j.n_clusters = nc;
  }

  j.sizes = (uint32_t *)malloc(sizeof(uint32_t) * (N ? N : 1));
  j.offsets = (uint64_t *)malloc(sizeof(uint64_t) * (N + 1));
  if (!j.sizes || !j.offsets) goto fail;
  run_parallel(&j, j.n_clusters, 0);
  run_parallel(&j, N, 1);
  j.offsets[0] = 0;
  for (uint64_t k = 0; k < N; ++k) j.offsets[k + 1] = j.offsets[k] + j.sizes[k];
  uint64_t T = j.offsets[N];
  j.tokens = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
  if (!j.tokens) goto fail;
  run_parallel(&j, j.n_clusters + (N - j.n_planted), 2);

  uint32_t n_distinct = 0;
  if (cfg->relabel) {
    j.freq = (uint32_t *)calloc(cfg->universe, sizeof(uint32_t));
    j.relabel = (uint32_t *)malloc(sizeof(uint32_t) * cfg->universe);
    if (!j.freq || !j.relabel) goto fail;
    run_parallel(&j, N, 3);
    freq_id *fi = (freq_id *)malloc(sizeof(freq_id) * cfg->universe);
    if (!fi) goto fail;
    uint32_t m = 0;
    for (uint32_t t = 0; t < cfg->universe; ++t)
      if (j.freq[t]) { fi[m].freq = j.freq[t]; fi[m].id = t; ++m; }
    qsort(fi, m, sizeof(freq_id), cmp_freq_id);
    for (uint32_t x = 0; x < m; ++x) j.relabel[fi[x].id] = x;
    free(fi);
    n_distinct = m;
  }
  run_parallel(&j, N, 4);
  if (!cfg->relabel) {
    /* count distinct ids for the report */
    uint8_t *seen = (uint8_t *)calloc(cfg->universe, 1);
    if (!seen) goto fail;
    for (uint64_t t = 0; t < T; ++t) seen[j.tokens[t]] = 1;
    for (uint32_t t = 0; t < cfg->universe; ++t) n_distinct += seen[t];
    free(seen);
  }

  if (cfg->shuffle && N > 1) {
    j.perm = (uint64_t *)malloc(sizeof(uint64_t) * N);
    j.offsets2 = (uint64_t *)malloc(sizeof(uint64_t) * (N + 1));
    j.tokens2 = (uint32_t *)malloc(sizeof(uint32_t) * (T ? T : 1));
    if (!j.perm || !j.offsets2 || !j.tokens2) goto fail;
    for (uint64_t k = 0; k < N; ++k) j.perm[k] = k;
    rng_t r;
    rng_stream(&r, cfg->seed, P_SHUFFLE, 0);
    for (uint64_t k = N - 1; k > 0; --k) {
      uint64_t pick = rng_next(&r) % (k + 1);
      uint64_t tmp = j.perm[k]; j.perm[k] = j.perm[pick]; j.perm[pick] = tmp;
    }
    j.offsets2[0] = 0;
    for (uint64_t k = 0; k < N; ++k)
      j.offsets2[k + 1] = j.offsets2[k] + (j.offsets[j.perm[k] + 1] - j.offsets[j.perm[k]]);
    run_parallel(&j, N, 5);
    free(j.offsets); free(j.tokens);
    j.offsets = j.offsets2; j.tokens = j.tokens2;
    j.offsets2 = NULL; j.tokens2 = NULL;
  }

  out->n_sets = N;
  out->n_tokens = T;
  out->offsets = j.offsets;
  out->tokens = j.tokens;
  out->n_distinct = n_distinct;
  j.offsets = NULL;
  j.tokens = NULL;
  rc = 0;
fail:
  free(j.g.cdf); free(j.cl_start); free(j.sizes); free(j.offsets); free(j.tokens);
  free(j.freq); free(j.relabel); free(j.perm); free(j.offsets2); free(j.tokens2);
  return rc;
}

void ssjgen_free(ssjgen_out *out) {
  if (!out) return;
  free(out->offsets);
  free(out->tokens);
  memset(out, 0, sizeof(*out));
}

/* FNV-1a 64 over the bytes of offsets then tokens (the collection's checksum). */
uint64_t ssjgen_checksum(const uint64_t *offsets, uint64_t n_sets, const uint32_t *tokens) {
  uint64_t h = 0xcbf29ce484222325ull;
  const unsigned char *p = (const unsigned char *)offsets;
  for (uint64_t i = 0; i < (n_sets + 1) * 8; ++i) { h ^= p[i]; h *= 0x100000001b3ull; }
  p = (const unsigned char *)tokens;
  uint64_t T = offsets[n_sets];
  for (uint64_t i = 0; i < T * 4; ++i) { h ^= p[i]; h *= 0x100000001b3ull; }
  return h;
}
