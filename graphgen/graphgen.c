/*
 * graphgen.c -- seeded synthetic graph inputs (RMAT, uniform random) in
 * canonical CSR form.
 *
 * This module only produces inputs.  It holds none of the PageRank or
 * partition-centric arithmetic; both the CPU oracle and the GPU library are
 * fed from it.
 *
 * Canonical form: self-loops dropped, duplicate (u,v) pairs dropped, every
 * row sorted ascending, int32 row offsets and column indices, isolated nodes
 * kept (n is fixed by the generator).
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used as a counter-based generator: draw
 * number c of stream key K is mix(K + (c+1)*gamma).  Every edge draw is a
 * pure function of (seed, edge index), so the output does not depend on the
 * thread count.
 *
 * RMAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each edge picks one of four
 * quadrants per level with probabilities a, b, c, d = 1-a-b-c; quadrants c
 * and d set the level's source bit, b and d its destination bit.  No noise
 * is added.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t gg_draw(uint64_t key, uint64_t ctr) {
  return gg_mix(key + (ctr + 1) * GG_GAMMA);
}

static inline uint64_t gg_key(uint64_t seed, uint64_t stream) {
  return gg_mix(gg_mix(seed + GG_GAMMA) + stream * GG_GAMMA);
}

/* floor(r * bound / 2^64) */
static inline uint64_t gg_bounded(uint64_t r, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

enum { GG_RMAT = 0, GG_UNIFORM = 1, GG_EDGES = 2 };

typedef struct {
  int kind;
  int scale;
  uint32_t ta, tab, tabc; /* cumulative quadrant thresholds on 32-bit draws */
  uint64_t key;
  int64_t n;
  int64_t ndraws;
  const int32_t* esrc; /* GG_EDGES */
  const int32_t* edst;
} gg_source;

static inline void gg_edge(const gg_source* s, int64_t e, int64_t* u, int64_t* v) {
  if (s->kind == GG_RMAT) {
    uint64_t su = 0, sv = 0;
    const int L = s->scale;
    const uint64_t base = (uint64_t)e * (uint64_t)((L + 1) / 2);
    for (int l = 0; l < L; l += 2) {
      uint64_t w = gg_draw(s->key, base + (uint64_t)(l / 2));
      for (int h = 0; h < 2 && l + h < L; ++h) {
        uint32_t r = (uint32_t)(h ? (w >> 32) : w);
        /* quadrant a [0,ta): (0,0); b [ta,tab): (0,1); c [tab,tabc): (1,0);
         * d [tabc,2^32): (1,1) -- written without branches, whose outcomes
         * are random */
        const int bu = r >= s->tab;
        const int bv = (r >= s->ta) ^ (r >= s->tab) ^ (r >= s->tabc);
        su = (su << 1) | (uint64_t)bu;
        sv = (sv << 1) | (uint64_t)bv;
      }
    }
    *u = (int64_t)su;
    *v = (int64_t)sv;
  } else if (s->kind == GG_UNIFORM) {
    uint64_t r0 = gg_draw(s->key, 2 * (uint64_t)e);
    uint64_t r1 = gg_draw(s->key, 2 * (uint64_t)e + 1);
    *u = (int64_t)gg_bounded(r0, (uint64_t)s->n);
    *v = (int64_t)gg_bounded(r1, (uint64_t)s->n);
  } else {
    *u = s->esrc[e];
    *v = s->edst[e];
  }
}

/* ---- row sorting -------------------------------------------------------- */
static void gg_sort_i32(int32_t* a, int64_t len) {
  if (len < 2) return;
  if (len <= 32) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t x = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
      a[j + 1] = x;
    }
    return;
  }
  /* LSD radix sort on the unsigned key, 11-bit digits (values are >= 0). */
  int32_t* tmp = (int32_t*)malloc((size_t)len * sizeof(int32_t));
  if (!tmp) abort();
  int32_t* from = a;
  int32_t* to = tmp;
  int32_t mx = 0;
  for (int64_t i = 0; i < len; ++i) if (a[i] > mx) mx = a[i];
  for (int shift = 0; shift < 32 && ((uint32_t)mx >> shift) != 0; shift += 11) {
    int64_t cnt[2049];
    memset(cnt, 0, sizeof(cnt));
    for (int64_t i = 0; i < len; ++i) cnt[(((uint32_t)from[i]) >> shift & 2047u) + 1]++;
    for (int d = 0; d < 2048; ++d) cnt[d + 1] += cnt[d];
    for (int64_t i = 0; i < len; ++i) to[cnt[((uint32_t)from[i]) >> shift & 2047u]++] = from[i];
    int32_t* t = from; from = to; to = t;
  }
  if (from != a) memcpy(a, from, (size_t)len * sizeof(int32_t));
  free(tmp);
}

static int64_t gg_unique(int32_t* a, int64_t len) {
  if (len == 0) return 0;
  int64_t w = 1;
  for (int64_t i = 1; i < len; ++i)
    if (a[i] != a[w - 1]) a[w++] = a[i];
  return w;
}

/* ---- state between the two calls ----------------------------------------- */
typedef struct {
  int64_t n;
  int64_t m;
  int64_t* start; /* n+1: slot ranges of tmp */
  int64_t* len;   /* n: kept entries per row after dedup */
  int32_t* tmp;
  int nthreads;
} gg_state;

static void gg_set_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Bucket every kept draw by its source row, then sort and dedup each row.
 * Draws are generated twice (the generator is counter-based): a first pass
 * counts, per thread, the draws of each coarse bucket of rows; a second pass
 * writes each draw as a (row, column) key to its bucket.  Each bucket is then
 * laid out row by row with a counting sort in cache, and every row is sorted
 * and deduplicated.  No atomics, so hub rows cause no contention. */
static gg_state* gg_build(const gg_source* s, int nthreads) {
  gg_set_threads(nthreads);
  const int64_t n = s->n;
  const int64_t nd = s->ndraws;
  gg_state* st = (gg_state*)calloc(1, sizeof(gg_state));
  if (!st) return NULL;
  st->n = n;
  st->nthreads = nthreads;
  st->start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  st->len = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!st->start || !st->len) abort();

  int bshift = 0; /* rows per bucket = 2^bshift, at most 4096 buckets */
  while ((((n - 1) >> bshift) + 1) > 4096) ++bshift;
  const int64_t nb = n > 0 ? ((n - 1) >> bshift) + 1 : 1;
  const int T = omp_get_max_threads();
  int64_t* hist = (int64_t*)calloc((size_t)T * (size_t)nb + 1, sizeof(int64_t));
  int64_t* boff = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
  if (!hist || !boff) abort();

#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const int64_t e0 = nd * t / T, e1 = nd * (t + 1) / T;
    int64_t* h = hist + (size_t)t * (size_t)nb;
    for (int64_t e = e0; e < e1; ++e) {
      int64_t u, v;
      gg_edge(s, e, &u, &v);
      if (u != v) h[u >> bshift]++;
    }
  }
  /* bucket-major, thread-minor exclusive offsets */
  int64_t acc = 0;
  for (int64_t b = 0; b < nb; ++b) {
    boff[b] = acc;
    for (int t = 0; t < T; ++t) {
      const int64_t c = hist[(size_t)t * (size_t)nb + b];
      hist[(size_t)t * (size_t)nb + b] = acc;
      acc += c;
    }
  }
  boff[nb] = acc;
  uint64_t* keys = (uint64_t*)malloc((size_t)(acc > 0 ? acc : 1) * sizeof(uint64_t));
  st->tmp = (int32_t*)malloc((size_t)(acc > 0 ? acc : 1) * sizeof(int32_t));
  if (!keys || !st->tmp) abort();

#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const int64_t e0 = nd * t / T, e1 = nd * (t + 1) / T;
    int64_t* cur = hist + (size_t)t * (size_t)nb;
    for (int64_t e = e0; e < e1; ++e) {
      int64_t u, v;
      gg_edge(s, e, &u, &v);
      if (u != v) keys[cur[u >> bshift]++] = ((uint64_t)u << 32) | (uint64_t)(uint32_t)v;
    }
  }
  free(hist);

  int64_t m = 0;
  const int64_t rows_per = (int64_t)1 << bshift;
#pragma omp parallel reduction(+ : m) num_threads(T)
  {
    int64_t* cnt = (int64_t*)malloc((size_t)(rows_per + 1) * sizeof(int64_t));
    if (!cnt) abort();
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t u0 = b << bshift;
      const int64_t nr = (u0 + rows_per <= n) ? rows_per : n - u0;
      const int64_t k0 = boff[b], k1 = boff[b + 1];
      memset(cnt, 0, (size_t)(nr + 1) * sizeof(int64_t));
      for (int64_t i = k0; i < k1; ++i) cnt[(int64_t)(keys[i] >> 32) - u0 + 1]++;
      for (int64_t r = 0; r < nr; ++r) {
        cnt[r + 1] += cnt[r];
        st->start[u0 + r] = k0 + cnt[r];
      }
      for (int64_t i = k0; i < k1; ++i) {
        const int64_t r = (int64_t)(keys[i] >> 32) - u0;
        st->tmp[k0 + cnt[r]++] = (int32_t)(uint32_t)keys[i];
      }
      for (int64_t r = 0; r < nr; ++r) {
        const int64_t u = u0 + r;
        const int64_t l = k0 + cnt[r] - st->start[u]; /* cnt[r] now ends row r */
        int32_t* row = st->tmp + st->start[u];
        gg_sort_i32(row, l);
        st->len[u] = gg_unique(row, l);
        m += st->len[u];
      }
    }
    free(cnt);
  }
  st->start[n] = acc;
  free(keys);
  free(boff);
  st->m = m;
  return st;
}

/* ---- exported API ------------------------------------------------------- */

void* gg_rmat(int scale, double edge_factor, double a, double b, double c, uint64_t seed,
              int nthreads) {
  if (scale < 1 || scale > 30 || edge_factor < 0) return NULL;
  gg_source s;
  memset(&s, 0, sizeof(s));
  s.kind = GG_RMAT;
  s.scale = scale;
  s.n = (int64_t)1 << scale;
  s.ndraws = (int64_t)(edge_factor * (double)s.n + 0.5);
  const double two32 = 4294967296.0;
  double ca = a, cab = a + b, cabc = a + b + c;
  s.ta = (uint32_t)(ca * two32 >= two32 ? 4294967295.0 : ca * two32);
  s.tab = (uint32_t)(cab * two32 >= two32 ? 4294967295.0 : cab * two32);
  s.tabc = (uint32_t)(cabc * two32 >= two32 ? 4294967295.0 : cabc * two32);
  s.key = gg_key(seed, 1);
  return gg_build(&s, nthreads);
}

void* gg_uniform(int64_t n, int64_t ndraws, uint64_t seed, int nthreads) {
  if (n < 1 || ndraws < 0) return NULL;
  gg_source s;
  memset(&s, 0, sizeof(s));
  s.kind = GG_UNIFORM;
  s.n = n;
  s.ndraws = ndraws;
  s.key = gg_key(seed, 3);
  return gg_build(&s, nthreads);
}

/* Canonicalise an explicit edge list (entries must lie in [0,n)). */
void* gg_from_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst, int nthreads) {
  if (n < 0 || ne < 0) return NULL;
  for (int64_t e = 0; e < ne; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return NULL;
  gg_source s;
  memset(&s, 0, sizeof(s));
  s.kind = GG_EDGES;
  s.n = n;
  s.ndraws = ne;
  s.esrc = src;
  s.edst = dst;
  return gg_build(&s, nthreads);
}

int64_t gg_nodes(void* h) { return ((gg_state*)h)->n; }
int64_t gg_edges(void* h) { return ((gg_state*)h)->m; }

static void gg_free_state(gg_state* st) {
  if (!st) return;
  free(st->start);
  free(st->len);
  free(st->tmp);
  free(st);
}

void gg_discard(void* h) { gg_free_state((gg_state*)h); }

/* Write the CSR into caller buffers (row_off: n+1, col: m) and free the
 * state.  Returns 0, or -1 when m does not fit int32 offsets. */
int gg_take(void* h, int32_t* row_off, int32_t* col) {
  gg_state* st = (gg_state*)h;
  if (st->m > 2147483647LL) { gg_free_state(st); return -1; }
  gg_set_threads(st->nthreads);
  const int64_t n = st->n;
  int64_t acc = 0;
  for (int64_t u = 0; u < n; ++u) {
    row_off[u] = (int32_t)acc;
    acc += st->len[u];
  }
  row_off[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < n; ++u)
    memcpy(col + row_off[u], st->tmp + st->start[u], (size_t)st->len[u] * sizeof(int32_t));
  gg_free_state(st);
  return 0;
}

/* Seeded uniform permutation (Fisher-Yates / Durstenfeld): newid[old]. */
int gg_perm_random(int64_t n, uint64_t seed, int32_t* newid) {
  const uint64_t key = gg_key(seed, 2);
  for (int64_t i = 0; i < n; ++i) newid[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)gg_bounded(gg_draw(key, (uint64_t)i), (uint64_t)i + 1);
    int32_t t = newid[i];
    newid[i] = newid[j];
    newid[j] = t;
  }
  return 0;
}

/* Relabelling by in-degree, descending; ties keep the ascending old ID
 * (a stable counting sort).  newid[old] = rank. */
int gg_perm_indegree(int64_t n, const int32_t* row_off, const int32_t* col, int32_t* newid,
                     int nthreads) {
  gg_set_threads(nthreads);
  const int64_t m = row_off[n];
  int64_t* indeg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!indeg) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) __atomic_fetch_add(&indeg[col[e]], 1, __ATOMIC_RELAXED);
  int64_t mx = 0;
  for (int64_t v = 0; v < n; ++v) if (indeg[v] > mx) mx = indeg[v];
  int64_t* first = (int64_t*)calloc((size_t)mx + 2, sizeof(int64_t));
  if (!first) { free(indeg); return -1; }
  for (int64_t v = 0; v < n; ++v) first[indeg[v]]++;
  /* descending degree: rank offset of degree D = count of nodes with degree > D */
  int64_t acc = 0;
  for (int64_t dg = mx; dg >= 0; --dg) {
    int64_t c = first[dg];
    first[dg] = acc;
    acc += c;
  }
  for (int64_t v = 0; v < n; ++v) newid[v] = (int32_t)(first[indeg[v]]++);
  free(first);
  free(indeg);
  return 0;
}

/* Apply newid to both endpoints; writes a canonical CSR of the same size. */
int gg_relabel(int64_t n, const int32_t* row_off, const int32_t* col, const int32_t* newid,
               int32_t* row_off_out, int32_t* col_out, int nthreads) {
  gg_set_threads(nthreads);
  int32_t* oldid = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!oldid) return -1;
  for (int64_t v = 0; v < n; ++v) {
    if (newid[v] < 0 || newid[v] >= n) { free(oldid); return -2; }
    oldid[newid[v]] = (int32_t)v;
  }
  int64_t acc = 0;
  for (int64_t w = 0; w < n; ++w) {
    int32_t u = oldid[w];
    row_off_out[w] = (int32_t)acc;
    acc += row_off[u + 1] - row_off[u];
  }
  row_off_out[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t w = 0; w < n; ++w) {
    int32_t u = oldid[w];
    int32_t* dst = col_out + row_off_out[w];
    int64_t l = row_off[u + 1] - row_off[u];
    for (int64_t j = 0; j < l; ++j) dst[j] = newid[col[row_off[u] + j]];
    gg_sort_i32(dst, l);
  }
  free(oldid);
  return 0;
}
