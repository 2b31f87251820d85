/*
 * oracle.c -- plain, slow, obviously correct CPU reference for PCPM PageRank.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and
 * the benchmark's CPU-baseline leg may load this file's library.  It shares
 * no code, header or table with the GPU library; it reads graphs from the
 * seeded input generator like the GPU side does.
 *
 * All floating point is FP64.  Summation order is fixed (blocks of
 * ORC_BLOCK nodes reduced in ascending order), so results do not depend on
 * the thread count.
 *
 * Contents
 *   orc_pagerank      Eq. 1 of Sec. 2.1, evaluated in the pull direction of
 *                     Alg. 1 (in-neighbours over the transposed adjacency),
 *                     with the mass of dangling nodes redistributed by the
 *                     teleport vector.  Plain PageRank uses t(v) = 1/|V|;
 *                     personalised PageRank passes its own t.
 *                     orc_pagerank_csc takes the transposed adjacency from
 *                     orc_transpose_into, so many runs on one graph (the
 *                     vectors of a personalised batch) transpose it once.
 *   orc_png_sizes,    The Partition-Node Graph layout of Sec. 3.1 and 3.3,
 *   orc_png_layout    written from its set definitions (equisized index
 *                     partitions of any size q, one update per (node, destination
 *                     partition), write offsets ordered by source partition
 *                     ID, MSB on the first destination ID of each message).
 *   orc_pcpm_iterate  One PageRank iteration carried out over that layout:
 *                     the scatter of Alg. 3 and the branch-avoiding gather of
 *                     Alg. 5 (update pointer read as "flags seen so far,
 *                     inclusive, minus one"), then the apply of Alg. 2.
 *   orc_step_at       One step of Eq. 1 from a given vector, evaluated only at
 *                     chosen nodes (a scan of all edges, no transpose), for
 *                     checks on graphs too large for full oracle runs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_BLOCK 65536
#define ORC_MSB 0x80000000u

static void orc_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Sum of f(v) over v in [0,n) in a fixed order: blocks in parallel, block
 * sums added in ascending block order. */
typedef double (*orc_term_fn)(int64_t v, const void* ctx);

static double orc_fixed_sum(int64_t n, orc_term_fn f, const void* ctx) {
  const int64_t nb = (n + ORC_BLOCK - 1) / ORC_BLOCK;
  double* part = (double*)calloc((size_t)(nb > 0 ? nb : 1), sizeof(double));
  if (!part) abort();
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    double s = 0.0;
    const int64_t hi = (b + 1) * ORC_BLOCK < n ? (b + 1) * ORC_BLOCK : n;
    for (int64_t v = b * ORC_BLOCK; v < hi; ++v) s += f(v, ctx);
    part[b] = s;
  }
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s += part[b];
  free(part);
  return s;
}

typedef struct {
  const int32_t* row_off;
  const double* x;
  const double* y;
} orc_sum_ctx;

static double orc_dangling_term(int64_t v, const void* c) {
  const orc_sum_ctx* k = (const orc_sum_ctx*)c;
  return (k->row_off[v + 1] == k->row_off[v]) ? k->x[v] : 0.0;
}

static double orc_l1_term(int64_t v, const void* c) {
  const orc_sum_ctx* k = (const orc_sum_ctx*)c;
  return fabs(k->y[v] - k->x[v]);
}

/* Transposed adjacency into caller arrays: in_off[n+2], in_src[m]; afterwards
 * in_off[v] .. in_off[v+1] is v's list of in-neighbours, sources ascending. */
int orc_transpose_into(int64_t n, const int32_t* row_off, const int32_t* col, int64_t* in_off, int32_t* in_src) {
  if (n <= 0) return -1;
  const int64_t m = row_off[n];
  memset(in_off, 0, ((size_t)n + 2) * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) in_off[(int64_t)col[e] + 2]++;
  for (int64_t v = 0; v < n; ++v) in_off[v + 2] += in_off[v + 1];
  /* in_off[v+1] is now the start of v's list; advance it while filling */
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) in_src[in_off[(int64_t)col[e] + 1]++] = (int32_t)u;
  return 0;
}

static int orc_transpose(int64_t n, const int32_t* row_off, const int32_t* col, int64_t** in_off_out,
                         int32_t** in_src_out) {
  const int64_t m = row_off[n];
  int64_t* in_off = (int64_t*)calloc((size_t)n + 2, sizeof(int64_t));
  int32_t* in_src = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!in_off || !in_src) { free(in_off); free(in_src); return -1; }
  orc_transpose_into(n, row_off, col, in_off, in_src);
  *in_off_out = in_off;
  *in_src_out = in_src;
  return 0;
}

/*
 * FP64 PageRank, pull direction (Eq. 1 / Alg. 1), dangling mass spread by t.
 *   x_0 = x0 if given, else t (t = 1/n everywhere when tele is NULL)
 *   D_i = sum of x_i(u) over dangling u (no out-edges)
 *   x_{i+1}(v) = (1-d) t(v) + d (sum_{u->v} x_i(u)/outdeg(u) + D_i t(v))
 *   res_i = sum_v |x_{i+1}(v) - x_i(v)|
 * Runs until res_i < tol (tol > 0) or max_iters iterations.
 * Returns 0, 1 when tol > 0 was never reached, negative on bad input.
 */
int orc_pagerank_csc(int64_t n, const int32_t* row_off, const int64_t* in_off, const int32_t* in_src, double d,
                     const double* tele, const double* x0, int max_iters, double tol, int nthreads, double* x_out,
                     double* res_hist, int32_t* iters_out, double* sec_per_iter) {
  orc_threads(nthreads);
  if (n <= 0 || max_iters < 0) return -1;
  double* x = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  double* spr = (double*)malloc((size_t)n * sizeof(double));
  if (!x || !y || !spr) abort();
  const double un = 1.0 / (double)n;
  for (int64_t v = 0; v < n; ++v) x[v] = x0 ? x0[v] : (tele ? tele[v] : un);

  int rc = (tol > 0.0) ? 1 : 0;
  int32_t it = 0;
  double t0 = omp_get_wtime();
  for (it = 0; it < max_iters;) {
    orc_sum_ctx ctx = {row_off, x, NULL};
    const double D = orc_fixed_sum(n, orc_dangling_term, &ctx);
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; ++u) {
      const int64_t od = row_off[u + 1] - row_off[u];
      spr[u] = od > 0 ? x[u] / (double)od : 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) s += spr[in_src[e]];
      const double t = tele ? tele[v] : un;
      y[v] = (1.0 - d) * t + d * (s + D * t);
    }
    ctx.y = y;
    const double res = orc_fixed_sum(n, orc_l1_term, &ctx);
    if (res_hist) res_hist[it] = res;
    double* sw = x; x = y; y = sw;
    ++it;
    if (tol > 0.0 && res < tol) { rc = 0; break; }
  }
  double t1 = omp_get_wtime();
  if (sec_per_iter) *sec_per_iter = it > 0 ? (t1 - t0) / it : 0.0;
  memcpy(x_out, x, (size_t)n * sizeof(double));
  if (iters_out) *iters_out = it;
  free(x); free(y); free(spr);
  return rc;
}

/* The same with the transposed adjacency formed here from the CSR. */
int orc_pagerank(int64_t n, const int32_t* row_off, const int32_t* col, double d, const double* tele,
                 const double* x0, int max_iters, double tol, int nthreads, double* x_out,
                 double* res_hist, int32_t* iters_out, double* sec_per_iter) {
  if (n <= 0 || max_iters < 0) return -1;
  int64_t* in_off = NULL;
  int32_t* in_src = NULL;
  if (orc_transpose(n, row_off, col, &in_off, &in_src) != 0) return -2;
  const int rc = orc_pagerank_csc(n, row_off, in_off, in_src, d, tele, x0, max_iters, tol, nthreads, x_out,
                                  res_hist, iters_out, sec_per_iter);
  free(in_off); free(in_src);
  return rc;
}

/*
 * One step of Eq. 1 from x (FP64, length n), at the nodes listed in nodes[s]
 * (distinct, in [0,n)):
 *   out[i] = (1-d) t(v) + d (sum_{u->v} x(u)/outdeg(u) + D t(v)),  v = nodes[i]
 * with D the dangling mass of x and t = tele (or 1/n when tele is NULL).
 * Every edge is scanned once; each thread keeps its own partial sums, added
 * in thread order.  Returns 0, negative on bad input.
 */
int orc_step_at(int64_t n, const int32_t* row_off, const int32_t* col, double d, const double* tele,
                const double* x, const int64_t* nodes, int64_t s, int nthreads, double* out) {
  orc_threads(nthreads);
  if (n <= 0 || s < 0) return -1;
  int32_t* slot = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!slot) return -2;
  for (int64_t v = 0; v < n; ++v) slot[v] = -1;
  for (int64_t i = 0; i < s; ++i) {
    if (nodes[i] < 0 || nodes[i] >= n || slot[nodes[i]] >= 0) { free(slot); return -1; }
    slot[nodes[i]] = (int32_t)i;
  }
  orc_sum_ctx ctx = {row_off, x, NULL};
  const double D = orc_fixed_sum(n, orc_dangling_term, &ctx);
  const int T = omp_get_max_threads();
  double* part = (double*)calloc((size_t)T * (size_t)(s > 0 ? s : 1), sizeof(double));
  if (!part) { free(slot); return -2; }
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    double* acc = part + (size_t)t * (size_t)s;
    const int64_t u0 = n * t / T, u1 = n * (t + 1) / T;
    for (int64_t u = u0; u < u1; ++u) {
      const int64_t od = row_off[u + 1] - row_off[u];
      for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) {
        const int32_t j = slot[col[e]];
        if (j >= 0) acc[j] += x[u] / (double)od;
      }
    }
  }
  const double un = 1.0 / (double)n;
  for (int64_t i = 0; i < s; ++i) {
    double sum = 0.0;
    for (int t = 0; t < T; ++t) sum += part[(size_t)t * (size_t)s + i];
    const double tv = tele ? tele[nodes[i]] : un;
    out[i] = (1.0 - d) * tv + d * (sum + D * tv);
  }
  free(part);
  free(slot);
  return 0;
}

/* ---- Partition-Node Graph, from its definitions ------------------------ */

int orc_png_sizes(int64_t n, const int32_t* row_off, const int32_t* col, int64_t q,
                  int64_t* k_out, int64_t* eprime_out) {
  if (n <= 0 || q <= 0) return -1;
  int64_t ep = 0;
  for (int64_t u = 0; u < n; ++u) {
    int64_t prev = -1;
    for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) {
      const int64_t pp = col[e] / q;
      if (pp != prev) { ++ep; prev = pp; }
    }
  }
  *k_out = (n + q - 1) / q;
  *eprime_out = ep;
  return 0;
}

/*
 * Canonical layout (all offsets int64):
 *   U(p,p')          ascending u in P_p with at least one out-neighbour in P_p'
 *   png_off[p][j]    sum_{p'<j} |U(p,p')|, j = 0..k   (local to partition p)
 *   png_src          concatenation over p, then p', of U(p,p')
 *   upd_start[j]     sum_{p'<j} sum_p |U(p,p')|, j = 0..k
 *   wo[p][p']        sum_{p''<p} |U(p'',p')|          (write offset, Sec. 3.1)
 *   did_start[j]     number of edges whose destination lies in P_0..P_{j-1}
 *   did              bin p' lists, for p ascending, u in U(p,p') ascending,
 *                    every v in N_o(u) within P_p' ascending; the first v of
 *                    each (u,p') message carries the MSB (Sec. 3.2)
 */
int orc_png_layout(int64_t n, const int32_t* row_off, const int32_t* col, int64_t q,
                   int64_t* png_off, int32_t* png_src, int64_t* upd_start, int64_t* wo,
                   int64_t* did_start, uint32_t* did) {
  if (n <= 0 || q <= 0) return -1;
  const int64_t k = (n + q - 1) / q;
  int64_t* cnt = (int64_t*)calloc((size_t)(k * k), sizeof(int64_t));
  int64_t* raw = (int64_t*)calloc((size_t)(k * k), sizeof(int64_t));
  int64_t* png_base = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
  int64_t* cur_png = (int64_t*)calloc((size_t)(k * k), sizeof(int64_t));
  int64_t* cur_did = (int64_t*)calloc((size_t)(k * k), sizeof(int64_t));
  if (!cnt || !raw || !png_base || !cur_png || !cur_did) abort();

  /* |U(p,p')| and the number of raw edges from P_p into P_p' */
  for (int64_t u = 0; u < n; ++u) {
    const int64_t p = u / q;
    int64_t prev = -1;
    for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) {
      const int64_t pp = col[e] / q;
      raw[p * k + pp]++;
      if (pp != prev) { cnt[p * k + pp]++; prev = pp; }
    }
  }
  for (int64_t p = 0; p < k; ++p) {
    int64_t s = 0;
    for (int64_t j = 0; j < k; ++j) { png_off[p * (k + 1) + j] = s; s += cnt[p * k + j]; }
    png_off[p * (k + 1) + k] = s;
    png_base[p + 1] = png_base[p] + s;
  }
  {
    int64_t s = 0, sr = 0;
    for (int64_t j = 0; j < k; ++j) {
      upd_start[j] = s;
      did_start[j] = sr;
      for (int64_t p = 0; p < k; ++p) { s += cnt[p * k + j]; sr += raw[p * k + j]; }
    }
    upd_start[k] = s;
    did_start[k] = sr;
  }
  for (int64_t j = 0; j < k; ++j) {
    int64_t s = 0, sr = 0;
    for (int64_t p = 0; p < k; ++p) {
      wo[p * k + j] = s;
      cur_did[p * k + j] = did_start[j] + sr;
      cur_png[p * k + j] = png_base[p] + png_off[p * (k + 1) + j];
      s += cnt[p * k + j];
      sr += raw[p * k + j];
    }
  }
  for (int64_t u = 0; u < n; ++u) {
    const int64_t p = u / q;
    int64_t prev = -1;
    for (int64_t e = row_off[u]; e < row_off[u + 1]; ++e) {
      const int64_t pp = col[e] / q;
      const int first = (pp != prev);
      if (first) { png_src[cur_png[p * k + pp]++] = (int32_t)u; prev = pp; }
      did[cur_did[p * k + pp]++] = (uint32_t)col[e] | (first ? ORC_MSB : 0u);
    }
  }
  free(cnt); free(raw); free(png_base); free(cur_png); free(cur_did);
  return 0;
}

/*
 * One FP64 iteration over the layout above:
 *   scatter (Alg. 3): for p, p', u in U(p,p'):
 *       update_bins[p'][wo[p][p'] + rank of u in U(p,p')] = x(u)/outdeg(u)
 *   gather (Alg. 5): per bin, ptr starts one before the bin; for every
 *       destination ID, ptr += MSB(id); acc[id & mask] += update_bins[p'][ptr]
 *   apply (Alg. 2): y(v) = (1-d) t(v) + d (acc(v) + D t(v)), D = dangling mass
 * Returns res = sum_v |y(v) - x(v)| through *res (may be NULL).
 */
int orc_pcpm_iterate(int64_t n, const int32_t* row_off, int64_t q, const int64_t* png_off,
                     const int32_t* png_src, const int64_t* upd_start, const int64_t* wo,
                     const int64_t* did_start, const uint32_t* did, double d, const double* tele,
                     const double* x, double* y, double* res) {
  const int64_t k = (n + q - 1) / q;
  double* upd = (double*)malloc((size_t)(upd_start[k] > 0 ? upd_start[k] : 1) * sizeof(double));
  double* acc = (double*)calloc((size_t)n, sizeof(double));
  if (!upd || !acc) abort();
  int64_t base = 0;
  for (int64_t p = 0; p < k; ++p) {
    for (int64_t pp = 0; pp < k; ++pp) {
      for (int64_t j = png_off[p * (k + 1) + pp]; j < png_off[p * (k + 1) + pp + 1]; ++j) {
        const int64_t u = png_src[base + j];
        const int64_t od = row_off[u + 1] - row_off[u];
        upd[upd_start[pp] + wo[p * k + pp] + (j - png_off[p * (k + 1) + pp])] = x[u] / (double)od;
      }
    }
    base += png_off[p * (k + 1) + k];
  }
  for (int64_t pp = 0; pp < k; ++pp) {
    const double* bin = upd + upd_start[pp];
    int64_t ptr = -1;
    for (int64_t e = did_start[pp]; e < did_start[pp + 1]; ++e) {
      const uint32_t id = did[e];
      ptr += (int64_t)(id >> 31);
      acc[id & ~ORC_MSB] += bin[ptr];
    }
  }
  orc_sum_ctx ctx = {row_off, x, NULL};
  const double D = orc_fixed_sum(n, orc_dangling_term, &ctx);
  const double un = 1.0 / (double)n;
  for (int64_t v = 0; v < n; ++v) {
    const double t = tele ? tele[v] : un;
    y[v] = (1.0 - d) * t + d * (acc[v] + D * t);
  }
  ctx.y = y;
  if (res) *res = orc_fixed_sum(n, orc_l1_term, &ctx);
  free(upd);
  free(acc);
  return 0;
}
