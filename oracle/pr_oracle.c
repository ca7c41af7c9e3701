/*
 * CPU oracle for Static and DF-P PageRank -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of what the GPU path
 * computes. Only the test suite, the smoke check and the benchmark's CPU
 * baseline call it; the product path never does. It shares no code with the
 * HIP library: it reads a canonical edge list and builds its own adjacency.
 *
 * Build: gcc -O2 -ffp-contract=off -shared -fPIC (no FMA contraction, so every
 * product and sum is rounded as written). Vertex loops run in ascending ID
 * order and every in-edge sum is accumulated in ascending source order.
 *
 * Paper: S. Sahu, "Efficient GPU Implementation of Static and Incrementally
 * Expanding DF-P PageRank for Dynamic Graphs" (arXiv 2404.08299).
 *   Eq. 1  (Sec. 3.1): R[v] = alpha * sum_{u in in(v)} R[u]/|out(u)| + (1-alpha)/|V|
 *   Eq. 2  (Sec. 4.3): closed-loop form for a vertex with a self-loop
 *   Alg. 1 (Static), Alg. 2 (DF*), Alg. 3 (updateRanks), Alg. 5 (marking)
 *
 * Readings of the paper taken here (where it is silent or garbled):
 *   - updateRanks leaves an unaffected vertex's new rank equal to its current
 *     rank (carry forward); the printed pseudocode only skips it.
 *   - a relative change above the frontier tolerance sets delta_N[v] = 1
 *     (the pseudocode prints 0; the prose says such vertices are marked).
 *   - convergence is L-infinity over all vertices with Delta <= tau, tested
 *     after each update; the returned ranks are the ones just computed.
 *
 * PPR, the weighted forward and the adjoint are not in the paper; they are
 * the textbook personalised PageRank iteration and its transposed fixed
 * point (derivation in the adjoint function's comment).
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_EINVAL = -1, OR_ENOMEM = -4 };

/* Adjacency built from an edge list (src[e] -> dst[e]). */
typedef struct {
  int32_t n;
  int64_t m;
  int64_t *in_off;   /* [n+1] */
  int32_t *in_src;   /* [m] sources of in-edges, ascending per row */
  int64_t *in_eid;   /* [m] index of that edge in the input list   */
  int64_t *out_off;  /* [n+1] */
  int32_t *out_tgt;  /* [m] targets of out-edges, ascending per row */
  int64_t *out_eid;  /* [m] */
  int32_t *out_deg;  /* [n] |out(u)| */
} adjacency;

static void adj_free(adjacency *a) {
  free(a->in_off); free(a->in_src); free(a->in_eid);
  free(a->out_off); free(a->out_tgt); free(a->out_eid); free(a->out_deg);
  memset(a, 0, sizeof(*a));
}

/* Stable counting sort of edge ids `ids` by key[id]; result in `out`. */
static int counting_sort(int32_t n, int64_t m, const int32_t *key, const int64_t *ids,
                         int64_t *out, int64_t *off /* [n+1] */) {
  memset(off, 0, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < m; ++i) off[key[ids[i]] + 1]++;
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!pos) return OR_ENOMEM;
  memcpy(pos, off, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < m; ++i) out[pos[key[ids[i]]]++] = ids[i];
  free(pos);
  return OR_OK;
}

static int adj_build(adjacency *a, int32_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  memset(a, 0, sizeof(*a));
  if (n <= 0 || m < 0 || !src || !dst) return OR_EINVAL;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return OR_EINVAL;
  a->n = n; a->m = m;
  a->in_off = malloc(sizeof(int64_t) * ((size_t)n + 1));
  a->out_off = malloc(sizeof(int64_t) * ((size_t)n + 1));
  a->in_src = malloc(sizeof(int32_t) * ((size_t)m + 1));
  a->out_tgt = malloc(sizeof(int32_t) * ((size_t)m + 1));
  a->in_eid = malloc(sizeof(int64_t) * ((size_t)m + 1));
  a->out_eid = malloc(sizeof(int64_t) * ((size_t)m + 1));
  a->out_deg = malloc(sizeof(int32_t) * (size_t)n);
  int64_t *ids = malloc(sizeof(int64_t) * ((size_t)m + 1));
  int64_t *tmp = malloc(sizeof(int64_t) * ((size_t)m + 1));
  if (!a->in_off || !a->out_off || !a->in_src || !a->out_tgt || !a->in_eid || !a->out_eid ||
      !a->out_deg || !ids || !tmp) {
    free(ids); free(tmp); adj_free(a); return OR_ENOMEM;
  }
  for (int64_t e = 0; e < m; ++e) ids[e] = e;
  /* in-lists: sort by source, then stably by destination (LSD radix) */
  if (counting_sort(n, m, src, ids, tmp, a->in_off) ||
      counting_sort(n, m, dst, tmp, a->in_eid, a->in_off)) {
    free(ids); free(tmp); adj_free(a); return OR_ENOMEM;
  }
  for (int64_t i = 0; i < m; ++i) a->in_src[i] = src[a->in_eid[i]];
  /* out-lists: sort by destination, then stably by source */
  if (counting_sort(n, m, dst, ids, tmp, a->out_off) ||
      counting_sort(n, m, src, tmp, a->out_eid, a->out_off)) {
    free(ids); free(tmp); adj_free(a); return OR_ENOMEM;
  }
  for (int64_t i = 0; i < m; ++i) a->out_tgt[i] = dst[a->out_eid[i]];
  for (int32_t u = 0; u < n; ++u) a->out_deg[u] = (int32_t)(a->out_off[u + 1] - a->out_off[u]);
  free(ids); free(tmp);
  return OR_OK;
}

static double linf_delta(int32_t n, const double *x, const double *y) {
  double d = 0.0;
  for (int32_t v = 0; v < n; ++v) {
    double t = fabs(x[v] - y[v]);
    if (t > d) d = t;
  }
  return d;
}

/* Adjacency over a caller's in-CSR (int32, rows ascending) and out-offsets;
 * the in-source array is borrowed, not copied. */
static int adj_wrap_csr(adjacency *a, int32_t n, const int32_t *in_off, const int32_t *in_src,
                        const int32_t *out_off) {
  memset(a, 0, sizeof(*a));
  if (n <= 0 || !in_off || !in_src || !out_off) return OR_EINVAL;
  a->n = n;
  a->m = in_off[n];
  a->in_off = malloc(sizeof(int64_t) * ((size_t)n + 1));
  a->out_deg = malloc(sizeof(int32_t) * (size_t)n);
  if (!a->in_off || !a->out_deg) { free(a->in_off); free(a->out_deg); return OR_ENOMEM; }
  for (int32_t v = 0; v <= n; ++v) a->in_off[v] = in_off[v];
  for (int32_t u = 0; u < n; ++u) a->out_deg[u] = out_off[u + 1] - out_off[u];
  a->in_src = (int32_t *)in_src;
  return OR_OK;
}

static double now_seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Static PageRank: Alg. 1 with the update of Eq. 1.
 * R = R_new = 1/|V| (or `init` when given: the Naive-dynamic variant of
 * Sec. 3.4.1 starts from the previous ranks); each iteration computes R_new
 * from R for every vertex, Delta = max_v |R_new[v] - R[v]|, swaps, and stops
 * when Delta <= tol, at most max_iter iterations.
 * Requires |out(u)| >= 1 for every u (the self-loop convention).
 * `seconds` (may be NULL) receives the wall time of the iteration loop.
 */
static int static_iterate(const adjacency *a, double alpha, double tol, int32_t max_iter,
                          const double *init, double *ranks, int32_t *iters, double *delta,
                          double *seconds) {
  const int32_t n = a->n;
  for (int32_t u = 0; u < n; ++u)
    if (a->out_deg[u] == 0) return OR_EINVAL;
  double *R = malloc(sizeof(double) * (size_t)n), *Rn = malloc(sizeof(double) * (size_t)n);
  if (!R || !Rn) { free(R); free(Rn); return OR_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = init ? init[v] : 1.0 / (double)n;
  const double C0 = (1.0 - alpha) / (double)n;
  int32_t it = 0;
  double d = 0.0;
  int converged = 0;
  const double t0 = now_seconds();
  while (it < max_iter) {
    for (int32_t v = 0; v < n; ++v) {
      double c = 0.0;
      for (int64_t i = a->in_off[v]; i < a->in_off[v + 1]; ++i) {
        int32_t u = a->in_src[i];
        c = c + R[u] / (double)a->out_deg[u];
      }
      Rn[v] = C0 + alpha * c;
    }
    d = linf_delta(n, Rn, R);
    double *t = R; R = Rn; Rn = t;
    ++it;
    if (d <= tol) { converged = 1; break; }
  }
  if (seconds) *seconds = now_seconds() - t0;
  memcpy(ranks, R, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  if (delta) *delta = d;
  free(R); free(Rn);
  return converged ? OR_OK : OR_NOT_CONVERGED;
}

int oracle_static(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, double alpha,
                  double tol, int32_t max_iter, const double *init, double *ranks,
                  int32_t *iters, double *delta) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(tol >= 0.0) || max_iter <= 0 || !ranks) return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  rc = static_iterate(&a, alpha, tol, max_iter, init, ranks, iters, delta, NULL);
  adj_free(&a);
  return rc;
}

/* Static PageRank over a given in-CSR (rows ascending by source) and
 * out-offsets, with the wall time of the iteration loop in `seconds`. Same
 * iteration as oracle_static; used to time the oracle without its own
 * adjacency construction. */
int oracle_static_csr(int32_t n, const int32_t *in_off, const int32_t *in_src,
                      const int32_t *out_off, double alpha, double tol, int32_t max_iter,
                      double *ranks, int32_t *iters, double *delta, double *seconds) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(tol >= 0.0) || max_iter <= 0 || !ranks) return OR_EINVAL;
  adjacency a;
  int rc = adj_wrap_csr(&a, n, in_off, in_src, out_off);
  if (rc) return rc;
  rc = static_iterate(&a, alpha, tol, max_iter, NULL, ranks, iters, delta, seconds);
  free(a.in_off);
  free(a.out_deg);
  return rc;
}

/* One update of a pull iteration for listed (row, vector) pairs only, from
 * the given R (n x ld, vertex-major; vector j is column j):
 *   out[i] = t + alpha * sum_{u in in(v)} x_u,  v = rows[i], j = cols ? cols[i] : 0,
 *   x_u = w ? w[e] * R[u][j] : R[u][j] / |out(u)|  (e the in-edge u -> v, in
 *         in-CSR order),
 *   t = s ? (1 - alpha) * s[v][j] : (1 - alpha)/|V|,
 * sources in ascending order, as in the full iterations: Eq. 1 (Static),
 * personalised PageRank (s per vector) and the weighted forward (w per
 * edge). For graphs too large for the full iteration here: a sample of one
 * step of a long run. */
int oracle_pull_rows(int32_t n, const int32_t *in_off, const int32_t *in_src,
                     const int32_t *out_off, const double *w, const double *R, int32_t ld,
                     const double *s, double alpha, int64_t k, const int32_t *rows,
                     const int32_t *cols, double *out) {
  if (n <= 0 || !in_off || !in_src || (!w && !out_off) || !R || ld <= 0 || k < 0 ||
      (k && (!rows || !out)))
    return OR_EINVAL;
  const double C0 = (1.0 - alpha) / (double)n;
  for (int64_t i = 0; i < k; ++i) {
    const int32_t v = rows[i], j = cols ? cols[i] : 0;
    if (v < 0 || v >= n || j < 0 || j >= ld) return OR_EINVAL;
    double c = 0.0;
    for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
      const int32_t u = in_src[e];
      const double x = R[(size_t)u * (size_t)ld + (size_t)j];
      if (w) c = c + w[e] * x;
      else c = c + x / (double)(out_off[u + 1] - out_off[u]);
    }
    const double t = s ? (1.0 - alpha) * s[(size_t)v * (size_t)ld + (size_t)j] : C0;
    out[i] = t + alpha * c;
  }
  return OR_OK;
}

/* expandAffected of Alg. 5: for each u with delta_N[u], mark every v in out(u). */
static void expand_affected(const adjacency *a, uint8_t *dV, const uint8_t *dN) {
  for (int32_t u = 0; u < a->n; ++u)
    if (dN[u])
      for (int64_t i = a->out_off[u]; i < a->out_off[u + 1]; ++i) dV[a->out_tgt[i]] = 1;
}

/*
 * Dynamic Frontier PageRank: Alg. 2 with updateRanks of Alg. 3 and the
 * marking of Alg. 5, on G^t given as an edge list.
 *   prune = 1: DF-P (Eq. 2 closed-loop update, pruning when the relative
 *              change is <= tau_p);
 *   prune = 0: DF (Eq. 1 update, no pruning).
 * The batch (deletions and insertions) must be the set differences between
 * G^{t-1} and G^t. Only insertion sources are read.
 * stats (may be NULL): [0] affected after initial marking, [1] maximum
 * affected at the start of an iteration, [2] in-edges processed (sum over
 * iterations of the in-degrees of the updated vertices), [3] vertices ever
 * affected.
 * trace (may be NULL): (max_iter + 1) x n bytes; row i is delta_V at the
 * start of iteration i (row 0 after the initial marking).
 */
static int dfp_run(const adjacency *ap, int64_t n_del, const int32_t *del_src,
                   const int32_t *del_dst, int64_t n_ins, const int32_t *ins_src,
                   const double *ranks_prev, double alpha, double tol, double tau_f,
                   double tau_p, int32_t max_iter, int32_t prune, double *ranks, int32_t *iters,
                   double *delta, int64_t *stats, uint8_t *trace) {
  const adjacency a = *ap;
  const int32_t n = a.n;
  for (int32_t u = 0; u < n; ++u)
    if (a.out_deg[u] == 0) return OR_EINVAL;
  for (int64_t i = 0; i < n_del; ++i)
    if (del_src[i] < 0 || del_src[i] >= n || del_dst[i] < 0 || del_dst[i] >= n) return OR_EINVAL;
  for (int64_t i = 0; i < n_ins; ++i)
    if (ins_src[i] < 0 || ins_src[i] >= n) return OR_EINVAL;
  double *R = malloc(sizeof(double) * (size_t)n), *Rn = malloc(sizeof(double) * (size_t)n);
  uint8_t *dV = calloc((size_t)n, 1), *dN = calloc((size_t)n, 1), *ever = calloc((size_t)n, 1);
  if (!R || !Rn || !dV || !dN || !ever) {
    free(R); free(Rn); free(dV); free(dN); free(ever); return OR_ENOMEM;
  }
  /* initialise both rank vectors from the previous ranks (Alg. 2) */
  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = ranks_prev[v];
  /* initialAffected (Alg. 5) */
  for (int64_t i = 0; i < n_del; ++i) { dN[del_src[i]] = 1; dV[del_dst[i]] = 1; }
  for (int64_t i = 0; i < n_ins; ++i) dN[ins_src[i]] = 1;
  expand_affected(&a, dV, dN);
  const double C0 = (1.0 - alpha) / (double)n;
  int64_t aff0 = 0, affmax = 0, edges = 0, ever_n = 0;
  for (int32_t v = 0; v < n; ++v) aff0 += dV[v];
  int32_t it = 0;
  double d = 0.0;
  int converged = 0;
  while (it < max_iter) {
    int64_t aff = 0;
    for (int32_t v = 0; v < n; ++v) { aff += dV[v]; if (dV[v]) ever[v] = 1; }
    if (aff > affmax) affmax = aff;
    if (trace) memcpy(trace + (size_t)it * (size_t)n, dV, (size_t)n);
    memset(dN, 0, (size_t)n);
    /* updateRanks (Alg. 3) */
    for (int32_t v = 0; v < n; ++v) {
      if (!dV[v]) { Rn[v] = R[v]; continue; }
      double c = 0.0;
      const double dv = (double)a.out_deg[v];
      for (int64_t i = a.in_off[v]; i < a.in_off[v + 1]; ++i) {
        int32_t u = a.in_src[i];
        c = c + R[u] / (double)a.out_deg[u];
      }
      edges += a.in_off[v + 1] - a.in_off[v];
      double r;
      if (prune) r = 1.0 / (1.0 - alpha / dv) * (C0 + alpha * (c - R[v] / dv)); /* Eq. 2 */
      else r = C0 + alpha * c;                                                   /* Eq. 1 */
      double dr = fabs(r - R[v]);
      double rel = dr / (r > R[v] ? r : R[v]);
      if (prune && rel <= tau_p) dV[v] = 0;
      if (rel > tau_f) dN[v] = 1;
      Rn[v] = r;
    }
    d = linf_delta(n, Rn, R);
    double *t = R; R = Rn; Rn = t;
    ++it;
    if (d <= tol) { converged = 1; break; }
    expand_affected(&a, dV, dN);
  }
  if (trace && it <= max_iter) memcpy(trace + (size_t)it * (size_t)n, dV, (size_t)n);
  for (int32_t v = 0; v < n; ++v) ever_n += ever[v];
  memcpy(ranks, R, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  if (delta) *delta = d;
  if (stats) { stats[0] = aff0; stats[1] = affmax; stats[2] = edges; stats[3] = ever_n; }
  free(R); free(Rn); free(dV); free(dN); free(ever);
  return converged ? OR_OK : OR_NOT_CONVERGED;
}

static int dfp_args_ok(double alpha, double tol, int32_t max_iter, const double *ranks,
                       const double *ranks_prev, int64_t n_del, const int32_t *del_src,
                       const int32_t *del_dst, int64_t n_ins, const int32_t *ins_src) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(tol >= 0.0) || max_iter <= 0 || !ranks || !ranks_prev)
    return 0;
  return !((n_del > 0 && (!del_src || !del_dst)) || (n_ins > 0 && !ins_src));
}

int oracle_dfp(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t n_del,
               const int32_t *del_src, const int32_t *del_dst, int64_t n_ins,
               const int32_t *ins_src, const double *ranks_prev, double alpha, double tol,
               double tau_f, double tau_p, int32_t max_iter, int32_t prune, double *ranks,
               int32_t *iters, double *delta, int64_t *stats, uint8_t *trace) {
  if (!dfp_args_ok(alpha, tol, max_iter, ranks, ranks_prev, n_del, del_src, del_dst, n_ins,
                   ins_src))
    return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  rc = dfp_run(&a, n_del, del_src, del_dst, n_ins, ins_src, ranks_prev, alpha, tol, tau_f, tau_p,
               max_iter, prune, ranks, iters, delta, stats, trace);
  adj_free(&a);
  return rc;
}

/* The same DF/DF-P run over a given G^t in both CSR views (int32, rows
 * ascending), without building an adjacency from an edge list: for graphs
 * whose edge-list construction is too slow here. */
int oracle_dfp_csr(int32_t n, const int32_t *in_off, const int32_t *in_src,
                   const int32_t *out_off, const int32_t *out_tgt, int64_t n_del,
                   const int32_t *del_src, const int32_t *del_dst, int64_t n_ins,
                   const int32_t *ins_src, const double *ranks_prev, double alpha, double tol,
                   double tau_f, double tau_p, int32_t max_iter, int32_t prune, double *ranks,
                   int32_t *iters, double *delta, int64_t *stats) {
  if (!dfp_args_ok(alpha, tol, max_iter, ranks, ranks_prev, n_del, del_src, del_dst, n_ins,
                   ins_src) || !out_tgt)
    return OR_EINVAL;
  adjacency a;
  int rc = adj_wrap_csr(&a, n, in_off, in_src, out_off);
  if (rc) return rc;
  a.out_off = malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!a.out_off) { free(a.in_off); free(a.out_deg); return OR_ENOMEM; }
  for (int32_t u = 0; u <= n; ++u) a.out_off[u] = out_off[u];
  a.out_tgt = (int32_t *)out_tgt;
  rc = dfp_run(&a, n_del, del_src, del_dst, n_ins, ins_src, ranks_prev, alpha, tol, tau_f, tau_p,
               max_iter, prune, ranks, iters, delta, stats, NULL);
  free(a.in_off); free(a.out_deg); free(a.out_off);
  return rc;
}

/*
 * Dynamic Traversal (Alg. 7, Sec. 3.4.2). Every vertex reachable from a
 * changed edge is affected; Eq. 1 iterations then run over that fixed set
 * from R^{t-1}, and every other vertex keeps its rank. Reachability starts
 * from the marking of Alg. 5 (deletion targets, and the out-neighbours of
 * every batch source, which include the source through its self-loop) and
 * is closed under out-edges by a breadth-first search. Alg. 7 prints its
 * closure loop expanding into the affected flags themselves; the closure is
 * its evident intent (the prose: all vertices reachable from u are flagged).
 * n_affected (optional) receives the size of the affected set.
 */
int oracle_dt(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t n_del,
              const int32_t *del_src, const int32_t *del_dst, int64_t n_ins,
              const int32_t *ins_src, const double *ranks_prev, double alpha, double tol,
              int32_t max_iter, double *ranks, int32_t *iters, double *delta,
              int64_t *n_affected) {
  if (!(alpha > 0.0 && alpha < 1.0) || !(tol >= 0.0) || max_iter <= 0 || !ranks || !ranks_prev)
    return OR_EINVAL;
  if ((n_del > 0 && (!del_src || !del_dst)) || (n_ins > 0 && !ins_src)) return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  for (int32_t u = 0; u < n; ++u)
    if (a.out_deg[u] == 0) { adj_free(&a); return OR_EINVAL; }
  for (int64_t i = 0; i < n_del; ++i)
    if (del_src[i] < 0 || del_src[i] >= n || del_dst[i] < 0 || del_dst[i] >= n) {
      adj_free(&a); return OR_EINVAL;
    }
  for (int64_t i = 0; i < n_ins; ++i)
    if (ins_src[i] < 0 || ins_src[i] >= n) { adj_free(&a); return OR_EINVAL; }
  double *R = malloc(sizeof(double) * (size_t)n), *Rn = malloc(sizeof(double) * (size_t)n);
  uint8_t *dV = calloc((size_t)n, 1), *dN = calloc((size_t)n, 1);
  int32_t *queue = malloc(sizeof(int32_t) * (size_t)n);
  if (!R || !Rn || !dV || !dN || !queue) {
    free(R); free(Rn); free(dV); free(dN); free(queue); adj_free(&a); return OR_ENOMEM;
  }
  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = ranks_prev[v];
  /* initialAffected, expandAffected (Alg. 5) */
  for (int64_t i = 0; i < n_del; ++i) { dV[del_dst[i]] = 1; dN[del_src[i]] = 1; }
  for (int64_t i = 0; i < n_ins; ++i) dN[ins_src[i]] = 1;
  expand_affected(&a, dV, dN);
  /* closure under out-edges: breadth-first search from every affected vertex */
  int64_t head = 0, tail = 0;
  for (int32_t v = 0; v < n; ++v)
    if (dV[v]) queue[tail++] = v;
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int64_t i = a.out_off[u]; i < a.out_off[u + 1]; ++i) {
      const int32_t v = a.out_tgt[i];
      if (!dV[v]) { dV[v] = 1; queue[tail++] = v; }
    }
  }
  if (n_affected) *n_affected = tail;
  /* Eq. 1 over the affected set, the rest carried forward */
  const double C0 = (1.0 - alpha) / (double)n;
  int32_t it = 0;
  double d = 0.0;
  int converged = 0;
  while (it < max_iter) {
    for (int32_t v = 0; v < n; ++v) {
      if (!dV[v]) { Rn[v] = R[v]; /* unreachable: unchanged */ continue; }
      double c = 0.0;
      for (int64_t i = a.in_off[v]; i < a.in_off[v + 1]; ++i) {
        const int32_t u = a.in_src[i];
        c = c + R[u] / (double)a.out_deg[u];
      }
      Rn[v] = C0 + alpha * c; /* Eq. 1 */
    }
    d = linf_delta(n, Rn, R);
    double *t = R; R = Rn; Rn = t;
    ++it;
    if (d <= tol) { converged = 1; break; }
  }
  memcpy(ranks, R, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  if (delta) *delta = d;
  free(R); free(Rn); free(dV); free(dN); free(queue); adj_free(&a);
  return converged ? OR_OK : OR_NOT_CONVERGED;
}

/*
 * Personalised PageRank with k teleport vectors (vertex-major, s[v*k + j]):
 *   R_j[v] = alpha * sum_{u in in(v)} R_j[u]/|out(u)| + (1-alpha) * s_j[v],
 * started from 1/|V|; each vector stops on its own when its L-infinity
 * change is <= tol. With s_j = 1/|V| everywhere this is Eq. 1.
 */
int oracle_ppr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t k,
               const double *s, double alpha, double tol, int32_t max_iter, double *ranks,
               int32_t *iters) {
  if (k <= 0 || !s || !ranks || !(alpha > 0.0 && alpha < 1.0) || max_iter <= 0) return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  double *R = malloc(sizeof(double) * (size_t)n), *Rn = malloc(sizeof(double) * (size_t)n);
  if (!R || !Rn) { free(R); free(Rn); adj_free(&a); return OR_ENOMEM; }
  int all = 1;
  for (int32_t j = 0; j < k; ++j) {
    for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = 1.0 / (double)n;
    int32_t it = 0;
    int conv = 0;
    while (it < max_iter) {
      for (int32_t v = 0; v < n; ++v) {
        double c = 0.0;
        for (int64_t i = a.in_off[v]; i < a.in_off[v + 1]; ++i) {
          int32_t u = a.in_src[i];
          c = c + R[u] / (double)a.out_deg[u];
        }
        Rn[v] = (1.0 - alpha) * s[(size_t)v * (size_t)k + (size_t)j] + alpha * c;
      }
      double d = linf_delta(n, Rn, R);
      double *t = R; R = Rn; Rn = t;
      ++it;
      if (d <= tol) { conv = 1; break; }
    }
    for (int32_t v = 0; v < n; ++v) ranks[(size_t)v * (size_t)k + (size_t)j] = R[v];
    if (iters) iters[j] = it;
    if (!conv) all = 0;
  }
  free(R); free(Rn); adj_free(&a);
  return all ? OR_OK : OR_NOT_CONVERGED;
}

/*
 * Weighted forward: r_v = alpha * sum_{u in in(v)} P_uv * r_u + (1-alpha) * s_v,
 * with P given per edge (w[e] for edge src[e] -> dst[e]), used as given.
 * Started from 1/|V| (or `init`); L-infinity stop as in Alg. 1.
 */
int oracle_weighted(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    const double *w, const double *s, double alpha, double tol, int32_t max_iter,
                    const double *init, double *ranks, int32_t *iters, double *delta) {
  if (!w || !s || !ranks || !(alpha > 0.0 && alpha < 1.0) || max_iter <= 0) return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  double *R = malloc(sizeof(double) * (size_t)n), *Rn = malloc(sizeof(double) * (size_t)n);
  if (!R || !Rn) { free(R); free(Rn); adj_free(&a); return OR_ENOMEM; }
  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = init ? init[v] : 1.0 / (double)n;
  int32_t it = 0;
  double d = 0.0;
  int conv = 0;
  while (it < max_iter) {
    for (int32_t v = 0; v < n; ++v) {
      double c = 0.0;
      for (int64_t i = a.in_off[v]; i < a.in_off[v + 1]; ++i)
        c = c + w[a.in_eid[i]] * R[a.in_src[i]];
      Rn[v] = (1.0 - alpha) * s[v] + alpha * c;
    }
    d = linf_delta(n, Rn, R);
    double *t = R; R = Rn; Rn = t;
    ++it;
    if (d <= tol) { conv = 1; break; }
  }
  memcpy(ranks, R, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  if (delta) *delta = d;
  free(R); free(Rn); adj_free(&a);
  return conv ? OR_OK : OR_NOT_CONVERGED;
}

/*
 * Adjoint of the weighted forward. With A[v][u] = P_uv, the forward fixed
 * point is r = alpha*A*r + (1-alpha)*s. For a loss L(r) with g = dL/dr,
 * lambda = (I - alpha*A^T)^{-1} g solves the transposed fixed point
 *   lambda_u = g_u + alpha * sum_{v in out(u)} P_uv * lambda_v,
 * iterated from lambda = 0 with an L-infinity stop (a contraction with
 * factor alpha when P is row-stochastic). Then
 *   dL/ds_v    = (1-alpha) * lambda_v,
 *   dL/dP_uv   = alpha * r_u * lambda_v    (per edge, input order).
 */
int oracle_adjoint(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                   const double *w, const double *r, const double *g, double alpha, double tol,
                   int32_t max_iter, double *grad_w, double *grad_s, double *lambda_out,
                   int32_t *iters) {
  if (!w || !r || !g || !(alpha > 0.0 && alpha < 1.0) || max_iter <= 0) return OR_EINVAL;
  adjacency a;
  int rc = adj_build(&a, n, m, src, dst);
  if (rc) return rc;
  double *L = calloc((size_t)n, sizeof(double)), *Ln = calloc((size_t)n, sizeof(double));
  if (!L || !Ln) { free(L); free(Ln); adj_free(&a); return OR_ENOMEM; }
  int32_t it = 0;
  int conv = 0;
  while (it < max_iter) {
    for (int32_t u = 0; u < n; ++u) {
      double c = 0.0;
      for (int64_t i = a.out_off[u]; i < a.out_off[u + 1]; ++i)
        c = c + w[a.out_eid[i]] * L[a.out_tgt[i]];
      Ln[u] = g[u] + alpha * c;
    }
    double d = linf_delta(n, Ln, L);
    double *t = L; L = Ln; Ln = t;
    ++it;
    if (d <= tol) { conv = 1; break; }
  }
  if (grad_s)
    for (int32_t v = 0; v < n; ++v) grad_s[v] = (1.0 - alpha) * L[v];
  if (grad_w)
    for (int64_t e = 0; e < m; ++e) grad_w[e] = alpha * r[src[e]] * L[dst[e]];
  if (lambda_out) memcpy(lambda_out, L, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  free(L); free(Ln); adj_free(&a);
  return conv ? OR_OK : OR_NOT_CONVERGED;
}
