/*
 * prhip -- Static and DF-P PageRank on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libprhip.so. Method: S. Sahu, "Efficient GPU Implementation of
 * Static and Incrementally Expanding DF-P PageRank for Dynamic Graphs"
 * (arXiv 2404.08299).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - All array pointers are DEVICE pointers owned by the caller (for example
 *    torch tensor storage on the current HIP device). A call borrows them for
 *    its duration only. The library owns nothing but its internal workspace,
 *    which it allocates on first use per device, keeps for reuse, and frees
 *    in pr_release(). Every array argument is checked before any work is
 *    enqueued: host memory (pageable or pinned) or memory of another device
 *    gives PR_EINVAL, and no kernel sees it.
 *  - Calls are synchronous with respect to the host: when a call returns,
 *    every output is complete on the stream given to pr_set_stream() (the
 *    default stream if none). Convergence is decided inside the call.
 *  - Vertex IDs are int32, ranks are FP64 (Sec. 5.1.2).
 *  - Input contract (Sec. 3.1, "dead ends"): every vertex has exactly one
 *    self-loop, so |out(u)| >= 1 for all u; rows hold no duplicates; each
 *    in-row lists its sources in ascending order. pr_validate_csr() checks
 *    this; the compute entry points trust it and read out of bounds if a
 *    caller breaks it.
 *  - Return value: PR_OK (0); PR_NOT_CONVERGED (1) when max_iter iterations
 *    ran without meeting the tolerance (the ranks are still written); a
 *    negative PR_E* code on error, with a message in pr_last_error(). The
 *    library never aborts, exits or prints. Calls from several host threads
 *    are serialised internally (they share one workspace per device).
 */
#ifndef PRHIP_H
#define PRHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_OK 0
#define PR_NOT_CONVERGED 1
#define PR_EINVAL (-1) /* bad argument: NULL, n <= 0, alpha outside (0,1), tol < 0, ... */
#define PR_EGRAPH (-2) /* pr_validate_csr: the graph breaks the input contract      */
#define PR_EBATCH (-3) /* a batch vertex ID is outside [0, n)                        */
#define PR_ENOMEM (-4) /* workspace allocation failed                                */
#define PR_EHIP (-5)   /* a HIP runtime call failed (message in pr_last_error)       */

/* Paper defaults (Sec. 5.1.2). */
#define PR_ALPHA 0.85
#define PR_TOL 1e-10
#define PR_FRONTIER_TOL 1e-6
#define PR_PRUNE_TOL 1e-6
#define PR_MAX_ITERATIONS 500

/*
 * One graph G(V, E) in both CSR views (Sec. 4.1, 4.3: G' drives the rank
 * pull, G drives the marking of affected vertices).
 *   n, m          |V| and |E| (self-loops included)
 *   in_offsets    [n+1] CSR of the transpose G': row v spans
 *   in_sources    [m]   in_sources[in_offsets[v] .. in_offsets[v+1]) = the
 *                       sources u of the edges u -> v, ascending
 *   out_offsets   [n+1] CSR of G: |out(u)| = out_offsets[u+1] - out_offsets[u]
 *   out_targets   [m]   targets of u's out-edges (read by pr_dfp only; may be
 *                       NULL for pr_static)
 */
typedef struct pr_csr {
  int32_t n;
  int32_t m;
  const int32_t *in_offsets;
  const int32_t *in_sources;
  const int32_t *out_offsets;
  const int32_t *out_targets;
} pr_csr;

/* A list of edges (src[i] -> dst[i]), i < count, device arrays. */
typedef struct pr_edges {
  const int32_t *src;
  const int32_t *dst;
  int32_t count;
} pr_edges;

/*
 * Static PageRank (Alg. 1; update of Eq. 1, Sec. 3.1):
 *   R[v] = alpha * sum_{u in in(v)} R[u] / |out(u)| + (1 - alpha) / n,
 * synchronous (two rank vectors), pull-based, no atomics on ranks. Starts
 * from R = 1/n, stops when max_v |R_new[v] - R[v]| <= tol (L-infinity) or
 * after max_iter iterations. The returned vector is the last one computed.
 *   csr        graph (in_* and out_offsets are read)
 *   ranks_out  [n] device, written
 */
int pr_static(const pr_csr *csr, double alpha, double tol, int max_iter, double *ranks_out);

/*
 * pr_static without any allocation, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments, update, stopping rule and return codes as pr_static; it never
 * calls hipMalloc, hipFree or another allocating routine. Its scratch is a
 * fixed device-resident array of PR_NOALLOC_SCRATCH_BYTES that each device
 * holds from the time the library's code is loaded on it until the process
 * ends, shared by every call on that device and left holding the last call's
 * contents (each call initialises what it reads). Calls that overlapped on
 * one device's array would race on it; they do not: a call returns only
 * after its device work has finished, calls within a process are serialised,
 * and each process that loads the library has its own copy of the array.
 * Limits: n <= PR_NOALLOC_MAX_N and about 44 n + 12 m / hub_chunk_edges
 * bytes of scratch (at most PR_NOALLOC_SCRATCH_BYTES); beyond them PR_EINVAL,
 * before any work is enqueued, with the reason in pr_last_error().
 * It runs without the gather-side relabel and the die split (every other
 * tuning field applies), so its ranks equal pr_static's under the tuning
 * relabel = 0, xcd_split_degree = 0 bit for bit, and pr_static's under any
 * other tuning up to summation-order rounding. The convergence flag is read
 * every 4 iterations (iters_per_sync is not used); profiling is not recorded.
 */
#define PR_NOALLOC_MAX_N (1 << 20)
#define PR_NOALLOC_SCRATCH_BYTES (64 << 20)
int pr_static_noalloc(const pr_csr *csr, double alpha, double tol, int max_iter,
                      double *ranks_out);

/*
 * DF-P PageRank (Alg. 2 with updateRanks of Alg. 3, partitioning of Alg. 4
 * and marking of Alg. 5; closed-loop update of Eq. 2, Sec. 4.3).
 *   csr_old     G^{t-1}; not read by the computation (kept for the interface
 *               of the method's problem statement, Sec. 3.3); may be NULL
 *   csr_new     G^t, both views (in_* for the rank pull, out_* for marking)
 *   deletions   Delta^- = E^{t-1} \ E^t (sources and targets are read)
 *   insertions  Delta^+ = E^t \ E^{t-1} (only sources are read, Sec. 4.3);
 *               either batch may have count 0 and NULL arrays
 *   ranks_prev  [n] R^{t-1}
 *   ranks_out   [n] written; may alias ranks_prev (in-place update)
 * An affected vertex is recomputed with Eq. 2, pruned (no longer affected)
 * when its relative change |r - R[v]| / max(r, R[v]) <= prune_tol, and flags
 * its out-neighbours for marking when that change > frontier_tol. A vertex
 * that is not affected keeps its rank. At most PR_MAX_ITERATIONS iterations.
 * Batch IDs outside [0, n) give PR_EBATCH (ranks_out is then unspecified).
 */
int pr_dfp(const pr_csr *csr_old, const pr_csr *csr_new, const pr_edges *deletions,
           const pr_edges *insertions, const double *ranks_prev, double alpha, double tol,
           double frontier_tol, double prune_tol, double *ranks_out);

/* Variants of the dynamic update selected by pr_dfp_ex's `mode`. */
#define PR_MODE_DFP 0 /* Dynamic Frontier with Pruning: Eq. 2 + pruning (Sec. 4.3)    */
#define PR_MODE_DF 1  /* Dynamic Frontier: Eq. 1, no pruning (Sec. 4.3, Alg. 3)       */
#define PR_MODE_ND 2  /* Naive-dynamic: Static from R^{t-1}, all vertices (Sec. 3.4.1) */
#define PR_MODE_DT 3  /* Dynamic Traversal: every vertex reachable from the batch,     */
                      /* Eq. 1 over that fixed set (Sec. 3.4.2, Alg. 7)              */

/* pr_dfp with an explicit iteration cap and update variant. */
int pr_dfp_ex(const pr_csr *csr_old, const pr_csr *csr_new, const pr_edges *deletions,
              const pr_edges *insertions, const double *ranks_prev, double alpha, double tol,
              double frontier_tol, double prune_tol, int max_iter, int mode, double *ranks_out);

/*
 * Personalised PageRank with k teleport vectors (Eq. 1 with the uniform
 * teleport (1-alpha)/|V| replaced by (1-alpha) * s_j[v]):
 *   R_j[v] = alpha * sum_{u in in(v)} R_j[u] / |out(u)| + (1 - alpha) * s_j[v].
 * All vectors start from 1/n and iterate together; vector j stops on its own
 * when max_v |R_j,new[v] - R_j[v]| <= tol and keeps that iterate.
 *   teleport   [n][k] device, vertex-major (s_j[v] at teleport[v*k + j])
 *   ranks_out  [n][k] device, vertex-major, written
 *   iters_out  [k] HOST array receiving each vector's iteration count, or NULL
 * PR_NOT_CONVERGED if some vector reached max_iter.
 */
int pr_ppr(const pr_csr *csr, const double *teleport, int k, double alpha, double tol,
           int max_iter, double *ranks_out, int32_t *iters_out);

/*
 * Static or personalised PageRank (Alg. 1 with Eq. 1's teleport term, or the
 * personalised term of pr_ppr) on num_graphs independent graphs in one
 * batched computation: the graphs are joined into one block-diagonal union,
 * every graph keeps its own teleport term and its own L-infinity stop (a
 * converged graph is no longer updated), and the iterations run as replays
 * of one captured hipGraph (several iterations per replay; the instantiated
 * graph is kept and updated in place by the next call of the same shape).
 * Many personalised vectors of one graph are run by passing that graph once
 * per vector. A graph with a uniform teleport gives the same bits as
 * pr_static on it with the same tuning; one with teleport s_g gives
 *   R[v] = alpha * sum_{u in in(v)} R[u] / |out(u)| + (1 - alpha) * s_g[v]
 * from R = 1/n_g (as pr_ppr with k = 1, up to the order of summation).
 *   graphs       [num_graphs] host array of graphs (device pointers inside;
 *                out_targets not read); total vertices and edges < 2^31
 *   num_graphs   1 .. 4096
 *   teleport     [num_graphs] host array of device pointers, [n_g] each
 *                (s_g; not normalised by the library), or NULL entries for
 *                the uniform term (1 - alpha)/n_g; the array itself may be
 *                NULL (every graph uniform)
 *   ranks_out    [num_graphs] host array of device pointers, [n_g] each
 *   iters_out    [num_graphs] host array for the iteration counts, or NULL
 */
int pr_static_batched(const pr_csr *graphs, int num_graphs, const double *const *teleport,
                      double alpha, double tol, int max_iter, double *const *ranks_out,
                      int32_t *iters_out);

/*
 * Weighted forward (PageRank with given transition weights and teleport):
 *   r_v = alpha * sum_{u in in(v)} P_uv * r_u + (1 - alpha) * s_v,
 * from r = 1/n, L-infinity stop as in pr_static. The weights are used as
 * given (no normalisation); with P_uv = 1/|out(u)| and s = 1/n this is Eq. 1.
 *   in_weights  [m] device, P_uv aligned with in_sources (in-CSR order)
 *   teleport    [n] device, s; NULL means s_v = 1/n with the term (1-alpha)/n
 *   ranks_out   [n] device, written
 */
int pr_weighted(const pr_csr *csr, const double *in_weights, const double *teleport,
                double alpha, double tol, int max_iter, double *ranks_out);

/*
 * Adjoint of pr_weighted. For a loss L(r) with g = dL/dr at the forward
 * solution r, the adjoint lambda solves lambda = g + alpha * A^T lambda
 * (A[v][u] = P_uv), i.e. lambda_u = g_u + alpha * sum_{v in out(u)} P_uv *
 * lambda_v, iterated from 0 with the same L-infinity stop (a pull over the
 * out-CSR; the weights are transposed into out-CSR order on the device).
 * Then
 *   grad_weights[e] = alpha * r_u * lambda_v   for in-edge e = (u -> v),
 *   grad_teleport[v] = (1 - alpha) * lambda_v.
 *   csr            both views (out_targets required; rows ascending)
 *   in_weights     [m] device, P_uv in in-CSR order (as for pr_weighted)
 *   ranks          [n] device, the forward solution r
 *   grad_ranks     [n] device, g
 *   grad_weights   [m] device, in-CSR order, or NULL
 *   grad_teleport  [n] device, or NULL
 *   lambda_out     [n] device, or NULL
 */
int pr_adjoint(const pr_csr *csr, const double *in_weights, const double *ranks,
               const double *grad_ranks, double alpha, double tol, int max_iter,
               double *grad_weights, double *grad_teleport, double *lambda_out);

/* Output views of pr_apply_batch: device arrays owned by the caller. */
typedef struct pr_csr_out {
  int32_t n, m;           /* n as in the input; m = input m - deletions + insertions */
  int32_t *in_offsets;    /* [n+1] */
  int32_t *in_sources;    /* [m]   */
  int32_t *out_offsets;   /* [n+1] (NULL: the out view is not built) */
  int32_t *out_targets;   /* [m]   (NULL with out_offsets)             */
} pr_csr_out;

/*
 * Applies a batch update on the device (Sec. 3.3): G^t = G^{t-1} minus the
 * deletions plus the insertions, both CSR views, rows ascending. The paper
 * does this on the host before its timed region; here it runs on the GPU,
 * so a dynamic pipeline never leaves the device.
 *   old          G^{t-1}; out_targets required when out->out_offsets is set
 *   deletions    pairs (src[i] -> dst[i]) present in G^{t-1}, no self-loops
 *   insertions   pairs absent from G^{t-1} (dst required here)
 *   out          G^t; out->n = old->n and out->m = old->m - deletions +
 *                insertions; its arrays must not alias old's
 * The batch must be normalised (the set differences): a repeated pair, a
 * deletion that is absent or an insertion that is present returns
 * PR_EBATCH (out then holds unspecified values; nothing is written outside
 * its arrays). Sorts the batch keys on the device (its own radix sort) and
 * allocates stream-ordered scratch.
 */
int pr_apply_batch(const pr_csr *old, const pr_edges *deletions, const pr_edges *insertions,
                   const pr_csr_out *out);

/*
 * Checks the input contract on the device: offsets start at 0, are
 * non-decreasing and end at m; every ID is in [0, n); rows are strictly
 * ascending (no duplicates); every vertex has its self-loop in both views;
 * both views have equal degree sums. Returns PR_OK or PR_EGRAPH (the first
 * violated rule is named in pr_last_error). out_targets may be NULL, in which
 * case only the in view and the out degrees are checked.
 */
int pr_validate_csr(const pr_csr *csr);

/*
 * Launch parameters of the kernels. The results do not depend on them
 * beyond the order of floating-point summation in the wave/workgroup
 * reductions (Alg. 4 leaves the degree threshold unspecified).
 *   lane_max_degree    in-degree <= this: one lane per vertex (Alg. 3,
 *                      thread-per-vertex kernel)
 *   wave_max_degree    in-degree <= this (and above lane_max_degree): one
 *                      64-lane wavefront per vertex (Alg. 3, block-per-vertex
 *                      kernel); above it: the split class (hub_chunk_edges)
 *   expand_lane_max_degree  out-degree <= this: one lane marks the
 *                      neighbours; up to wave_max_degree one wavefront;
 *                      above it one workgroup per chunk of out-edges (Alg. 5)
 *   iters_per_sync     iterations in flight before the host reads a
 *                      convergence flag (1 = read after every iteration;
 *                      with k > 1 the host waits on iteration i-k+1 while
 *                      later ones run, and iterations enqueued after
 *                      convergence exit at once on the device)
 *   hub_chunk_edges    edges per chunk of the split class: a vertex with
 *                      degree above wave_max_degree is cut into chunks of
 *                      this many edges, one workgroup each; their partial
 *                      sums are added in chunk order (0 = default 4096)
 *   grid_blocks        workgroups of the fixed-size launches that stride over
 *                      the work (0 = as many as can be resident at once)
 *   relabel            gather-side locality renumbering (degree-based
 *                      grouping of the sources, built inside each call):
 *                      1 on, 0 off, -1 automatic (on when n >= 2^20). Rows and
 *                      their summation order are unchanged.
 *   xcd_split_degree   0: off. Otherwise in-degree >= this (and above
 *                      lane_max_degree) selects the die-split class, which
 *                      replaces the wavefront class above this degree and
 *                      the split class: the sources are cut into 8
 *                      contiguous ranges of about equal out-edge count, a
 *                      row's sources in range x are summed (in chunks of
 *                      hub_chunk_edges, one wavefront each) by workgroups on
 *                      accelerator die x, whose L2 then holds only that
 *                      range's contributions, and the partial sums are added
 *                      in range and chunk order. With relabel on, the
 *                      grouping is done inside each range. Must be 0 or >= 2.
 *   expand_pull_per_mille  DF/DF-P expandAffected direction: when the
 *                      frontier (vertices whose neighbours are to be marked)
 *                      holds more than this many thousandths of the
 *                      vertices, every unaffected vertex is marked if one of
 *                      its in-neighbours is in the frontier (pull, over a
 *                      frontier bitmap); otherwise the frontier's out-edges
 *                      are marked (push). Both give the same set. 0 = always
 *                      push; 0..1000.
 */
typedef struct pr_tuning {
  int32_t lane_max_degree;
  int32_t wave_max_degree;
  int32_t expand_lane_max_degree;
  int32_t iters_per_sync;
  int32_t hub_chunk_edges;
  int32_t grid_blocks;
  int32_t relabel;
  int32_t xcd_split_degree;
  int32_t expand_pull_per_mille;
  int32_t frontier_list;
  int32_t chain_numbering;
  int32_t ppr_chunk_edges;
} pr_tuning;

/* frontier_list       DF/DF-P/DT: 1 = after each marking the affected set is
 *                     compacted into a list, and the rank update's lane class
 *                     and the apply/marking step run over that list (tiles
 *                     of 256 affected vertices); 0 = both sweep ID tiles of
 *                     every vertex and skip the unaffected ones. The same
 *                     ranks either way (bit for bit).
 * chain_numbering     DF/DF-P/DT with relabel and the die split on. 1: the
 *                     gather-side numbering is kept from one such call to
 *                     the next on graphs of the same n, and each call maps
 *                     its in-CSR from the mapping the previous call left (a
 *                     streamed copy of the rows whose sources match, a
 *                     lookup elsewhere; nothing about the caller's arrays
 *                     is assumed); the numbering is rebuilt once the
 *                     entries not found that way, summed since it was
 *                     built, pass 1/8 of the edges. 0: numbering and
 *                     mapping built inside each call (the next such call
 *                     releases what was kept). -1 (automatic): 1 when
 *                     n >= 2^23, where the numbering no longer fits the
 *                     dies' L2 caches and a fresh map's lookups miss, else
 *                     0 without the release. The same ranks either way (bit
 *                     for bit). Keeping it costs 16 m + 12 n bytes of device
 *                     memory beyond the workspace; when that cannot be
 *                     allocated the call builds the numbering itself.
 * ppr_chunk_edges     pr_ppr: a row with at most this many in-edges is
 *                     summed whole by one wavefront (lane = vector); a longer
 *                     row is summed in chunks of this many edges whose
 *                     partial rows are added in chunk order, and with the
 *                     die split on it is cut by source range first (the die
 *                     split's threshold is then this + 1, whatever
 *                     xcd_split_degree says beyond 0). 0 = default 256;
 *                     16 .. 2^20.
 * Defaults: lane_max_degree 128, wave_max_degree 4096, expand_lane_max_degree
 * 32, iters_per_sync 2, hub_chunk_edges 4096, grid_blocks 0, relabel -1,
 * xcd_split_degree 129, expand_pull_per_mille 20, frontier_list 1,
 * chain_numbering -1, ppr_chunk_edges 256. */

/* Set (NULL = defaults) or read the process-wide tuning. PR_EINVAL if a
 * field is out of range (degrees < 0, lane > wave, iters_per_sync < 1,
 * xcd_split_degree == 1, frontier_list not 0 or 1, chain_numbering not in
 * -1 .. 1,
 * ppr_chunk_edges not 0 or in 16 .. 2^20). */
int pr_set_tuning(const pr_tuning *t);
int pr_get_tuning(pr_tuning *t);

/*
 * Statistics of the calling thread's last compute call.
 *   iterations         rank updates performed (Alg. 1/2 loop count)
 *   converged          1 if the tolerance was met
 *   final_delta        L-infinity change of the last iteration
 *   affected_initial   DF-P: affected vertices after the initial marking
 *                      (only at profiling level 2, else -1)
 *   rank_kernel_ms     with profiling on: summed device time of the fused
 *                      rank-update launches of the performed iterations
 *   rank_kernel_launches  number of those launches
 *   total_ms           with profiling on: device time of the whole call
 */
typedef struct pr_stats {
  int32_t iterations;
  int32_t converged;
  double final_delta;
  int64_t affected_initial;
  double rank_kernel_ms;
  int32_t rank_kernel_launches;
  int32_t numbering;         /* gather-side numbering of the call: 0 none, 1 built */
                             /* by it, 2 kept from an earlier DF/DF-P/DT call     */
  double total_ms;
  int64_t affected_max;      /* DF/DF-P/DT, profiling level 2: largest affected set */
  int64_t edges_processed;   /* of an iteration, and the in-edges of the affected */
                             /* vertices summed over the iterations (-1: n/a)    */
  double reserved[2];
} pr_stats;

int pr_last_stats(pr_stats *out);

/* Profiling of this thread's calls: 0 off; 1 HIP events around the call and
 * around every rank-update launch (rank_kernel_ms, total_ms); 2 as 1, plus
 * the affected-set counters of DF/DF-P/DT (affected_initial, affected_max,
 * edges_processed), which add a counting pass per iteration. PR_EINVAL for
 * other levels. */
int pr_set_profiling(int level);

/* Stream for this thread's subsequent calls (a hipStream_t; NULL = default). */
void pr_set_stream(void *hip_stream);

/* Message for this thread's last failure ("" if none). */
const char *pr_last_error(void);

/* Free the cached workspace of every device. */
void pr_release(void);

#ifdef __cplusplus
}
#endif

#endif /* PRHIP_H */
