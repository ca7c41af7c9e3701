// Static PageRank over many graphs at once on gfx950.
//
// The graphs are concatenated into one union CSR (vertex and edge bases per
// graph, block-diagonal), so the fixed-grid rank update, its partition and
// its locality renumbering run once over all of them. Each vertex carries its
// graph id: the teleport term is (1 - alpha) / n_g of its own graph (or
// (1 - alpha) s_g[v] with the graph's own personalised teleport vector), its
// |change| goes into its graph's maximum (workgroup tables in LDS, then one
// row per workgroup), and once graph g meets the tolerance its vertices are
// no longer updated, so every graph stops exactly where pr_static on it alone
// would stop, with the same per-vertex summation order (bit-identical
// results). The iteration counter lives on the device, so one hipGraph holds
// an even and an odd iteration and is replayed until every graph is done.
#pragma once
#include "kernels.h"

namespace prhip {

// One graph of a batch, as the union build reads it.
struct BatchDesc {
  const int *in_off, *in_src, *out_off;
  int vb, eb;  // first vertex and first edge of the graph in the union
  int n, m;
};

// Index g with base[g] <= x < base[g + 1] (base ascending, base[G] = total).
__device__ __forceinline__ int find_base(const int *__restrict__ base, int G, int x) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Union CSR: offsets and sources shifted by the graph's bases; gid[v] = g.
// Vertices and edges are taken in runs of kUnionRun consecutive elements per
// workgroup: the graph of a run's first element is found once (binary search
// over the bases), and each thread steps to the next graph only when its
// element crosses that graph's base, so the copy streams instead of
// searching per element.
constexpr int kUnionRun = 16 * kBlock;
__global__ __launch_bounds__(kBlock) void k_union_build(
    const BatchDesc *__restrict__ d, const int *__restrict__ vbase, const int *__restrict__ ebase,
    int G, int N, int M, int *__restrict__ in_off, int *__restrict__ in_src,
    int *__restrict__ out_off, int *__restrict__ gid) {
  const long long rstride = (long long)gridDim.x * kUnionRun;
  for (long long r0 = (long long)blockIdx.x * kUnionRun; r0 < N; r0 += rstride) {
    const int r1 = (int)min((long long)N, r0 + kUnionRun);
    int g = find_base(vbase, G, (int)r0);
    int next = vbase[g + 1], vb = d[g].vb, eb = d[g].eb;
    const int *io = d[g].in_off, *oo = d[g].out_off;
    for (int v = (int)r0 + threadIdx.x; v < r1; v += kBlock) {
      while (v >= next) {
        ++g;
        next = vbase[g + 1];
        vb = d[g].vb;
        eb = d[g].eb;
        io = d[g].in_off;
        oo = d[g].out_off;
      }
      in_off[v] = eb + io[v - vb];
      out_off[v] = eb + oo[v - vb];
      gid[v] = g;
    }
  }
  for (long long r0 = (long long)blockIdx.x * kUnionRun; r0 < M; r0 += rstride) {
    const int r1 = (int)min((long long)M, r0 + kUnionRun);
    int g = find_base(ebase, G, (int)r0);
    int next = ebase[g + 1], vb = d[g].vb, eb = d[g].eb;
    const int *src = d[g].in_src;
    for (int e = (int)r0 + threadIdx.x; e < r1; e += kBlock) {
      while (e >= next) {
        ++g;
        next = ebase[g + 1];
        vb = d[g].vb;
        eb = d[g].eb;
        src = d[g].in_src;
      }
      in_src[e] = vb + src[e - eb];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    in_off[N] = M;
    out_off[N] = M;
  }
}

// Output policy of the batched update (see rank_update in kernels.h). The
// teleport term of graph g is (1 - alpha)/n_g (C0g[g]) unless tele[g] is set:
// then it is (1 - alpha) * tele[g][v - vb[g]], personalised PageRank on that
// graph (the form of pr_ppr and pr_weighted: the product first, then + alpha c).
struct BatchOut {
  const int *out_off;
  const int *pos;
  const int *gid;
  const double *C0g;
  const double *const *tele;  // [G] device pointers (null entries: uniform), or null
  const int *vb;              // [G + 1] first vertex of each graph
  const int *gdone;
  const double *R;
  double *Rn, *Xn;
  double alpha;
  unsigned long long *s_gmax;  // LDS: per-graph maximum |change| (bit patterns)
  __device__ __forceinline__ double finish(int v, double c) const {
    const int g = gid[v];
    const double *t = tele ? tele[g] : nullptr;
    const double r = t ? (1.0 - alpha) * t[v - vb[g]] + alpha * c : C0g[g] + alpha * c;
    st_nt(Rn + v, r);
    Xn[xpos(pos, v)] = r / (double)(ld_nt(out_off + v + 1) - ld_nt(out_off + v));
    return fabs(r - ld_nt(R + v));
  }
  __device__ __forceinline__ bool active(int v) const { return !gdone[gid[v]]; }
  __device__ __forceinline__ void inactive(int) const {}
  // non-negative doubles order like their bit patterns
  __device__ __forceinline__ void note(int v, double d) const {
    atomicMax(&s_gmax[gid[v]], (unsigned long long)__double_as_longlong(d));
  }
};

__device__ __forceinline__ void clear_table(unsigned long long *s, int G) {
  for (int g = threadIdx.x; g < G; g += kBlock) s[g] = 0ULL;
  __syncthreads();
}

__device__ __forceinline__ void flush_table(const unsigned long long *s, int G, double *row) {
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += kBlock) row[g] = __longlong_as_double((long long)s[g]);
}

// gpart: [gridDim.x (+ finalize blocks)][G] per-workgroup per-graph maxima.
template <int LG>
__global__ __launch_bounds__(kBlock) void k_rank_batched(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ out_off, const int *__restrict__ pos, const double *__restrict__ X,
    const double *__restrict__ R, double *__restrict__ Rn, double *__restrict__ Xn,
    const int *__restrict__ hi, const int *__restrict__ counts,
    const int *__restrict__ hub_start, const int *__restrict__ chunk_hub,
    double *__restrict__ hub_part, int CH, int n, int t1, const int4 *__restrict__ xitems,
    const int *__restrict__ xoff, const int *__restrict__ gid, const double *__restrict__ C0g,
    const double *const *__restrict__ tele, const int *__restrict__ vb,
    const int *__restrict__ gdone, int G, double alpha, double *__restrict__ gpart, int *tq,
    const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  extern __shared__ unsigned long long s_gmax[];
  clear_table(s_gmax, G);
  const BatchOut out{out_off, pos, gid, C0g, tele, vb, gdone, R, Rn, Xn, alpha, s_gmax};
  rank_update<false, LG>(in_off, in_src, nullptr, X, hi, counts, hub_start, chunk_hub, hub_part, CH,
                         n, t1, xitems, xoff, out, nullptr, nullptr, nullptr, tq);
  flush_table(s_gmax, G, gpart + (size_t)blockIdx.x * G);
}

__global__ __launch_bounds__(kBlock) void k_hub_finalize_batched(
    const int *__restrict__ hi, const int *__restrict__ counts, const int *__restrict__ hub_start,
    const double *__restrict__ hub_part, const int *__restrict__ out_off,
    const int *__restrict__ pos, const double *__restrict__ R, double *__restrict__ Rn,
    double *__restrict__ Xn, const int *__restrict__ gid, const double *__restrict__ C0g,
    const double *const *__restrict__ tele, const int *__restrict__ vb,
    const int *__restrict__ gdone, int G, double alpha, double *__restrict__ gpart,
    int *__restrict__ tq, const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) tq[threadIdx.x] = 0;  // next launch's queues
  extern __shared__ unsigned long long s_gmax[];
  clear_table(s_gmax, G);
  const BatchOut out{out_off, pos, gid, C0g, tele, vb, gdone, R, Rn, Xn, alpha, s_gmax};
  hub_finalize(hi, counts, hub_start, hub_part, out, nullptr);
  flush_table(s_gmax, G, gpart + (size_t)blockIdx.x * G);
}

// Per-graph convergence for the current iteration (ctrl->iters updates so
// far): one workgroup per graph reduces its column of gpart.
__global__ __launch_bounds__(kBlock) void k_batched_final(const double *__restrict__ gpart, int np,
                                                          int G, int *__restrict__ gdone,
                                                          int *__restrict__ giters,
                                                          double *__restrict__ gdelta,
                                                          const Ctrl *__restrict__ ctrl,
                                                          double tol) {
  if (ctrl->done) return;
  __shared__ double lds[kWavesPerBlock];
  const int g = blockIdx.x;
  if (gdone[g]) return;  // uniform over the workgroup
  double m = 0.0;
  for (int b = threadIdx.x; b < np; b += kBlock) m = fmax(m, gpart[(size_t)b * G + g]);
  m = block_max<kBlock>(m, lds);
  if (threadIdx.x == 0) {
    gdelta[g] = m;
    giters[g] = ctrl->iters + 1;
    if (m <= tol) gdone[g] = 1;
  }
}

// Advances the device iteration counter; done once every graph converged or
// max_iter updates ran.
__global__ __launch_bounds__(kBlock) void k_batched_done(const int *__restrict__ gdone, int G,
                                                         Ctrl *__restrict__ ctrl, int max_iter) {
  if (ctrl->done) return;
  __shared__ int open;
  if (threadIdx.x == 0) open = 0;
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += kBlock)
    if (!gdone[g]) open = 1;  // benign: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) {
    ctrl->iters += 1;
    if (!open || ctrl->iters >= max_iter) ctrl->done = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_batched_init(int N, int G, const int *__restrict__ gid,
                                                         const int *__restrict__ vbase,
                                                         const int *__restrict__ out_off,
                                                         const int *__restrict__ pos,
                                                         double *__restrict__ R,
                                                         double *__restrict__ X, int *gdone,
                                                         int *giters, int *__restrict__ tq) {
  const int stride = gridDim.x * kBlock;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) tq[threadIdx.x] = 0;  // first launch's queues
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < N; v += stride) {
    const int g = gid[v];
    const double r = 1.0 / (double)(vbase[g + 1] - vbase[g]);
    R[v] = r;
    X[xpos(pos, v)] = r / (double)(out_off[v + 1] - out_off[v]);
  }
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < G; g += stride) {
    gdone[g] = 0;
    giters[g] = 0;
  }
}

// out[g][v - vb] = buffer (giters[g] & 1) of the union vector.
__global__ __launch_bounds__(kBlock) void k_batched_out(int N, const int *__restrict__ gid,
                                                        const int *__restrict__ vbase,
                                                        const int *__restrict__ giters,
                                                        const double *__restrict__ b0,
                                                        const double *__restrict__ b1,
                                                        double *const *__restrict__ outs) {
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < N; v += gridDim.x * kBlock) {
    const int g = gid[v];
    outs[g][v - vbase[g]] = (giters[g] & 1) ? b1[v] : b0[v];
  }
}

}  // namespace prhip
