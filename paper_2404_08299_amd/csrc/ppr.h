// Personalised PageRank with K teleport vectors on gfx950.
//
//   R_k[v] = alpha * sum_{u in in(v)} R_k[u] / |out(u)| + (1 - alpha) * s_k[v]
//
// (Eq. 1 of the paper with the uniform teleport 1/|V| replaced by a
// per-vector teleport distribution.) All K vectors iterate together from
// 1/|V|; each one stops on its own when its L-infinity change is <= tol and
// is frozen from then on.
//
// Layout: vertex-major [n][K] for ranks R, contributions X (gather-side
// numbering, as for Static) and the teleport matrix. A wavefront owns one
// vertex and lane k owns vector k (K is processed in slices of 64), so one
// in-edge gathers one contiguous row X[u][0..K) and every lane sums its
// vector's contributions in row order: rows of in-degree <= CH are summed
// sequentially (bit-identical to a sequential FP64 sum); longer rows are cut
// into chunks of CH edges, one wavefront per chunk, whose partial rows are
// added in chunk order by a second kernel.
#pragma once
#include "kernels.h"

namespace prhip {

// Rows of X for one in-edge range, sequential in edge order, for lane k.
__device__ __forceinline__ double ppr_row_sum(const int *__restrict__ src,
                                              const double *__restrict__ X, int K, int k,
                                              int e0, int e1) {
  double c = 0.0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    const int u0 = ld_nt(src + e), u1 = ld_nt(src + e + 1), u2 = ld_nt(src + e + 2),
              u3 = ld_nt(src + e + 3);
    const double x0 = X[(size_t)u0 * K + k], x1 = X[(size_t)u1 * K + k],
                 x2 = X[(size_t)u2 * K + k], x3 = X[(size_t)u3 * K + k];
    c = c + x0;
    c = c + x1;
    c = c + x2;
    c = c + x3;
  }
  for (; e < e1; ++e) c = c + X[(size_t)ld_nt(src + e) * K + k];
  return c;
}

// One PPR iteration. Work items: chunks of the split class (rows with
// in-degree > CH, listed in hi[n1 + i] with their chunk plan) first,
// wavefront gw of W taking items gw, gw + W, ...; then all other vertices,
// 64 consecutive rows per take from per-die row queues.
// vdone[k] marks frozen vectors (their lanes neither read nor write).
// pmax: per-workgroup, per-vector maxima [gridDim.x][K].
__global__ __launch_bounds__(kBlock) void k_ppr_rank(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ out_off, const int *__restrict__ pos, const int *__restrict__ hi,
    const int *__restrict__ counts, const int *__restrict__ hub_start,
    const int *__restrict__ chunk_hub, const uint8_t *__restrict__ deg_split, int CH, int n,
    int K, const double *__restrict__ X, const double *__restrict__ R, double *__restrict__ Rn,
    double *__restrict__ Xn, const double *__restrict__ S, const uint8_t *__restrict__ tnz,
    double *__restrict__ part, const int *__restrict__ vdone, double alpha,
    double *__restrict__ pmax,
    const int4 *__restrict__ xitems, const int *__restrict__ xoff, int *rq,
    const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  extern __shared__ double s_max[];  // [kWavesPerBlock][K]
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int k = lane; k < K; k += kWave) s_max[wid * K + k] = 0.0;
  const int n1 = counts[kInWave], nch = counts[kInChunks];
  const int W = gridDim.x * kWavesPerBlock;
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  const double oma = 1.0 - alpha;
  if (xitems) {
    // long rows cut by source range: list x ({partial, e0, e1, vertex} items)
    // is summed by the workgroups on die x, one wavefront per item
    const int B = gridDim.x;
    const int x0 = B >= kXcds ? (int)blockIdx.x % kXcds : (int)blockIdx.x;
    const int xstep = B >= kXcds ? kXcds : B;
    const int loc = B >= kXcds ? (int)blockIdx.x / kXcds : 0;
    const int nloc = B >= kXcds ? (B - 1 - x0) / kXcds + 1 : 1;
    for (int x = x0; x < kXcds; x += xstep)
      for (int j = xoff[x] + loc * kWavesPerBlock + wid; j < xoff[x + 1];
           j += nloc * kWavesPerBlock) {
        const int4 it = xitems[j];
        for (int k = lane; k < K; k += kWave)
          if (!vdone[k]) part[(size_t)it.x * K + k] = ppr_row_sum(in_src, X, K, k, it.y, it.z);
      }
  }
  // chunks of long rows: partial row sums
  for (int c = gw; !xitems && c < nch; c += W) {
    const int i = chunk_hub[c];
    const int v = hi[n1 + i];
    const int r0 = in_off[v], r1 = in_off[v + 1];
    const int e0 = r0 + (c - hub_start[i]) * CH, e1 = min(e0 + CH, r1);
    for (int k = lane; k < K; k += kWave)
      if (!vdone[k]) part[(size_t)c * K + k] = ppr_row_sum(in_src, X, K, k, e0, e1);
  }
  // other rows: full sums and the update, in runs of 64 consecutive rows.
  // Run c belongs to die c mod 8 (as when runs are dealt round robin); a
  // wavefront takes its die's next run from that die's counter in rq (8
  // atomic counters the previous kernel on the stream cleared), loads the
  // run's metadata (one row per lane) in one round trip and walks its rows
  // one by one. Row costs vary with in-degree, so wavefronts that drew short
  // rows take more runs. Every wavefront leaves once its counter passes n.
  // A grid of fewer than 8 workgroups has no workgroup on some dies: then
  // all runs come from the one counter rq[0].
  const bool per_die = gridDim.x >= kXcds;
  const int die = per_die ? (int)blockIdx.x % kXcds : 0, stride = per_die ? kXcds : 1;
  for (;;) {
    int run = 0;
    if (lane == 0) run = die + stride * atomicAdd(rq + die, 1);
    const long long first = (long long)__shfl(run, 0) * kWave;
    if (first >= n) break;
    const int r0 = (int)first;
    const long long vl = (long long)r0 + lane;
    int me0 = 0, me1 = 0, mdeg = 1, mpx = 0, mt = 0;
    bool ok = false;
    if (vl < n && !deg_split[vl]) {
      ok = true;
      me0 = in_off[vl];
      me1 = in_off[vl + 1];
      mdeg = out_off[vl + 1] - out_off[vl];
      mpx = xpos(pos, (int)vl);
      mt = tnz[vl];
    }
    unsigned long long mask = __ballot(ok);
    while (mask) {
      const int j = __ffsll(mask) - 1;
      mask &= mask - 1;
      const int v = r0 + j;
      const int e0 = __shfl(me0, j), e1 = __shfl(me1, j), t = __shfl(mt, j);
      const double d = (double)__shfl(mdeg, j);
      const size_t px = (size_t)__shfl(mpx, j) * K, pv = (size_t)v * K;
      for (int k = lane; k < K; k += kWave) {
        if (vdone[k]) continue;
        const double c = ppr_row_sum(in_src, X, K, k, e0, e1);
        const double r = oma * (t ? S[pv + k] : 0.0) + alpha * c;
        st_nt(Rn + pv + k, r);
        Xn[px + k] = r / d;
        s_max[wid * K + k] = fmax(s_max[wid * K + k], fabs(r - R[pv + k]));
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += kBlock) {
    double mx = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) mx = fmax(mx, s_max[w * K + k]);
    pmax[(size_t)blockIdx.x * K + k] = mx;
  }
}

// Long rows: add the chunk partials in chunk order and update.
// pmax: [gridDim.x][K] after the rank kernel's partials.
__global__ __launch_bounds__(kBlock) void k_ppr_finalize(
    const int *__restrict__ out_off, const int *__restrict__ pos, const int *__restrict__ hi,
    const int *__restrict__ counts, const int *__restrict__ hub_start, int K,
    const double *__restrict__ part, const double *__restrict__ R, double *__restrict__ Rn,
    double *__restrict__ Xn, const double *__restrict__ S, const uint8_t *__restrict__ tnz,
    const int *__restrict__ vdone, double alpha, double *__restrict__ pmax,
    int *__restrict__ rq, const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) rq[threadIdx.x] = 0;  // next launch's row queues
  extern __shared__ double s_max[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int k = lane; k < K; k += kWave) s_max[wid * K + k] = 0.0;
  const int n1 = counts[kInWave], n2 = counts[kInSplit];
  const int W = gridDim.x * kWavesPerBlock;
  const double oma = 1.0 - alpha;
  for (int i = blockIdx.x * kWavesPerBlock + wid; i < n2; i += W) {
    const int v = hi[n1 + i];
    const double d = (double)(out_off[v + 1] - out_off[v]);
    const size_t px = (size_t)xpos(pos, v) * K, pv = (size_t)v * K;
    for (int k = lane; k < K; k += kWave) {
      if (vdone[k]) continue;
      // the row's partial rows in chunk order, four loads in flight
      double c = 0.0;
      int q = hub_start[i];
      const int q1 = hub_start[i + 1];
      for (; q + 4 <= q1; q += 4) {
        const double p0 = part[(size_t)q * K + k], p1 = part[(size_t)(q + 1) * K + k];
        const double p2 = part[(size_t)(q + 2) * K + k], p3 = part[(size_t)(q + 3) * K + k];
        c = c + p0;
        c = c + p1;
        c = c + p2;
        c = c + p3;
      }
      for (; q < q1; ++q) c = c + part[(size_t)q * K + k];
      const double r = oma * (tnz[v] ? S[pv + k] : 0.0) + alpha * c;
      Rn[pv + k] = r;
      Xn[px + k] = r / d;
      s_max[wid * K + k] = fmax(s_max[wid * K + k], fabs(r - R[pv + k]));
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += kBlock) {
    double mx = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) mx = fmax(mx, s_max[w * K + k]);
    pmax[(size_t)blockIdx.x * K + k] = mx;
  }
}

// Per-vector maxima of the np partial rows of pmax ([np][K]) in
// kPprColBlocks row chunks, cmax[chunk][k]: a wavefront's lanes read 64
// consecutive vectors of one row at a time (coalesced), the four wavefronts
// of a workgroup split the chunk's rows.
constexpr int kPprColBlocks = 64;

__global__ __launch_bounds__(kBlock) void k_ppr_colmax(const double *__restrict__ pmax, int np,
                                                       int K, double *__restrict__ cmax,
                                                       const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  __shared__ double s_m[kWavesPerBlock][kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int r0 = (int)((long long)np * blockIdx.x / gridDim.x);
  const int r1 = (int)((long long)np * (blockIdx.x + 1) / gridDim.x);
  for (int k0 = 0; k0 < K; k0 += kWave) {
    const int k = k0 + lane;
    double m = 0.0;
    if (k < K)
      for (int r = r0 + wid; r < r1; r += kWavesPerBlock) m = fmax(m, pmax[(size_t)r * K + k]);
    s_m[wid][lane] = m;
    __syncthreads();
    if (wid == 0 && k < K) {
      double t = s_m[0][lane];
      for (int i = 1; i < kWavesPerBlock; ++i) t = fmax(t, s_m[i][lane]);
      cmax[(size_t)blockIdx.x * K + k] = t;
    }
    __syncthreads();
  }
}

// Per-vector convergence: vector k's maximum over the nb chunk maxima (one
// thread per vector); a vector meeting tol is frozen with its iteration
// count. ctrl->done once every vector is frozen.
__global__ __launch_bounds__(kBlock) void k_ppr_linf(const double *__restrict__ cmax, int nb,
                                                     int K, int *__restrict__ vdone,
                                                     int *__restrict__ viters,
                                                     double *__restrict__ vdelta, Ctrl *ctrl,
                                                     double tol, int it) {
  if (ctrl->done) return;
  __shared__ int s_open;
  if (threadIdx.x == 0) s_open = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += kBlock) {
    if (vdone[k]) continue;
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, cmax[(size_t)b * K + k]);
    vdelta[k] = m;
    viters[k] = it + 1;
    if (m <= tol) vdone[k] = 1;
    else s_open = 1;  // every writer stores 1
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ctrl->iters = it + 1;
    if (!s_open) ctrl->done = 1;
  }
}

// R = 1/n for every vector, its contributions X, per-vector state cleared.
__global__ __launch_bounds__(kBlock) void k_ppr_init(int n, int K, const int *__restrict__ out_off,
                                                     const int *__restrict__ pos, double *R,
                                                     double *__restrict__ X, int *vdone,
                                                     int *viters, int *__restrict__ rq) {
  const size_t total = (size_t)n * K;
  if (blockIdx.x == 0 && threadIdx.x < kXcds) rq[threadIdx.x] = 0;  // first launch's row queues
  const double r0 = 1.0 / (double)n;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (size_t)gridDim.x * kBlock) {
    const int v = (int)(i / K), k = (int)(i % K);
    R[i] = r0;
    X[(size_t)xpos(pos, v) * K + k] = r0 / (double)(out_off[v + 1] - out_off[v]);
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < K; k += kBlock) { vdone[k] = 0; viters[k] = 0; }
  }
}

// Flag of the split class per vertex (in-degree > CH).
__global__ __launch_bounds__(kBlock) void k_split_flags(const int *__restrict__ in_off, int n,
                                                        int CH, uint8_t *__restrict__ f) {
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
    f[v] = (in_off[v + 1] - in_off[v]) > CH;
}

// tnz[v] = 1 when any teleport entry of vertex v is non-zero (a wavefront per
// vertex, lanes over the vectors): rows of all zeros need not be read, since
// (1 - alpha) * 0 + alpha * c is exactly alpha * c.
__global__ __launch_bounds__(kBlock) void k_tele_flags(const double *__restrict__ S, int n, int K,
                                                       uint8_t *__restrict__ tnz) {
  const int lane = threadIdx.x & (kWave - 1);
  for (long long v = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; v < n;
       v += (long long)gridDim.x * kWavesPerBlock) {
    bool any = false;
    for (int k = lane; k < K; k += kWave) any = any || S[v * K + k] != 0.0;
    const bool nz = __ballot(any) != 0;
    if (lane == 0) tnz[v] = nz ? 1 : 0;
  }
}

// out[v][k] = buf[viters[k] & 1][v][k]: each vector's final iterate.
__global__ __launch_bounds__(kBlock) void k_ppr_gather_out(int n, int K,
                                                           const double *__restrict__ b0,
                                                           const double *__restrict__ b1,
                                                           const int *__restrict__ viters,
                                                           double *__restrict__ out) {
  const size_t total = (size_t)n * K;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (size_t)gridDim.x * kBlock) {
    const int k = (int)(i % K);
    out[i] = (viters[k] & 1) ? b1[i] : b0[i];
  }
}

}  // namespace prhip
