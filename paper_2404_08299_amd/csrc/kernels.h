// gfx950 kernels for Static and DF-P PageRank.
//
// Layout in HBM (all device arrays, int32 IDs, FP64 ranks):
//   in_offsets[n+1], in_sources[m]     transpose G' (rank pull)
//   out_offsets[n+1], out_targets[m]   G (out-degrees, marking)
//   R, X (Static): ranks and contributions X[u] = R[u]/|out(u)|, two
//                  buffers each, swapped every iteration
//   R, T (DF-P):   one rank vector plus a staging vector for the new ranks
//                  of the vertices updated in this iteration
//   dV, dN, cv:    uint8 flags: affected, neighbours-to-mark, updated-now
//   hi:            partition output, vertices of the wavefront class then
//                  of the workgroup class, each ascending (Alg. 4)
//
// Vertex classes by degree (Alg. 4 with two thresholds): lane-per-vertex
// (deg <= t1), wavefront-per-vertex (t1 < deg <= t2), workgroup-per-vertex
// (deg > t2). The lane class is not materialised: tiles of 256 consecutive
// vertex IDs are swept and the lanes whose vertex belongs to another class
// sit out, which keeps the lane class in ID order (coalesced offsets, rank
// and flag accesses) without a permutation array.
//
// One fused launch per rank update holds three block ranges:
//   [0, nb2)            one workgroup per workgroup-class vertex
//   [nb2, nb2+nb1)      four wavefronts, one vertex each (wavefront class)
//   [nb2+nb1, ...)      one 256-vertex ID tile, one lane per vertex
// so the long rows are dispatched first. Every block writes the maximum
// |R_new - R| of its vertices to partials[block]; a second small kernel
// reduces them (Sec. 4.1, convergence detection).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave.h"

namespace prhip {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPartTile = 1024;  // vertices per partition block
constexpr int kFinalBlock = 1024;

// Device-side control block of one call.
struct Ctrl {
  int done;       // set once an iteration met the tolerance
  int iters;      // rank updates performed (valid once done, or at max_iter)
  int err;        // nonzero: a batch vertex ID was out of range
  int pad;
  double delta;   // L-infinity change of the last performed iteration
  long long aux[4];
};

__device__ __forceinline__ int deg_class(int deg, int t1, int t2) {
  return deg <= t1 ? 0 : (deg <= t2 ? 1 : 2);
}

__device__ __forceinline__ int wave_sum_int(int x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__global__ void k_ctrl_reset(Ctrl *ctrl) {
  if (threadIdx.x == 0) {
    ctrl->done = 0;
    ctrl->iters = 0;
    ctrl->err = 0;
    ctrl->pad = 0;
    ctrl->delta = 0.0;
    for (int i = 0; i < 4; ++i) ctrl->aux[i] = 0;
  }
}

// ------------------------------------------------------------ partition
// Alg. 4 as a stable split into three classes in three passes: per-tile class
// counts, one exclusive scan over the tiles, then a scatter that ranks each
// vertex inside its tile with wavefront ballots.

__global__ __launch_bounds__(kBlock) void k_part_count(const int *__restrict__ off, int n, int t1,
                                                       int t2, int *__restrict__ tile_counts,
                                                       int ntiles) {
  const int tile = blockIdx.x;
  int c1 = 0, c2 = 0;
#pragma unroll
  for (int k = 0; k < kPartTile / kBlock; ++k) {
    const int v = tile * kPartTile + k * kBlock + threadIdx.x;
    if (v < n) {
      const int c = deg_class(off[v + 1] - off[v], t1, t2);
      c1 += (c == 1);
      c2 += (c == 2);
    }
  }
  __shared__ int s[2][kWavesPerBlock];
  c1 = wave_sum_int(c1);
  c2 = wave_sum_int(c2);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { s[0][w] = c1; s[1][w] = c2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) { a += s[0][i]; b += s[1][i]; }
    tile_counts[tile] = a;
    tile_counts[ntiles + tile] = b;
  }
}

// Exclusive scan of tile_counts[cls][0..ntiles) in place; counts[cls] = total.
__global__ __launch_bounds__(kFinalBlock) void k_part_scan(int *__restrict__ tile_counts,
                                                           int ntiles, int *__restrict__ counts) {
  __shared__ int wsum[kFinalBlock / kWave];
  __shared__ int total_s;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int per = (ntiles + kFinalBlock - 1) / kFinalBlock;
  for (int cls = 0; cls < 2; ++cls) {
    int *tc = tile_counts + (size_t)cls * ntiles;
    const int beg = min(tid * per, ntiles), end = min(beg + per, ntiles);
    int s = 0;
    for (int i = beg; i < end; ++i) s += tc[i];
    // inclusive wave scan
    int x = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int i = 0; i < kFinalBlock / kWave; ++i) { int t = wsum[i]; wsum[i] = run; run += t; }
      total_s = run;
    }
    __syncthreads();
    int run = wsum[w] + x - s;  // exclusive prefix of this thread's chunk
    for (int i = beg; i < end; ++i) { int t = tc[i]; tc[i] = run; run += t; }
    if (tid == 0) counts[cls] = total_s;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_part_scatter(const int *__restrict__ off, int n,
                                                         int t1, int t2,
                                                         const int *__restrict__ tile_counts,
                                                         int ntiles,
                                                         const int *__restrict__ counts,
                                                         int *__restrict__ hi) {
  const int tile = blockIdx.x;
  __shared__ int s1[kWavesPerBlock], s2[kWavesPerBlock];
  int base1 = tile_counts[tile];
  int base2 = counts[0] + tile_counts[ntiles + tile];
  const int w = threadIdx.x / kWave;
  for (int k = 0; k < kPartTile / kBlock; ++k) {
    const int v = tile * kPartTile + k * kBlock + threadIdx.x;
    const int c = (v < n) ? deg_class(off[v + 1] - off[v], t1, t2) : 0;
    int tot1, tot2;
    const int p1 = wave_prefix_count(c == 1, &tot1);
    const int p2 = wave_prefix_count(c == 2, &tot2);
    if ((threadIdx.x & (kWave - 1)) == 0) { s1[w] = tot1; s2[w] = tot2; }
    __syncthreads();
    int o1 = 0, o2 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
      if (i < w) { o1 += s1[i]; o2 += s2[i]; }
      a1 += s1[i];
      a2 += s2[i];
    }
    if (c == 1) hi[base1 + o1 + p1] = v;
    if (c == 2) hi[base2 + o2 + p2] = v;
    base1 += a1;
    base2 += a2;
    __syncthreads();
  }
}

// ------------------------------------------------------------ Static
// R = 1/n, X = R / |out(v)| (Alg. 1 initialisation). With `init` the start
// vector is given (Naive-dynamic, Sec. 3.4.1).
__global__ __launch_bounds__(kBlock) void k_static_init(int n, const int *__restrict__ out_off,
                                                        const double *init, double *R,
                                                        double *__restrict__ X) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n) {
    const double r = init ? init[v] : 1.0 / (double)n;
    R[v] = r;
    X[v] = r / (double)(out_off[v + 1] - out_off[v]);
  }
}

// Sequential in-row sum of X over sources, ascending (four loads in flight,
// additions in row order).
__device__ __forceinline__ double row_sum_seq(const int *__restrict__ src,
                                              const double *__restrict__ X, int e0, int e1) {
  double c = 0.0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    const int u0 = src[e], u1 = src[e + 1], u2 = src[e + 2], u3 = src[e + 3];
    const double x0 = X[u0], x1 = X[u1], x2 = X[u2], x3 = X[u3];
    c = c + x0;
    c = c + x1;
    c = c + x2;
    c = c + x3;
  }
  for (; e < e1; ++e) c = c + X[src[e]];
  return c;
}

// Eq. 1 for one vertex: R_new, its contribution, and |R_new - R|.
__device__ __forceinline__ double static_finish(int v, double c, const int *__restrict__ out_off,
                                                const double *__restrict__ R,
                                                double *__restrict__ Rn,
                                                double *__restrict__ Xn, double C0,
                                                double alpha) {
  const double r = C0 + alpha * c;
  Rn[v] = r;
  Xn[v] = r / (double)(out_off[v + 1] - out_off[v]);
  return fabs(r - R[v]);
}

__global__ __launch_bounds__(kBlock) void k_rank_static(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ out_off, const double *__restrict__ X, const double *__restrict__ R,
    double *__restrict__ Rn, double *__restrict__ Xn, const int *__restrict__ hi, int n1,
    int nb2, int nb1, int n, int t1, double C0, double alpha, double *__restrict__ partials,
    const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  __shared__ double lds[kWavesPerBlock];
  double dmax = 0.0;
  const int b = blockIdx.x;
  if (b < nb2) {  // workgroup per vertex
    const int v = hi[n1 + b];
    const int e0 = in_off[v], e1 = in_off[v + 1];
    double c = 0.0;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) c += X[in_src[e]];
    c = block_sum<kBlock>(c, lds);
    if (threadIdx.x == 0) dmax = static_finish(v, c, out_off, R, Rn, Xn, C0, alpha);
  } else if (b < nb2 + nb1) {  // wavefront per vertex
    const int lane = threadIdx.x & (kWave - 1);
    const int i = (b - nb2) * kWavesPerBlock + (int)threadIdx.x / kWave;
    if (i < n1) {
      const int v = hi[i];
      const int e0 = in_off[v], e1 = in_off[v + 1];
      double c = 0.0;
      for (int e = e0 + lane; e < e1; e += kWave) c += X[in_src[e]];
      c = wave_sum(c);
      if (lane == 0) dmax = static_finish(v, c, out_off, R, Rn, Xn, C0, alpha);
    }
  } else {  // lane per vertex over an ID tile
    const int v = (b - nb2 - nb1) * kBlock + (int)threadIdx.x;
    if (v < n) {
      const int e0 = in_off[v], e1 = in_off[v + 1];
      if (e1 - e0 <= t1) {
        const double c = row_sum_seq(in_src, X, e0, e1);
        dmax = static_finish(v, c, out_off, R, Rn, Xn, C0, alpha);
      }
    }
  }
  dmax = block_max<kBlock>(dmax, lds);
  if (threadIdx.x == 0) partials[b] = dmax;
}

// Second stage of the L-infinity norm; records the iteration's outcome.
__global__ __launch_bounds__(kFinalBlock) void k_linf_final(const double *__restrict__ partials,
                                                           int np, Ctrl *__restrict__ ctrl,
                                                           double tol, int it) {
  if (ctrl->done) return;
  __shared__ double lds[kFinalBlock / kWave];
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += kFinalBlock) m = fmax(m, partials[i]);
  m = block_max<kFinalBlock>(m, lds);
  if (threadIdx.x == 0) {
    ctrl->delta = m;
    ctrl->iters = it + 1;
    if (m <= tol) ctrl->done = 1;
  }
}

// ------------------------------------------------------------ DF / DF-P
__global__ __launch_bounds__(kBlock) void k_dfp_init(int n, const double *__restrict__ prev,
                                                     double *__restrict__ R, uint8_t *dV,
                                                     uint8_t *dN, uint8_t *cv) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n) {
    if (prev != R) R[v] = prev[v];
    dV[v] = 0;
    dN[v] = 0;
    cv[v] = 0;
  }
}

// initialAffected (Alg. 5): deletion (u, v) sets dN[u] and dV[v]; insertion
// (u, .) sets dN[u]. Out-of-range IDs are skipped and reported in ctrl->err.
__global__ __launch_bounds__(kBlock) void k_mark_initial(const int *__restrict__ del_src,
                                                         const int *__restrict__ del_dst, int nd,
                                                         const int *__restrict__ ins_src, int ni,
                                                         int n, uint8_t *dV, uint8_t *dN,
                                                         Ctrl *ctrl) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nd) {
    const int u = del_src[i], v = del_dst[i];
    if (u >= 0 && u < n && v >= 0 && v < n) {
      dN[u] = 1;
      dV[v] = 1;
    } else {
      ctrl->err = 1;
    }
  } else if (i < nd + ni) {
    const int u = ins_src[i - nd];
    if (u >= 0 && u < n) dN[u] = 1;
    else ctrl->err = 1;
  }
}

// Sequential in-row sum of R[u]/|out(u)| (DF-P gathers ranks and degrees
// directly: only affected rows are read, so no per-vertex contribution pass).
__device__ __forceinline__ double row_sum_seq_rd(const int *__restrict__ src,
                                                 const int *__restrict__ out_off,
                                                 const double *__restrict__ R, int e0, int e1) {
  double c = 0.0;
  int e = e0;
  for (; e + 2 <= e1; e += 2) {
    const int u0 = src[e], u1 = src[e + 1];
    const double r0 = R[u0], r1 = R[u1];
    const int d0 = out_off[u0 + 1] - out_off[u0], d1 = out_off[u1 + 1] - out_off[u1];
    c = c + r0 / (double)d0;
    c = c + r1 / (double)d1;
  }
  for (; e < e1; ++e) {
    const int u = src[e];
    c = c + R[u] / (double)(out_off[u + 1] - out_off[u]);
  }
  return c;
}

// updateRanks (Alg. 3) for one affected vertex v with in-row sum c.
// prune: Eq. 2 closed-loop update plus pruning (DF-P); else Eq. 1 (DF).
// Returns |r - R[v]| for the L-infinity norm.
template <bool PRUNE>
__device__ __forceinline__ double dfp_finish(int v, double c, const int *__restrict__ out_off,
                                             const double *__restrict__ R,
                                             double *__restrict__ T, uint8_t *dV, uint8_t *dN,
                                             uint8_t *cv, double C0, double alpha, double tau_f,
                                             double tau_p) {
  const double Rv = R[v];
  const double d = (double)(out_off[v + 1] - out_off[v]);
  double r;
  if (PRUNE) r = 1.0 / (1.0 - alpha / d) * (C0 + alpha * (c - Rv / d));
  else r = C0 + alpha * c;
  const double dr = fabs(r - Rv);
  const double rel = dr / fmax(r, Rv);
  if (PRUNE && rel <= tau_p) dV[v] = 0;
  if (rel > tau_f) dN[v] = 1;
  T[v] = r;
  cv[v] = 1;
  return dr;
}

template <bool PRUNE>
__global__ __launch_bounds__(kBlock) void k_rank_dfp(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ out_off, const double *__restrict__ R, double *__restrict__ T,
    uint8_t *dV, uint8_t *dN, uint8_t *cv, const int *__restrict__ hi, int n1, int nb2, int nb1,
    int n, int t1, double C0, double alpha, double tau_f, double tau_p,
    double *__restrict__ partials, const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  __shared__ double lds[kWavesPerBlock];
  double dmax = 0.0;
  const int b = blockIdx.x;
  if (b < nb2) {
    const int v = hi[n1 + b];
    if (dV[v]) {  // uniform over the block
      const int e0 = in_off[v], e1 = in_off[v + 1];
      double c = 0.0;
      for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
        const int u = in_src[e];
        c += R[u] / (double)(out_off[u + 1] - out_off[u]);
      }
      c = block_sum<kBlock>(c, lds);
      if (threadIdx.x == 0)
        dmax = dfp_finish<PRUNE>(v, c, out_off, R, T, dV, dN, cv, C0, alpha, tau_f, tau_p);
    }
  } else if (b < nb2 + nb1) {
    const int lane = threadIdx.x & (kWave - 1);
    const int i = (b - nb2) * kWavesPerBlock + (int)threadIdx.x / kWave;
    if (i < n1) {
      const int v = hi[i];
      if (dV[v]) {  // uniform over the wavefront
        const int e0 = in_off[v], e1 = in_off[v + 1];
        double c = 0.0;
        for (int e = e0 + lane; e < e1; e += kWave) {
          const int u = in_src[e];
          c += R[u] / (double)(out_off[u + 1] - out_off[u]);
        }
        c = wave_sum(c);
        if (lane == 0)
          dmax = dfp_finish<PRUNE>(v, c, out_off, R, T, dV, dN, cv, C0, alpha, tau_f, tau_p);
      }
    }
  } else {
    const int v = (b - nb2 - nb1) * kBlock + (int)threadIdx.x;
    if (v < n && dV[v]) {
      const int e0 = in_off[v], e1 = in_off[v + 1];
      if (e1 - e0 <= t1) {
        const double c = row_sum_seq_rd(in_src, out_off, R, e0, e1);
        dmax = dfp_finish<PRUNE>(v, c, out_off, R, T, dV, dN, cv, C0, alpha, tau_f, tau_p);
      }
    }
  }
  dmax = block_max<kBlock>(dmax, lds);
  if (threadIdx.x == 0) partials[b] = dmax;
}

// After the convergence check of iteration `it`: copy the new ranks of the
// vertices updated in it (the swap of Alg. 2; vertices not updated keep
// their rank), then, unless it converged, expandAffected (Alg. 5): every u
// with dN[u] marks out(u) in dV and clears dN[u] (the clearing of dN at the
// start of the next iteration in Alg. 2). Lane per vertex for out-degree
// <= t_exp over ID tiles; a wavefront per vertex of the high out-degree
// list. dV stores are all 1s (benign races, no atomics). it = -1 is the
// initial expansion.
__global__ __launch_bounds__(kBlock) void k_apply_expand(
    const int *__restrict__ out_off, const int *__restrict__ out_tgt, double *__restrict__ R,
    const double *__restrict__ T, uint8_t *dV, uint8_t *dN, uint8_t *cv,
    const int *__restrict__ hi_out, int no1, int nbo1, int n, int t_exp,
    const Ctrl *__restrict__ ctrl, int it) {
  const int done = ctrl->done;
  if (done && ctrl->iters < it + 1) return;  // converged before this iteration
  const bool expand = !done;
  const int b = blockIdx.x;
  if (b < nbo1) {
    if (!expand) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int i = b * kWavesPerBlock + (int)threadIdx.x / kWave;
    if (i < no1) {
      const int u = hi_out[i];
      if (dN[u]) {
        const int e0 = out_off[u], e1 = out_off[u + 1];
        for (int e = e0 + lane; e < e1; e += kWave) dV[out_tgt[e]] = 1;
        if (lane == 0) dN[u] = 0;
      }
    }
  } else {
    const int v = (b - nbo1) * kBlock + (int)threadIdx.x;
    if (v < n) {
      if (cv[v]) {
        R[v] = T[v];
        cv[v] = 0;
      }
      if (expand && dN[v]) {
        const int e0 = out_off[v], e1 = out_off[v + 1];
        if (e1 - e0 <= t_exp) {
          for (int e = e0; e < e1; ++e) dV[out_tgt[e]] = 1;
          dN[v] = 0;
        }
      }
    }
  }
}

// Count of affected vertices (profiling only).
__global__ __launch_bounds__(kBlock) void k_count_flags(const uint8_t *__restrict__ f, int n,
                                                        Ctrl *ctrl, int slot) {
  int c = 0;
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) c += f[v] != 0;
  c = wave_sum_int(c);
  if ((threadIdx.x & (kWave - 1)) == 0 && c) atomicAdd((unsigned long long *)&ctrl->aux[slot],
                                                     (unsigned long long)c);
}

// ------------------------------------------------------------ validation
// Pass 1 reads only offsets; pass 2 (run only when pass 1 found nothing)
// reads the rows. Error bits: 1 offsets, 2 ID range, 4 row order, 8 missing
// self-loop, 16 out view, 32 degree sums.
__global__ __launch_bounds__(kBlock) void k_validate_offsets(const int *__restrict__ off, int n,
                                                             int m, int *err, int bit) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n) {
    if (off[v + 1] < off[v]) atomicOr(err, bit);
    if (v == 0 && (off[0] != 0 || off[n] != m)) atomicOr(err, bit);
  }
}

__global__ __launch_bounds__(kBlock) void k_validate_rows(const int *__restrict__ off,
                                                          const int *__restrict__ idx, int n,
                                                          int *err, int shift) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const int e0 = off[v], e1 = off[v + 1];
  bool self = false;
  int prev = -1;
  for (int e = e0; e < e1; ++e) {
    const int u = idx[e];
    if (u < 0 || u >= n) { atomicOr(err, 2 << shift); return; }
    if (u <= prev) atomicOr(err, 4 << shift);
    prev = u;
    self |= (u == v);
  }
  if (!self) atomicOr(err, 8 << shift);
}

}  // namespace prhip
