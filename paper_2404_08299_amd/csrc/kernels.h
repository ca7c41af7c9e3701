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
//                  of the split class, each ascending (Alg. 4)
//   hub_start, chunk_hub, hub_part: the split class cut into chunks of a
//                  fixed number of edges, and one partial sum per chunk
//
// Vertex classes by degree (Alg. 4 with two thresholds):
//   lane class      deg <= t1        one lane per vertex, sequential sum
//   wavefront class t1 < deg <= t2   one 64-lane wavefront per vertex
//   split class     deg > t2         the row is cut into chunks of CH edges;
//                                    one workgroup per chunk writes a partial
//                                    sum, a second kernel adds the partials
//                                    of each vertex in chunk order
// The lane class is not materialised: 256-vertex ID tiles are swept and the
// lanes whose vertex is in another class sit out, so the lane class stays in
// ID order (coalesced offsets, rank and flag accesses) without a permutation.
//
// Launch shape: a fixed grid of B workgroups (about eight per compute unit)
// strides over the three classes, so every workgroup gets a similar mix of
// work whatever the class sizes, the class counts never travel to the host,
// and a launch made after convergence exits in a few microseconds. Each
// workgroup writes the maximum |R_new - R| of its vertices to
// partials[blockIdx]; a one-workgroup kernel reduces the B + F partials
// (Sec. 4.1, convergence detection).
//
// Candidates of the wavefront and split classes are checked lane-parallel
// (a ballot over 64 candidates, or one chunk per thread) and only the
// selected ones are processed cooperatively, so sweeping those lists in DF-P
// costs one round of loads per 64 candidates.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave.h"

namespace prhip {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPartTile = 1024;  // vertices per partition block
constexpr int kFinalBlock = 1024;
constexpr int kHubFinalizeBlocks = 512;
constexpr int kXcds = 8;  // accelerator dies; workgroup b is dispatched to die b mod 8
constexpr int kLaneStage = 1536;  // contributions staged in LDS per round of a lane-class tile

// Device-side control block of one call.
struct Ctrl {
  int done;       // set once an iteration met the tolerance
  int iters;      // rank updates performed (valid once done, or at max_iter)
  int err;        // nonzero: a batch vertex ID was out of range
  int pad;
  double delta;   // L-infinity change of the last performed iteration
  // 0 affected after the initial marking, 2-3 frontier sizes (by parity),
  // 4 affected this iteration, 5 largest affected set, 6 in-edges processed
  long long aux[8];
};

// Device array of class counts, written by the partition and plan kernels.
enum CountSlot {
  kInWave = 0,     // in-degree wavefront class size (n1)
  kInSplit = 1,    // in-degree split class size (n2)
  kOutWave = 2,    // out-degree wavefront class size
  kOutSplit = 3,   // out-degree split class size
  kInChunks = 4,   // chunks of the in-degree split class
  kOutChunks = 5,  // chunks of the out-degree split class
  kDtChanged = 6,  // a closure level of Dynamic Traversal marked a vertex
  kAffList = 8,    // per iteration parity p: slot 8 + 2p the affected list's size,
                   // 9 + 2p the rank update's tile queue over it
  kTileQueue = 12, // slots 12 .. 19: per-die work queues of the Static and batched
                   // rank updates (tiles) and of the PPR update (runs of rows)
  kMapMiss = 20,   // entries a mapping from a kept mapping did not find there
  kCands = 21,     // per iteration parity p: slot 21 + p the size of the list of
                   // frontier vertices in the out-degree wavefront class
  kMapRows = 23,   // rows a mapping from a kept mapping leaves to k_map_rows_kept
  kNumCounts = 24
};

// Streamed data (CSR arrays, a vertex's own rank, new ranks) is read and
// written with the non-temporal hint so that it does not push the gathered
// contribution vector out of the caches.
template <class T>
__device__ __forceinline__ T ld_nt(const T *p) {
  return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void st_nt(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Position of vertex v in the contribution vector (the gather-side
// numbering; identity when no relabelling is in use).
__device__ __forceinline__ int xpos(const int *__restrict__ pos, int v) {
  return pos ? ld_nt(pos + v) : v;
}

__device__ __forceinline__ int deg_class(int deg, int t1, int t2) {
  return deg <= t1 ? 0 : (deg <= t2 ? 1 : 2);
}

__device__ __forceinline__ int wave_sum_int(int x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Exclusive scan over an NT-thread workgroup; *total gets the sum.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int s, int *total) {
  __shared__ int wsum[NT / kWave];
  __shared__ int tot;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  int x = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < NT / kWave; ++i) { const int t = wsum[i]; wsum[i] = run; run += t; }
    tot = run;
  }
  __syncthreads();
  const int r = wsum[w] + x - s;
  *total = tot;
  __syncthreads();
  return r;
}
__device__ __forceinline__ int block_exclusive_scan_1024(int s, int *total) {
  return block_exclusive_scan<kFinalBlock>(s, total);
}

__global__ void k_ctrl_reset(Ctrl *ctrl) {
  if (threadIdx.x == 0) {
    ctrl->done = 0;
    ctrl->iters = 0;
    ctrl->err = 0;
    ctrl->pad = 0;
    ctrl->delta = 0.0;
    for (int i = 0; i < 8; ++i) ctrl->aux[i] = 0;
  }
}

// ------------------------------------------------------------ partition
// Alg. 4 as a stable split into three classes in three passes: per-tile class
// counts, one exclusive scan over the tiles, then a scatter that ranks each
// vertex inside its tile with wavefront ballots. Output: hi = [wavefront
// class ascending][split class ascending]; counts[slot], counts[slot + 1].

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

// Exclusive scan of each class row rows[cls][0..len) in place, one
// workgroup per class (blockIdx.x); totals[cls] = the row's sum. Rows are
// `ntiles` apart; len = ntiles, or *dlen when given (a count on the device).
__global__ __launch_bounds__(kFinalBlock) void k_scan_rows(int *__restrict__ rows, int ntiles,
                                                           int *__restrict__ totals,
                                                           const int *__restrict__ dlen) {
  int *tc = rows + (size_t)blockIdx.x * ntiles;
  if (dlen) ntiles = min(ntiles, *dlen);
  const int per = (ntiles + kFinalBlock - 1) / kFinalBlock;
  const int beg = min((int)threadIdx.x * per, ntiles), end = min(beg + per, ntiles);
  int s = 0;
  for (int i = beg; i < end; ++i) s += tc[i];
  int total;
  int run = block_exclusive_scan_1024(s, &total);
  for (int i = beg; i < end; ++i) { const int x = tc[i]; tc[i] = run; run += x; }
  if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// The same scan for long rows, in three launches over tiles of kScanTile
// entries (grid: tiles x rows): tile sums into tsum (ntmax per row), a
// k_scan_rows pass over tsum, then every tile rescanned from its offset.
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int scan_row_len(int stride, const int *dlen) {
  return dlen ? min(stride, *dlen) : stride;
}

__global__ __launch_bounds__(kBlock) void k_rows_tile_sums(const int *__restrict__ rows, int stride,
                                                           const int *__restrict__ dlen,
                                                           int *__restrict__ tsum, int ntmax) {
  const int len = scan_row_len(stride, dlen);
  const int *row = rows + (size_t)blockIdx.y * stride;
  const int base = blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = base + k * kBlock + (int)threadIdx.x;
    if (i < len) s += row[i];
  }
  int total;
  (void)block_exclusive_scan<kBlock>(s, &total);
  if (threadIdx.x == 0) tsum[(size_t)blockIdx.y * ntmax + blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_rows_tile_apply(int *__restrict__ rows, int stride,
                                                            const int *__restrict__ dlen,
                                                            const int *__restrict__ tsum,
                                                            int ntmax) {
  __shared__ int s_v[kScanTile];
  const int len = scan_row_len(stride, dlen);
  int *row = rows + (size_t)blockIdx.y * stride;
  const int base = blockIdx.x * kScanTile;
  if (base >= len) return;  // the whole workgroup: before any barrier
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kBlock + tid;
    s_v[i] = base + i < len ? row[base + i] : 0;
  }
  __syncthreads();
  int *mine = s_v + tid * kScanItems;
  int loc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) loc += mine[k];
  int total;
  int run = block_exclusive_scan<kBlock>(loc, &total) + tsum[(size_t)blockIdx.y * ntmax + blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int x = mine[k];
    mine[k] = run;
    run += x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = k * kBlock + tid;
    if (base + i < len) row[base + i] = s_v[i];
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

// Chunk plan of the split class: vertex i of the class (hi[n1 + i]) owns
// chunks [hub_start[i], hub_start[i+1]) of CH edges each (the last one
// shorter); chunk_hub[c] = i. counts[chunk_slot] = number of chunks.
__global__ __launch_bounds__(kFinalBlock) void k_hub_plan(const int *__restrict__ off,
                                                          const int *__restrict__ hi,
                                                          int *__restrict__ counts, int slot,
                                                          int chunk_slot, int CH,
                                                          int *__restrict__ hub_start,
                                                          int *__restrict__ chunk_hub) {
  const int n1 = counts[slot], n2 = counts[slot + 1];
  const int tid = threadIdx.x;
  const int per = (n2 + kFinalBlock - 1) / kFinalBlock;
  const int beg = min(tid * per, n2), end = min(beg + per, n2);
  int s = 0;
  for (int i = beg; i < end; ++i) {
    const int v = hi[n1 + i];
    s += (off[v + 1] - off[v] + CH - 1) / CH;
  }
  int total;
  int run = block_exclusive_scan_1024(s, &total);
  for (int i = beg; i < end; ++i) {
    const int v = hi[n1 + i];
    const int cnt = (off[v + 1] - off[v] + CH - 1) / CH;
    hub_start[i] = run;
    for (int c = 0; c < cnt; ++c) chunk_hub[run + c] = i;
    run += cnt;
  }
  if (tid == 0) {
    hub_start[n2] = total;
    counts[chunk_slot] = total;
  }
}

// ------------------------------------------------------------ XCD split plan
// Each accelerator die (XCD) has its own L2. The gather side is cut into
// kXcds contiguous source ranges of about equal out-edge count, and every
// split-class row into the kXcds segments of its (ascending) sources that fall
// in each range. Segment x of every row is summed by the workgroups on die x,
// so each L2 caches only its own range of the contributions. Segments are cut
// into chunks of at most CH edges; the chunk partials of a row are laid out
// row-major (range 0 first, chunks in order), so hub_finalize adds them in one
// fixed order.
//
// Range starts of graph g, rs[g][0..kXcds] (first = the graph's first
// vertex, last = its end): the first vertex whose out-edge prefix reaches
// x * m_g / kXcds, rounded to partition tiles of the graph's own numbering.
// Graph g spans vertices vb[g] .. vb[g+1] (vb = null: one graph of n vertices),
// so a graph of a batch is cut exactly as it is when run alone.
__global__ void k_xcd_ranges(const int *__restrict__ goff, const int *__restrict__ vb, int n,
                             int *__restrict__ rs) {
  const int g = blockIdx.x, x = threadIdx.x;
  if (x > kXcds) return;
  const int v0 = vb ? vb[g] : 0, v1 = vb ? vb[g + 1] : n;
  const int ng = v1 - v0;
  int v = 0;
  if (x == kXcds) {
    v = ng;
  } else if (x > 0) {
    const long long e0 = goff[v0];
    const long long target = e0 + (long long)(goff[v1] - e0) * x / kXcds;
    int lo = v0, hi = v1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((long long)goff[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    v = min(ng, (lo - v0 + kPartTile / 2) / kPartTile * kPartTile);
  }
  rs[g * (kXcds + 1) + x] = v0 + v;
}

// First position p in [lo, hi) with idx[p] >= key (idx ascending there).
__device__ __forceinline__ int lower_bound_idx(const int *__restrict__ idx, int lo, int hi,
                                               int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (idx[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// End of segment x of row [r0, r1) given the end of segment x - 1.
__device__ __forceinline__ int xseg_end(const int *__restrict__ idx, const int *__restrict__ rs,
                                        int prev, int r1, int x) {
  return x == kXcds - 1 ? r1 : lower_bound_idx(idx, prev, r1, rs[x + 1]);
}

// mat[x][i] = chunks of segment x of split row i, mat[kXcds][i] = the row's
// total, for the n2 rows of the class (nb >= n2 is the row stride of mat).
// gid (batches): graph of each row, whose ranges are rs[gid[v]].
__global__ __launch_bounds__(kBlock) void k_xsplit_count(
    const int *__restrict__ off, const int *__restrict__ idx, const int *__restrict__ hi,
    const int *__restrict__ counts, int slot, const int *__restrict__ rs_all,
    const int *__restrict__ gid, int CH, int nb, int *__restrict__ mat) {
  const int n1 = counts[slot], n2 = min(counts[slot + 1], nb);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n2; i += gridDim.x * kBlock) {
    int tot = 0;
    const int v = hi[n1 + i];
    const int *rs = rs_all + (gid ? gid[v] : 0) * (kXcds + 1);
    const int r1 = off[v + 1];
    int prev = off[v];
    for (int x = 0; x < kXcds; ++x) {
      const int e = xseg_end(idx, rs, prev, r1, x);
      const int c = (e - prev + CH - 1) / CH;
      mat[(size_t)x * nb + i] = c;
      tot += c;
      prev = e;
    }
    mat[(size_t)kXcds * nb + i] = tot;
  }
}

// After the exclusive scans of the rows of mat (totals in tot[0..kXcds]):
// work item {partial index, e0, e1, vertex} of every chunk, list x at
// xoff[x] .. xoff[x + 1]; hub_start[i] = first partial of split row i.
__global__ __launch_bounds__(kBlock) void k_xsplit_fill(
    const int *__restrict__ off, const int *__restrict__ idx, const int *__restrict__ hi,
    int *__restrict__ counts, int slot, int chunk_slot, const int *__restrict__ rs_all,
    const int *__restrict__ gid, int CH, int nb, const int *__restrict__ mat,
    const int *__restrict__ tot, int *__restrict__ xoff, int *__restrict__ hub_start,
    int4 *__restrict__ items) {
  const int n1 = counts[slot], n2 = counts[slot + 1];
  int base[kXcds];
  int run = 0;
#pragma unroll
  for (int x = 0; x < kXcds; ++x) {
    base[x] = run;
    run += tot[x];
  }
  if (blockIdx.x == 0 && threadIdx.x <= kXcds) {
    int a = 0;
    for (int x = 0; x < (int)threadIdx.x; ++x) a += tot[x];
    xoff[threadIdx.x] = a;
    if (threadIdx.x == 0) {
      hub_start[n2] = tot[kXcds];
      counts[chunk_slot] = tot[kXcds];
    }
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n2; i += gridDim.x * kBlock) {
    const int v = hi[n1 + i];
    const int *rs = rs_all + (gid ? gid[v] : 0) * (kXcds + 1);
    const int r1 = off[v + 1];
    int p = mat[(size_t)kXcds * nb + i];
    hub_start[i] = p;
    int prev = off[v];
    for (int x = 0; x < kXcds; ++x) {
      const int e = xseg_end(idx, rs, prev, r1, x);
      const int cnt = (e - prev + CH - 1) / CH;
      int4 *dst = items + base[x] + mat[(size_t)x * nb + i];
      for (int k = 0; k < cnt; ++k) {
        const int e0 = prev + k * CH;
        dst[k] = make_int4(p + k, e0, min(e0 + CH, e), v);
      }
      p += cnt;
      prev = e;
    }
  }
}

// ------------------------------------------------------------ Static init
// R = r0 (1/n in Alg. 1), X = R / |out(v)| (or R when weighted). With
// `init` the start vector is given (Naive-dynamic, Sec. 3.4.1); it may alias R.
__global__ __launch_bounds__(kBlock) void k_static_init(int n, const int *__restrict__ out_off,
                                                        const int *__restrict__ pos,
                                                        const double *init, double r0,
                                                        int weighted, double *R,
                                                        double *__restrict__ X,
                                                        int *__restrict__ tq) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (tq && v < kXcds) tq[v] = 0;  // the first rank update's tile queues
  if (v < n) {
    const double r = init ? init[v] : r0;
    R[v] = r;
    X[xpos(pos, v)] = weighted ? r : r / (double)(out_off[v + 1] - out_off[v]);
  }
}

// ------------------------------------------------------------ row sums
// Sequential in-row sum of the contributions, ascending (four gathers in
// flight, additions in row order, so the result equals a plain sequential
// sum). Unweighted: X[src[e]]; weighted: wt[e] * X[src[e]].
template <bool WEIGHTED>
__device__ __forceinline__ double row_sum_seq(const int *__restrict__ src,
                                              const double *__restrict__ wt,
                                              const double *__restrict__ X, int e0, int e1) {
  double c = 0.0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    const int u0 = ld_nt(src + e), u1 = ld_nt(src + e + 1), u2 = ld_nt(src + e + 2),
              u3 = ld_nt(src + e + 3);
    double x0 = X[u0], x1 = X[u1], x2 = X[u2], x3 = X[u3];
    if (WEIGHTED) {
      x0 = ld_nt(wt + e) * x0;
      x1 = ld_nt(wt + e + 1) * x1;
      x2 = ld_nt(wt + e + 2) * x2;
      x3 = ld_nt(wt + e + 3) * x3;
    }
    c = c + x0;
    c = c + x1;
    c = c + x2;
    c = c + x3;
  }
  for (; e < e1; ++e) {
    const double x = X[ld_nt(src + e)];
    c = c + (WEIGHTED ? ld_nt(wt + e) * x : x);
  }
  return c;
}

// Contribution of in-edge e.
template <bool WEIGHTED>
__device__ __forceinline__ double contrib(int e, const int *__restrict__ src,
                                          const double *__restrict__ wt,
                                          const double *__restrict__ X) {
  const double x = X[ld_nt(src + e)];
  return WEIGHTED ? ld_nt(wt + e) * x : x;
}

// Strided partial sum over [e0, e1) with stride S starting at e0 + t, four
// independent accumulators combined in a fixed order.
template <int S, bool WEIGHTED>
__device__ __forceinline__ double strided_sum(int e0, int e1, int t, const int *__restrict__ src,
                                              const double *__restrict__ wt,
                                              const double *__restrict__ X) {
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  int e = e0 + t;
  for (; e + 3 * S < e1; e += 4 * S) {
    c0 += contrib<WEIGHTED>(e, src, wt, X);
    c1 += contrib<WEIGHTED>(e + S, src, wt, X);
    c2 += contrib<WEIGHTED>(e + 2 * S, src, wt, X);
    c3 += contrib<WEIGHTED>(e + 3 * S, src, wt, X);
  }
  for (; e < e1; e += S) c0 += contrib<WEIGHTED>(e, src, wt, X);
  return (c0 + c1) + (c2 + c3);
}

// ------------------------------------------------------------ finishing
// Finishing of a full pull for one vertex:
//   r = C0 + alpha * c                    (Eq. 1, uniform teleport), or
//   r = tscale * tele[v] + alpha * c      (given teleport term),
// then R_new[v] = r, the gather-side value X[pos(v)] = r / |out(v)|
// (unweighted) or r (weighted), and |r - R[v]| is returned.
struct StaticOut {
  const int *out_off;
  const int *pos;
  const double *R;
  double *Rn, *Xn;
  double C0, alpha;
  const double *tele;
  double tscale;
  bool weighted;
  __device__ __forceinline__ double finish(int v, double c) const {
    const double r = tele ? tscale * ld_nt(tele + v) + alpha * c : C0 + alpha * c;
    st_nt(Rn + v, r);
    Xn[xpos(pos, v)] =
        weighted ? r : r / (double)(ld_nt(out_off + v + 1) - ld_nt(out_off + v));
    return fabs(r - ld_nt(R + v));
  }
  __device__ __forceinline__ bool active(int) const { return true; }
  __device__ __forceinline__ void inactive(int) const {}
  __device__ __forceinline__ void note(int, double) const {}
};

template <bool PRUNE>
struct DynOut {
  const int *out_off;
  const double *R;
  double *T;
  uint8_t *dV, *dN, *cv;
  double C0, alpha, tau_f, tau_p;
  // updateRanks (Alg. 3) for one affected vertex: Eq. 2 (DF-P) or Eq. 1
  // (DF), pruning (DF-P), frontier flag, staged new rank. Returns |r - R[v]|.
  __device__ __forceinline__ double finish(int v, double c) const {
    const double Rv = R[v];
    const double d = (double)(out_off[v + 1] - out_off[v]);
    double r;
    if (PRUNE) r = 1.0 / (1.0 - alpha / d) * (C0 + alpha * (c - Rv / d));
    else r = C0 + alpha * c;
    const double dr = fabs(r - Rv);
    const double rel = dr / fmax(r, Rv);
    if (PRUNE && rel <= tau_p) dV[v] = 0;
    dN[v] = rel > tau_f ? 1 : 0;
    T[v] = r;
    cv[v] = 1;
    return dr;
  }
  // only affected vertices are updated; the others clear their dN flag
  __device__ __forceinline__ bool active(int v) const { return dV[v] != 0; }
  __device__ __forceinline__ void inactive(int v) const { dN[v] = 0; }
  __device__ __forceinline__ void note(int, double) const {}
};

// ------------------------------------------------------------ rank update
// One rank update (Alg. 3 / Eq. 1 for Static, Eq. 2 for DF-P) over all three
// classes; see the file comment for the launch shape. The output policy
// `out` decides which vertices are updated (active: all for Static; those
// with dV set for DF/DF-P), what an inactive vertex does (DF/DF-P clears its
// dN flag, which is the clearing of delta_N at the start of the iteration in
// Alg. 2), computes the new value (finish) and may record its |change|
// elsewhere (note). partials may be null (no per-workgroup maximum).
// Die-split items of one die's list, dealt out in groups of G = 2^LG
// consecutive items, group g to wavefront g mod Wd: slot s of wavefront gwx
// (s = 0, 1, ...) holds item beg + (gwx + (s >> LG) * Wd) * G + (s & (G - 1)).
// Every item of the list is in exactly one slot of one wavefront. Lists long
// enough to give every wavefront kItemSpread groups of 16 keep runs of 16
// consecutive items together (LG = 4); shorter ones are spread item by item
// (LG = 0), so that no wavefront of the die sits idle while others work
// through consecutive chunks of a long row. The host picks LG from the list
// lengths and launches that instantiation (a mapping chosen inside the
// kernel, at run time, made the loop about a third slower).
constexpr int kItemSpread = 8;
template <int LG>
__device__ __forceinline__ long long item_of(int beg, int gwx, long long s, long long Wd) {
  return beg + ((gwx + (s >> LG) * Wd) << LG) + (s & ((1 << LG) - 1));
}

// LIST (DF/DF-P/DT): the lane class runs over alist[0 .. acount[0]), the
// vertices affected in this iteration (compacted after the previous marking,
// see k_compact_affected), 256 to a tile, instead of over ID tiles of every
// vertex; vertices not in the list had their dN flag cleared by the
// compaction, which is what `inactive` does in the ID-tile sweep.
// Tile queues: with more tiles than workgroups, the lane class's tiles are
// taken from atomic counters that the previous kernel on the stream cleared,
// instead of being dealt round robin, so workgroups that finished their
// long-row work early take more tiles; a workgroup leaves once its counter
// passes the last tile.
//  - tq (Static, batched; may be null): 8 counters, one per die; die x's
//    workgroups take the round robin's tiles x, x + 8, x + 16, ... from
//    counter x.
//  - LIST: a sparse list (at most n/4 affected vertices), whose tiles are
//    few and of very uneven cost, is shared out by the whole chip from one
//    counter (acount[1], cleared by the compaction); a denser list is dealt
//    round robin, like the ID tiles it then resembles.
// Measured and not kept: one counter for all Static tiles, each die taking
// the tiles of its own vertex range, and workgroups moving on to other dies'
// counters once theirs ran out were all slower; so was claiming the next
// tile before summing the current one.
template <bool WEIGHTED, int LG, class Out, bool LIST = false>
__device__ __forceinline__ void rank_update(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const double *__restrict__ wt, const double *__restrict__ X, const int *__restrict__ hi,
    const int *__restrict__ counts,
    const int *__restrict__ hub_start, const int *__restrict__ chunk_hub,
    double *__restrict__ hub_part, int CH, int n, int t1, const int4 *__restrict__ xitems,
    const int *__restrict__ xoff, const Out &out, double *__restrict__ partials,
    const int *__restrict__ alist = nullptr, int *acount = nullptr, int *tq = nullptr) {
  __shared__ double lds[kWavesPerBlock];
  __shared__ int s_v[kBlock], s_e0[kBlock], s_e1[kBlock], s_c[kBlock];
  __shared__ int s_wcnt[kWavesPerBlock];
  const int n1 = counts[kInWave], nch = counts[kInChunks];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int B = gridDim.x;
  double dmax = 0.0;

  // 1a) split class cut by source range (xitems set): list x is summed by the
  // workgroups on die x, one wavefront per chunk. With fewer than kXcds
  // workgroups, workgroup b takes lists b, b + B, ...
  if (xitems) {
    const int x0 = B >= kXcds ? (int)blockIdx.x % kXcds : (int)blockIdx.x;
    const int xstep = B >= kXcds ? kXcds : B;
    const int loc = B >= kXcds ? (int)blockIdx.x / kXcds : 0;
    const int nloc = B >= kXcds ? (B - 1 - x0) / kXcds + 1 : 1;
    // a wavefront loads 64 items {partial, e0, e1, vertex} (one per lane),
    // keeps those of active vertices and sums them one by one; the items are
    // dealt out to the Wd wavefronts of the die by item_of
    const long long Wd = (long long)nloc * kWavesPerBlock;
    const int gwx = loc * kWavesPerBlock + wid;
    for (int x = x0; x < kXcds; x += xstep) {
      const int beg = xoff[x], end = xoff[x + 1];
      for (long long k0 = 0; item_of<LG>(beg, gwx, k0, Wd) < end; k0 += kWave) {
        const long long j = item_of<LG>(beg, gwx, k0 + lane, Wd);
        int4 it = make_int4(0, 0, 0, 0);
        bool f = false;
        if (j < end) {
          it = xitems[j];
          f = out.active(it.w);
        }
        unsigned long long big = __ballot(f);
        while (big) {
          const int k = __ffsll(big) - 1;
          big &= big - 1;
          const int p = __shfl(it.x, k), e0 = __shfl(it.y, k), e1 = __shfl(it.z, k);
          double c = strided_sum<kWave, WEIGHTED>(e0, e1, lane, in_src, wt, X);
          c = wave_sum(c);
          if (lane == 0) hub_part[p] = c;
        }
      }
    }
  }
  // 1b) split class: this workgroup's chunks are blockIdx + k*B; in each
  // round thread tid checks one of them, and the selected ones are summed by
  // the whole workgroup.
  for (long long base = blockIdx.x; !xitems && base < nch; base += (long long)kBlock * B) {
    const long long cl = base + (long long)tid * B;
    const int c = cl < nch ? (int)cl : 0;
    bool f = false;
    int v = 0, e0 = 0, e1 = 0;
    if (cl < nch) {
      const int i = chunk_hub[c];
      v = hi[n1 + i];
      f = out.active(v);
      const int r0 = in_off[v], r1 = in_off[v + 1];
      e0 = r0 + (c - hub_start[i]) * CH;
      e1 = min(e0 + CH, r1);
    }
    int wtot;
    const int p = wave_prefix_count(f, &wtot);
    if (lane == 0) s_wcnt[wid] = wtot;
    __syncthreads();
    int off = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
      if (i < wid) off += s_wcnt[i];
      cnt += s_wcnt[i];
    }
    if (f) { s_c[off + p] = c; s_v[off + p] = v; s_e0[off + p] = e0; s_e1[off + p] = e1; }
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      double s = strided_sum<kBlock, WEIGHTED>(s_e0[k], s_e1[k], tid, in_src, wt, X);
      s = block_sum<kBlock>(s, lds);
      if (tid == 0) hub_part[s_c[k]] = s;
    }
    __syncthreads();
  }

  // 2) wavefront class: wavefront gw takes candidates gw + k*W, 64 at a time
  {
    const int W = B * kWavesPerBlock;
    const int gw = blockIdx.x * kWavesPerBlock + wid;
    for (long long k0 = 0; gw + k0 * W < n1; k0 += kWave) {
      const long long ii = gw + (k0 + lane) * W;
      int v = -1, r0 = 0, r1 = 0;
      bool f = false;
      if (ii < n1) {
        v = hi[ii];
        f = out.active(v);
        if (!f) out.inactive(v);
        else {
          r0 = in_off[v];
          r1 = in_off[v + 1];
        }
      }
      unsigned long long big = __ballot(f);
      while (big) {
        const int j = __ffsll(big) - 1;
        big &= big - 1;
        const int vv = __shfl(v, j), e0 = __shfl(r0, j), e1 = __shfl(r1, j);
        double c = strided_sum<kWave, WEIGHTED>(e0, e1, lane, in_src, wt, X);
        c = wave_sum(c);
        if (lane == 0) {
          const double d = out.finish(vv, c);
          dmax = fmax(dmax, d);
          out.note(vv, d);
        }
      }
    }
  }

  // 3) lane class over 256-vertex ID tiles. The tile's lane-class rows are
  // laid end to end (exclusive scan of their degrees); the workgroup gathers
  // their contributions edge-parallel into LDS, kLaneStage per round, and
  // each lane then adds its own row's values in row order, carrying its sum
  // across rounds: the sequential order of the oracle, so bit-identical.
  {
    __shared__ int s_off[kBlock + 1];
    __shared__ double s_val[kLaneStage];
    __shared__ int s_tile;
    const int nrows = LIST ? acount[0] : n;
    const int ntiles = (nrows + kBlock - 1) / kBlock;
    int *queue = (ntiles > B && B >= kXcds && (!LIST || nrows <= n / 4))
                     ? (LIST ? acount + 1 : tq)
                     : nullptr;
    const int qd = (int)blockIdx.x % kXcds;
    for (int t = blockIdx.x;; t += B) {
      if (queue) {
        if (tid == 0) {
          if (LIST) s_tile = atomicAdd(queue, 1);
          else s_tile = qd + kXcds * atomicAdd(queue + qd, 1);
        }
        __syncthreads();
        t = s_tile;
      }
      if (t >= ntiles) break;
      const int i = t * kBlock + tid;
      const int v = LIST ? (i < nrows ? alist[i] : n) : i;
      int e0 = 0, cnt = 0;
      bool act = false;
      if (v < n) {
        e0 = ld_nt(in_off + v);
        const int e1 = ld_nt(in_off + v + 1);
        if (e1 - e0 <= t1) {
          if (out.active(v)) {
            act = true;
            cnt = e1 - e0;
          } else {
            out.inactive(v);
          }
        }
      }
      int total;
      const int off = block_exclusive_scan<kBlock>(cnt, &total);
      s_off[tid] = off;
      s_e0[tid] = e0;
      if (tid == 0) s_off[kBlock] = total;
      __syncthreads();
      double c = 0.0;
      for (int c0 = 0; c0 < total; c0 += kLaneStage) {
        const int c1 = min(c0 + kLaneStage, total);
        for (int k = c0 + tid; k < c1; k += kBlock) {
          int lo = 0, hi = kBlock;  // the row r with s_off[r] <= k < s_off[r + 1]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= k) lo = mid;
            else hi = mid;
          }
          s_val[k - c0] = contrib<WEIGHTED>(s_e0[lo] + (k - s_off[lo]), in_src, wt, X);
        }
        __syncthreads();
        if (act) {
          const int k1 = min(off + cnt, c1);
          for (int k = max(off, c0); k < k1; ++k) c = c + s_val[k - c0];
        }
        __syncthreads();
      }
      if (act) {
        const double d = out.finish(v, c);
        dmax = fmax(dmax, d);
        out.note(v, d);
      }
    }
  }

  if (partials) {
    dmax = block_max<kBlock>(dmax, lds);
    if (tid == 0) partials[blockIdx.x] = dmax;
  }
}

// One full pull (Static, Naive-dynamic, the weighted forward and the
// adjoint iteration). in_src: the row indices in the gather-side numbering
// (pos); wt: per-edge weights aligned with them (WEIGHTED); X, Xn: gathered
// values in that numbering; R, Rn: the iterate in vertex order.
template <bool WEIGHTED, int LG>
__global__ __launch_bounds__(kBlock) void k_rank_static(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const double *__restrict__ wt, const int *__restrict__ out_off,
    const int *__restrict__ pos, const double *__restrict__ X, const double *__restrict__ R,
    double *__restrict__ Rn, double *__restrict__ Xn, const int *__restrict__ hi,
    const int *__restrict__ counts, const int *__restrict__ hub_start,
    const int *__restrict__ chunk_hub, double *__restrict__ hub_part, int CH, int n, int t1,
    const int4 *__restrict__ xitems, const int *__restrict__ xoff, double C0, double alpha,
    const double *__restrict__ tele, double tscale, double *__restrict__ partials,
    int *tq, const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  const StaticOut out{out_off, pos, R, Rn, Xn, C0, alpha, tele, tscale, WEIGHTED};
  rank_update<WEIGHTED, LG>(in_off, in_src, wt, X, hi, counts, hub_start, chunk_hub, hub_part, CH,
                            n, t1, xitems, xoff, out, partials, nullptr, nullptr, tq);
}

// LIST: the lane class runs over the compacted affected list
// (alist[0 .. acount[0]), tiles taken from the queue acount[1]), and the
// count of the other list (*anext) is cleared for the compaction that follows
// this iteration's marking.
template <bool PRUNE, int LG, bool LIST>
__global__ __launch_bounds__(kBlock) void k_rank_dfp(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ out_off, const double *__restrict__ X, const double *__restrict__ R,
    double *__restrict__ T, uint8_t *dV, uint8_t *dN, uint8_t *cv, const int *__restrict__ hi,
    const int *__restrict__ counts, const int *__restrict__ hub_start,
    const int *__restrict__ chunk_hub, double *__restrict__ hub_part, int CH, int n, int t1,
    const int4 *__restrict__ xitems, const int *__restrict__ xoff, double C0, double alpha,
    double tau_f, double tau_p, double *__restrict__ partials, const int *__restrict__ alist,
    int *acount, int *__restrict__ anext, const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  if (LIST && blockIdx.x == 0 && threadIdx.x == 0) *anext = 0;
  const DynOut<PRUNE> out{out_off, R, T, dV, dN, cv, C0, alpha, tau_f, tau_p};
  rank_update<false, LG, DynOut<PRUNE>, LIST>(in_off, in_src, nullptr, X, hi, counts, hub_start,
                                              chunk_hub, hub_part, CH, n, t1, xitems, xoff, out,
                                              partials, alist, acount);
}

// Split-class vertices: add the chunk partials in chunk order and finish.
template <class Out>
__device__ __forceinline__ void hub_finalize(const int *__restrict__ hi,
                                             const int *__restrict__ counts,
                                             const int *__restrict__ hub_start,
                                             const double *__restrict__ hub_part, const Out &out,
                                             double *__restrict__ partials) {
  __shared__ double lds[kWavesPerBlock];
  const int n1 = counts[kInWave], n2 = counts[kInSplit];
  double dmax = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n2; i += gridDim.x * kBlock) {
    const int v = hi[n1 + i];
    if (!out.active(v)) {
      out.inactive(v);
      continue;
    }
    double c = 0.0;
    for (int k = hub_start[i]; k < hub_start[i + 1]; ++k) c = c + hub_part[k];
    const double d = out.finish(v, c);
    dmax = fmax(dmax, d);
    out.note(v, d);
  }
  if (partials) {
    dmax = block_max<kBlock>(dmax, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = dmax;
  }
}

__global__ __launch_bounds__(kBlock) void k_hub_finalize_static(
    const int *__restrict__ hi, const int *__restrict__ counts, const int *__restrict__ hub_start,
    const double *__restrict__ hub_part, const int *__restrict__ out_off,
    const int *__restrict__ pos, const double *__restrict__ R, double *__restrict__ Rn,
    double *__restrict__ Xn, double C0, double alpha, const double *__restrict__ tele,
    double tscale, int weighted, double *__restrict__ partials, int *__restrict__ tq,
    const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  if (tq && blockIdx.x == 0 && threadIdx.x < kXcds) tq[threadIdx.x] = 0;  // next launch's queues
  const StaticOut out{out_off, pos, R, Rn, Xn, C0, alpha, tele, tscale, weighted != 0};
  hub_finalize(hi, counts, hub_start, hub_part, out, partials);
}

template <bool PRUNE>
__global__ __launch_bounds__(kBlock) void k_hub_finalize_dfp(
    const int *__restrict__ hi, const int *__restrict__ counts, const int *__restrict__ hub_start,
    const double *__restrict__ hub_part, const int *__restrict__ out_off,
    const double *__restrict__ R, double *__restrict__ T, uint8_t *dV, uint8_t *dN, uint8_t *cv,
    double C0, double alpha, double tau_f, double tau_p, double *__restrict__ partials,
    const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  const DynOut<PRUNE> out{out_off, R, T, dV, dN, cv, C0, alpha, tau_f, tau_p};
  hub_finalize(hi, counts, hub_start, hub_part, out, partials);
}

// Second stage of the L-infinity norm; records the iteration's outcome.
__global__ __launch_bounds__(kFinalBlock) void k_linf_final(const double *__restrict__ partials,
                                                           int np, Ctrl *__restrict__ ctrl,
                                                           double tol, int it) {
  if (ctrl->done) return;
  __shared__ double lds[kFinalBlock / kWave];
  double m0 = 0.0, m1 = 0.0;
  int i = threadIdx.x;
  for (; i + kFinalBlock < np; i += 2 * kFinalBlock) {
    m0 = fmax(m0, partials[i]);
    m1 = fmax(m1, partials[i + kFinalBlock]);
  }
  if (i < np) m0 = fmax(m0, partials[i]);
  double m = block_max<kFinalBlock>(fmax(m0, m1), lds);
  if (threadIdx.x == 0) {
    ctrl->delta = m;
    ctrl->iters = it + 1;
    if (m <= tol) ctrl->done = 1;
  }
}

// ------------------------------------------------------------ DF / DF-P
// R = R^{t-1} (Alg. 2), its contributions X (gather-side numbering), and
// cleared flags.
// acount (may be null): the affected-list count, cleared for the first
// compaction.
__global__ __launch_bounds__(kBlock) void k_dfp_init(int n, const int *__restrict__ out_off,
                                                     const int *__restrict__ pos,
                                                     const double *prev, double *R,
                                                     double *__restrict__ X, uint8_t *dV,
                                                     uint8_t *dN, uint8_t *cv,
                                                     int *__restrict__ acount) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (acount && v == 0) *acount = 0;
  if (v < n) {
    const double r = prev[v];
    if (prev != R) R[v] = r;
    X[xpos(pos, v)] = r / (double)(out_off[v + 1] - out_off[v]);
    dV[v] = 0;
    dN[v] = 0;
    cv[v] = 0;
  }
}

// initialAffected (Alg. 5): deletion (u, v) sets dN[u] and dV[v]; insertion
// (u, .) sets dN[u]. Out-of-range IDs are skipped and reported in ctrl->err.
// cand (may be null): the sources in the out-degree wavefront class
// (t_exp < |out| <= wmax) are listed for the initial expansion, as
// k_expand_cands lists the later frontiers (a source of several batch edges
// may appear more than once; marking twice changes nothing).
__global__ __launch_bounds__(kBlock) void k_mark_initial(const int *__restrict__ del_src,
                                                         const int *__restrict__ del_dst, int nd,
                                                         const int *__restrict__ ins_src, int ni,
                                                         int n, uint8_t *dV, uint8_t *dN,
                                                         const int *__restrict__ out_off,
                                                         int t_exp, int wmax,
                                                         int *__restrict__ cand,
                                                         int *__restrict__ ccount, Ctrl *ctrl) {
  const int i = blockIdx.x * kBlock + threadIdx.x, lane = threadIdx.x & (kWave - 1);
  int u = -1;  // the frontier vertex this thread sets
  if (i < nd) {
    const int s = del_src[i], v = del_dst[i];
    if (s >= 0 && s < n && v >= 0 && v < n) {
      u = s;
      dV[v] = 1;
    } else {
      ctrl->err = 1;
    }
  } else if (i < nd + ni) {
    const int s = ins_src[i - nd];
    if (s >= 0 && s < n) u = s;
    else ctrl->err = 1;
  }
  if (u >= 0) dN[u] = 1;
  if (!cand) return;
  bool c = false;
  if (u >= 0) {
    const int d = out_off[u + 1] - out_off[u];
    c = d > t_exp && d <= wmax;
  }
  const unsigned long long mask = __ballot(c);
  if (!mask) return;
  int base = 0;
  if (lane == 0) base = atomicAdd(ccount, __popcll(mask));
  base = __shfl(base, 0);
  const int at = base + __popcll(mask & ((1ull << lane) - 1));
  if (c && at < n) cand[at] = u;  // a longer list (count > n) is not used
}

// markNeighbors (Alg. 5) for one target: a store of 1, skipped when the flag
// is already set (a read is cheaper than a partial-line write when most
// targets are already affected). All writers store the same value.
__device__ __forceinline__ void mark(uint8_t *dV, int v) {
  if (!dV[v]) dV[v] = 1;
}

// The affected set after a marking, compacted: every v with dV[v] is
// appended to list. A vertex that is not affected has its dN flag cleared:
// the clearing of delta_N at the start of the next iteration (Alg. 2), which
// the rank update then skips for the vertices it does not visit. Workgroup b
// owns a contiguous run of rounds of kCompactRun vertices (16 per thread,
// read as one 16-byte load of each flag array; the flag arrays are 256-byte
// aligned and padded to a multiple of 256). A first pass counts its affected
// vertices and clears dN, one atomic add reserves its slots in the list, and
// a second pass (the flags again, now from L2) writes them in ascending
// order. The list is ascending inside each workgroup's run and the runs land
// in atomic order, which varies run to run; the results do not, since each
// vertex is summed by its own lane in row order whatever tile it lands in.
// One atomic per workgroup, not per round: many adds on one address queue up.
// It also clears `queue`, the 8 per-die counters the next rank update takes
// its list tiles from.
constexpr int kCompactPer = 16;
constexpr int kCompactRun = kBlock * kCompactPer;
__device__ __forceinline__ uint32_t affected_bits(const uint8_t *__restrict__ dV, int v0, int n) {
  if (v0 >= n) return 0;
  const uint4 f = *(const uint4 *)(dV + v0);
  const uint32_t w[4] = {f.x, f.y, f.z, f.w};
  uint32_t keep = 0;  // bit j: vertex v0 + j is affected
#pragma unroll
  for (int j = 0; j < kCompactPer; ++j)
    if (v0 + j < n && ((w[j >> 2] >> (8 * (j & 3))) & 0xFF) != 0) keep |= 1u << j;
  return keep;
}
__global__ __launch_bounds__(kBlock) void k_compact_affected(const uint8_t *__restrict__ dV,
                                                             uint8_t *__restrict__ dN, int n,
                                                             int *__restrict__ list,
                                                             int *__restrict__ count,
                                                             int *__restrict__ queue,
                                                             const Ctrl *__restrict__ ctrl) {
  if (ctrl->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;  // tile queue of the next rank update
  __shared__ int s_base;
  const int tid = threadIdx.x;
  const long long rounds = ((long long)n + kCompactRun - 1) / kCompactRun;
  const long long per = (rounds + gridDim.x - 1) / gridDim.x;
  const long long q0 = (long long)blockIdx.x * per, q1 = min(rounds, q0 + per);
  // pass 1: count, and clear dN of the vertices that are not affected
  int mine = 0;
  for (long long q = q0; q < q1; ++q) {
    const int v0 = (int)(q * kCompactRun) + tid * kCompactPer;
    const uint32_t keep = affected_bits(dV, v0, n);
    mine += __popc(keep);
    if (v0 < n) {
      const uint4 fn = *(const uint4 *)(dN + v0);
      uint32_t wn[4] = {fn.x, fn.y, fn.z, fn.w};
      bool clear = false;
#pragma unroll
      for (int j = 0; j < kCompactPer; ++j) {
        const uint32_t sh = 8 * (j & 3);
        if (v0 + j < n && !((keep >> j) & 1) && ((wn[j >> 2] >> sh) & 0xFF) != 0) {
          wn[j >> 2] &= ~(0xFFu << sh);
          clear = true;
        }
      }
      if (clear) *(uint4 *)(dN + v0) = make_uint4(wn[0], wn[1], wn[2], wn[3]);
    }
  }
  int total;
  (void)block_exclusive_scan<kBlock>(mine, &total);
  if (tid == 0) s_base = total ? atomicAdd(count, total) : 0;
  __syncthreads();
  int base = s_base;
  // pass 2: write the affected vertices in order
  for (long long q = q0; q < q1 && total; ++q) {
    const int v0 = (int)(q * kCompactRun) + tid * kCompactPer;
    uint32_t keep = affected_bits(dV, v0, n);
    int rt;
    int at = base + block_exclusive_scan<kBlock>(__popc(keep), &rt);
    while (keep) {
      const int j = __ffs(keep) - 1;
      keep &= keep - 1;
      list[at++] = v0 + j;
    }
    base += rt;
  }
}

// The frontier's vertices of the out-degree wavefront class (t_exp < |out| <=
// wmax), listed for expandAffected of iteration `it` from that iteration's
// affected list, which holds every vertex with dN set. Workgroup b owns a
// contiguous run of rounds of kCandRun list entries (16 per thread, strided
// by the workgroup) and reserves each round's slots with one atomic add.
// Skipped when the marking will not push (converged, or the frontier is
// pulled). The other parity's count is cleared for the next iteration.
constexpr int kCandPer = 16;
constexpr int kCandRun = kBlock * kCandPer;
__global__ __launch_bounds__(kBlock) void k_expand_cands(
    const int *__restrict__ alist, const int *__restrict__ acount, const uint8_t *__restrict__ dN,
    const int *__restrict__ out_off, int t_exp, int wmax, long long pull_thresh,
    int *__restrict__ cand, int *__restrict__ ccount, int *__restrict__ cnext,
    const Ctrl *__restrict__ ctrl, int it) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *cnext = 0;
  if (ctrl->done || (pull_thresh >= 0 && ctrl->aux[2 + (it & 1)] > pull_thresh)) return;
  __shared__ int s_base;
  const int L = *acount, tid = threadIdx.x;
  const long long rounds = ((long long)L + kCandRun - 1) / kCandRun;
  const long long per = (rounds + gridDim.x - 1) / gridDim.x;
  const long long q0 = (long long)blockIdx.x * per, q1 = min(rounds, q0 + per);
  for (long long q = q0; q < q1; ++q) {
    int vv[kCandPer];
    uint32_t keep = 0;
#pragma unroll
    for (int k = 0; k < kCandPer; ++k) {
      const long long i = q * kCandRun + k * kBlock + tid;
      vv[k] = 0;
      if (i < L) {
        const int v = alist[i];
        vv[k] = v;
        if (dN[v]) {
          const int d = out_off[v + 1] - out_off[v];
          if (d > t_exp && d <= wmax) keep |= 1u << k;
        }
      }
    }
    int total;
    int at = block_exclusive_scan<kBlock>(__popc(keep), &total);
    if (tid == 0) s_base = total ? atomicAdd(ccount, total) : 0;
    __syncthreads();
    at += s_base;
#pragma unroll
    for (int k = 0; k < kCandPer; ++k)
      if ((keep >> k) & 1u) cand[at++] = vv[k];
    __syncthreads();  // s_base is rewritten by the next round
  }
}

// After the convergence check of iteration `it`: copy the new ranks of the
// vertices updated in it, with their contributions (the swap of Alg. 2;
// vertices not updated keep their rank), then, unless it converged, expandAffected (Alg. 5): every u
// with dN[u] marks out(u) in dV. Out-degree classes as for the rank update:
// lane per vertex over ID tiles, a wavefront per vertex, or one workgroup per
// chunk of out-edges. dV stores are all 1s (benign races, no atomics).
// it = -1 is the initial expansion. cand (with ccount): the wavefront-class
// vertices of the frontier (k_expand_cands, k_mark_initial), else, or when
// the count exceeds n, every wavefront-class vertex is checked.
__global__ __launch_bounds__(kBlock) void k_apply_expand(
    const int *__restrict__ out_off, const int *__restrict__ out_tgt, const int *__restrict__ pos,
    double *__restrict__ R, double *__restrict__ X, const double *__restrict__ T, uint8_t *dV,
    const uint8_t *dN, uint8_t *cv,
    const int *__restrict__ hi_out, const int *__restrict__ counts,
    const int *__restrict__ hub_start, const int *__restrict__ chunk_hub, int CH, int n,
    int t_exp, const int *__restrict__ rt, long long pull_thresh, int do_mark,
    const int *__restrict__ alist, const int *__restrict__ acount,
    const int *__restrict__ cand, const int *__restrict__ ccount,
    const Ctrl *__restrict__ ctrl, int it) {
  const int done = ctrl->done;
  if (done && ctrl->iters < it + 1) return;  // converged before this iteration
  // pull_thresh >= 0: k_pull_mark did the marking when the frontier was
  // larger; do_mark = 0: the apply step only (the affected set is fixed)
  const bool expand =
      do_mark && !done && (pull_thresh < 0 || ctrl->aux[2 + (it & 1)] <= pull_thresh);
  __shared__ int s_e0[kBlock], s_e1[kBlock];
  __shared__ int s_wcnt[kWavesPerBlock];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int B = gridDim.x;
  if (expand && rt) {
    // Wavefront and split classes cut by target range: the workgroups on die
    // x mark only targets in [rt[x], rt[x+1]), found by binary search in the
    // ascending out-row, so the flags they read and write stay in that die's
    // L2. Candidates: the wavefront-class rows, then the split-class chunks.
    // wavefront-class candidates [0, nw), then split-class chunks
    const int n1 = counts[kOutWave], nch = counts[kOutChunks];
    const bool listed = cand && *ccount <= n;
    const int nw = listed ? *ccount : n1;
    const long long ncand = (long long)nw + nch;
    const int x0 = B >= kXcds ? (int)blockIdx.x % kXcds : (int)blockIdx.x;
    const int xstep = B >= kXcds ? kXcds : B;
    const int loc = B >= kXcds ? (int)blockIdx.x / kXcds : 0;
    const int nloc = B >= kXcds ? (B - 1 - x0) / kXcds + 1 : 1;
    const long long Wx = (long long)nloc * kWavesPerBlock;
    const int gwx = loc * kWavesPerBlock + wid;
    for (int x = x0; x < kXcds; x += xstep) {
      const int lo_t = rt[x], hi_t = rt[x + 1];
      for (long long k0 = 0; gwx + k0 * Wx < ncand; k0 += kWave) {
        const long long ii = gwx + (k0 + lane) * Wx;
        bool f = false;
        int a = 0, b = 0;
        if (ii < nw) {
          const int u = listed ? cand[ii] : hi_out[ii];
          f = listed || dN[u] != 0;
          a = out_off[u];
          b = out_off[u + 1];
        } else if (ii < ncand) {
          const int c = (int)(ii - nw);
          const int i = chunk_hub[c];
          const int u = hi_out[n1 + i];
          f = dN[u] != 0;
          a = out_off[u] + (c - hub_start[i]) * CH;
          b = min(a + CH, out_off[u + 1]);
        }
        // each lane finds its candidate's targets in the range
        int s0 = 0, s1 = 0;
        if (f) {
          s0 = lower_bound_idx(out_tgt, a, b, lo_t);
          s1 = lower_bound_idx(out_tgt, s0, b, hi_t);
        }
        unsigned long long mask = __ballot(s1 > s0);
        while (mask) {
          const int j = __ffsll(mask) - 1;
          mask &= mask - 1;
          const int ss0 = __shfl(s0, j), ss1 = __shfl(s1, j);
          for (int e = ss0 + lane; e < ss1; e += kWave) mark(dV, ld_nt(out_tgt + e));
        }
      }
    }
  } else if (expand) {
    const int n1 = counts[kOutWave], nch = counts[kOutChunks];
    // split class: chunks blockIdx + k*B, one per thread and round
    for (long long base = blockIdx.x; base < nch; base += (long long)kBlock * B) {
    const long long cl = base + (long long)tid * B;
    const int c = cl < nch ? (int)cl : 0;
    bool f = false;
    int e0 = 0, e1 = 0;
    if (cl < nch) {
      const int i = chunk_hub[c];
      const int u = hi_out[n1 + i];
      f = dN[u] != 0;
      e0 = out_off[u] + (c - hub_start[i]) * CH;
      e1 = min(e0 + CH, out_off[u + 1]);
    }
    int wtot;
    const int p = wave_prefix_count(f, &wtot);
    if (lane == 0) s_wcnt[wid] = wtot;
    __syncthreads();
    int off = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
      if (i < wid) off += s_wcnt[i];
      cnt += s_wcnt[i];
    }
    if (f) { s_e0[off + p] = e0; s_e1[off + p] = e1; }
    __syncthreads();
    for (int k = 0; k < cnt; ++k)
      for (int e = s_e0[k] + tid; e < s_e1[k]; e += kBlock) mark(dV, ld_nt(out_tgt + e));
    __syncthreads();
    }
    // wavefront class
    const bool listed = cand && *ccount <= n;
    const int nw = listed ? *ccount : n1;
    const int W = B * kWavesPerBlock;
    const int gw = blockIdx.x * kWavesPerBlock + wid;
    for (long long k0 = 0; gw + k0 * W < nw; k0 += kWave) {
      const long long ii = gw + (k0 + lane) * W;
      int u = -1;
      bool g = false;
      if (ii < nw) {
        u = listed ? cand[ii] : hi_out[ii];
        g = listed || dN[u] != 0;
      }
      unsigned long long mask = __ballot(g);
      while (mask) {
        const int j = __ffsll(mask) - 1;
        mask &= mask - 1;
        const int uu = __shfl(u, j);
        const int a = out_off[uu], b = out_off[uu + 1];
        for (int e = a + lane; e < b; e += kWave) mark(dV, ld_nt(out_tgt + e));
      }
    }
  }
  // lane class and the apply step over ID tiles, or over the iteration's
  // affected list (alist): every vertex updated in this iteration (cv set)
  // and every vertex with dN set is in it
  const int nrows = alist ? *acount : n;
  const int ntiles = (nrows + kBlock - 1) / kBlock;
  for (int t = blockIdx.x; t < ntiles; t += B) {
    const int i = t * kBlock + tid;
    const int v = alist ? (i < nrows ? alist[i] : n) : i;
    if (v < n) {
      if (cv[v]) {
        const double r = T[v];
        R[v] = r;
        X[xpos(pos, v)] = r / (double)(out_off[v + 1] - out_off[v]);
        cv[v] = 0;
      }
      if (expand && dN[v]) {
        const int e0 = out_off[v], e1 = out_off[v + 1];
        if (e1 - e0 <= t_exp)
          for (int e = e0; e < e1; ++e) mark(dV, ld_nt(out_tgt + e));
      }
    }
  }
}

// ------------------------------------------------------------ pull expansion
// The frontier of iteration `it` as a bitmap, bit v of fb[v / 32] = dN[v]
// (dN bytes are 0 or 1), over fb's words [w0, n/32) with stride ws.
__device__ __forceinline__ int frontier_words(const uint8_t *__restrict__ dN, int n,
                                              uint32_t *__restrict__ fb, long long w0,
                                              long long ws) {
  const int nw = (n + 31) / 32;
  int cnt = 0;
  for (long long w = w0; w < nw; w += ws) {
    const int v0 = (int)w * 32;
    uint32_t word = 0;
    if (v0 + 32 <= n && (reinterpret_cast<uintptr_t>(dN) & 3) == 0) {
      const uint32_t *q = reinterpret_cast<const uint32_t *>(dN + v0);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t b = q[k] & 0x01010101u;  // byte i's low bit at bit 8i
        word |= ((b | (b >> 7) | (b >> 14) | (b >> 21)) & 0xFu) << (4 * k);
      }
    } else {
      for (int b = 0; v0 + b < n; ++b)
        if (dN[v0 + b]) word |= 1u << b;
    }
    fb[w] = word;
    cnt += __popc(word);
  }
  return cnt;
}

__device__ __forceinline__ void frontier_add(int cnt, Ctrl *ctrl, int it) {
  cnt = wave_sum_int(cnt);
  if ((threadIdx.x & (kWave - 1)) == 0 && cnt)
    atomicAdd((unsigned long long *)&ctrl->aux[2 + (it & 1)], (unsigned long long)cnt);
}

// A list of at most n / kFrontierListShare vertices is counted over rather
// than the n flags swept.
constexpr int kFrontierListShare = 8;

// The frontier's bitmap and its size added to ctrl->aux[2 + (it & 1)]; the
// other counter is cleared for the next iteration. With the iteration's
// affected list (alist, acount: it holds every vertex with dN set) and gate
// >= 0: a short list is counted here and the bitmap is built only when the
// frontier is larger than gate (when the marking pulls); a long list leaves
// everything to the sweep, as without a list.
__global__ __launch_bounds__(kBlock) void k_frontier(const uint8_t *__restrict__ dN, int n,
                                                     uint32_t *__restrict__ fb, Ctrl *ctrl,
                                                     int it, long long gate,
                                                     const int *__restrict__ acount) {
  if (ctrl->done) return;
  const bool listed = acount && (long long)*acount * kFrontierListShare <= n;
  if (listed && ctrl->aux[2 + (it & 1)] <= gate) return;
  if (!listed && blockIdx.x == 0 && threadIdx.x == 0) ctrl->aux[2 + ((it + 1) & 1)] = 0;
  const int cnt = frontier_words(dN, n, fb, (long long)blockIdx.x * kBlock + threadIdx.x,
                                 (long long)gridDim.x * kBlock);
  if (!listed) frontier_add(cnt, ctrl, it);
}

// The size of the frontier of iteration `it` counted over that iteration's
// affected list, when the list is short (see k_frontier), into
// ctrl->aux[2 + (it & 1)]; the other counter is cleared for the next
// iteration.
__global__ __launch_bounds__(kBlock) void k_frontier_count(const int *__restrict__ alist,
                                                           const int *__restrict__ acount,
                                                           const uint8_t *__restrict__ dN, int n,
                                                           Ctrl *ctrl, int it) {
  if (ctrl->done) return;
  const int L = *acount;
  if ((long long)L * kFrontierListShare > n) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->aux[2 + ((it + 1) & 1)] = 0;
  int cnt = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < L; i += gridDim.x * kBlock)
    cnt += dN[alist[i]] != 0;
  frontier_add(cnt, ctrl, it);
}

__device__ __forceinline__ bool in_frontier(const uint32_t *__restrict__ fb, int u) {
  return (fb[u >> 5] >> (u & 31)) & 1u;
}

// Whether wavefront-uniform edge range [a, b) of in_src holds a frontier
// vertex (stops at the first 64-edge step that finds one).
__device__ __forceinline__ bool wave_any_frontier(const int *__restrict__ in_src,
                                                  const uint32_t *__restrict__ fb, int a, int b,
                                                  int lane) {
  for (int e0 = a; e0 < b; e0 += kWave) {
    const int e = e0 + lane;
    if (__ballot(e < b && in_frontier(fb, in_src[e]))) return true;
  }
  return false;
}

// expandAffected (Alg. 5) in the pull direction, used when the frontier of
// iteration `it` has more than `thresh` vertices: an unaffected vertex v
// becomes affected when one of its in-neighbours is in the frontier, which
// is the set that marking out(u) for every frontier vertex u produces.
// Rows above the lane class are checked one wavefront per row (wavefront
// class) or per chunk (top class: die-split items {p, e0, e1, v} when
// xitems is set, else the split-class chunks), lane-class rows one lane each.
__global__ __launch_bounds__(kBlock) void k_pull_mark(
    const int *__restrict__ in_off, const int *__restrict__ in_src,
    const int *__restrict__ hi_in, const int *__restrict__ counts,
    const int *__restrict__ hub_start, const int *__restrict__ chunk_hub, int CH,
    const int4 *__restrict__ xitems, const int *__restrict__ xoff,
    const uint32_t *__restrict__ fb, uint8_t *dV, int n, int t1, long long thresh,
    uint8_t *newly, int *changed, const Ctrl *__restrict__ ctrl, int it) {
  if (ctrl->done || ctrl->aux[2 + (it & 1)] <= thresh) return;
  // newly (optional): flags of the vertices marked here, and *changed = 1
  auto set = [&](int v) {
    dV[v] = 1;
    if (newly) {
      newly[v] = 1;
      *changed = 1;
    }
  };
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int B = gridDim.x;
  const long long W = (long long)B * kWavesPerBlock;
  const int gw = blockIdx.x * kWavesPerBlock + wid;
  const int n1 = counts[kInWave];
  // top class, chunk by chunk
  const long long nchunks = xitems ? (long long)xoff[kXcds] : (long long)counts[kInChunks];
  for (long long k0 = 0; gw + k0 * W < nchunks; k0 += kWave) {
    const long long c = gw + (k0 + lane) * W;
    int v = 0, a = 0, b = 0;
    bool need = false;
    if (c < nchunks) {
      if (xitems) {
        const int4 itm = xitems[c];
        v = itm.w;
        a = itm.y;
        b = itm.z;
      } else {
        const int i = chunk_hub[c];
        v = hi_in[n1 + i];
        a = in_off[v] + ((int)c - hub_start[i]) * CH;
        b = min(a + CH, in_off[v + 1]);
      }
      need = !dV[v];
    }
    unsigned long long mask = __ballot(need);
    while (mask) {
      const int j = __ffsll(mask) - 1;
      mask &= mask - 1;
      const int vv = __shfl(v, j), aa = __shfl(a, j), bb = __shfl(b, j);
      if (wave_any_frontier(in_src, fb, aa, bb, lane) && lane == 0) set(vv);
    }
  }
  // wavefront class, one wavefront per row
  for (long long k0 = 0; gw + k0 * W < n1; k0 += kWave) {
    const long long ii = gw + (k0 + lane) * W;
    int v = 0;
    bool need = false;
    if (ii < n1) {
      v = hi_in[ii];
      need = !dV[v];
    }
    unsigned long long mask = __ballot(need);
    while (mask) {
      const int j = __ffsll(mask) - 1;
      mask &= mask - 1;
      const int vv = __shfl(v, j);
      if (wave_any_frontier(in_src, fb, in_off[vv], in_off[vv + 1], lane) && lane == 0)
        set(vv);
    }
  }
  // lane class over ID tiles
  const int ntiles = (n + kBlock - 1) / kBlock;
  for (int t = blockIdx.x; t < ntiles; t += B) {
    const int v = t * kBlock + tid;
    if (v < n && !dV[v]) {
      const int e0 = in_off[v], e1 = in_off[v + 1];
      if (e1 - e0 <= t1) {
        for (int e = e0; e < e1; ++e)
          if (in_frontier(fb, in_src[e])) {
            set(v);
            break;
          }
      }
    }
  }
}

// ------------------------------------------------------------ adjoint
// Row of edge e in a CSR (offsets[row] <= e < offsets[row + 1]).
__device__ __forceinline__ int row_of_edge(const int *__restrict__ off, int n, int e) {
  int lo = 0, hi = n;  // invariant: off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Weights in out-CSR order: for in-edge e = (u -> v), P_out at the position
// of v in u's (ascending) out-row gets in_w[e]. Entries of an out-row whose
// in-edge is missing (views inconsistent) keep 0.
__global__ __launch_bounds__(kBlock) void k_transpose_weights(
    const int *__restrict__ in_off, const int *__restrict__ in_src, const double *__restrict__ in_w,
    const int *__restrict__ out_off, const int *__restrict__ out_tgt, int n, int m,
    double *__restrict__ out_w) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < m; e += gridDim.x * kBlock) {
    const int v = row_of_edge(in_off, n, e);
    const int u = in_src[e];
    int lo = out_off[u], hi = out_off[u + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (out_tgt[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    if (lo < out_off[u + 1] && out_tgt[lo] == v) out_w[lo] = in_w[e];
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ a, size_t len, double x) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < len;
       i += (size_t)gridDim.x * kBlock)
    a[i] = x;
}

// Gradients from the adjoint solution lambda: d/dP_uv = alpha * r_u * lambda_v
// for every in-edge (in-CSR order), d/ds_v = (1 - alpha) * lambda_v.
__global__ __launch_bounds__(kBlock) void k_adjoint_grads(
    const int *__restrict__ in_off, const int *__restrict__ in_src, int n, int m,
    const double *__restrict__ r, const double *__restrict__ lam, double alpha,
    double *__restrict__ grad_w, double *__restrict__ grad_s) {
  const int stride = gridDim.x * kBlock;
  if (grad_w)
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) {
      const int v = row_of_edge(in_off, n, e);
      grad_w[e] = alpha * r[in_src[e]] * lam[v];
    }
  if (grad_s)
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
      grad_s[v] = (1.0 - alpha) * lam[v];
}

// ------------------------------------------------------------ locality
// Gather-side renumbering by degree-based grouping: vertices are grouped by
// floor(log2(out-degree)), highest group first, and keep their ID order
// inside a group. The contributions of high out-degree vertices (the sources
// most in-edges read) then share cache lines. It is a stable partition into
// kGroups classes, the k-class form of Alg. 4: per-tile class counts, one
// exclusive scan over the class-major counts, a ranking scatter.
constexpr int kGroups = 32;

__device__ __forceinline__ int group_key(int outdeg) {  // 0 = highest degrees
  // kGroups - 1 - floor(log2(outdeg)) = clz(outdeg); clamped for safety
  return min(__clz(outdeg), kGroups - 1);
}

__global__ __launch_bounds__(kBlock) void k_group_count(const int *__restrict__ out_off, int n,
                                                        int *__restrict__ counts, int ntiles) {
  __shared__ int c[kGroups];
  if (threadIdx.x < kGroups) c[threadIdx.x] = 0;
  __syncthreads();
  for (int k = 0; k < kPartTile / kBlock; ++k) {
    const int v = blockIdx.x * kPartTile + k * kBlock + threadIdx.x;
    if (v < n) atomicAdd(&c[group_key(out_off[v + 1] - out_off[v])], 1);
  }
  __syncthreads();
  if (threadIdx.x < kGroups) counts[(size_t)threadIdx.x * ntiles + blockIdx.x] = c[threadIdx.x];
}

// base[g][tile]: exclusive prefix of group g's counts over the tiles;
// totals[g]: group sizes (the group's first position is their prefix sum).
// With source ranges rs (tile-aligned, see k_xcd_ranges) the grouping is done
// inside each range, so range x keeps the positions rs[x] .. rs[x+1]: the
// contributions a die gathers stay contiguous. rs = null: one range.
__global__ __launch_bounds__(kBlock) void k_group_scatter(const int *__restrict__ out_off, int n,
                                                          const int *__restrict__ base,
                                                          const int *__restrict__ totals,
                                                          int ntiles, const int *__restrict__ rs,
                                                          int *__restrict__ newid) {
  __shared__ int s_base[kGroups];
  __shared__ int s_cnt[kWavesPerBlock][kGroups];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x < kGroups) {
    // tiles [t0, t1) form this tile's range; prefix(g, t) = members of group
    // g in tiles before t (totals[g] at t = ntiles)
    int r0 = 0, t0 = 0, t1 = ntiles;
    if (rs) {
      int x = 0;
      while (x < kXcds - 1 && rs[x + 1] <= (int)blockIdx.x * kPartTile) ++x;
      r0 = rs[x];
      t0 = rs[x] / kPartTile;
      t1 = (rs[x + 1] + kPartTile - 1) / kPartTile;
    }
    auto prefix = [&](int g, int t) {
      return t < ntiles ? base[(size_t)g * ntiles + t] : totals[g];
    };
    int gb = r0;
    for (int g = 0; g < (int)threadIdx.x; ++g) gb += prefix(g, t1) - prefix(g, t0);
    s_base[threadIdx.x] =
        gb + base[(size_t)threadIdx.x * ntiles + blockIdx.x] - prefix(threadIdx.x, t0);
  }
  for (int k = 0; k < kPartTile / kBlock; ++k) {
    const int v = blockIdx.x * kPartTile + k * kBlock + threadIdx.x;
    const int key = v < n ? group_key(out_off[v + 1] - out_off[v]) : -1;
    int rank = 0;
    for (int g = 0; g < kGroups; ++g) {
      int tot;
      const int p = wave_prefix_count(key == g, &tot);
      if (key == g) rank = p;
      if (lane == 0) s_cnt[w][g] = tot;
    }
    __syncthreads();
    if (v < n) {
      int off = s_base[key] + rank;
      for (int i = 0; i < w; ++i) off += s_cnt[i][key];
      newid[v] = off;
    }
    __syncthreads();
    if (threadIdx.x < kGroups) {
      int a = 0;
      for (int i = 0; i < kWavesPerBlock; ++i) a += s_cnt[i][threadIdx.x];
      s_base[threadIdx.x] += a;
    }
    __syncthreads();
  }
}

// dst[e] = newid[src[e]]: the in-CSR sources in the gather-side numbering
// (rows keep their order, so every row sum runs in the original order).
__global__ __launch_bounds__(kBlock) void k_map_sources(const int *__restrict__ src, int m,
                                                        const int *__restrict__ newid,
                                                        int *__restrict__ dst) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < m; e += gridDim.x * kBlock)
    st_nt(dst + e, newid[ld_nt(src + e)]);
}

// A mapping kept from an earlier in-CSR of the same vertex set under the
// same numbering: its row offsets, its sources and their numbers, with
// old_map[p] == newid[old_raw[p]] at every p < old_m. A source u read at
// entry e may take old_map[p] for any p with old_raw[p] == u, wherever p
// lies; the guess p = e + old_off[v] - off[v] (v = e's row) finds it in every
// row that an update left alone, so the random newid reads are left to the
// rows it changed. Maps written with the copies (raw_out, off_out) are the
// next call's kept mapping, and the invariant carries over.
//   MODE 0: dst[e] = newid[src[e]]
//   MODE 1: the same, also writing raw_out and off_out
//   MODE 2: as MODE 1, probing the kept mapping first
struct MapCache {
  const int *old_off, *old_raw, *old_map;
  int old_m;
  int *raw_out, *off_out;
  int *miss;  // MODE 2: entries not found by the guess (one atomic per wavefront)
};

// Entries [a, b) of a run whose kept positions are e + shift (MODE 2), e.g.
// the rows of a wavefront that all kept their offsets' shift: every lane keeps
// kMapUnroll strides of the wavefront in flight (their loads first, then the
// lookups of the entries not found, then the stores), the last pass with the
// strides past b switched off.
constexpr int kMapUnroll = 8;

template <int MODE>
__device__ __forceinline__ void map_run(const int *__restrict__ src,
                                        const int *__restrict__ newid, int *__restrict__ dst,
                                        int a, int b, int shift, const MapCache &c, int &miss) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int e = a + lane; e - lane < b; e += kMapUnroll * kWave) {
    int u[kMapUnroll], o[kMapUnroll], mm[kMapUnroll];
#pragma unroll
    for (int k = 0; k < kMapUnroll; ++k) {
      const int ek = e + k * kWave;
      u[k] = 0;
      o[k] = 0;
      mm[k] = 0;
      if (ek < b) {
        u[k] = ld_nt(src + ek);
        if (MODE == 2) {
          const int p = ek + shift;
          const bool in = (unsigned)p < (unsigned)c.old_m;
          o[k] = in ? ld_nt(c.old_raw + p) : -1;  // sources are >= 0
          mm[k] = in ? ld_nt(c.old_map + p) : 0;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMapUnroll; ++k) {
      const int ek = e + k * kWave;
      if (ek < b) {
        int id;
        if (MODE == 2 && o[k] == u[k]) {
          id = mm[k];
        } else {
          id = newid[u[k]];
          if (MODE == 2) ++miss;
        }
        st_nt(dst + ek, id);
        if (MODE >= 1) st_nt(c.raw_out + ek, u[k]);
      }
    }
  }
}

// Entries [a, b) of ONE row (MODE 2), four wavefront-wide chunks at a time,
// all loaded at the current shift. When every entry is found where guessed
// the chunks are stored as loaded. Otherwise each chunk looks for its
// entries not found among its own 64 kept entries: rows are ascending, so
// the kept entries a wavefront loads at e + shift are ascending too, and a
// cross-lane binary search finds an entry that an update moved by fewer
// than 64 places. The four searches are independent (their shuffles
// overlap); the entries still not found are looked up in the numbering
// together, and the shift that the last entry found by a search shows is
// carried to the rest of the row.
__device__ __forceinline__ void map_row_kept(const int *__restrict__ src,
                                             const int *__restrict__ newid,
                                             int *__restrict__ dst, int a, int b, int shift,
                                             const MapCache &c, int &miss) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int cb = a; cb < b; cb += 4 * kWave) {
    int u[4], o[4], mm[4];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = cb + k * kWave + lane, p = e + shift;
      const bool in = (unsigned)p < (unsigned)c.old_m;
      u[k] = e < b ? ld_nt(src + e) : 0;
      // places outside the kept entries read as -1 below and +infinity above
      o[k] = in ? ld_nt(c.old_raw + p) : (p < 0 ? -1 : 0x7fffffff);
      mm[k] = in ? ld_nt(c.old_map + p) : 0;
      ok = ok && (e >= b || o[k] == u[k]);
    }
    if (__ballot(!ok) != 0) {
      int carry = 0;
      bool carried = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool v = cb + k * kWave + lane < b;
        const bool want = v && o[k] != u[k];
        if (!__ballot(want)) continue;
        int lo = 0;  // last lane j with o_j <= u
#pragma unroll
        for (int st = kWave / 2; st >= 1; st >>= 1) {
          const int oj = __shfl(o[k], lo + st);
          if (lo + st < kWave && oj <= u[k]) lo += st;
        }
        const int oj = __shfl(o[k], lo), mj = __shfl(mm[k], lo);
        const bool found = want && oj == u[k];  // u >= 0 never equals the fillers
        if (found) {
          mm[k] = mj;
          o[k] = u[k];
        }
        const unsigned long long fb = __ballot(found);
        if (fb) {
          const int L = 63 - __clzll(fb);
          carry = __shfl(lo - lane, L);
          carried = true;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (cb + k * kWave + lane < b && o[k] != u[k]) {
          mm[k] = newid[u[k]];
          ++miss;
        }
      if (carried) shift += carry;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = cb + k * kWave + lane;
      if (e < b) {
        st_nt(dst + e, mm[k]);
        st_nt(c.raw_out + e, u[k]);
      }
    }
  }
}

template <int MODE>
__device__ __forceinline__ void map_misses(int miss, const MapCache &c) {
  if (MODE != 2) return;
  miss = wave_sum_int(miss);
  if ((threadIdx.x & (kWave - 1)) == 0 && miss) atomicAdd(c.miss, miss);
}

// The same renumbering split by the die-split plan. Rows with at least T
// in-edges are mapped item by item, list x by the workgroups on die x (the
// items of list x have their sources in range x, so the newid entries a die
// reads are that range's eighth of the table, as the rank kernel's gathers
// are). A wavefront loads 64 items, one per lane, dealt out as in the rank
// kernel (item_of), and maps them one after the other with all its lanes.
// MODE 2 takes only the items of rows with at least min_len entries (the
// others go to k_map_short).
template <int LG, int MODE>
__global__ __launch_bounds__(kBlock) void k_map_split(const int4 *__restrict__ xitems,
                                                      const int *__restrict__ xoff,
                                                      const int *__restrict__ row_off,
                                                      const int *__restrict__ src,
                                                      const int *__restrict__ newid,
                                                      int *__restrict__ dst, MapCache c,
                                                      int min_len) {
  const int B = gridDim.x, lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int x0 = B >= kXcds ? (int)blockIdx.x % kXcds : (int)blockIdx.x;
  const int xstep = B >= kXcds ? kXcds : B;
  const int loc = B >= kXcds ? (int)blockIdx.x / kXcds : 0;
  const int nloc = B >= kXcds ? (B - 1 - x0) / kXcds + 1 : 1;
  const long long Wd = (long long)nloc * kWavesPerBlock;
  const int gwx = loc * kWavesPerBlock + wid;
  int miss = 0;
  for (int x = x0; x < kXcds; x += xstep) {
    const int beg = xoff[x], end = xoff[x + 1];
    for (long long k0 = 0; item_of<LG>(beg, gwx, k0, Wd) < end; k0 += kWave) {
      const long long j = item_of<LG>(beg, gwx, k0 + lane, Wd);
      const int4 it = j < end ? xitems[j] : make_int4(0, 0, 0, 0);
      bool take = j < end;
      int sh = 0;  // the shift of the item's row between the two layouts
      if (MODE == 2 && take) {
        const int r0 = row_off[it.w];
        take = row_off[it.w + 1] - r0 >= min_len;
        sh = c.old_off[it.w] - r0;
      }
      unsigned long long vm = __ballot(take);
      while (vm) {
        const int q = __ffsll(vm) - 1;
        vm &= vm - 1;
        const int e0 = __shfl(it.y, q), e1 = __shfl(it.z, q), shq = __shfl(sh, q);
        if (MODE == 2) map_row_kept(src, newid, dst, e0, e1, shq, c, miss);
        else map_run<MODE>(src, newid, dst, e0, e1, 0, c, miss);
      }
    }
  }
  map_misses<MODE>(miss, c);
}

// Rows with fewer than T in-edges: a wavefront takes 64 consecutive rows and
// cuts them into segments, maximal runs of consecutive such rows (which lie
// end to end in memory) with one shift to the kept layout (MODE 2; 0
// otherwise), and maps each segment as one run. In MODE 2, when the 64 rows
// hold more than kKeptGroupLen entries, their rows of at least kKeptRowLen
// entries are listed in dlist instead (one atomic per wavefront), and
// k_map_rows_kept maps them a wavefront each: the long rows of a graph can
// cluster in a few groups of 64 (on preferential-attachment graphs the early
// vertices hold most in-edges), and one wavefront streaming all of them would
// hold up the whole launch. A row of at least kKeptRowLen entries whose
// length changed (the next row's shift differs from its own) is listed there
// too, since its walk with the in-row search (map_row_kept) is slower than a
// stream; in a shorter changed row the entries after the change are looked
// up. MODE >= 1 also copies the row offsets.
constexpr int kKeptRowLen = 256;
constexpr int kKeptGroupLen = 16384;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_map_short(const int *__restrict__ in_off,
                                                      const int *__restrict__ src, int n, int T,
                                                      const int *__restrict__ newid,
                                                      int *__restrict__ dst, MapCache c,
                                                      int *__restrict__ dlist,
                                                      int *__restrict__ dcount) {
  const int lane = threadIdx.x & (kWave - 1);
  const long long nw = (long long)gridDim.x * kWavesPerBlock;
  int miss = 0;
  long long wv = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  // the offsets of the wavefront's next 64 rows (and their kept ones), loaded
  // while the current rows are mapped
  int ne0 = 0, ne1 = 0, no0 = 0, no1 = 0;
  auto fetch = [&](long long g) {
    const long long rr = g * kWave + lane;
    if (rr < n) {
      ne0 = in_off[rr];
      ne1 = in_off[rr + 1];
      if (MODE == 2) {
        no0 = c.old_off[rr];
        no1 = c.old_off[rr + 1];
      }
    }
  };
  if (wv * kWave < n) fetch(wv);
  for (; wv * kWave < n; wv += nw) {
    const int r = (int)(wv * kWave) + lane;
    const int ce0 = ne0, ce1 = ne1, co0 = no0, co1 = no1;
    if ((wv + nw) * kWave < n) fetch(wv + nw);
    int e0 = 0, cnt = 0, sh = 0, d = 0;
    bool mine = false, alone = false;
    if (r < n) {
      e0 = ce0;
      const int e1 = ce1;
      d = e1 - e0;
      mine = d < T;
      if (mine) cnt = d;
      if (MODE == 2) {
        sh = co0 - e0;
        alone = mine && d >= kKeptRowLen && co1 - e1 != sh;
      }
      if (MODE >= 1) {
        c.off_out[r] = e0;
        if (r == n - 1) c.off_out[n] = e1;
      }
    }
    if (MODE == 2) {
      const bool heavy = wave_sum_int(cnt) > kKeptGroupLen;  // every lane takes part
      const bool later = alone || (mine && d >= kKeptRowLen && heavy);
      const unsigned long long lm = __ballot(later);
      if (lm) {
        int base = 0;
        if (lane == 0) base = atomicAdd(dcount, __popcll(lm));
        base = __shfl(base, 0);
        if (later) {
          dlist[base + __popcll(lm & ((1ull << lane) - 1))] = r;
          mine = false;
          cnt = 0;
        }
      }
    }
    // a segment starts at a row of this kernel unless the previous row is
    // one too, of the same shift
    const int psh = __shfl_up(sh, 1);
    const bool pmine = __shfl_up((int)mine, 1) != 0;
    const bool start = mine && (lane == 0 || !pmine || psh != sh);
    // ... and ends before the next start or the next row not of this kernel
    const unsigned long long starts = __ballot(start), stops = __ballot(!mine) | starts;
    int x = cnt;  // inclusive scan of the lengths of this kernel's rows
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    unsigned long long sm = starts;
    while (sm) {
      const int j = __ffsll(sm) - 1;
      sm &= sm - 1;
      const unsigned long long after = stops & ~((2ull << j) - 1);
      const int jend = after ? __ffsll(after) - 1 : kWave;  // rows j .. jend - 1
      // entries of rows j .. jend - 1, end to end
      const int len = __shfl(x, jend - 1) - __shfl(x, j) + __shfl(cnt, j);
      const int a = __shfl(e0, j), shj = __shfl(sh, j);
      map_run<MODE>(src, newid, dst, a, a + len, shj, c, miss);
    }
  }
  map_misses<MODE>(miss, c);
}

// The rows k_map_short listed (MODE 2), a wavefront per row, each walked from
// its offsets' shift with the in-row search.
__global__ __launch_bounds__(kBlock) void k_map_rows_kept(const int *__restrict__ in_off,
                                                          const int *__restrict__ src,
                                                          const int *__restrict__ newid,
                                                          int *__restrict__ dst, MapCache c,
                                                          const int *__restrict__ dlist,
                                                          const int *__restrict__ dcount) {
  const int L = *dcount;
  const int W = gridDim.x * kWavesPerBlock;
  int miss = 0;
  for (int i = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; i < L; i += W) {
    const int r = dlist[i];
    const int e0 = in_off[r], e1 = in_off[r + 1];
    map_row_kept(src, newid, dst, e0, e1, c.old_off[r] - e0, c, miss);
  }
  map_misses<2>(miss, c);
}

// Count of affected vertices (profiling only).
__global__ __launch_bounds__(kBlock) void k_count_flags(const uint8_t *__restrict__ f, int n,
                                                        Ctrl *ctrl, int slot) {
  int c = 0;
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) c += f[v] != 0;
  c = wave_sum_int(c);
  if ((threadIdx.x & (kWave - 1)) == 0 && c)
    atomicAdd((unsigned long long *)&ctrl->aux[slot], (unsigned long long)c);
}

// Profiling of DF/DF-P/DT: the affected vertices an iteration is about to
// update, and their in-edges; k_affected_fold keeps the largest set and
// adds the edges to the running total.
__global__ __launch_bounds__(kBlock) void k_count_affected(const uint8_t *__restrict__ dV,
                                                           const int *__restrict__ in_off, int n,
                                                           Ctrl *ctrl) {
  if (ctrl->done) return;
  int c = 0;
  long long e = 0;
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
    if (dV[v]) {
      ++c;
      e += in_off[v + 1] - in_off[v];
    }
  c = wave_sum_int(c);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) e += __shfl_xor(e, o);
  if ((threadIdx.x & (kWave - 1)) == 0 && (c || e)) {
    atomicAdd((unsigned long long *)&ctrl->aux[4], (unsigned long long)c);
    atomicAdd((unsigned long long *)&ctrl->aux[6], (unsigned long long)e);
  }
}
__global__ void k_affected_fold(Ctrl *ctrl) {
  if (threadIdx.x == 0 && !ctrl->done) {
    if (ctrl->aux[4] > ctrl->aux[5]) ctrl->aux[5] = ctrl->aux[4];
    ctrl->aux[4] = 0;
  }
}

// ------------------------------------------------------------ validation
// Pass 1 reads only offsets; pass 2 (run only when pass 1 found nothing)
// reads the rows. Error bits: 1 / 16 offsets (in / out view), then
// 2, 4, 8 (in view) and 32, 64, 128 (out view) for an ID out of range, a row
// not strictly ascending, a missing self-loop.
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
