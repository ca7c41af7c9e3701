// Batch update of a CSR view on the device: G^t = G^{t-1} minus deletions
// plus insertions (Sec. 3.3; the paper applies batches on the host, outside
// its timed region). One view at a time: rows keyed by `row`, entries by
// `col` (the in-view uses row = target, col = source; the out-view the
// reverse). Rows stay ascending.
//
//  1. keys (row << 32 | col) of the deletions and of the insertions, sorted
//     (least-significant-digit radix sort over the bits IDs below n can set),
//     duplicates rejected;
//  2. per-row change counts, new degrees, new offsets (multi-workgroup scan);
//  3. one pass over the rows: a wavefront owns 64 consecutive rows; it copies
//     their unchanged short rows edge-parallel, laid end to end, then handles
//     its changed or long rows together: every kept old entry and every
//     insertion goes to its rank in the merged row, found by binary search
//     over the row's (sorted) deletions and insertions. A deletion that is
//     not in the row or an insertion that already is raises the error flag.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "apply.h"

namespace prhip_apply {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kScanTile = 1024;   // offsets per workgroup in the scan
constexpr int kLongRow = 4096;    // longer rows are cut into chunks of this many entries

using u64 = unsigned long long;

__device__ __forceinline__ u64 key_of(int row, int col) { return ((u64)(unsigned)row << 32) | (unsigned)col; }
__device__ __forceinline__ int row_of(u64 k) { return (int)(k >> 32); }
__device__ __forceinline__ int col_of(u64 k) { return (int)(k & 0xFFFFFFFFu); }

// keys of a batch in the view's orientation; IDs outside [0, n) set err bit 1
__global__ __launch_bounds__(kBlock) void k_keys(const int *__restrict__ row, const int *__restrict__ col,
                                                 int k, int n, u64 *__restrict__ keys, int *err) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    const int r = row[i], c = col[i];
    if (r < 0 || r >= n || c < 0 || c >= n) {
      atomicOr(err, 1);
      keys[i] = key_of(0, 0);
    } else {
      keys[i] = key_of(r, c);
    }
  }
}

// ------------------------------------------------------------ radix sort
// Keys are sorted by 8-bit digits, least significant first, and only the
// digits that IDs below n can set (a row or column ID of b bits leaves the
// others 0). Each pass is a stable counting sort. A list of at most
// kRsSmall keys is sorted by one workgroup in one launch, the keys held in
// registers and moved through LDS. A longer one takes three launches per
// pass: per-tile digit histograms (tiles of kRsTile keys, stored tile-major),
// a scan of each digit's column over the tiles (one workgroup per digit),
// and a scatter: digit d of tile t starts where all smaller digits, and
// digit d of the earlier tiles, end (each scatter workgroup scans the 256
// digit totals itself).
// Either way a key's place within its tile is its rank among the tile's keys
// with the same digit, in input order: rounds of kBlock keys in order; in a
// round the lanes of a wavefront with the same digit are found with eight
// ballots, and the wavefronts before it and the rounds before add their
// counts, kept per digit in LDS.
constexpr int kRsBins = 256;
constexpr int kRsPer = 4;                 // keys per thread in a tile of the long path
constexpr int kRsTile = kBlock * kRsPer;
constexpr int kRsSmallPer = 16;           // keys per thread on the one-workgroup path
constexpr int kRsSmall = kBlock * kRsSmallPer;
constexpr int kRsWaves = kBlock / kWave;
static_assert(kRsBins == kBlock, "one digit per thread");

__device__ __forceinline__ int rs_digit(u64 k, int sh) { return (int)((k >> sh) & 0xFFu); }

// Place of this thread's key (digit d; valid = it exists) in a round: the
// count of the digit before the round (s_run[d]) plus its rank in the
// round. s_w must be zero on entry; on return s_run holds the counts after
// the round and s_w is zero again.
__device__ __forceinline__ int rs_rank(bool valid, int d, int *s_run, int (*s_w)[kRsBins]) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  unsigned long long same = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool on = (d >> bit) & 1;
    const unsigned long long bb = __ballot(valid && on);
    same &= on ? bb : ~bb;
  }
  const int r = __popcll(same & ((1ull << lane) - 1));
  if (valid && r == 0) s_w[w][d] = __popcll(same);
  __syncthreads();
  int pos = 0;
  if (valid) {
    pos = s_run[d] + r;
    for (int j = 0; j < w; ++j) pos += s_w[j][d];
  }
  __syncthreads();
  int add = 0;
#pragma unroll
  for (int j = 0; j < kRsWaves; ++j) {
    add += s_w[j][tid];
    s_w[j][tid] = 0;
  }
  s_run[tid] += add;
  __syncthreads();
  return pos;
}

// one workgroup sorts keys[0 .. cnt), cnt <= kRsSmall, in place
__global__ __launch_bounds__(kBlock) void k_rs_small(u64 *__restrict__ keys, int cnt, int b) {
  __shared__ u64 buf[kRsSmall];
  __shared__ int s_run[kRsBins];
  __shared__ int s_w[kRsWaves][kRsBins];
  const int tid = threadIdx.x;
  u64 v[kRsSmallPer];
#pragma unroll
  for (int k = 0; k < kRsSmallPer; ++k) {
    const int i = k * kBlock + tid;
    v[k] = i < cnt ? keys[i] : 0;
  }
  for (int j = 0; j < kRsWaves; ++j) s_w[j][tid] = 0;
  for (int half = 0; half < 2; ++half)
    for (int lo = 0; lo < b; lo += 8) {
      const int sh = 32 * half + lo;
      s_run[tid] = 0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kRsSmallPer; ++k)
        if (k * kBlock + tid < cnt) atomicAdd(&s_run[rs_digit(v[k], sh)], 1);
      __syncthreads();
      if (tid == 0) {  // exclusive scan over the digits
        int run = 0;
        for (int d = 0; d < kRsBins; ++d) {
          const int x = s_run[d];
          s_run[d] = run;
          run += x;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kRsSmallPer; ++k) {
        if (k * kBlock >= cnt) break;  // rounds past the keys (uniform)
        const bool valid = k * kBlock + tid < cnt;
        const int pos = rs_rank(valid, rs_digit(v[k], sh), s_run, s_w);
        if (valid) buf[pos] = v[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kRsSmallPer; ++k) {
        const int i = k * kBlock + tid;
        if (i < cnt) v[k] = buf[i];
      }
      __syncthreads();
    }
#pragma unroll
  for (int k = 0; k < kRsSmallPer; ++k) {
    const int i = k * kBlock + tid;
    if (i < cnt) keys[i] = v[k];
  }
}

// hist[t * kRsBins + d] = keys of tile t with digit d
__global__ __launch_bounds__(kBlock) void k_rs_hist(const u64 *__restrict__ keys, int cnt, int sh,
                                                    int *__restrict__ hist) {
  __shared__ int h[kRsBins];
  const int tid = threadIdx.x, t = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  for (int k = 0; k < kRsPer; ++k) {
    const long long i = (long long)t * kRsTile + k * kBlock + tid;
    if (i < cnt) atomicAdd(&h[rs_digit(keys[i], sh)], 1);
  }
  __syncthreads();
  hist[(size_t)t * kRsBins + tid] = h[tid];
}

// Exclusive scan over the workgroup (kBlock threads); *total gets the sum.
__device__ __forceinline__ int rs_block_scan(int x, int *total) {
  __shared__ int wsum[kRsWaves];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  int v = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) wsum[w] = v;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int j = 0; j < kRsWaves; ++j) {
    if (j < w) before += wsum[j];
    all += wsum[j];
  }
  __syncthreads();
  *total = all;
  return before + v - x;
}

// Column d of the tile-major histograms (workgroup d): each entry becomes
// the count of digit d in the tiles before it, and tot[d] the column's sum.
__global__ __launch_bounds__(kBlock) void k_rs_colscan(int *__restrict__ hist, int ntiles,
                                                       int *__restrict__ tot) {
  const int d = blockIdx.x;
  int carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += kBlock) {
    const int t = t0 + (int)threadIdx.x;
    const size_t i = (size_t)t * kRsBins + d;
    const int x = t < ntiles ? hist[i] : 0;
    int sum;
    const int ex = rs_block_scan(x, &sum);
    if (t < ntiles) hist[i] = carry + ex;
    carry += sum;
  }
  if (threadIdx.x == 0) tot[d] = carry;
}

// out[start of (digit, tile) + rank within the tile] = key
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const u64 *__restrict__ in,
                                                       u64 *__restrict__ out, int cnt, int sh,
                                                       const int *__restrict__ start,
                                                       const int *__restrict__ tot) {
  __shared__ int s_run[kRsBins];
  __shared__ int s_w[kRsWaves][kRsBins];
  const int tid = threadIdx.x, t = blockIdx.x;
  int all;
  s_run[tid] = rs_block_scan(tot[tid], &all) + start[(size_t)t * kRsBins + tid];
  for (int j = 0; j < kRsWaves; ++j) s_w[j][tid] = 0;
  __syncthreads();
  for (int k = 0; k < kRsPer; ++k) {
    const long long i = (long long)t * kRsTile + k * kBlock + tid;
    const bool valid = i < cnt;
    const u64 key = valid ? in[i] : 0;
    const int pos = rs_rank(valid, rs_digit(key, sh), s_run, s_w);
    if (valid) out[pos] = key;
  }
}

// sorts keys[0 .. cnt) (IDs below n in both halves); the result is in
// *keys or *tmp, returned through *sorted
void rs_sort(u64 *keys, u64 *tmp, int cnt, int n, int *hist, hipStream_t s, u64 **sorted) {
  int b = 0;  // bits of an ID below n
  while (b < 31 && (1ll << b) < n) ++b;
  if (cnt <= kRsSmall) {
    if (b > 0) hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(kBlock), 0, s, keys, cnt, b);
    *sorted = keys;
    return;
  }
  const int ntiles = (int)(((long long)cnt + kRsTile - 1) / kRsTile);
  u64 *src = keys, *dst = tmp;
  for (int half = 0; half < 2; ++half)
    for (int lo = 0; lo < b; lo += 8) {
      const int sh = 32 * half + lo;
      hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(kBlock), 0, s, (const u64 *)src, cnt, sh,
                         hist);
      hipLaunchKernelGGL(k_rs_colscan, dim3(kRsBins), dim3(kBlock), 0, s, hist, ntiles,
                         hist + (size_t)kRsBins * ntiles);
      hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kBlock), 0, s, (const u64 *)src, dst,
                         cnt, sh, (const int *)hist, (const int *)hist + (size_t)kRsBins * ntiles);
      u64 *x = src;
      src = dst;
      dst = x;
    }
  *sorted = src;
}

// per-row counts of a sorted key list (cnt zeroed before); a repeated key
// sets err bit 2
__global__ __launch_bounds__(kBlock) void k_count(const u64 *__restrict__ keys, int k, int *cnt, int *err) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    if (i > 0 && keys[i] == keys[i - 1]) atomicOr(err, 2);
    atomicAdd(&cnt[row_of(keys[i])], 1);
  }
}

// new degree of every row, summed per tile of kScanTile rows
__global__ __launch_bounds__(kBlock) void k_tile_sums(const int *__restrict__ off, const int *__restrict__ dcnt,
                                                      const int *__restrict__ icnt, int n, int *__restrict__ deg,
                                                      int *__restrict__ tsum) {
  __shared__ int part[kBlock / kWave];
  int s = 0;
  for (int q = 0; q < kScanTile / kBlock; ++q) {
    const int r = blockIdx.x * kScanTile + q * kBlock + threadIdx.x;
    if (r < n) {
      const int d = off[r + 1] - off[r] - dcnt[r] + icnt[r];
      deg[r] = d;
      s += d;
    }
  }
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    tsum[blockIdx.x] = t;
  }
}

// exclusive scan of the tile sums in place (one workgroup, sequential chunks)
__global__ __launch_bounds__(kBlock) void k_scan_tiles(int *__restrict__ tsum, int nt) {
  __shared__ int part[kBlock];
  const int per = (nt + kBlock - 1) / kBlock;
  const int b = min((int)threadIdx.x * per, nt), e = min(b + per, nt);
  int s = 0;
  for (int i = b; i < e; ++i) s += tsum[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < kBlock; ++i) {
      const int t = part[i];
      part[i] = run;
      run += t;
    }
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int i = b; i < e; ++i) {
    const int t = tsum[i];
    tsum[i] = run;
    run += t;
  }
}

// new offsets: tile base + exclusive scan inside the tile; new_off[n] = m'
__global__ __launch_bounds__(kBlock) void k_offsets(const int *__restrict__ deg, const int *__restrict__ tsum, int n,
                                                    int m_new, int *__restrict__ new_off) {
  __shared__ int part[kBlock / kWave];
  __shared__ int carry;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) carry = tsum[blockIdx.x];
  __syncthreads();
  for (int q = 0; q < kScanTile / kBlock; ++q) {
    const int r = blockIdx.x * kScanTile + q * kBlock + threadIdx.x;
    const int d = r < n ? deg[r] : 0;
    int x = d;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) part[w] = x;
    __syncthreads();
    int base = carry;
    for (int i = 0; i < w; ++i) base += part[i];
    if (r < n) new_off[r] = base + x - d;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int i = 0; i < kBlock / kWave; ++i) t += part[i];
      carry += t;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) new_off[n] = m_new;
}

// the scanned total must be m_new (err bit 16), the degrees non-negative
__global__ void k_check_total(const int *__restrict__ new_off, const int *__restrict__ deg, int n, int m_new,
                              int *err) {
  if (threadIdx.x == 0 && (n == 0 ? m_new != 0 : new_off[n - 1] + deg[n - 1] != m_new)) atomicOr(err, 16);
}
__global__ __launch_bounds__(kBlock) void k_check_deg(const int *__restrict__ deg, int n, int *err) {
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock)
    if (deg[r] < 0) atomicOr(err, 16);
}

// first index of row r's keys in a sorted list
__device__ __forceinline__ int first_of_row(const u64 *__restrict__ keys, int k, int r) {
  int lo = 0, hi = k;
  const u64 t = key_of(r, 0);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// number of entries in sorted cols [a, b) (of one row) below c
__device__ __forceinline__ int count_below_key(const u64 *__restrict__ keys, int a, int b, int c) {
  int lo = a, hi = b;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col_of(keys[mid]) < c) lo = mid + 1;
    else hi = mid;
  }
  return lo - a;
}
__device__ __forceinline__ int count_below(const int *__restrict__ cols, int a, int b, int c) {
  int lo = a, hi = b;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cols[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo - a;
}

// Rebuild every row of at most kLongRow entries (longer rows: k_long_rows).
// err bit 4: a deletion not in its row; bit 8: an insertion already in its
// row. Every write stays inside the row's new range [new_off[r],
// new_off[r+1]) and below m_new, whatever the batch: an invalid batch leaves
// unspecified output, never a write out of bounds.
__device__ __forceinline__ void put(int *__restrict__ new_cols, int m_new, int *err, int pos, int lo,
                                    int hi, int c) {
  if (pos >= lo && pos < hi && pos >= 0 && pos < m_new) new_cols[pos] = c;
  else atomicOr(err, 32);
}

__global__ __launch_bounds__(kBlock) void k_rows(const int *__restrict__ off, const int *__restrict__ cols,
                                                 const u64 *__restrict__ dk, int nd, const u64 *__restrict__ ik,
                                                 int ni, const int *__restrict__ dcnt,
                                                 const int *__restrict__ icnt, int n,
                                                 const int *__restrict__ new_off, int m_new,
                                                 int *__restrict__ new_cols, int *err) {
  const int lane = threadIdx.x & (kWave - 1);
  const long long nw = (long long)gridDim.x * (kBlock / kWave);
  for (long long wv = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; wv * kWave < n; wv += nw) {
    const int r = (int)(wv * kWave) + lane;
    bool special = false, lng = false;
    int o0 = 0, cnt = 0, no = 0, ne = 0;
    if (r < n) {
      // all of the row's metadata in one round trip
      o0 = off[r];
      const int o1 = off[r + 1], dc = dcnt[r], ic = icnt[r];
      no = new_off[r];
      ne = new_off[r + 1];
      lng = o1 - o0 > kLongRow;
      special = !lng && (dc != 0 || ic != 0);
      if (!lng && !special) cnt = o1 - o0;
    }
    if (__ballot(special || lng) == 0) {
      // no changed or long row among the 64: their entries are one run with
      // one shift in both arrays, copied with eight loads per lane in flight
      int total = cnt;
      for (int o = kWave / 2; o > 0; o >>= 1) total += __shfl_xor(total, o);
      const int s0 = __shfl(o0, 0), d0 = __shfl(no, 0), d1 = d0 + total;
      for (int k0 = 0; k0 < total; k0 += 8 * kWave) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + u * kWave + lane;
          v[u] = k < total ? cols[s0 + k] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + u * kWave + lane;
          if (k < total) put(new_cols, m_new, err, d0 + k, d0, d1, v[u]);
        }
      }
      continue;
    }
    // Unchanged rows keep their entries, shifted: laid end to end (a
    // wavefront scan of their lengths) they are copied edge-parallel, four
    // entries per lane in flight, so a wavefront's loads and stores are
    // contiguous runs. Entry k of the run belongs to the last row j whose
    // start excl_j is <= k.
    int x = cnt;
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    const int excl = x - cnt, total = __shfl(x, kWave - 1);
    for (int k0 = 0; k0 < total; k0 += 4 * kWave) {
      int dst[4], dlo[4], dhi[4], val[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = min(k0 + u * kWave + lane, total - 1);
        int lo = 0, hi = kWave;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (__shfl(excl, mid) <= k) lo = mid;
          else hi = mid;
        }
        const int b = __shfl(excl, lo), s0 = __shfl(o0, lo);
        dlo[u] = __shfl(no, lo);
        dhi[u] = __shfl(ne, lo);
        dst[u] = dlo[u] + (k - b);
        val[u] = cols[s0 + (k - b)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k0 + u * kWave + lane < total) put(new_cols, m_new, err, dst[u], dlo[u], dhi[u], val[u]);
    }
    // changed rows, one at a time by the whole wavefront
    unsigned long long mask = __ballot(special);
    while (mask) {
      const int j = __ffsll(mask) - 1;
      mask &= mask - 1;
      const int rr = (int)(wv * kWave) + j;
      const int o0 = off[rr], o1 = off[rr + 1], no = new_off[rr], ne = new_off[rr + 1];
      const int nd_r = dcnt[rr], ni_r = icnt[rr];
      const int da = nd_r ? first_of_row(dk, nd, rr) : 0, db = da + nd_r;
      const int ia = ni_r ? first_of_row(ik, ni, rr) : 0, ib = ia + ni_r;
      // kept old entries
      for (int i = o0 + lane; i < o1; i += kWave) {
        const int c = cols[i];
        const int dbelow = nd_r ? count_below_key(dk, da, db, c) : 0;
        if (dbelow < nd_r && col_of(dk[da + dbelow]) == c) continue;  // deleted
        const int ibelow = ni_r ? count_below_key(ik, ia, ib, c) : 0;
        put(new_cols, m_new, err, no + (i - o0) - dbelow + ibelow, no, ne, c);
      }
      // insertions
      for (int q = ia + lane; q < ib; q += kWave) {
        const int c = col_of(ik[q]);
        const int obelow = count_below(cols, o0, o1, c);
        if (obelow < o1 - o0 && cols[o0 + obelow] == c) atomicOr(err, 8);
        const int dbelow = nd_r ? count_below_key(dk, da, db, c) : 0;
        put(new_cols, m_new, err, no + obelow - dbelow + (q - ia), no, ne, c);
      }
      // every deletion must be present
      for (int q = da + lane; q < db; q += kWave) {
        const int c = col_of(dk[q]);
        const int obelow = count_below(cols, o0, o1, c);
        if (!(obelow < o1 - o0 && cols[o0 + obelow] == c)) atomicOr(err, 4);
      }
    }
  }
}

// rowat[k] = the row holding old entry k * kLongRow, for k < nbk (entries
// beyond off[n] are never named). Each such entry lies in exactly one row.
__global__ __launch_bounds__(kBlock) void k_rowat(const int *__restrict__ off, int n, int nbk,
                                                  int *__restrict__ rowat) {
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    const int o0 = off[r], o1 = off[r + 1];
    for (long long k = ((long long)o0 + kLongRow - 1) / kLongRow; k * kLongRow < o1 && k < nbk; ++k)
      rowat[k] = r;
  }
}

// Rows longer than kLongRow, cut into the chunks [b * kLongRow, (b+1) *
// kLongRow) of the old entries, one workgroup per chunk. A long row
// overlapping chunk b holds entry b * kLongRow or starts inside the chunk and
// then holds entry (b + 1) * kLongRow: it is rowat[b] or rowat[b + 1]. The
// workgroup of the chunk where a changed row starts also places its
// insertions and checks its deletions.
__global__ __launch_bounds__(kBlock) void k_long_rows(const int *__restrict__ off, const int *__restrict__ cols,
                                                      const u64 *__restrict__ dk, int nd,
                                                      const u64 *__restrict__ ik, int ni,
                                                      const int *__restrict__ dcnt,
                                                      const int *__restrict__ icnt, int n,
                                                      const int *__restrict__ rowat, int nbk,
                                                      const int *__restrict__ new_off, int m_new,
                                                      int *__restrict__ new_cols, int *err) {
  const int tid = threadIdx.x;
  for (int b = blockIdx.x; b < nbk; b += gridDim.x) {
    const long long c0 = (long long)b * kLongRow, c1 = c0 + kLongRow;
    const int cand[2] = {rowat[b], b + 1 < nbk ? rowat[b + 1] : -1};
    for (int t = 0; t < 2; ++t) {
      const int L = cand[t];
      if (L < 0 || L >= n || (t == 1 && L == cand[0])) continue;
      const int o0 = off[L], o1 = off[L + 1];
      if (o1 - o0 <= kLongRow) continue;
      const int lo = (int)max((long long)o0, c0), hi = (int)min((long long)o1, c1);
      const int no = new_off[L], ne = new_off[L + 1];
      const int nd_r = dcnt[L], ni_r = icnt[L];
      if (nd_r == 0 && ni_r == 0) {
        // unchanged: a shifted copy, sixteen entries per thread in flight
        int v[kLongRow / kBlock];
#pragma unroll
        for (int u = 0; u < kLongRow / kBlock; ++u) {
          const int i = lo + u * kBlock + tid;
          v[u] = i < hi ? cols[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kLongRow / kBlock; ++u) {
          const int i = lo + u * kBlock + tid;
          if (i < hi) put(new_cols, m_new, err, no + (i - o0), no, ne, v[u]);
        }
        continue;
      }
      const int da = nd_r ? first_of_row(dk, nd, L) : 0, db = da + nd_r;
      const int ia = ni_r ? first_of_row(ik, ni, L) : 0, ib = ia + ni_r;
      for (int i = lo + tid; i < hi; i += kBlock) {
        const int c = cols[i];
        const int dbelow = nd_r ? count_below_key(dk, da, db, c) : 0;
        if (dbelow < nd_r && col_of(dk[da + dbelow]) == c) continue;  // deleted
        const int ibelow = ni_r ? count_below_key(ik, ia, ib, c) : 0;
        put(new_cols, m_new, err, no + (i - o0) - dbelow + ibelow, no, ne, c);
      }
      if (o0 >= c0 && o0 < c1) {
        for (int q = ia + tid; q < ib; q += kBlock) {
          const int c = col_of(ik[q]);
          const int obelow = count_below(cols, o0, o1, c);
          if (obelow < o1 - o0 && cols[o0 + obelow] == c) atomicOr(err, 8);
          const int dbelow = nd_r ? count_below_key(dk, da, db, c) : 0;
          put(new_cols, m_new, err, no + obelow - dbelow + (q - ia), no, ne, c);
        }
        for (int q = da + tid; q < db; q += kBlock) {
          const int c = col_of(dk[q]);
          const int obelow = count_below(cols, o0, o1, c);
          if (!(obelow < o1 - o0 && cols[o0 + obelow] == c)) atomicOr(err, 4);
        }
      }
    }
  }
}

int grid_for(long long work) {
  long long b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

}  // namespace prhip_apply

using namespace prhip_apply;

// See apply.h.
int prhip_apply_view(int n, const int *off, const int *cols, int m_old, int m_new, const int *del_row,
                     const int *del_col, int nd, const int *ins_row, const int *ins_col, int ni,
                     int *new_off, int *new_cols, hipStream_t s, int *err_out, const char **what) {
  *err_out = 0;
  *what = nullptr;
  const int nt = (n + kScanTile - 1) / kScanTile;
  const int nbk = (int)(((long long)m_old + kLongRow - 1) / kLongRow);  // long-row chunks
  // scratch: keys in/out for both lists, counts, degrees, tile sums, error
  // word, the row of every chunk start
  size_t bytes = 0;
  u64 *dk_in = nullptr, *dk = nullptr, *ik_in = nullptr, *ik = nullptr;
  int *dcnt = nullptr, *icnt = nullptr, *deg = nullptr, *tsum = nullptr, *err = nullptr;
  void *tmp = nullptr;
  hipError_t e = hipSuccess;
  auto done = [&](hipError_t code, const char *msg) {
    (void)hipFreeAsync(dk_in, s); (void)hipFreeAsync(dk, s); (void)hipFreeAsync(ik_in, s);
    (void)hipFreeAsync(ik, s); (void)hipFreeAsync(dcnt, s); (void)hipFreeAsync(tmp, s);
    if (code != hipSuccess && !*what) *what = msg;
    return (int)code;
  };
  // radix sort: per-tile digit histograms of the longer list
  const long long kmax = nd > ni ? nd : ni;
  const size_t nhist = (size_t)kRsBins * (size_t)((kmax + kRsTile - 1) / kRsTile + 1);
  bytes = (size_t)(nd + 1) * 2 * sizeof(u64) + (size_t)(ni + 1) * 2 * sizeof(u64);
  if ((e = hipMallocAsync((void **)&dk_in, (size_t)(nd + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&dk, (size_t)(nd + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&ik_in, (size_t)(ni + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&ik, (size_t)(ni + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&dcnt, ((size_t)3 * n + nt + 16 + nbk + 1) * sizeof(int), s)) != hipSuccess ||
      (e = hipMallocAsync(&tmp, nhist * sizeof(int), s)) != hipSuccess)
    return done(e, "scratch allocation");
  (void)bytes;
  icnt = dcnt + n;
  deg = icnt + n;
  tsum = deg + n;
  err = tsum + nt + 8;
  int *rowat = err + 8;
  if ((e = hipMemsetAsync(dcnt, 0, (size_t)2 * n * sizeof(int), s)) != hipSuccess ||
      (e = hipMemsetAsync(err, 0, sizeof(int), s)) != hipSuccess ||
      (e = hipMemsetAsync(rowat, 0xff, (size_t)(nbk + 1) * sizeof(int), s)) != hipSuccess)
    return done(e, "memset");
  // the sorted lists (dk_in / dk and ik_in / ik are each other's ping-pong)
  const u64 *dsorted = dk, *isorted = ik;
  if (nd > 0) {
    hipLaunchKernelGGL(k_keys, dim3(grid_for(nd)), dim3(kBlock), 0, s, del_row, del_col, nd, n, dk_in, err);
    u64 *out = nullptr;
    rs_sort(dk_in, dk, nd, n, (int *)tmp, s, &out);
    dsorted = out;
    hipLaunchKernelGGL(k_count, dim3(grid_for(nd)), dim3(kBlock), 0, s, dsorted, nd, dcnt, err);
  }
  if (ni > 0) {
    hipLaunchKernelGGL(k_keys, dim3(grid_for(ni)), dim3(kBlock), 0, s, ins_row, ins_col, ni, n, ik_in, err);
    u64 *out = nullptr;
    rs_sort(ik_in, ik, ni, n, (int *)tmp, s, &out);
    isorted = out;
    hipLaunchKernelGGL(k_count, dim3(grid_for(ni)), dim3(kBlock), 0, s, isorted, ni, icnt, err);
  }
  hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kBlock), 0, s, off, (const int *)dcnt, (const int *)icnt, n,
                     deg, tsum);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, s, tsum, nt);
  hipLaunchKernelGGL(k_offsets, dim3(nt), dim3(kBlock), 0, s, (const int *)deg, (const int *)tsum, n, m_new,
                     new_off);
  hipLaunchKernelGGL(k_check_total, dim3(1), dim3(64), 0, s, (const int *)new_off, (const int *)deg, n, m_new,
                     err);
  hipLaunchKernelGGL(k_check_deg, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, (const int *)deg, n, err);
  hipLaunchKernelGGL(k_rows, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, off, cols, dsorted, nd,
                     isorted, ni, (const int *)dcnt, (const int *)icnt, n, (const int *)new_off,
                     m_new, new_cols, err);
  if (nbk > 0) {
    hipLaunchKernelGGL(k_rowat, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, off, n, nbk, rowat);
    hipLaunchKernelGGL(k_long_rows, dim3(nbk < 65536 ? nbk : 65536), dim3(kBlock), 0, s, off, cols,
                       dsorted, nd, isorted, ni, (const int *)dcnt, (const int *)icnt, n,
                       (const int *)rowat, nbk, (const int *)new_off, m_new, new_cols, err);
  }
  if ((e = hipGetLastError()) != hipSuccess) return done(e, "kernel launch");
  int h_err = 0;
  if ((e = hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return done(e, "error readback");
  *err_out = h_err;
  return done(hipSuccess, nullptr);
}
