// Batch update of a CSR view on the device: G^t = G^{t-1} minus deletions
// plus insertions (Sec. 3.3; the paper applies batches on the host, outside
// its timed region). One view at a time: rows keyed by `row`, entries by
// `col` (the in-view uses row = target, col = source; the out-view the
// reverse). Rows stay ascending.
//
//  1. keys (row << 32 | col) of the deletions and of the insertions, sorted
//     (rocPRIM radix sort), duplicates rejected;
//  2. per-row change counts, new degrees, new offsets (multi-workgroup scan);
//  3. one pass over the rows: a wavefront owns 64 consecutive rows; it copies
//     their unchanged short rows edge-parallel, laid end to end, then handles
//     its changed or long rows together: every kept old entry and every
//     insertion goes to its rank in the merged row, found by binary search
//     over the row's (sorted) deletions and insertions. A deletion that is
//     not in the row or an insertion that already is raises the error flag.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

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
  size_t tmp_d = 0, tmp_i = 0;
  hipError_t e = hipSuccess;
  auto done = [&](hipError_t code, const char *msg) {
    (void)hipFreeAsync(dk_in, s); (void)hipFreeAsync(dk, s); (void)hipFreeAsync(ik_in, s);
    (void)hipFreeAsync(ik, s); (void)hipFreeAsync(dcnt, s); (void)hipFreeAsync(tmp, s);
    if (code != hipSuccess && !*what) *what = msg;
    return (int)code;
  };
  if ((e = rocprim::radix_sort_keys(nullptr, tmp_d, (u64 *)nullptr, (u64 *)nullptr, (unsigned)nd, 0, 64, s)) != hipSuccess ||
      (e = rocprim::radix_sort_keys(nullptr, tmp_i, (u64 *)nullptr, (u64 *)nullptr, (unsigned)ni, 0, 64, s)) != hipSuccess)
    return done(e, "radix sort size query");
  const size_t tmp_b = tmp_d > tmp_i ? tmp_d : tmp_i;
  bytes = (size_t)(nd + 1) * 2 * sizeof(u64) + (size_t)(ni + 1) * 2 * sizeof(u64);
  if ((e = hipMallocAsync((void **)&dk_in, (size_t)(nd + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&dk, (size_t)(nd + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&ik_in, (size_t)(ni + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&ik, (size_t)(ni + 1) * sizeof(u64), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&dcnt, ((size_t)3 * n + nt + 16 + nbk + 1) * sizeof(int), s)) != hipSuccess ||
      (e = hipMallocAsync(&tmp, tmp_b + 16, s)) != hipSuccess)
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
  if (nd > 0) {
    hipLaunchKernelGGL(k_keys, dim3(grid_for(nd)), dim3(kBlock), 0, s, del_row, del_col, nd, n, dk_in, err);
    size_t tb = tmp_d;
    if ((e = rocprim::radix_sort_keys(tmp, tb, dk_in, dk, (unsigned)nd, 0, 64, s)) != hipSuccess)
      return done(e, "radix sort");
    hipLaunchKernelGGL(k_count, dim3(grid_for(nd)), dim3(kBlock), 0, s, (const u64 *)dk, nd, dcnt, err);
  }
  if (ni > 0) {
    hipLaunchKernelGGL(k_keys, dim3(grid_for(ni)), dim3(kBlock), 0, s, ins_row, ins_col, ni, n, ik_in, err);
    size_t tb = tmp_i;
    if ((e = rocprim::radix_sort_keys(tmp, tb, ik_in, ik, (unsigned)ni, 0, 64, s)) != hipSuccess)
      return done(e, "radix sort");
    hipLaunchKernelGGL(k_count, dim3(grid_for(ni)), dim3(kBlock), 0, s, (const u64 *)ik, ni, icnt, err);
  }
  hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kBlock), 0, s, off, (const int *)dcnt, (const int *)icnt, n,
                     deg, tsum);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, s, tsum, nt);
  hipLaunchKernelGGL(k_offsets, dim3(nt), dim3(kBlock), 0, s, (const int *)deg, (const int *)tsum, n, m_new,
                     new_off);
  hipLaunchKernelGGL(k_check_total, dim3(1), dim3(64), 0, s, (const int *)new_off, (const int *)deg, n, m_new,
                     err);
  hipLaunchKernelGGL(k_check_deg, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, (const int *)deg, n, err);
  hipLaunchKernelGGL(k_rows, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, off, cols, (const u64 *)dk, nd,
                     (const u64 *)ik, ni, (const int *)dcnt, (const int *)icnt, n, (const int *)new_off,
                     m_new, new_cols, err);
  if (nbk > 0) {
    hipLaunchKernelGGL(k_rowat, dim3(grid_for((long long)n)), dim3(kBlock), 0, s, off, n, nbk, rowat);
    hipLaunchKernelGGL(k_long_rows, dim3(nbk < 65536 ? nbk : 65536), dim3(kBlock), 0, s, off, cols,
                       (const u64 *)dk, nd, (const u64 *)ik, ni, (const int *)dcnt, (const int *)icnt, n,
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
