// Batch update of a CSR view on the device: G^t = G^{t-1} minus deletions
// plus insertions (Sec. 3.3; the paper applies batches on the host, outside
// its timed region). One view at a time: rows keyed by `row`, entries by
// `col` (the in-view uses row = target, col = source; the out-view the
// reverse). Rows stay ascending.
//
//  1. keys (row << 32 | col) of the deletions and of the insertions, sorted
//     (rocPRIM radix sort), duplicates rejected;
//  2. per-row change counts, new degrees, new offsets (multi-workgroup scan);
//  3. one pass over the rows: a wavefront owns 64 consecutive rows; its lanes
//     copy their unchanged short rows, then the wavefront handles its changed
//     or long rows together: every kept old entry and every insertion goes to
//     its rank in the merged row, found by binary search over the row's
//     (sorted) deletions and insertions. A deletion that is not in the row or
//     an insertion that already is raises the error flag.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <cstdint>

#include "apply.h"

namespace prhip_apply {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kScanTile = 1024;   // offsets per workgroup in the scan
constexpr int kShortRow = 64;     // rows up to this long are copied by one lane

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

// Rebuild every row. err bit 4: a deletion not in its row; bit 8: an
// insertion already in its row. Every write stays inside the row's new range
// [new_off[r], new_off[r+1]) and below m_new, whatever the batch: an invalid
// batch leaves unspecified output, never a write out of bounds.
__global__ __launch_bounds__(kBlock) void k_rows(const int *__restrict__ off, const int *__restrict__ cols,
                                                 const u64 *__restrict__ dk, int nd, const u64 *__restrict__ ik,
                                                 int ni, const int *__restrict__ dcnt,
                                                 const int *__restrict__ icnt, int n,
                                                 const int *__restrict__ new_off, int m_new,
                                                 int *__restrict__ new_cols, int *err) {
  auto put = [&](int pos, int lo, int hi, int c) {
    if (pos >= lo && pos < hi && pos >= 0 && pos < m_new) new_cols[pos] = c;
    else atomicOr(err, 32);
  };
  const int lane = threadIdx.x & (kWave - 1);
  const long long nw = (long long)gridDim.x * (kBlock / kWave);
  for (long long wv = (long long)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; wv * kWave < n; wv += nw) {
    const int r = (int)(wv * kWave) + lane;
    bool special = false;
    if (r < n) {
      const int o0 = off[r], o1 = off[r + 1];
      special = dcnt[r] != 0 || icnt[r] != 0 || o1 - o0 > kShortRow;
      if (!special) {
        const int no = new_off[r], ne = new_off[r + 1];
        for (int i = o0; i < o1; ++i) put(no + (i - o0), no, ne, cols[i]);
      }
    }
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
        put(no + (i - o0) - dbelow + ibelow, no, ne, c);
      }
      // insertions
      for (int q = ia + lane; q < ib; q += kWave) {
        const int c = col_of(ik[q]);
        const int obelow = count_below(cols, o0, o1, c);
        if (obelow < o1 - o0 && cols[o0 + obelow] == c) atomicOr(err, 8);
        const int dbelow = nd_r ? count_below_key(dk, da, db, c) : 0;
        put(no + obelow - dbelow + (q - ia), no, ne, c);
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

int grid_for(long long work) {
  long long b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

}  // namespace prhip_apply

using namespace prhip_apply;

// See apply.h.
int prhip_apply_view(int n, const int *off, const int *cols, int m_new, const int *del_row,
                     const int *del_col, int nd, const int *ins_row, const int *ins_col, int ni,
                     int *new_off, int *new_cols, hipStream_t s, int *err_out, const char **what) {
  *err_out = 0;
  *what = nullptr;
  const int nt = (n + kScanTile - 1) / kScanTile;
  // scratch: keys in/out for both lists, counts, degrees, tile sums, error word
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
      (e = hipMallocAsync((void **)&dcnt, ((size_t)3 * n + nt + 16) * sizeof(int), s)) != hipSuccess ||
      (e = hipMallocAsync(&tmp, tmp_b + 16, s)) != hipSuccess)
    return done(e, "scratch allocation");
  (void)bytes;
  icnt = dcnt + n;
  deg = icnt + n;
  tsum = deg + n;
  err = tsum + nt + 8;
  if ((e = hipMemsetAsync(dcnt, 0, (size_t)2 * n * sizeof(int), s)) != hipSuccess ||
      (e = hipMemsetAsync(err, 0, sizeof(int), s)) != hipSuccess)
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
  if ((e = hipGetLastError()) != hipSuccess) return done(e, "kernel launch");
  int h_err = 0;
  if ((e = hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return done(e, "error readback");
  *err_out = h_err;
  return done(hipSuccess, nullptr);
}
