// Wavefront-level (64-lane) and workgroup-level reductions for gfx950.
//
// FP64 values move through DPP as two 32-bit halves. The reduction tree is
// fixed (quad_perm pairs, quad_perm quads, row_shr 4, row_shr 8, row_bcast15,
// row_bcast31), so results are deterministic run to run. The full result
// lands in lane 63 and is broadcast with v_readlane. Every lane of the
// wavefront must be active when these are called: lanes without data pass
// the identity (0 for sums, 0 for the max of non-negative values).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prhip {

constexpr int kWave = 64;

// DPP control words (GFX9 encoding).
constexpr int DPP_QUAD_1032 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_SHR4 = 0x114;
constexpr int DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xFFFFFFFFLL);
  int hi = (int)(b >> 32);
  // old = 0: lanes with no valid source (or outside ROW_MASK) read 0 / 0.0
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, BANK_MASK, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, BANK_MASK, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFLL), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct OpSum {
  __device__ __forceinline__ double operator()(double a, double b) const { return a + b; }
};
struct OpMax {  // for non-negative values
  __device__ __forceinline__ double operator()(double a, double b) const { return fmax(a, b); }
};

// Reduction over the 64 lanes; the result is returned to every lane.
template <class Op>
__device__ __forceinline__ double wave_reduce(double x, Op op) {
  x = op(x, dpp_move<DPP_QUAD_1032>(x));
  x = op(x, dpp_move<DPP_QUAD_2301>(x));
  x = op(x, dpp_move<DPP_ROW_SHR4>(x));
  x = op(x, dpp_move<DPP_ROW_SHR8>(x));
  x = op(x, dpp_move<DPP_ROW_BCAST15, 0xA>(x));
  x = op(x, dpp_move<DPP_ROW_BCAST31, 0xC>(x));
  return readlane_d(x, 63);
}

__device__ __forceinline__ double wave_sum(double x) { return wave_reduce(x, OpSum()); }
__device__ __forceinline__ double wave_max(double x) { return wave_reduce(x, OpMax()); }

// Workgroup max of non-negative values (blockDim.x == NT, a multiple of 64).
// `lds` needs NT/64 doubles. Every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_max(double x, double *lds) {
  x = wave_max(x);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = x;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) r = fmax(r, lds[i]);
  __syncthreads();
  return r;
}

// Workgroup sum in a fixed order (wave sums, then waves 0..NT/64-1).
template <int NT>
__device__ __forceinline__ double block_sum(double x, double *lds) {
  x = wave_sum(x);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = x;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) r = r + lds[i];
  __syncthreads();
  return r;
}

// Exclusive prefix count of `pred` over the lanes of this wavefront, and the
// wavefront total.
__device__ __forceinline__ int wave_prefix_count(bool pred, int *total) {
  const unsigned long long mask = __ballot(pred);
  *total = __popcll(mask);
  const unsigned lo = (unsigned)(mask & 0xFFFFFFFFULL), hi = (unsigned)(mask >> 32);
  return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0));
}

}  // namespace prhip
