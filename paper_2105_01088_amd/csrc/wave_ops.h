// Wave-level helpers shared by the panel kernels (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace sgs {

// Pivot search key: |v| as an ordered bit pattern with its low 16 bits
// replaced by 0xffff - row, so one unsigned 64-bit maximum yields the largest
// entry (to 36 mantissa bits, far inside what partial pivoting needs) and, on
// ties, the smallest row.  0 means "no candidate".
__device__ __forceinline__ unsigned long long pivot_key(double v, int row) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
  return (bits & ~0xffffull) | (unsigned long long)(0xffff - row);
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// Maximum over the 64 lanes of a wave (every lane active), returned uniform.
// DPP within rows of 16 lanes (swap neighbours, swap pairs, half-row mirror,
// row mirror), then the four row results are read as scalars.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = umax64(v, dpp_u64<0xb1>(v));   // quad_perm [1,0,3,2]
  v = umax64(v, dpp_u64<0x4e>(v));   // quad_perm [2,3,0,1]
  v = umax64(v, dpp_u64<0x141>(v));  // row_half_mirror
  v = umax64(v, dpp_u64<0x140>(v));  // row_mirror
  return umax64(umax64(readlane_u64(v, 0), readlane_u64(v, 16)),
                umax64(readlane_u64(v, 32), readlane_u64(v, 48)));
}

// Maximum over lanes 0..7 (every lane active), returned uniform: swap
// neighbours, swap pairs, half-row mirror, then lane 0 read as a scalar.
__device__ __forceinline__ unsigned long long max8_u64(unsigned long long v) {
  v = umax64(v, dpp_u64<0xb1>(v));
  v = umax64(v, dpp_u64<0x4e>(v));
  v = umax64(v, dpp_u64<0x141>(v));
  return readlane_u64(v, 0);
}

// Lane `src` (a constant) of v, as a wave-uniform value (scalar registers).
// A uniform row is read from LDS one element per lane and broadcast this way:
// one LDS access per wave instead of one per element, and the FMAs that use
// it take the scalar operand directly.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace sgs
