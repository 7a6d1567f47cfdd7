// device_common.h -- small device helpers shared by the lattice kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Koren-limited correction of an upwind face value (Hundsdorfer et al.
// 1995, the limiter the paper uses in Sec. 2): with dp the difference toward
// the downwind cell and dm the difference on the upwind side, the correction
// is psi(dm/dp) * dp, psi(t) = max(0, min(1, 1/3 + t/6, t)).  Multiplying
// through by dp turns the three-way min/max into two medians:
//   psi*dp = med3(dp, med3(dp/3 + dm/6, dm, 0), 0),
// which is 0 whenever dp and dm differ in sign and needs no division.
__device__ __forceinline__ float koren(float dp, float dm) {
  const float c = __builtin_fmaf(dm, 1.0f / 6.0f, dp * (1.0f / 3.0f));
  return __builtin_amdgcn_fmed3f(dp, __builtin_amdgcn_fmed3f(c, dm, 0.0f),
                                 0.0f);
}

__device__ __forceinline__ double med3d(double a, double b, double c) {
  return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

__device__ __forceinline__ double koren(double dp, double dm) {
  const double c = fma(dm, 1.0 / 6.0, dp * (1.0 / 3.0));
  return med3d(dp, med3d(c, dm, 0.0), 0.0);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fma_t(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

template <typename T>
__device__ __forceinline__ T pos(T a) {
  return a > T(0) ? a : T(0);
}
template <typename T>
__device__ __forceinline__ T neg(T a) {
  return a < T(0) ? a : T(0);
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8).  Re-number them so that each XCD walks one contiguous range of
// logical workgroups: neighbouring tiles (which share the cache lines at
// their edges) then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int xcd = b & 7, k = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// Lane-to-lane exchange inside a wavefront (ds_bpermute; no LDS storage).
__device__ __forceinline__ float lane_read(float v, int src) {
  return __int_as_float(
      __builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) |
                              (unsigned int)lo);
}

// Row-based addressing: the base of a velocity row and the per-cell stride
// are wave-uniform (scalar registers); each lane adds one 32-bit byte
// offset.  Every offset inside a row stays below 2^32.
// The empty asm pins the uniform cell base in scalar registers and keeps
// the compiler from re-associating it with the lane offset (which would
// hoist one 64-bit per-lane address per cell out of the row loop).
#define LAT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T row_load(const T* row, uint32_t cell_off,
                                      uint32_t lane_off) {
  const char* b = (const char*)row + cell_off;
  asm("" : "+s"(b));
  return *(const LAT_GLOBAL T*)((const LAT_GLOBAL char*)b + lane_off);
}
// NT: non-temporal stores, for a pass whose output is too large to stay in
// the caches for the next pass (the pass itself never reads a finished row
// again).  Measured on the 2D pass at 512^2 x 33^2 (1.14 GB): 1.9 % shorter;
// on a 76 MB state that the next kernel reads at once, longer.
template <bool NT, typename T>
__device__ __forceinline__ void row_store(T* row, uint32_t cell_off,
                                          uint32_t lane_off, T v) {
  char* b = (char*)row + cell_off;
  asm("" : "+s"(b));
  LAT_GLOBAL T* const q = (LAT_GLOBAL T*)((LAT_GLOBAL char*)b + lane_off);
  if constexpr (NT)
    __builtin_nontemporal_store(v, q);
  else
    *q = v;
}
// Store from the lanes with ok only (the cell base is pinned before the
// lane mask is applied).
template <bool NT, typename T>
__device__ __forceinline__ void row_store_if(T* row, uint32_t cell_off,
                                             uint32_t lane_off, T v, bool ok) {
  char* b = (char*)row + cell_off;
  asm("" : "+s"(b));
  LAT_GLOBAL T* const q = (LAT_GLOBAL T*)((LAT_GLOBAL char*)b + lane_off);
  if (ok) {
    if constexpr (NT)
      __builtin_nontemporal_store(v, q);
    else
      *q = v;
  }
}

}  // namespace lat
