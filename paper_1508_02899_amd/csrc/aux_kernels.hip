// aux_kernels.hip -- FP64 conservation moments, density, flow checks and
// copies for the lattice library (gfx950).
#include <float.h>

#include "device_common.h"
#include "lattice_internal.h"

namespace lat {
namespace {

constexpr int kBlock = 256;

// Fixed-order block reduction of one double per thread: a pairwise tree in
// LDS, the same pairing on every run, so results are bit-reproducible.
__device__ double block_sum(double v, double* sh) {
  const int t = (int)threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// One workgroup per velocity plane: sum of the plane's sites in FP64.
// When the plane is 16-byte aligned and a whole number of 16-byte pieces,
// thread t adds pieces t, t+256, ... (coalesced 16-byte loads, one FP64
// partial sum per element of a piece, combined in a fixed order);
// otherwise sites t, t+256, ... one by one.  Then the tree.  The order of
// the additions depends only on the plane size, so repeated calls give the
// same bits.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int n = 2;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_plane_sums(const T* __restrict__ f,
                                                       int64_t sites,
                                                       int64_t pitch,
                                                       double* __restrict__ out) {
  __shared__ double sh[kBlock];
  using V = typename Vec16<T>::type;
  constexpr int NE = Vec16<T>::n;
  const T* p = f + (size_t)blockIdx.x * (size_t)pitch;
  double acc = 0.0;
  if (sites % NE == 0 && ((uintptr_t)p & 15) == 0) {  // uniform
    const V* q = reinterpret_cast<const V*>(p);
    const int64_t n = sites / NE;
    double a[NE] = {};
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const V v = q[i];
      const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int k = 0; k < NE; ++k) a[k] += (double)e[k];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) acc += a[k];
  } else {
    for (int64_t i = threadIdx.x; i < sites; i += kBlock) acc += (double)p[i];
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Weighted combination of the plane sums: M = w sum S_j, P_k = w sum S_j v_k,
// Q_k = w sum S_j v_k^2 with v = (j - h) dv per component, and the variance
// sum_k Q_k/M - |P/M|^2.  Single workgroup, fixed order.
__global__ __launch_bounds__(kBlock) void k_moments_final(
    const double* __restrict__ ps, int nv, int dim, double w, double dv,
    const int* __restrict__ flag, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  const int h = (nv - 1) / 2;
  const int nplanes = dim == 1 ? nv : nv * nv;
  double m = 0, px = 0, py = 0, qx = 0, qy = 0;
  for (int j = threadIdx.x; j < nplanes; j += kBlock) {
    const double s = ps[j];
    const double vx = (double)((dim == 1 ? j : j % nv) - h) * dv;
    const double vy = dim == 2 ? (double)(j / nv - h) * dv : 0.0;
    m += s;
    px += s * vx;
    qx += s * vx * vx;
    py += s * vy;
    qy += s * vy * vy;
  }
  m = block_sum(m, sh);
  px = block_sum(px, sh);
  py = block_sum(py, sh);
  qx = block_sum(qx, sh);
  qy = block_sum(qy, sh);
  if (threadIdx.x == 0) {
    out[0] = w * m;
    out[1] = w * px;
    out[2] = w * py;
    out[3] = w * qx;
    out[4] = w * qy;
    const double var = (qx + qy) / m - ((px / m) * (px / m) + (py / m) * (py / m));
    out[5] = var;
    out[6] = (double)*flag;
  }
}

// rho[site] = dvd * sum_j f[j][site], FP64, j in order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_density(const T* __restrict__ f,
                                                    int64_t sites,
                                                    int64_t pitch, int nplanes,
                                                    double dvd,
                                                    double* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= sites) return;
  double acc = 0.0;
  for (int j = 0; j < nplanes; ++j) acc += (double)f[(size_t)j * pitch + i];
  rho[i] = dvd * acc;
}

// Flow check: flag |= 1 if some |u| exceeds umax_ok (>= when strict) or is
// not finite.  Grid-stride, one atomic per offending wavefront.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cfl_check(const T* __restrict__ u,
                                                      int64_t n, T umax_ok,
                                                      int strict,
                                                      int* __restrict__ flag) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += stride) {
    const T a = u[i] < T(0) ? -u[i] : u[i];
    const bool ok = strict ? (a < umax_ok) : (a <= umax_ok);  // NaN -> !ok
    bad |= !ok;
  }
  if (__any(bad) && ((int)threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// max |u| into out (out must hold 0 beforehand); NaN propagates as +inf.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_absmax(const T* __restrict__ u,
                                                   int64_t n,
                                                   unsigned long long* out) {
  __shared__ double sh[kBlock];
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += stride) {
    double a = (double)u[i];
    a = a < 0 ? -a : a;
    if (!(a <= DBL_MAX)) a = __longlong_as_double(0x7ff0000000000000LL);
    m = a > m ? a : m;
  }
  const int t = (int)threadIdx.x;
  sh[t] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = sh[t] > sh[t + w] ? sh[t] : sh[t + w];
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (t == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ __launch_bounds__(kBlock) void k_copy16(const uint4* __restrict__ s,
                                                   uint4* __restrict__ d,
                                                   int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += stride)
    d[i] = s[i];
}

__global__ void k_copy1(const unsigned char* __restrict__ s,
                        unsigned char* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void k_clear(int* flag) { *flag = 0; }

__global__ void k_flag_out(const int* flag, int32_t* status) {
  *status = *flag;
}

__global__ void k_clear_u64(unsigned long long* p) { *p = 0ull; }

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_moments(const void* f, int64_t sites, int64_t pitch,
                          int nv, int dim, int f64, double w, double dv,
                          double* plane_sums, const int* flag, double* out,
                          hipStream_t s) {
  const int nplanes = dim == 1 ? nv : nv * nv;
  if (f64)
    hipLaunchKernelGGL(k_plane_sums<double>, dim3(nplanes), dim3(kBlock), 0, s,
                       (const double*)f, sites, pitch, plane_sums);
  else
    hipLaunchKernelGGL(k_plane_sums<float>, dim3(nplanes), dim3(kBlock), 0, s,
                       (const float*)f, sites, pitch, plane_sums);
  hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(kBlock), 0, s, plane_sums,
                     nv, dim, w, dv, flag, out);
  return hipGetLastError();
}

hipError_t launch_density(const void* f, int64_t sites, int64_t pitch,
                          int nplanes, int f64, double dvd, double* rho,
                          hipStream_t s) {
  const int g = (int)((sites + kBlock - 1) / kBlock);
  if (f64)
    hipLaunchKernelGGL(k_density<double>, dim3(g), dim3(kBlock), 0, s,
                       (const double*)f, sites, pitch, nplanes, dvd, rho);
  else
    hipLaunchKernelGGL(k_density<float>, dim3(g), dim3(kBlock), 0, s,
                       (const float*)f, sites, pitch, nplanes, dvd, rho);
  return hipGetLastError();
}

hipError_t launch_cfl_check(const void* u, int64_t n, double umax_ok,
                            int strict, int f64, int* flag, hipStream_t s) {
  const int g = grid_for(n);
  if (f64)
    hipLaunchKernelGGL(k_cfl_check<double>, dim3(g), dim3(kBlock), 0, s,
                       (const double*)u, n, umax_ok, strict, flag);
  else
    hipLaunchKernelGGL(k_cfl_check<float>, dim3(g), dim3(kBlock), 0, s,
                       (const float*)u, n, (float)umax_ok, strict, flag);
  return hipGetLastError();
}

hipError_t launch_absmax(const void* u, int64_t n, int f64, double* out,
                         hipStream_t s) {
  auto* o = reinterpret_cast<unsigned long long*>(out);
  hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(1), 0, s, o);
  const int g = grid_for(n);
  if (f64)
    hipLaunchKernelGGL(k_absmax<double>, dim3(g), dim3(kBlock), 0, s,
                       (const double*)u, n, o);
  else
    hipLaunchKernelGGL(k_absmax<float>, dim3(g), dim3(kBlock), 0, s,
                       (const float*)u, n, o);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes,
                       hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 > 0 && ((uintptr_t)dst % 16) == 0 && ((uintptr_t)src % 16) == 0) {
    hipLaunchKernelGGL(k_copy16, dim3(grid_for(n16)), dim3(kBlock), 0, s,
                       (const uint4*)src, (uint4*)dst, n16);
    const int64_t done = n16 * 16;
    const int64_t rest = bytes - done;
    if (rest > 0)
      hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, s,
                         (const unsigned char*)src + done,
                         (unsigned char*)dst + done, rest);
  } else if (bytes > 0) {
    hipLaunchKernelGGL(k_copy1, dim3((int)((bytes + 255) / 256)), dim3(256), 0,
                       s, (const unsigned char*)src, (unsigned char*)dst,
                       bytes);
  }
  return hipGetLastError();
}

hipError_t launch_clear_flag(int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(1), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_flag_out(const int* flag, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_out, dim3(1), dim3(1), 0, s, flag, status);
  return hipGetLastError();
}

}  // namespace lat
