// flows.hip -- carrier-flow synthesis on the device from Fourier mode tables
// (gfx950), so that long runs need no prestaged velocity field.
//
// The flows are the random Fourier flows of Sec. 3 (1D: a sum of modes whose
// amplitudes are redrawn or evolve as Ornstein-Uhlenbeck processes, Eq. 7)
// and the incompressible 2D flows of Sec. 4 (u = (d_y psi, -d_x psi) from a
// streamfunction).  The host draws the mode amplitudes (one table row per
// time slice); this file evaluates them on the lattice sites.  Phases are
// exact: the angle 2 pi k j / n is formed from the integer (k j) mod n.
#include <math.h>

#include "../../include/lattice.h"
#include "lattice_struct.h"

namespace lat {
namespace {

constexpr int kFlowBlock = 256;

__device__ __forceinline__ void phase(int64_t k, int64_t j, int64_t n,
                                      float* c, float* s) {
  int64_t p = (k * j) % n;
  if (p < 0) p += n;
  sincospif(2.0f * (float)p / (float)n, s, c);
}
__device__ __forceinline__ void phase(int64_t k, int64_t j, int64_t n,
                                      double* c, double* s) {
  int64_t p = (k * j) % n;
  if (p < 0) p += n;
  sincospi(2.0 * (double)p / (double)n, s, c);
}

// 1D: u[s][ix] = sum_k a_k cos(2 pi k ix / nx) + b_k sin(...), k = 1..K.
// coef[s][k-1] = (a, b).  One thread per site, one grid row per slice.
template <typename T>
__global__ __launch_bounds__(kFlowBlock) void k_flow1d(
    const float* __restrict__ coef, int K, int64_t nx, T* __restrict__ u) {
  const int64_t ix = (int64_t)blockIdx.x * kFlowBlock + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (ix >= nx) return;
  const float* c = coef + (size_t)s * K * 2;
  T acc = 0;
  for (int k = 1; k <= K; ++k) {
    T cs, sn;
    phase(k, ix, nx, &cs, &sn);
    acc += (T)c[2 * (k - 1)] * cs + (T)c[2 * (k - 1) + 1] * sn;
  }
  u[(size_t)s * nx + ix] = acc;
}

// 2D, pass 1 (along x): for every ky row of the table and every ix,
//   A[ky][ix] = sum_kx c[ky][kx] e^{2 pi i kx ix / nx}
//   B[ky][ix] = sum_kx (-i gx kx) c[ky][kx] e^{2 pi i kx ix / nx}
// with gx = 2 pi / (nx dx).  coef[s][ky + K][kx] = (re, im), kx = 0..K.
template <typename T>
__global__ __launch_bounds__(kFlowBlock) void k_flow2d_x(
    const float* __restrict__ coef, int K, int64_t nx, T gx,
    T* __restrict__ A, T* __restrict__ B) {
  const int64_t ix = (int64_t)blockIdx.x * kFlowBlock + threadIdx.x;
  const int row = blockIdx.y;  // ky + K, 0 .. 2K
  const int64_t s = blockIdx.z;
  if (ix >= nx) return;
  const int nky = 2 * K + 1;
  const float* c = coef + ((size_t)s * nky + row) * (K + 1) * 2;
  T ar = 0, ai = 0, br = 0, bi = 0;
  for (int kx = 0; kx <= K; ++kx) {
    T cs, sn;
    phase(kx, ix, nx, &cs, &sn);
    const T cr = (T)c[2 * kx], ci = (T)c[2 * kx + 1];
    const T er = cr * cs - ci * sn, ei = cr * sn + ci * cs;  // c e^{i th}
    ar += er;
    ai += ei;
    // (-i gx kx)(er + i ei) = gx kx (ei - i er)
    br += gx * (T)kx * ei;
    bi -= gx * (T)kx * er;
  }
  const size_t o = (((size_t)s * nky + row) * nx + ix) * 2;
  A[o] = ar;
  A[o + 1] = ai;
  B[o] = br;
  B[o + 1] = bi;
}

// 2D, pass 2 (along y): one block row per (slice, iy);
//   u_x(ix, iy) = Re sum_ky (i gy ky) A[ky][ix] e^{2 pi i ky iy / ny}
//   u_y(ix, iy) = Re sum_ky B[ky][ix] e^{2 pi i ky iy / ny}
template <typename T>
__global__ __launch_bounds__(kFlowBlock) void k_flow2d_y(
    const T* __restrict__ A, const T* __restrict__ B, int K, int64_t nx,
    int64_t ny, T gy, T* __restrict__ u) {
  __shared__ T tw[2 * 129];  // twiddles of this row, K <= 64
  const int64_t iy = blockIdx.y;
  const int64_t s = blockIdx.z;
  const int nky = 2 * K + 1;
  for (int r = threadIdx.x; r < nky; r += kFlowBlock) {
    T cs, sn;
    phase(r - K, iy, ny, &cs, &sn);
    tw[2 * r] = cs;
    tw[2 * r + 1] = sn;
  }
  __syncthreads();
  const int64_t ix = (int64_t)blockIdx.x * kFlowBlock + threadIdx.x;
  if (ix >= nx) return;
  T ux = 0, uy = 0;
  for (int r = 0; r < nky; ++r) {
    const size_t o = (((size_t)s * nky + r) * nx + ix) * 2;
    const T cs = tw[2 * r], sn = tw[2 * r + 1];
    // Re((i gy ky)(ar + i ai)(cs + i sn)) = -gy ky (ai cs + ar sn)
    ux -= gy * (T)(r - K) * (A[o + 1] * cs + A[o] * sn);
    // Re((br + i bi)(cs + i sn)) = br cs - bi sn
    uy += B[o] * cs - B[o + 1] * sn;
  }
  const size_t plane = (size_t)nx * ny;
  u[((size_t)s * 2) * plane + iy * nx + ix] = ux;
  u[((size_t)s * 2 + 1) * plane + iy * nx + ix] = uy;
}

template <typename T>
hipError_t flow2d(const float* coef, int K, int64_t nx, int64_t ny, double dx,
                  int64_t ns, T* u, hipStream_t st) {
  const int nky = 2 * K + 1;
  T* work = nullptr;
  const size_t n = (size_t)ns * nky * nx * 2;
  hipError_t e = hipMallocAsync((void**)&work, 2 * n * sizeof(T), st);
  if (e != hipSuccess) return e;
  const T gx = (T)(2.0 * M_PI / ((double)nx * dx));
  const T gy = (T)(2.0 * M_PI / ((double)ny * dx));
  const unsigned bx = (unsigned)((nx + kFlowBlock - 1) / kFlowBlock);
  hipLaunchKernelGGL(k_flow2d_x<T>, dim3(bx, nky, (unsigned)ns),
                     dim3(kFlowBlock), 0, st, coef, K, nx, gx, work, work + n);
  hipLaunchKernelGGL(k_flow2d_y<T>, dim3(bx, (unsigned)ny, (unsigned)ns),
                     dim3(kFlowBlock), 0, st, work, work + n, K, nx, ny, gy, u);
  e = hipGetLastError();
  const hipError_t f = hipFreeAsync(work, st);
  return e != hipSuccess ? e : f;
}

}  // namespace
}  // namespace lat

extern "C" {

int lattice_flow1d_modes(lattice_t* L, int32_t nmodes, const float* coef,
                         int64_t n_slices, void* u) {
  if (!L) return LATTICE_EINVAL;
  const lattice_desc& d = L->d;
  if (d.dim != 1 || !coef || !u || nmodes < 1 || n_slices < 1 ||
      n_slices > 65535)
    return LATTICE_EINVAL;
  const dim3 grid((unsigned)((d.nx + lat::kFlowBlock - 1) / lat::kFlowBlock),
                  (unsigned)n_slices);
  if (d.dtype == LATTICE_F64)
    hipLaunchKernelGGL(lat::k_flow1d<double>, grid, dim3(lat::kFlowBlock), 0,
                       L->stream, coef, nmodes, (int64_t)d.nx, (double*)u);
  else
    hipLaunchKernelGGL(lat::k_flow1d<float>, grid, dim3(lat::kFlowBlock), 0,
                       L->stream, coef, nmodes, (int64_t)d.nx, (float*)u);
  return hipGetLastError() == hipSuccess ? LATTICE_OK : LATTICE_EHIP;
}

int lattice_flow2d_modes(lattice_t* L, int32_t kmax, const float* coef,
                         int64_t n_slices, void* u) {
  if (!L) return LATTICE_EINVAL;
  const lattice_desc& d = L->d;
  if (d.dim != 2 || !coef || !u || kmax < 1 || kmax > 64 || n_slices < 1 ||
      n_slices > 65535 || d.ny > 65535 || 2 * kmax >= d.nx ||
      2 * kmax >= d.ny)
    return LATTICE_EINVAL;
  const hipError_t e =
      d.dtype == LATTICE_F64
          ? lat::flow2d<double>(coef, kmax, d.nx, d.ny, d.dx, n_slices,
                                (double*)u, L->stream)
          : lat::flow2d<float>(coef, kmax, d.nx, d.ny, d.dx, n_slices,
                               (float*)u, L->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return LATTICE_EHIP;
  }
  return LATTICE_OK;
}

}  // extern "C"
