// s1.hip -- Eulerian first-order velocity structure function of the
// phase-space density (Eq. 11, Sec. 3.1), gfx950.
//
//   S1(r) = < sum_{j,j'} f_j(x) f_j'(x + r) |v_j - v_j'| >_x
//           / < sum_{j,j'} f_j(x) f_j'(x + r) >_x.
//
// With h_j(y) = sum_j' |v_j - v_j'| f_j'(y) (velocity units of dv), the
// numerator is < sum_j f_j(x) h_j(x + r) >_x and the denominator
// < rho(x) rho(x + r) >_x (rho = sum_j f_j; every dv factor but the one of
// |v - v'| cancels).  1D: h by a direct sum over j' per site.  2D:
// |v_J - v_J'| = dv |J - J'| (Euclidean on the velocity square), so h is
// the product of the state (sites x nv^2) with the fixed nv^2 x nv^2 matrix
// of index distances -- a plain GEMM, done by rocBLAS.  The correlation
// sums for each requested separation are FP64 with fixed-order reductions.
// In 2D the separation r is taken along x and along y and the two
// estimates are averaged.
#include <math.h>

#include <rocblas/rocblas.h>

#include "../../include/lattice.h"
#include "lattice_struct.h"

namespace lat {
namespace {

constexpr int kS1Block = 256;

// 1D: h[j][x] = sum_j' |j - j'| f[j'][x]
template <typename T>
__global__ __launch_bounds__(kS1Block) void k_s1_h1d(const T* __restrict__ f,
                                                     int64_t nx, int nv,
                                                     T* __restrict__ h) {
  const int64_t x = (int64_t)blockIdx.x * kS1Block + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= nx) return;
  T acc = 0;
  for (int jp = 0; jp < nv; ++jp)
    acc += (T)(jp > j ? jp - j : j - jp) * f[(size_t)jp * nx + x];
  h[(size_t)j * nx + x] = acc;
}

// 2D distance matrix D[J'][J] = |J - J'| on the nv x nv index square
template <typename T>
__global__ __launch_bounds__(kS1Block) void k_s1_dist(int nv, T* __restrict__ D) {
  const int64_t n2 = (int64_t)nv * nv;
  const int64_t i = (int64_t)blockIdx.x * kS1Block + threadIdx.x;
  if (i >= n2 * n2) return;
  const int64_t a = i / n2, b = i - a * n2;
  const int ay = (int)(a / nv), ax = (int)(a - ay * nv);
  const int by = (int)(b / nv), bx = (int)(b - by * nv);
  const double dxv = ax - bx, dyv = ay - by;
  D[i] = (T)sqrt(dxv * dxv + dyv * dyv);
}

__device__ void block_sum2(double& a, double& b, double* sa, double* sb) {
  const int t = (int)threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
#pragma unroll
  for (int w = kS1Block / 2; w > 0; w >>= 1) {
    if (t < w) {
      sa[t] += sa[t + w];
      sb[t] += sb[t + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

// Partial sums over a block of sites of (sum_J f_J(x) h_J(x'), rho(x)
// rho(x')) with x' = x shifted by r along x (axis 0) or y (axis 1),
// periodic.  partial[(k * 2 + axis) * nblocks + block][2].
template <typename T>
__global__ __launch_bounds__(kS1Block) void k_s1_corr(
    const T* __restrict__ f, int64_t fpitch, const T* __restrict__ h,
    int64_t nx, int64_t ny, int nplanes, const int32_t* __restrict__ rs,
    int naxes, double* __restrict__ partial) {
  __shared__ double sa[kS1Block], sb[kS1Block];
  const int64_t sites = nx * ny;
  const int64_t i = (int64_t)blockIdx.x * kS1Block + threadIdx.x;
  const int k = blockIdx.y / naxes, axis = blockIdx.y - k * naxes;
  const int64_t r = rs[k];
  double num = 0.0, den = 0.0;
  if (i < sites) {
    const int64_t y = i / nx, x = i - y * nx;
    int64_t j;
    if (axis == 0) {
      int64_t xs = (x + r) % nx;
      j = y * nx + xs;
    } else {
      int64_t ys = (y + r) % ny;
      j = ys * nx + x;
    }
    double ra = 0.0, rb = 0.0;
    for (int J = 0; J < nplanes; ++J) {
      const double a = (double)f[(size_t)J * fpitch + i];
      num += a * (double)h[(size_t)J * sites + j];
      ra += a;
      rb += (double)f[(size_t)J * fpitch + j];
    }
    den = ra * rb;
  }
  block_sum2(num, den, sa, sb);
  if (threadIdx.x == 0) {
    const size_t o = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
    partial[o] = num;
    partial[o + 1] = den;
  }
}

// One block per (separation, axis): fixed-order sum of the partials.
__global__ __launch_bounds__(kS1Block) void k_s1_final(
    const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  __shared__ double sa[kS1Block], sb[kS1Block];
  const double* p = partial + (size_t)blockIdx.x * nblocks * 2;
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < nblocks; j += kS1Block) {
    a += p[2 * j];
    b += p[2 * j + 1];
  }
  block_sum2(a, b, sa, sb);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = a;
    out[2 * blockIdx.x + 1] = b;
  }
}

}  // namespace
}  // namespace lat

extern "C" int lattice_s1(lattice_t* L, const void* f, double dt, int32_t nr,
                          const int32_t* r, double* out) {
  if (!L) return LATTICE_EINVAL;
  const lattice_desc& d = L->d;
  if (!f || !r || !out || nr < 1 || nr > 4096 || !(dt > 0.0) ||
      !isfinite(dt))
    return LATTICE_EINVAL;
  for (int k = 0; k < nr; ++k)
    if (r[k] < 0) return LATTICE_EINVAL;
  const bool f64 = d.dtype == LATTICE_F64;
  const size_t el = f64 ? 8 : 4;
  const int64_t sites = L->sites;
  const int naxes = d.dim == 2 ? 2 : 1;
  const int nb = (int)((sites + lat::kS1Block - 1) / lat::kS1Block);
  const int64_t np = L->nplanes;
  hipStream_t st = L->stream;
  // workspace: h (state-sized), the distance matrix (2D), separations,
  // partials and the per-(separation, axis) sums
  const size_t nD = d.dim == 2 ? (size_t)np * np : 0;
  const size_t bytes = el * ((size_t)L->cells + nD) + sizeof(int32_t) * nr +
                       sizeof(double) * 2 * ((size_t)nr * naxes * nb +
                                             (size_t)nr * naxes) +
                       64;
  char* w = nullptr;
  if (hipMalloc((void**)&w, bytes) != hipSuccess) return LATTICE_ENOMEM;
  void* h = w;
  void* D = w + el * (size_t)L->cells;
  int32_t* dr = (int32_t*)(w + el * ((size_t)L->cells + nD));
  double* partial =
      (double*)(((uintptr_t)(dr + nr) + 15) & ~(uintptr_t)15);
  double* sums = partial + 2 * (size_t)nr * naxes * nb;
  int rc = LATTICE_OK;
  rocblas_handle handle = nullptr;
  hipError_t e = hipMemcpyAsync(dr, r, sizeof(int32_t) * nr,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess && d.dim == 1) {
    const dim3 g((unsigned)((d.nx + lat::kS1Block - 1) / lat::kS1Block),
                 (unsigned)d.nv);
    if (f64)
      hipLaunchKernelGGL(lat::k_s1_h1d<double>, g, dim3(lat::kS1Block), 0, st,
                         (const double*)f, (int64_t)d.nx, d.nv, (double*)h);
    else
      hipLaunchKernelGGL(lat::k_s1_h1d<float>, g, dim3(lat::kS1Block), 0, st,
                         (const float*)f, (int64_t)d.nx, d.nv, (float*)h);
    e = hipGetLastError();
  } else if (e == hipSuccess) {
    const unsigned gd = (unsigned)((nD + lat::kS1Block - 1) / lat::kS1Block);
    if (f64)
      hipLaunchKernelGGL(lat::k_s1_dist<double>, dim3(gd), dim3(lat::kS1Block),
                         0, st, d.nv, (double*)D);
    else
      hipLaunchKernelGGL(lat::k_s1_dist<float>, dim3(gd), dim3(lat::kS1Block),
                         0, st, d.nv, (float*)D);
    e = hipGetLastError();
    // column-major view: F (sites x np, ld = the plane pitch), D (np x np),
    // h = F D (sites x np, ld sites)
    if (e == hipSuccess &&
        (rocblas_create_handle(&handle) != rocblas_status_success ||
         rocblas_set_stream(handle, st) != rocblas_status_success))
      rc = LATTICE_EHIP;
    if (rc == LATTICE_OK && e == hipSuccess) {
      rocblas_status bs;
      if (f64) {
        const double one = 1.0, zero = 0.0;
        bs = rocblas_dgemm(handle, rocblas_operation_none,
                           rocblas_operation_none, (rocblas_int)sites,
                           (rocblas_int)np, (rocblas_int)np, &one,
                           (const double*)f, (rocblas_int)L->pitch,
                           (const double*)D, (rocblas_int)np, &zero,
                           (double*)h, (rocblas_int)sites);
      } else {
        const float one = 1.f, zero = 0.f;
        bs = rocblas_sgemm(handle, rocblas_operation_none,
                           rocblas_operation_none, (rocblas_int)sites,
                           (rocblas_int)np, (rocblas_int)np, &one,
                           (const float*)f, (rocblas_int)L->pitch,
                           (const float*)D, (rocblas_int)np, &zero,
                           (float*)h, (rocblas_int)sites);
      }
      if (bs != rocblas_status_success) rc = LATTICE_EHIP;
    }
  }
  if (e != hipSuccess) rc = LATTICE_EHIP;
  if (rc == LATTICE_OK) {
    const dim3 g((unsigned)nb, (unsigned)(nr * naxes));
    if (f64)
      hipLaunchKernelGGL(lat::k_s1_corr<double>, g, dim3(lat::kS1Block), 0, st,
                         (const double*)f, L->pitch, (const double*)h,
                         (int64_t)d.nx,
                         (int64_t)(d.dim == 2 ? d.ny : 1), (int)np, dr, naxes,
                         partial);
    else
      hipLaunchKernelGGL(lat::k_s1_corr<float>, g, dim3(lat::kS1Block), 0, st,
                         (const float*)f, L->pitch, (const float*)h,
                         (int64_t)d.nx,
                         (int64_t)(d.dim == 2 ? d.ny : 1), (int)np, dr, naxes,
                         partial);
    hipLaunchKernelGGL(lat::k_s1_final, dim3((unsigned)(nr * naxes)),
                       dim3(lat::kS1Block), 0, st, partial, nb, sums);
    e = hipGetLastError();
  }
  double* hs = nullptr;
  if (rc == LATTICE_OK && e == hipSuccess) {
    hs = new double[2 * (size_t)nr * naxes];
    e = hipMemcpyAsync(hs, sums, sizeof(double) * 2 * nr * naxes,
                       hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    rc = LATTICE_EHIP;
  }
  if (rc == LATTICE_OK) {
    const double dv = (double)d.vstride * d.dx / dt;
    for (int k = 0; k < nr; ++k) {
      double s = 0.0;
      for (int a = 0; a < naxes; ++a) {
        const double* q = hs + 2 * ((size_t)k * naxes + a);
        s += dv * q[0] / q[1];
      }
      out[k] = s / naxes;
      if (!isfinite(out[k])) rc = LATTICE_ENONFINITE;
    }
  }
  delete[] hs;
  if (handle) rocblas_destroy_handle(handle);
  (void)hipFree(w);
  return rc;
}
