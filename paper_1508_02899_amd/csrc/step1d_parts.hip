// step1d_parts.hip -- fused streaming + collision pass for 1D lattices with
// each site's velocity column split over P lanes (gfx950).
//
// The one-lane-per-site pass (step1d.hip) gives nx lanes: a short lattice
// (a few thousand to tens of thousands of sites) then leaves most of the
// chip idle.  Here P lanes share a column and a workgroup updates a tile of
// G consecutive sites through LDS (parts1d.h).
#include "lattice_internal.h"
#include "parts1d.h"

namespace lat {
namespace {

template <typename T, int NV, int P, int WGW, bool KOREN>
__global__ __launch_bounds__(64 * WGW) void k_step1d_parts(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int step_mod, int init_off,
    int jump, int nsub, T alpha_scale, T beta, T D, int nblocks) {
  using C = Parts1D<T, NV, P, WGW>;
  __shared__ T tile[C::SIZE];
  if (*flag != 0) return;  // uniform over the grid
  const int xg = xcd_remap(blockIdx.x, nblocks);
  parts1d_tile<T, NV, P, WGW, KOREN>(fin, fout, u, tile, nx, nx, xg * C::G,
                                     step_mod, init_off, jump, nsub,
                                     alpha_scale, beta, D);
}

template <typename T, int NV>
hipError_t launch_nv(const StepArgs& a, hipStream_t s) {
  constexpr int P = PartsShape<T, NV>::P, WGW = PartsShape<T, NV>::WGW;
  constexpr int G = Parts1D<T, NV, P, WGW>::G;
  const int nx = (int)a.nx;
  const int nblocks = (nx + G - 1) / G;
  const int h = (NV - 1) / 2;
  const int step_mod = a.shift % nx;
  const int init_off = (int)(((int64_t)a.shift * h) % nx);
  const int jump = (int)(((int64_t)P * step_mod) % nx);
  const T as = (T)a.alpha_scale, be = (T)a.beta, D = (T)a.D;
  if (a.koren)
    hipLaunchKernelGGL((k_step1d_parts<T, NV, P, WGW, true>), dim3(nblocks),
                       dim3(64 * WGW), 0, s, (const T*)a.fin, (T*)a.fout,
                       (const T*)a.u, a.flag, nx, step_mod, init_off, jump,
                       a.nsub_inline, as, be, D, nblocks);
  else
    hipLaunchKernelGGL((k_step1d_parts<T, NV, P, WGW, false>), dim3(nblocks),
                       dim3(64 * WGW), 0, s, (const T*)a.fin, (T*)a.fout,
                       (const T*)a.u, a.flag, nx, step_mod, init_off, jump,
                       a.nsub_inline, as, be, D, nblocks);
  return hipGetLastError();
}

}  // namespace

bool step1d_parts_supported(int nv, int f64) {
  return nv == 17 || nv == 33 || nv == 65 || (nv == 129 && !f64);
}

hipError_t launch_step1d_parts(const StepArgs& a, hipStream_t s) {
  if (!step1d_parts_supported(a.nv, a.f64) || a.nx < 1 ||
      a.nx > 0x7FFFFFFF)
    return hipErrorInvalidValue;
  if (a.f64) {
    switch (a.nv) {
      case 17: return launch_nv<double, 17>(a, s);
      case 33: return launch_nv<double, 33>(a, s);
      default: return launch_nv<double, 65>(a, s);
    }
  }
  switch (a.nv) {
    case 17: return launch_nv<float, 17>(a, s);
    case 33: return launch_nv<float, 33>(a, s);
    case 65: return launch_nv<float, 65>(a, s);
    default: return launch_nv<float, 129>(a, s);
  }
}

}  // namespace lat
