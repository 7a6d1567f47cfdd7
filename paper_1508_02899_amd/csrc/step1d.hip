// step1d.hip -- fused streaming + collision pass for 1D lattices (gfx950).
//
// One lane owns one spatial site and holds that site's whole velocity
// column (capacity CAP >= nv, runtime nv) in registers:
//   1. pull streaming (Sec. 2 of the paper): cell j of site x comes from
//      site x - shift*(j-h); for a fixed j the lanes of a wavefront read
//      consecutive addresses, so every load is one coalesced 256-byte run;
//   2. nsub_inline times: drift (Eq. 5 force at cell centres, upwind or
//      Koren-limited split fluxes, zero flux at the two outer faces), then
//      diffusion (finite-difference face fluxes, Eq. 4);
//   3. coalesced stores of the column to the output state.
// Each state element is read once and written once per pass.
#include "column1d.h"
#include "lattice_internal.h"

namespace lat {
namespace {

template <typename T, int CAP, bool KOREN>
__global__ __launch_bounds__(256) void k_step1d(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int nv, int h, int step_mod,
    int init_off, int nsub, T alpha_scale, T beta, T D, int nblocks) {
  if (*flag != 0) return;
  const int b = xcd_remap(blockIdx.x, nblocks);
  const int x = b * 256 + (int)threadIdx.x;
  if (x >= nx) return;
  column1d<T, CAP, KOREN>(fin, fout, x, nx, nx, nv, h, step_mod, init_off, nsub,
                          u[x] * alpha_scale, beta, D);
}

template <typename T, int CAP>
hipError_t launch_cap(const StepArgs& a, hipStream_t s) {
  const int nx = (int)a.nx;
  const int nblocks = (nx + 255) / 256;
  const int h = (a.nv - 1) / 2;
  const int step_mod = a.shift % nx;
  const int init_off = (int)(((int64_t)a.shift * h) % nx);
  const T as = (T)a.alpha_scale, be = (T)a.beta, D = (T)a.D;
  if (a.koren)
    hipLaunchKernelGGL((k_step1d<T, CAP, true>), dim3(nblocks), dim3(256), 0,
                       s, (const T*)a.fin, (T*)a.fout, (const T*)a.u, a.flag,
                       nx, a.nv, h, step_mod, init_off, a.nsub_inline, as, be,
                       D, nblocks);
  else
    hipLaunchKernelGGL((k_step1d<T, CAP, false>), dim3(nblocks), dim3(256), 0,
                       s, (const T*)a.fin, (T*)a.fout, (const T*)a.u, a.flag,
                       nx, a.nv, h, step_mod, init_off, a.nsub_inline, as, be,
                       D, nblocks);
  return hipGetLastError();
}

hipError_t launch_f32(const StepArgs& a, hipStream_t s) {
  if (a.nv <= 9) return launch_cap<float, 9>(a, s);
  if (a.nv <= 17) return launch_cap<float, 17>(a, s);
  if (a.nv <= 33) return launch_cap<float, 33>(a, s);
  if (a.nv <= 65) return launch_cap<float, 65>(a, s);
  return launch_cap<float, 129>(a, s);
}

hipError_t launch_f64(const StepArgs& a, hipStream_t s) {
  if (a.nv <= 9) return launch_cap<double, 9>(a, s);
  if (a.nv <= 17) return launch_cap<double, 17>(a, s);
  if (a.nv <= 33) return launch_cap<double, 33>(a, s);
  return launch_cap<double, 65>(a, s);
}

}  // namespace

bool step1d_supported(int nv, int f64) {
  return nv >= 3 && (nv & 1) && nv <= (f64 ? 65 : 129);
}

// Up to this many sites the split-column pass (step1d_parts.hip) runs
// instead: it keeps P lanes per site busy where one lane per site would
// leave most of the chip idle.
constexpr int64_t kPartsMaxSites = 1 << 19;

hipError_t launch_step1d(const StepArgs& a, hipStream_t s) {
  if (!step1d_supported(a.nv, a.f64) || a.nx < 1) return hipErrorInvalidValue;
  if (a.nx <= kPartsMaxSites && step1d_parts_supported(a.nv, a.f64))
    return launch_step1d_parts(a, s);
  return a.f64 ? launch_f64(a, s) : launch_f32(a, s);
}

}  // namespace lat
