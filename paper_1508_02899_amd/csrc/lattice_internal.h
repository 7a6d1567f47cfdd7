// lattice_internal.h -- launch interfaces between the C-ABI host code and
// the HIP kernels of the phase-space lattice library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// One streaming + collision pass over the whole lattice (Sec. 2 of the
// paper: exact streaming, then drift, then diffusion).  shift = 0 gives a
// collision-only pass (used for the extra sub-steps when nsub > 1).
struct StepArgs {
  const void* fin;   // state before the pass
  void* fout;        // state after the pass (distinct from fin)
  const void* u;     // flow slice for this pass: [dim][ny][nx]
  const int* flag;   // sticky device flag: nonzero -> pass is a no-op
  int64_t nx, ny;
  int64_t pitch;     // elements between velocity planes of fin / fout
  int nv;
  int shift;         // cells moved per velocity index (vstride or 0)
  int nsub_inline;   // 1D only: collision sub-steps done inside the pass
  double alpha_scale;  // dt_s / (dv tau_p): drift of cell j in cell widths
  double beta;         // dt_s / tau_p       is alpha_scale*u - beta*(j-h)
  double D;            // kappa dt_s / dv^2
  int koren;
  int f64;
};

// Which velocity lattices have a compiled kernel.
bool step1d_supported(int nv, int f64);
bool step2d_supported(int nv, int f64);
// The 2D kernel addresses one vy row (nv planes, plane pitch elements
// apart) with 32-bit byte offsets from the row's base (lattice_init already
// caps a row below 2^31 bytes; the launcher re-checks).
inline bool step2d_offsets_fit(int nv, int64_t pitch, size_t elem) {
  return (uint64_t)nv * (uint64_t)pitch * elem < 0xFFFFFFFFull;
}

hipError_t launch_step1d(const StepArgs& a, hipStream_t s);
// The split-column 1D pass (P lanes per site) for the velocity lattices it
// is compiled for; launch_step1d picks it for short lattices.
bool step1d_parts_supported(int nv, int f64);
hipError_t launch_step1d_parts(const StepArgs& a, hipStream_t s);
hipError_t launch_step2d(const StepArgs& a, hipStream_t s);

// Sticky CFL / finiteness check of the u slices: sets flag |= 1 when some
// |u| exceeds umax_ok (strict: |u| >= umax_ok) or is not finite.
hipError_t launch_cfl_check(const void* u, int64_t n, double umax_ok,
                            int strict, int f64, int* flag, hipStream_t s);
// max |u| over n values into *out (FP64 on device, reset inside).
hipError_t launch_absmax(const void* u, int64_t n, int f64, double* out,
                         hipStream_t s);

// FP64 sums of every velocity plane (plane_sums[nplanes]; planes pitch
// elements apart) followed by the weighted combination into
// out[6] = {M, Px, Py, Qx, Qy, variance}; out[6] = the sticky flag's value
// (so that one copy brings both back).
hipError_t launch_moments(const void* f, int64_t sites, int64_t pitch,
                          int nv, int dim, int f64, double w, double dv,
                          double* plane_sums, const int* flag, double* out,
                          hipStream_t s);
// rho[site] = dvd * sum_j f[j][site] in FP64.
// <rho_r^2> on tilings r = 2^k sites, k = 0..levels-1 (observables.hip).
constexpr int kRhoMaxLevels = 32;
int64_t rho_r2_partials(int dim, int64_t nx, int64_t ny, int levels);
hipError_t launch_rho_r2(const double* rho, int dim, int64_t nx, int64_t ny,
                         int levels, double* work, double* partial,
                         double* out, hipStream_t s);
hipError_t launch_density(const void* f, int64_t sites, int64_t pitch,
                          int nplanes, int f64, double dvd, double* rho,
                          hipStream_t s);

hipError_t launch_copy(void* dst, const void* src, int64_t bytes,
                       hipStream_t s);
hipError_t launch_clear_flag(int* flag, hipStream_t s);
// *status = *flag (stream-ordered; a kernel, so that it can be captured).
hipError_t launch_flag_out(const int* flag, int32_t* status, hipStream_t s);

}  // namespace lat
