// step2d_dispatch.hip -- picks the compiled 2D pass for (nv, dtype).
#include "lattice_internal.h"

namespace lat {
hipError_t step2d_f32_a(const StepArgs& a, hipStream_t s);
hipError_t step2d_f32_b(const StepArgs& a, hipStream_t s);
hipError_t step2d_f32_c(const StepArgs& a, hipStream_t s);
hipError_t step2d_f32_d(const StepArgs& a, hipStream_t s);
hipError_t step2d_f64(const StepArgs& a, hipStream_t s);

bool step2d_supported(int nv, int f64) {
  if (f64) return nv == 3 || nv == 5 || nv == 9 || nv == 17 || nv == 33;
  if (nv >= 3 && nv <= 21 && (nv & 1)) return true;
  return nv == 25 || nv == 33 || nv == 65;
}

hipError_t launch_step2d(const StepArgs& a, hipStream_t s) {
  if (!step2d_supported(a.nv, a.f64) || a.nx < 1 || a.ny < 1)
    return hipErrorInvalidValue;
  if (a.f64) return step2d_f64(a, s);
  if (a.nv <= 11) return step2d_f32_a(a, s);
  if (a.nv <= 21) return step2d_f32_b(a, s);
  if (a.nv <= 33) return step2d_f32_c(a, s);
  return step2d_f32_d(a, s);
}
}  // namespace lat
