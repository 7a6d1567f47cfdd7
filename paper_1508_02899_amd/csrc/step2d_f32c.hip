// step2d_f32c.hip -- FP32 2D pass instantiations for nv = 25, 33.
#include "step2d.h"

namespace lat {
hipError_t step2d_f32_c(const StepArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 25: return launch_step2d_nv<float, 25, 4>(a, s);
    case 33: return launch_step2d_nv<float, 33, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace lat
