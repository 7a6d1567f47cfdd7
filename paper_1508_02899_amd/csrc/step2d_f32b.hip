// step2d_f32b.hip -- FP32 2D pass instantiations for nv = 13..21.
#include "step2d.h"

namespace lat {
hipError_t step2d_f32_b(const StepArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 13: return launch_step2d_nv<float, 13, 2>(a, s);
    case 15: return launch_step2d_nv<float, 15, 2>(a, s);
    case 17: return launch_step2d_nv<float, 17, 2>(a, s);
    case 19: return launch_step2d_nv<float, 19, 2>(a, s);
    case 21: return launch_step2d_nv<float, 21, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace lat
