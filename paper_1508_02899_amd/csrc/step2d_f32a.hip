// step2d_f32a.hip -- FP32 2D pass instantiations for nv = 3..11.
#include "step2d.h"

namespace lat {
hipError_t step2d_f32_a(const StepArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 3: return launch_step2d_nv<float, 3, 1>(a, s);
    case 5: return launch_step2d_nv<float, 5, 1>(a, s);
    case 7: return launch_step2d_nv<float, 7, 1>(a, s);
    case 9: return launch_step2d_nv<float, 9, 1>(a, s);
    case 11: return launch_step2d_nv<float, 11, 2>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace lat
