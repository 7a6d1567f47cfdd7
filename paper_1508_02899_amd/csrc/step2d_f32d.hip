// step2d_f32d.hip -- FP32 2D pass instantiation for nv = 65.
#include "step2d.h"

namespace lat {
hipError_t step2d_f32_d(const StepArgs& a, hipStream_t s) {
  switch (a.nv) {
    // 8 parts of 9 cells: the register footprint of the nv = 33 kernel
    // (2 waves per SIMD; 4 parts of 17 cells left one)
    case 65: return launch_step2d_nv<float, 65, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace lat
