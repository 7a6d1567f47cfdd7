// step2d_f64.hip -- FP64 2D pass instantiations.
#include "step2d.h"

namespace lat {
hipError_t step2d_f64(const StepArgs& a, hipStream_t s) {
  switch (a.nv) {
    case 3: return launch_step2d_nv<double, 3, 1>(a, s);
    case 5: return launch_step2d_nv<double, 5, 1>(a, s);
    case 9: return launch_step2d_nv<double, 9, 2>(a, s);
    case 17: return launch_step2d_nv<double, 17, 4>(a, s);
    case 33: return launch_step2d_nv<double, 33, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace lat
