// dirac_sweep2d_f64_hi.hip -- FP64-state lowest-order passes of 3 to 5 steps
// (instances of the 1-D / 2-D fused-pass kernel; see dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

const void* kernel2d_lie_f64_hi(int depth, int axes_code, int mode, int nc) {
  switch (depth) {
    case 3: return kernel2d_axes<double, LieStep, 3>(axes_code, mode, nc);
    case 4: return kernel2d_axes<double, LieStep, 4>(axes_code, mode, nc);
    case 5: return kernel2d_axes<double, LieStep, 5>(axes_code, mode, nc);
    default: return nullptr;
  }
}

}  // namespace dirac
