// dirac_sweep2d_f64_lo.hip -- FP64-state lowest-order passes of 1 and 2 steps
// (instances of the 1-D / 2-D fused-pass kernel; see dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

const void* kernel2d_lie_f64_lo(int depth, int axes_code, int mode, int nc) {
  switch (depth) {
    case 1: return kernel2d_axes<double, LieStep, 1>(axes_code, mode, nc);
    case 2: return kernel2d_axes<double, LieStep, 2>(axes_code, mode, nc);
    default: return nullptr;
  }
}

}  // namespace dirac
