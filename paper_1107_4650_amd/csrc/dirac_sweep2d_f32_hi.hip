// dirac_sweep2d_f32_hi.hip -- FP32-state lowest-order passes of 3 to 5 steps
// (instances of the 1-D / 2-D fused-pass kernel; see dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

const void* kernel2d_lie_f32_hi(int depth, int axes_code, int mode, int nc) {
  switch (depth) {
    case 3: return kernel2d_axes<float, LieStep, 3>(axes_code, mode, nc);
    case 4: return kernel2d_axes<float, LieStep, 4>(axes_code, mode, nc);
    case 5: return kernel2d_axes<float, LieStep, 5>(axes_code, mode, nc);
    default: return nullptr;
  }
}

}  // namespace dirac
