// dirac_sweep2d_strang.hip -- second-order passes of 1 to 3 steps, both state types
// (instances of the 1-D / 2-D fused-pass kernel; see dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

const void* kernel2d_strang(bool fp64, int depth, int axes_code, int mode, int nc) {
  if (fp64) {
    switch (depth) {
      case 1: return kernel2d_axes<double, StrangStep, 1>(axes_code, mode, nc);
      case 2: return kernel2d_axes<double, StrangStep, 2>(axes_code, mode, nc);
      case 3: return kernel2d_axes<double, StrangStep, 3>(axes_code, mode, nc);
      default: return nullptr;
    }
  }
  switch (depth) {
    case 1: return kernel2d_axes<float, StrangStep, 1>(axes_code, mode, nc);
    case 2: return kernel2d_axes<float, StrangStep, 2>(axes_code, mode, nc);
    case 3: return kernel2d_axes<float, StrangStep, 3>(axes_code, mode, nc);
    default: return nullptr;
  }
}

}  // namespace dirac
