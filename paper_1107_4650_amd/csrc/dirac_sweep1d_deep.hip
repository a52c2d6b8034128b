// dirac_sweep1d_deep.hip -- 1-D lowest-order passes of kDeep1D steps
// (instances of the 1-D / 2-D fused-pass kernel; see dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

template <typename T, int AX, int NC>
static const void* deep_mode(int mode) {
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_sweep2d<T, LieStep, kDeep1D, AX, -1, 0, NC>);
    case 1: return reinterpret_cast<const void*>(&k_sweep2d<T, LieStep, kDeep1D, AX, -1, 1, NC>);
    case 2: return reinterpret_cast<const void*>(&k_sweep2d<T, LieStep, kDeep1D, AX, -1, 2, NC>);
    default: return nullptr;
  }
}

template <typename T, int NC>
static const void* deep_axis(int axis, int mode) {
  switch (axis) {
    case 0: return deep_mode<T, 0, NC>(mode);
    case 1: return deep_mode<T, 1, NC>(mode);
    case 2: return deep_mode<T, 2, NC>(mode);
    default: return nullptr;
  }
}

template <typename T>
static const void* deep_nc(int axis, int mode, int nc) {
  if (nc == 2) return deep_axis<T, 2>(axis, mode);
  if (nc == 4) return deep_axis<T, 4>(axis, mode);
  return nullptr;
}

const void* kernel1d_deep(bool fp64, int axis, int mode, int nc) {
  return fp64 ? deep_nc<double>(axis, mode, nc) : deep_nc<float>(axis, mode, nc);
}

}  // namespace dirac
