// dirac_sweep2d_obs.hip -- the 2-D lowest-order passes that also sum the
// observables of the state they store (instances of k_sweep2d_obs; see
// dirac_sweep2d_kernels.h)
#include "dirac_sweep2d_kernels.h"

namespace dirac {

template <typename T, int K>
static const void* obs_mode(int mode) {
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_sweep2d_obs<T, K, 0>);
    case 1: return reinterpret_cast<const void*>(&k_sweep2d_obs<T, K, 1>);
    case 2: return reinterpret_cast<const void*>(&k_sweep2d_obs<T, K, 2>);
    default: return nullptr;
  }
}

template <typename T>
static const void* obs_depth(int depth, int mode) {
  switch (depth) {
    case 1: return obs_mode<T, 1>(mode);
    case 2: return obs_mode<T, 2>(mode);
    case 3: return obs_mode<T, 3>(mode);
    case 4: return obs_mode<T, 4>(mode);
    case 5: return obs_mode<T, 5>(mode);
    default: return nullptr;
  }
}

const void* kernel2d_obs(bool fp64, int depth, int mode) {
  return fp64 ? obs_depth<double>(depth, mode) : obs_depth<float>(depth, mode);
}

}  // namespace dirac
