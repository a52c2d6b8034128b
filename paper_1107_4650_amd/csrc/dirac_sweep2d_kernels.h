// dirac_sweep2d_kernels.h -- the 1-D / 2-D fused-pass kernel template and the
// tables that map (layout, phase mode) to its instances.  Included by the
// translation units that instantiate one group of instances each (FP32 and
// FP64 lowest-order passes of 1-2 and 3-5 steps, second-order passes), so
// that they compile in parallel.  Internal to libdirac.
#pragma once
#include <type_traits>

#include "dirac_device.h"
#include "dirac_launch.h"
#include "dirac_sweep_impl.h"

namespace dirac {

// K full steps of scheme S per launch on a 1-D line or a 2-D plane (64 - 2X
// output columns per wave, X = x transports of the pass; march segments of
// H rows in 2-D)
template <typename T, class S, int K, int AX0, int AX1, int MODE, int NC = 4>
__global__ __launch_bounds__(256, sweep2d_min_blocks(sizeof(T) == 8, K, K * S::kStages, MODE))
void k_sweep2d(const T* __restrict__ src, T* __restrict__ dst, const double* __restrict__ V,
               SweepArgs a) {
  static_assert(NC == 4 || AX1 < 0, "two-component states are 1-D lines");
  constexpr int X = halo_lanes<S>(K);
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  const int64_t tile = blk * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  const int64_t strip = tile % a.nstrips;
  const int64_t seg = tile / a.nstrips;
  const int64_t xs = strip * strip_width(X) - X;  // lanes X .. 63 - X are written
  if constexpr (AX1 < 0) {
    one_row<T, S, K, AX0, MODE, NC>(src, dst, V, a, xs, lane, X);  // 1-D: one row, no march
  } else {
    const int64_t jb = seg * a.H;
    const int64_t je = (jb + a.H < a.ny) ? jb + a.H : a.ny;
    // even segments march up, odd ones down
    march_dir<T, S, K, AX0, AX1, MODE>(src, dst, V, a, xs, lane, jb, je, (seg & 1) == 0, X);
  }
}

// K lowest-order steps of a 2-D plane (grid axes 0 and 1, four components),
// as k_sweep2d, summing the observables of the cells the wave stores (each
// lane those of its column); the wave's totals (a fixed butterfly over its
// lanes) go to partials[tile], the Neumaier pairs of the kQ sums, for the
// final reduction in tile order
template <typename T, int K, int MODE>
__global__ __launch_bounds__(256, sweep2d_min_blocks(sizeof(T) == 8, K, K, MODE))
void k_sweep2d_obs(const T* __restrict__ src, T* __restrict__ dst, const double* __restrict__ V,
                   SweepArgs a, ObsArgs o, double* __restrict__ partials) {
  constexpr int X = halo_lanes<LieStep>(K);
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  const int64_t tile = blk * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  const int64_t strip = tile % a.nstrips;
  const int64_t seg = tile / a.nstrips;
  const int64_t xs = strip * strip_width(X) - X;
  const int64_t jb = seg * a.H;
  const int64_t je = (jb + a.H < a.ny) ? jb + a.H : a.ny;
  NSum acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = NSum{0.0, 0.0};
  march_dir<T, LieStep, K, 0, 1, MODE, true>(src, dst, V, a, xs, lane, jb, je, (seg & 1) == 0,
                                             X, acc, &o);
  obs_column_close(acc, xs + lane, o);  // lanes that stored nothing hold zeros
  wave_merge(acc);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      partials[(tile * kQ + q) * 2 + 0] = acc[q].s;
      partials[(tile * kQ + q) * 2 + 1] = acc[q].c;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers: the 1-D / 2-D kernel for (type, depth, axes, phase mode)
// ---------------------------------------------------------------------------
template <typename T, class S, int K, int AX0, int AX1, int NC>
const void* kernel2d_mode(int mode) {
  constexpr bool kField = NC == 4 &&
      K <= field_max_depth(sizeof(T) == 8, std::is_same<S, StrangStep>::value);
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_sweep2d<T, S, K, AX0, AX1, 0, NC>);
    case 1: return reinterpret_cast<const void*>(&k_sweep2d<T, S, K, AX0, AX1, 1, NC>);
    case 2: return reinterpret_cast<const void*>(&k_sweep2d<T, S, K, AX0, AX1, 2, NC>);
    case 3:
      if constexpr (kField)
        return reinterpret_cast<const void*>(&k_sweep2d<T, S, K, AX0, AX1, 3, NC>);
      else
        return nullptr;
    case 4:
      if constexpr (kField)
        return reinterpret_cast<const void*>(&k_sweep2d<T, S, K, AX0, AX1, 4, NC>);
      else
        return nullptr;
    default: return nullptr;
  }
}

template <typename T, class S, int K>
const void* kernel2d_axes(int axes_code, int mode, int nc) {
  if (nc == 2) {  // two-component 1-D lines
    switch (axes_code) {
      case 0: return kernel2d_mode<T, S, K, 0, -1, 2>(mode);
      case 1: return kernel2d_mode<T, S, K, 1, -1, 2>(mode);
      case 2: return kernel2d_mode<T, S, K, 2, -1, 2>(mode);
      default: return nullptr;
    }
  }
  switch (axes_code) {
    case 0: return kernel2d_mode<T, S, K, 0, -1, 4>(mode);
    case 1: return kernel2d_mode<T, S, K, 1, -1, 4>(mode);
    case 2: return kernel2d_mode<T, S, K, 2, -1, 4>(mode);
    case 10: return kernel2d_mode<T, S, K, 0, 1, 4>(mode);
    case 20: return kernel2d_mode<T, S, K, 0, 2, 4>(mode);
    case 21: return kernel2d_mode<T, S, K, 1, 2, 4>(mode);
    default: return nullptr;
  }
}

// the instance groups (nullptr for combinations that are not built)
const void* kernel2d_lie_f32_lo(int depth, int axes_code, int mode, int nc);  // 1-2 steps
const void* kernel2d_lie_f32_hi(int depth, int axes_code, int mode, int nc);  // 3-5 steps
const void* kernel2d_lie_f64_lo(int depth, int axes_code, int mode, int nc);
const void* kernel2d_lie_f64_hi(int depth, int axes_code, int mode, int nc);
const void* kernel2d_strang(bool fp64, int depth, int axes_code, int mode, int nc);
// k_sweep2d_obs for (type, depth 1..5, phase mode 0..2), else nullptr
const void* kernel2d_obs(bool fp64, int depth, int mode);
// the 1-D pass of kDeep1D lowest-order steps for (type, axis, phase mode
// 0..2, stored components), else nullptr
const void* kernel1d_deep(bool fp64, int axis, int mode, int nc);

}  // namespace dirac
