// dirac_launch.h -- host-side launch interface between the plan code and the
// kernels of the Dirac sweep.  Internal to libdirac.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dirac_device.h"

namespace dirac {

constexpr int kTY3D_F32 = 4;  // y rows per wave in the 3-D plane tile
constexpr int kTY3D_F64 = 2;
// two-step 3-D pass: y rows of a workgroup tile (four waves; FP32, FP64 state)
constexpr int kTY3D2_F32 = 8;
constexpr int kTY3D2_F64 = 8;
// 3-D passes fuse at most two lowest-order steps, on rows of fewer than 2^28
// cells (per-lane offsets are 32-bit)
__host__ __device__ constexpr int max_depth3d(bool) { return 2; }
constexpr int64_t kMaxRow3DFused = int64_t(1) << 28;
// 1-D / 2-D passes fuse up to kMaxDepth full lowest-order steps, or up to 3
// second-order steps.  A wave of 64 lanes writes 64 - 2X columns, X
// being the x transports of the pass (one per lowest-order step, two per
// second-order step).  FP64 passes of more than two stages need more
// registers than two waves per SIMD have: they run one wave per SIMD, the
// compiler parking part of the working set in the accumulation registers.
constexpr int kMaxDepth = 5;
constexpr int kMaxDepthF64 = 5;
// 1-D lines of at most kDeep1DMaxCells cells without a vector potential also
// run passes of kDeep1D lowest-order steps (each wave writes 64 - 2 kDeep1D =
// 16 cells): such a line's pass is short next to a kernel launch, so fewer,
// deeper passes win, while on longer lines the fourfold arithmetic of the
// deep pass costs more than the launches it saves
constexpr int kDeep1D = 24;
constexpr int64_t kDeep1DMaxCells = 65536;
__host__ __device__ constexpr int max_depth(bool fp64, bool strang) {
  return strang ? 3 : (fp64 ? kMaxDepthF64 : kMaxDepth);
}
// resident 256-thread blocks per CU the 1-D / 2-D kernel is compiled for, by
// the steps and stages (steps x stages per step) of its pass and its phase
// mode (modes 3 and 4, the static and the pulsed vector potential, carry more
// per row)
__host__ __device__ constexpr int sweep2d_min_blocks(bool fp64, int depth, int stages, int mode) {
  return ((fp64 && stages > 2) || ((mode == 3 || mode == 4) && (fp64 ? depth > 1 : stages > 3)))
             ? 1
             : 2;
}
// reverse (adjoint) passes fuse up to this many reverse steps
constexpr int kMaxRevDepthF32 = 3;
constexpr int kMaxRevDepthF64 = 2;
// passes whose local step carries a vector potential (phase mode 3) hold
// nine doubles of factors per row in flight: they fuse at most 3 lowest-order
// steps (FP64 passes of 2 or 3 at one wave per SIMD), second-order ones 1
__host__ __device__ constexpr int field_max_depth(bool /*fp64*/, bool strang) {
  return strang ? 1 : 3;
}
__host__ __device__ constexpr int strip_width(int xlanes) { return 64 - 2 * xlanes; }
__host__ __device__ constexpr int pass_xlanes(bool strang, int depth) {
  return strang ? 2 * depth : depth;
}

struct SweepArgs {
  int64_t nx, ny, nz;  // cells along grid dims 0, 1, 2 (1 where absent)
  int periodic;
  int H;               // cells per march segment (y in 2-D, z in 3-D)
  int64_t nstrips;     // ceil(nx / output columns per wave)
  int64_t nseg;        // march segments
  int64_t nyblk;       // 3-D: ceil(ny / TY)
  int64_t ntiles;      // waves with work
  int xcd_remap;       // blocks dealt XCD-contiguously (grid a multiple of 8)
  int axes_code;       // 1-D: axis; 2-D: 10*axis0 + axis1 with axis1 > axis0 ... see plan
  PhaseK ph;
  // phase mode 3: field integrals At, planar (x, y, z blocks of `cells`);
  // phase mode 4: the pulse's field profile P in the same layout
  const double* At;
  PulseK pulse;        // phase mode 4 (and 3-D passes with pulse_on)
  int pulse_on;        // 3-D passes: the field integral is P times the pulse's F
  int64_t cells;
  int nc;              // components stored per cell: 4, or 2 (two-component 1-D line)
};

struct ResidentArgs {
  int64_t n;
  int64_t nsteps;
  int periodic;
  PhaseK ph;
  int nc;              // components stored per cell: 4 or 2
};

struct ObsArgs {
  int64_t n0, n1, n2;
  int ndim;
  int nc;              // components stored per cell: 4 or 2
  double dx;
  double xmin0, xmin1, xmin2;
  double x_b;
};

// `depth` full steps (second order if `strang`) src -> dst in one pass over
// a 1-D / 2-D grid (tiling made for strip_width(pass_xlanes(strang, depth)));
// `blocks` 256-thread workgroups
hipError_t launch_sweep2d(bool fp64, bool strang, int depth, const void* src, void* dst,
                          const double* V, const SweepArgs& a, int blocks, hipStream_t st);
// the same lowest-order pass on a 2-D grid (phase modes 0-2, four components),
// which also sums the observables of the cells it stores: 10 doubles per wave
// with work (a.ntiles of them) at `partials`, reduced by launch_obs_final
hipError_t launch_sweep2d_obs(bool fp64, int depth, const void* src, void* dst, const double* V,
                              const SweepArgs& a, const ObsArgs& o, double* partials, int blocks,
                              hipStream_t st);
// true if launch_sweep2d_obs has a kernel for this depth and phase mode
bool sweep2d_obs_available(bool fp64, int depth, int mode);
// kDeep1D lowest-order steps src -> dst in one pass over a 1-D line (phase
// modes 0-2; tiling made for strip_width(kDeep1D))
hipError_t launch_sweep1d_deep(bool fp64, const void* src, void* dst, const double* V,
                               const SweepArgs& a, int blocks, hipStream_t st);
// the two-step 3-D pass (phase modes 0-2) that also sums the observables of
// the cells it stores: 10 doubles per wave (4 per workgroup tile, a.ntiles
// tiles) at `partials`, reduced by launch_obs_final
hipError_t launch_sweep3d_obs(bool fp64, const void* src, void* dst, const double* V,
                              const SweepArgs& a, const ObsArgs& o, double* partials, int blocks,
                              hipStream_t st);
// `depth` (1 or 2) full steps src -> dst in one pass over a 3-D grid (tiling
// made by the 3-D tiler for that depth)
hipError_t launch_sweep3d(bool fp64, int depth, const void* src, void* dst, const double* V,
                          const SweepArgs& a, int blocks, hipStream_t st);
// resident 256-thread blocks per CU of the sweep kernel for this layout,
// phase mode and depth (0 if the runtime cannot tell)
int sweep_occupancy(bool fp64, bool strang, int ndim, int axes_code, int mode, int depth,
                    int nc);
// the same for the 3-D kernels
int occupancy3d(bool fp64, int mode, int depth);
// nsteps >= 1 second-order steps src -> dst on a 3-D grid (Sec. 2.4) in
// nsteps + 1 passes through `mid` and `mid2` (state buffers distinct from src,
// dst and each other; src == dst is allowed), or, with mid2 = NULL, through
// mid and dst (src != dst); a needs nx, ny, nz, periodic and ph
hipError_t launch_strang3d(bool fp64, const void* src, void* dst, void* mid, void* mid2,
                           const double* V, const SweepArgs& a, int64_t nsteps, hipStream_t st);
// nsteps in place in one workgroup of `threads` threads, `spt` cells each
hipError_t launch_resident1d(bool fp64, int axis, void* psi, const double* V,
                             const ResidentArgs& a, int spt, int threads, hipStream_t st);

// observables: per-block partials (kObsDoubles per block) then final pass
constexpr int kObsBlocks = 512;
constexpr int kObsDoubles = 10;  // Neumaier pairs of the five sums
hipError_t launch_observables(bool fp64, const void* psi, const ObsArgs& a, double* partials,
                              double* out5, hipStream_t st);
// the final pass alone: n partials (10 doubles each) in index order -> out5
hipError_t launch_obs_final(const double* partials, int64_t n, const ObsArgs& a, double* out5,
                            hipStream_t st);

}  // namespace dirac
