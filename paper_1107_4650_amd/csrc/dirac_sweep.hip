// dirac_sweep.hip -- fused one-pass time step of the Dirac sweep on gfx950.
//
// One launch advances the whole grid by one full step S = D T_last ... T_first
// (lowest-order splitting, Sec. 2.1; transports eq:sol_dis_1-3; local step
// eq:sol_dis_4), reading psi once and writing it once.
//
// Work decomposition (2-D, and 1-D as the one-row case):
//   * a wave64 holds 64 consecutive x cells (lane l: cell xs + l) and writes
//     the 62 middle ones; their x neighbours all sit in the wave, so the x
//     transport is a DPP wave shift with no halo loads;
//   * the wave marches along y over a segment of H rows, keeping the y movers
//     of the two previous rows in registers, so every row of psi is loaded
//     once per segment (plus one halo row at each end);
//   * even segments march up, odd segments march down: the halo rows shared
//     by two neighbouring segments are then read by both near the same time
//     (both at their start or both at their end) and hit in L2;
//   * blocks are remapped so that each XCD receives a contiguous band of
//     segments (workgroups are dealt to the 8 XCDs round-robin).
// Passes of K fused steps (temporal blocking) write the 64 - 2K middle cells
// of a wave and advance them by K full steps per read and write of psi.
// The kernel template is in dirac_sweep2d_kernels.h and its instances in the
// dirac_sweep2d_*.hip units; this file holds the 1-D resident kernel, the
// dispatch and the launchers.  3-D grids: dirac_sweep3d.hip.
#include "dirac_device.h"
#include "dirac_launch.h"
#include "dirac_sweep_impl.h"
#include "dirac_sweep2d_kernels.h"

namespace dirac {

// ---------------------------------------------------------------------------
// 1-D resident kernel: a whole 1-D instance lives in one workgroup's
// registers for all its steps; neighbour movers cross thread boundaries
// through LDS.  Thread t holds cells [t*SPT, (t+1)*SPT).  The per-cell
// arithmetic is the same as in k_sweep2d, so results are bit-identical.
// ---------------------------------------------------------------------------
template <typename T, int AX, int SPT, int NC>
__global__ __launch_bounds__(1024) void k_resident1d(T* __restrict__ psi,
                                                     const double* __restrict__ V,
                                                     ResidentArgs a) {
  __shared__ Mov<T> lds_r[2][1024];
  __shared__ Mov<T> lds_l[2][1024];
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const int64_t n = a.n;
  Site<T> s[SPT];
  typename Stored<T>::type f[SPT];  // as the tiled passes keep them, for the same bits
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int64_t x = static_cast<int64_t>(t) * SPT + k;
    if (x < n) {
      load_cell<NC, AX>(psi, x, s[k]);
      f[k] = Stored<T>::of(phase_factors((a.ph.mode == 2) ? V[x] : 0.0, a.ph));
    } else {
      zero(s[k]);
      f[k] = Stored<T>::of(phase_factors(0.0, a.ph));
    }
  }
  for (int64_t step = 0; step < a.nsteps; ++step) {
    const int buf = static_cast<int>(step & 1);
    {
      Mov<T> r, l, tmp;
      Axis<AX, T>::movers(s[SPT - 1], r, tmp);
      Axis<AX, T>::movers(s[0], tmp, l);
      lds_r[buf][t] = r;
      lds_l[buf][t] = l;
    }
    __syncthreads();
    Mov<T> rprev, lnext, scratch;
    if (t > 0) rprev = lds_r[buf][t - 1];
    else if (a.periodic) rprev = lds_r[buf][nthr - 1];
    else zero(rprev);
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      if (k < SPT - 1) {
        Axis<AX, T>::movers(s[k + 1], scratch, lnext);
      } else {
        if (t < nthr - 1) lnext = lds_l[buf][t + 1];
        else if (a.periodic) lnext = lds_l[buf][0];
        else zero(lnext);
      }
      Mov<T> rcur;
      Axis<AX, T>::movers(s[k], rcur, scratch);
      Axis<AX, T>::combine(rprev, lnext, s[k]);
      rprev = rcur;
      if (a.ph.mode == 0) {
        const T sc = scale_of<T>(a.ph);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[k].v[j] *= sc;
      } else {
        apply_factors(s[k], f[k]);
      }
      const int64_t x = static_cast<int64_t>(t) * SPT + k;
      if (x >= n) zero(s[k]);  // cells beyond the wall stay empty
    }
    // double-buffered LDS slots: one barrier per step is enough
  }
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int64_t x = static_cast<int64_t>(t) * SPT + k;
    if (x < n) store_cell<NC, AX>(psi, x, s[k]);
  }
}

// nullptr for combinations that are not built (depths beyond max_depth)
static const void* kernel2d(bool fp64, bool strang, int depth, int axes_code, int mode, int nc) {
  if (strang) return kernel2d_strang(fp64, depth, axes_code, mode, nc);
  static_assert(kMaxDepth <= 5 && kMaxDepthF64 <= 5, "kernels are built for depths 1 to 5");
  if (depth < 1 || depth > (fp64 ? kMaxDepthF64 : kMaxDepth)) return nullptr;
  if (fp64)
    return depth <= 2 ? kernel2d_lie_f64_lo(depth, axes_code, mode, nc)
                      : kernel2d_lie_f64_hi(depth, axes_code, mode, nc);
  return depth <= 2 ? kernel2d_lie_f32_lo(depth, axes_code, mode, nc)
                    : kernel2d_lie_f32_hi(depth, axes_code, mode, nc);
}

hipError_t launch_sweep2d(bool fp64, bool strang, int depth, const void* src, void* dst,
                          const double* V, const SweepArgs& a, int blocks, hipStream_t st) {
  const void* fn = kernel2d(fp64, strang, depth, a.axes_code, a.ph.mode, a.nc);
  if (!fn || blocks <= 0) return hipErrorInvalidValue;
  SweepArgs args = a;
  void* kargs[] = {const_cast<void**>(&src), &dst, const_cast<double**>(&V), &args};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
}

hipError_t launch_sweep2d_obs(bool fp64, int depth, const void* src, void* dst, const double* V,
                              const SweepArgs& a, const ObsArgs& o, double* partials, int blocks,
                              hipStream_t st) {
  const void* fn = kernel2d_obs(fp64, depth, a.ph.mode);
  if (!fn || blocks <= 0 || a.axes_code != 10 || a.nc != 4) return hipErrorInvalidValue;
  SweepArgs args = a;
  ObsArgs oargs = o;
  void* kargs[] = {const_cast<void**>(&src), &dst, const_cast<double**>(&V), &args, &oargs,
                   &partials};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
}

hipError_t launch_sweep1d_deep(bool fp64, const void* src, void* dst, const double* V,
                               const SweepArgs& a, int blocks, hipStream_t st) {
  const void* fn = kernel1d_deep(fp64, a.axes_code, a.ph.mode, a.nc);
  if (!fn || blocks <= 0) return hipErrorInvalidValue;
  SweepArgs args = a;
  void* kargs[] = {const_cast<void**>(&src), &dst, const_cast<double**>(&V), &args};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
}

bool sweep2d_obs_available(bool fp64, int depth, int mode) {
  return kernel2d_obs(fp64, depth, mode) != nullptr;
}

// ---- occupancy queries (resident 256-thread blocks per CU) -------------------
static int occ_of(const void* kernel) {
  if (!kernel) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int sweep_occupancy(bool fp64, bool strang, int ndim, int axes_code, int mode, int depth,
                    int nc) {
  if (ndim == 3) return occupancy3d(fp64, mode, depth);
  return occ_of(kernel2d(fp64, strang, depth, axes_code, mode, nc));
}

template <typename T, int AX, int SPT>
static hipError_t launch_res_t(void* psi, const double* V, const ResidentArgs& a, int threads,
                               hipStream_t st) {
  if (a.nc == 2)
    hipLaunchKernelGGL((k_resident1d<T, AX, SPT, 2>), dim3(1), dim3(threads), 0, st,
                       static_cast<T*>(psi), V, a);
  else
    hipLaunchKernelGGL((k_resident1d<T, AX, SPT, 4>), dim3(1), dim3(threads), 0, st,
                       static_cast<T*>(psi), V, a);
  return hipGetLastError();
}

template <typename T, int AX>
static hipError_t launch_res_spt(void* psi, const double* V, const ResidentArgs& a, int spt,
                                 int threads, hipStream_t st) {
  switch (spt) {
    case 1: return launch_res_t<T, AX, 1>(psi, V, a, threads, st);
    case 2: return launch_res_t<T, AX, 2>(psi, V, a, threads, st);
    case 4: return launch_res_t<T, AX, 4>(psi, V, a, threads, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_resident1d(bool fp64, int axis, void* psi, const double* V,
                             const ResidentArgs& a, int spt, int threads, hipStream_t st) {
  if (fp64) {
    switch (axis) {
      case 0: return launch_res_spt<double, 0>(psi, V, a, spt, threads, st);
      case 1: return launch_res_spt<double, 1>(psi, V, a, spt, threads, st);
      default: return launch_res_spt<double, 2>(psi, V, a, spt, threads, st);
    }
  }
  switch (axis) {
    case 0: return launch_res_spt<float, 0>(psi, V, a, spt, threads, st);
    case 1: return launch_res_spt<float, 1>(psi, V, a, spt, threads, st);
    default: return launch_res_spt<float, 2>(psi, V, a, spt, threads, st);
  }
}

}  // namespace dirac
