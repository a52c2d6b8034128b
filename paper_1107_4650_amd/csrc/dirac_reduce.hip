// dirac_reduce.hip -- deterministic FP64 compensated reductions for the
// observables (norm, mean coordinates, probability beyond x_b; the R/T
// integrals of Sec. 5.2.1 on the cell grid).
//
// Each thread keeps Neumaier (sum, compensation) pairs over a fixed set of
// cells (a contiguous range per block, strided by the block size); pairs are
// merged with an exact two-sum in a fixed shuffle tree, then across the four
// waves of the block, then in a final one-block pass over the per-block
// partials in block order.  The grid size is fixed, so results do not depend
// on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/libdirac.h"
#include "dirac_launch.h"
#include "dirac_obs.h"
#include "dirac_plan.h"

namespace dirac {

template <int NQ>
__device__ void block_reduce(NSum (&acc)[NQ], NSum (*lds)[4]) {
  wave_merge(acc);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q][wave] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      NSum t = lds[q][0];
      for (int w = 1; w < 4; ++w) nmerge(t, lds[q][w]);
      acc[q] = t;
    }
  }
}

// |psi|^2 of one cell over its stored components, in FP64 (a two-component
// line stores a pair whose partners are zero, so the sum is the same)
template <typename T, int NC>
__device__ __forceinline__ void load_obs(const T* __restrict__ psi, int64_t c, T (&s)[2 * NC]) {
  if constexpr (NC == 4) {
    Site<T> q;
    load_site(psi + c * 8, q);
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = q.v[k];
  } else {
    load_pair(psi + c * 4, s[0], s[1], s[2], s[3]);
  }
}

// Block b sums the contiguous cells [b * per, min((b + 1) * per, ncell)),
// per a multiple of 256, thread t the cells b * per + t + 256 j.  A thread
// derives its cell's grid coordinates once and then advances them by 256
// cells per iteration (a wrap of the x index moves the row on), so no cell
// needs an integer division.  Cells are loaded kObsBatch at a time, their
// addresses linear in j, so the loads of a batch are in flight together.
constexpr int kObsBatch = 4;

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_obs_partial(const T* __restrict__ psi, ObsArgs a,
                                                     double* __restrict__ partials) {
  __shared__ NSum lds[kQ][4];
  NSum acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = NSum{0.0, 0.0};
  const int64_t ncell = a.n0 * a.n1 * a.n2;
  const int64_t per = ((ncell + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
  const int64_t cb = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t ce = cb + per < ncell ? cb + per : ncell;
  int64_t c = cb + threadIdx.x;
  // coordinates of this thread's first cell
  int64_t i0 = c % a.n0, r = c / a.n0;
  int64_t i1 = r % a.n1, i2 = r / a.n1;
  T s[kObsBatch][2 * NC];
  auto load_batch = [&](int64_t cc) {
#pragma unroll
    for (int j = 0; j < kObsBatch; ++j) {
      if (cc + 256 * j < ce) {
        load_obs<T, NC>(psi, cc + 256 * j, s[j]);
      } else {
#pragma unroll
        for (int k = 0; k < 2 * NC; ++k) s[j][k] = T(0);
      }
    }
  };
  if (c < ce) load_batch(c);
  for (; c < ce; c += 256 * kObsBatch) {
    double rho_b[kObsBatch];
#pragma unroll
    for (int j = 0; j < kObsBatch; ++j) {
      double rho = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * NC; ++k) {
        const double v = static_cast<double>(s[j][k]);
        rho = fma(v, v, rho);
      }
      rho_b[j] = rho;
    }
    // the next batch is in flight while this one is summed
    if (c + 256 * kObsBatch < ce) load_batch(c + 256 * kObsBatch);
#pragma unroll
    for (int j = 0; j < kObsBatch; ++j) {
      if (c + 256 * j < ce) {
        const double rho = rho_b[j];
        const double x0 = a.xmin0 + (static_cast<double>(i0) + 0.5) * a.dx;
        nadd(acc[0], rho);
        nadd(acc[1], x0 * rho);
        if (a.ndim > 1) nadd(acc[2], (a.xmin1 + (static_cast<double>(i1) + 0.5) * a.dx) * rho);
        if (a.ndim > 2) nadd(acc[3], (a.xmin2 + (static_cast<double>(i2) + 0.5) * a.dx) * rho);
        if (x0 > a.x_b) nadd(acc[4], rho);
      }
      // advance the coordinates by 256 cells
      i0 += 256;
      while (i0 >= a.n0) {
        i0 -= a.n0;
        if (++i1 == a.n1) {
          i1 = 0;
          ++i2;
        }
      }
    }
  }
  block_reduce<kQ>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      partials[(static_cast<int64_t>(blockIdx.x) * kQ + q) * 2 + 0] = acc[q].s;
      partials[(static_cast<int64_t>(blockIdx.x) * kQ + q) * 2 + 1] = acc[q].c;
    }
  }
}

__global__ __launch_bounds__(256) void k_obs_final(const double* __restrict__ partials,
                                                   int64_t nblk, ObsArgs a,
                                                   double* __restrict__ out5) {
  __shared__ NSum lds[kQ][4];
  NSum acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = NSum{0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const NSum p{partials[(static_cast<int64_t>(b) * kQ + q) * 2],
                   partials[(static_cast<int64_t>(b) * kQ + q) * 2 + 1]};
      nmerge(acc[q], p);
    }
  }
  block_reduce<kQ>(acc, lds);
  if (threadIdx.x == 0) {
    double dV = a.dx;
    for (int d = 1; d < a.ndim; ++d) dV *= a.dx;
    const double S = acc[0].s + acc[0].c;
    out5[0] = dV * S;
    out5[1] = (S != 0.0) ? (acc[1].s + acc[1].c) / S : 0.0;
    out5[2] = (a.ndim > 1 && S != 0.0) ? (acc[2].s + acc[2].c) / S : 0.0;
    out5[3] = (a.ndim > 2 && S != 0.0) ? (acc[3].s + acc[3].c) / S : 0.0;
    out5[4] = dV * (acc[4].s + acc[4].c);
  }
}

hipError_t launch_observables(bool fp64, const void* psi, const ObsArgs& a, double* partials,
                              double* out5, hipStream_t st) {
  if (fp64) {
    if (a.nc == 2)
      hipLaunchKernelGGL((k_obs_partial<double, 2>), dim3(kObsBlocks), dim3(256), 0, st,
                         static_cast<const double*>(psi), a, partials);
    else
      hipLaunchKernelGGL((k_obs_partial<double, 4>), dim3(kObsBlocks), dim3(256), 0, st,
                         static_cast<const double*>(psi), a, partials);
  } else {
    if (a.nc == 2)
      hipLaunchKernelGGL((k_obs_partial<float, 2>), dim3(kObsBlocks), dim3(256), 0, st,
                         static_cast<const float*>(psi), a, partials);
    else
      hipLaunchKernelGGL((k_obs_partial<float, 4>), dim3(kObsBlocks), dim3(256), 0, st,
                         static_cast<const float*>(psi), a, partials);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_obs_final(partials, kObsBlocks, a, out5, st);
}

hipError_t launch_obs_final(const double* partials, int64_t n, const ObsArgs& a, double* out5,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, st, partials, n, a, out5);
  return hipGetLastError();
}

}  // namespace dirac

// ===========================================================================
// dl_observables_noalloc: the observables of a state without a plan and
// without any allocation.  The per-block partial sums live in a file-scope
// device array; the host reaches it through the address that
// hipGetSymbolAddress returns for the current device (looked up on the first
// call on each device and kept), never through the array's name.
// ===========================================================================
namespace {

constexpr int kScratchDoubles = dirac::kObsBlocks * dirac::kQ * 2;  // 40 KiB
static_assert(kScratchDoubles >= dirac::kObsBlocks * dirac::kQ * 2,
              "scratch must hold the partials of every block");

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// device address of this device's scratch array
int scratch_of_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dirac::set_hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return dirac::set_error(DL_ERR_ARG, "device index beyond the scratch table (64 devices)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dirac::set_hip_error(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return DL_OK;
}

}  // namespace

extern "C" int dl_observables_noalloc(const dl_grid* g, double dx, dl_dtype dtype, unsigned flags,
                                      const void* psi, double x_b, double* out, void* stream) {
  using namespace dirac;
  if (!g) return set_error(DL_ERR_ARG, "grid is NULL");
  if (g->ndim < 1 || g->ndim > 3) return set_error(DL_ERR_ARG, "ndim must be 1..3");
  int64_t cells = 1;
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < 1 || g->n[d] > (int64_t(1) << 31))
      return set_error(DL_ERR_ARG, "cell count of a grid dimension out of range");
    if (!std::isfinite(g->xmin[d])) return set_error(DL_ERR_ARG, "xmin not finite");
    if (cells > (int64_t(1) << 40) / g->n[d])
      return set_error(DL_ERR_ARG, "grid beyond 2^40 cells");
    cells *= g->n[d];
  }
  if (!std::isfinite(dx) || dx <= 0.0) return set_error(DL_ERR_ARG, "dx must be finite and > 0");
  if (dtype != DL_C64 && dtype != DL_C128) return set_error(DL_ERR_DTYPE, "unknown dtype");
  if (flags & ~DL_BISPINOR) return set_error(DL_ERR_ARG, "only DL_BISPINOR is a valid flag");
  const bool pair = (flags & DL_BISPINOR) != 0;
  if (pair && g->ndim != 1) return set_error(DL_ERR_ARG, "two-component states are 1-D lines");
  int rc = check_state_ptr(psi, "psi");
  if (rc) return rc;
  if ((rc = check_f64_ptr(out, "out", false))) return rc;
  if (std::isnan(x_b)) return set_error(DL_ERR_ARG, "x_b is NaN");
  // the partials of kObsBlocks blocks, 2 * kQ doubles each, must fit the array
  if (int64_t(kObsBlocks) * kQ * 2 > kScratchDoubles)
    return set_error(DL_ERR_ARG, "reduction partials exceed the static scratch");
  double* sp = nullptr;
  if ((rc = scratch_of_current_device(&sp))) return rc;
  ObsArgs a{};
  a.n0 = g->n[0];
  a.n1 = g->ndim > 1 ? g->n[1] : 1;
  a.n2 = g->ndim > 2 ? g->n[2] : 1;
  a.ndim = g->ndim;
  a.dx = dx;
  a.xmin0 = g->xmin[0];
  a.xmin1 = g->ndim > 1 ? g->xmin[1] : 0.0;
  a.xmin2 = g->ndim > 2 ? g->xmin[2] : 0.0;
  a.x_b = x_b;
  a.nc = pair ? 2 : 4;
  hipError_t e = launch_observables(dtype == DL_C128, psi, a, sp, out,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DL_OK : set_hip_error(e, "observables launch");
}
