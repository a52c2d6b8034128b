// dirac_obs.h -- the compensated FP64 sums behind the observables (norm, mean
// coordinates, probability beyond x_b), shared by the standalone reduction
// kernels and the sweep passes that accumulate them as they store their last
// step.  Internal to libdirac.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dirac_device.h"
#include "dirac_launch.h"

namespace dirac {

// Neumaier (sum, compensation) pair
struct NSum {
  double s, c;
};

__device__ __forceinline__ void nadd(NSum& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

// merge b into a: two-sum of the sums, compensations added
__device__ __forceinline__ void nmerge(NSum& a, const NSum& b) {
  const double t = a.s + b.s;
  const double bb = t - a.s;
  const double err = (a.s - (t - bb)) + (b.s - bb);
  a.c = a.c + b.c + err;
  a.s = t;
}

__device__ __forceinline__ NSum shfl_xor(const NSum& v, int m) {
  NSum r;
  r.s = __shfl_xor(v.s, m, 64);
  r.c = __shfl_xor(v.c, m, 64);
  return r;
}

constexpr int kQ = 5;  // |psi|^2, x0|psi|^2, x1|psi|^2, x2|psi|^2, [x0 > x_b]|psi|^2
static_assert(2 * kQ == kObsDoubles, "a partial holds one Neumaier pair per sum");

// the wave's pairs merged in a fixed butterfly; every lane ends with the total
template <int NQ>
__device__ __forceinline__ void wave_merge(NSum (&acc)[NQ]) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) nmerge(acc[q], shfl_xor(acc[q], m));
  }
}

// |psi|^2 of a stored cell in FP64, components in storage order
template <typename T>
__device__ __forceinline__ double cell_density(const Site<T>& s) {
  double rho = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double v = static_cast<double>(s.v[k]);
    rho = fma(v, v, rho);
  }
  return rho;
}

// A lane that stores the cells of one column of a 2-D grid keeps two sums,
// |psi|^2 and y |psi|^2 (cell centres at xmin + (i + 1/2) dx); the column's
// x |psi|^2 and its part beyond x_b follow from the first once the column is
// done (obs_column_close), since x is the same for all its cells.
template <typename T>
__device__ __forceinline__ void obs_add_cell(NSum* acc, const Site<T>& s, int64_t row,
                                             const ObsArgs& o) {
  const double rho = cell_density(s);
  nadd(acc[0], rho);
  nadd(acc[2], (o.xmin1 + (static_cast<double>(row) + 0.5) * o.dx) * rho);
}

// the same for a stored cell of a 3-D grid: |psi|^2, y |psi|^2, z |psi|^2
template <typename T>
__device__ __forceinline__ void obs_add_cell3(NSum* acc, const Site<T>& s, int64_t row,
                                              int64_t plane, const ObsArgs& o) {
  const double rho = cell_density(s);
  nadd(acc[0], rho);
  nadd(acc[2], (o.xmin1 + (static_cast<double>(row) + 0.5) * o.dx) * rho);
  nadd(acc[3], (o.xmin2 + (static_cast<double>(plane) + 0.5) * o.dx) * rho);
}

// x (s + c) as a pair: the product's rounding error (exact, by fma) joins the
// compensation
__device__ __forceinline__ NSum nscale(const NSum& a, double x) {
  NSum r;
  r.s = x * a.s;
  r.c = fma(x, a.c, fma(x, a.s, -r.s));
  return r;
}

// the column sums of acc[1] (x |psi|^2) and acc[4] (|psi|^2 beyond x_b) from
// acc[0], for a lane whose cells all lie in column `col`
__device__ __forceinline__ void obs_column_close(NSum* acc, int64_t col, const ObsArgs& o) {
  const double x0 = o.xmin0 + (static_cast<double>(col) + 0.5) * o.dx;
  acc[1] = nscale(acc[0], x0);
  acc[4] = (x0 > o.x_b) ? acc[0] : NSum{0.0, 0.0};
}

}  // namespace dirac
