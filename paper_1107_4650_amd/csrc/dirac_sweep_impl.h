// dirac_sweep_impl.h -- per-wave building blocks of the fused step, shared
// by the single-plan kernels and the batched kernel so that both run the same
// per-cell arithmetic.  Internal to libdirac.
//
// A wave64 owns a strip of 64 consecutive x cells (lane l holds cell x0+l).
// The x transport takes the left neighbour's right movers and the right
// neighbour's left movers with DPP wave shifts; lane 0 also loads the cell
// left of the strip and lane 63 the cell right of it, and the lane just past
// the last cell stands for the cell beyond the wall.  In 2-D the wave marches
// along y over a segment of rows, keeping the y movers of the two previous
// rows in registers, so every row is loaded once per segment plus one halo
// row at each end.
#pragma once
#include "dirac_device.h"
#include "dirac_launch.h"

namespace dirac {

// ---------------------------------------------------------------------------
// row loading with walls / wrap-around
// ---------------------------------------------------------------------------
template <typename T> struct Row {
  Site<T> m;  // this lane's cell
  Site<T> h;  // lane 0: cell left of the strip; lane 63: cell right of it
  double v;   // potential at the output cell of this row
};

// Load cell row `j` (a row index of a 2-D plane, possibly outside [0, ny))
// of the plane starting at `plane`; returns zeros for cells beyond a wall.
template <typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ plane, int64_t nx, int64_t ny,
                                         int periodic, int64_t x0, int lane, int64_t j,
                                         Row<T>& R) {
  zero(R.m);
  zero(R.h);
  if (j < 0 || j >= ny) {
    if (!periodic) return;
    j = (j < 0) ? j + ny : j - ny;
  }
  const T* row = plane + j * nx * 8;
  const int64_t x = x0 + lane;
  int64_t xm = x;
  if (x == nx && periodic) xm = 0;
  if (xm < nx) load_site(row + xm * 8, R.m);
  int64_t hx = -2;
  if (lane == 0) hx = x0 - 1;
  if (lane == 63) hx = x0 + 64;
  if (hx == -1) hx = periodic ? nx - 1 : -2;
  if (hx == nx) hx = periodic ? 0 : -2;
  if (hx >= 0 && hx < nx) load_site(row + hx * 8, R.h);
}

// x transport of one row held across the wave (result is 2x the transport).
template <typename T, int AX>
__device__ __forceinline__ void x_transport(const Row<T>& R, Site<T>& phi) {
  Mov<T> r, l, hr, hl, rL, lR;
  Axis<AX, T>::movers(R.m, r, l);
  Axis<AX, T>::movers(R.h, hr, hl);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rL.v[k] = dpp_from_left(hr.v[k], r.v[k]);
    lR.v[k] = dpp_from_right(hl.v[k], l.v[k]);
  }
  Axis<AX, T>::combine(rL, lR, phi);
}

__device__ __forceinline__ int64_t wrap_or_neg(int64_t j, int64_t n, int periodic) {
  if (j >= 0 && j < n) return j;
  if (!periodic) return -1;
  return j < 0 ? j + n : j - n;
}

// ---------------------------------------------------------------------------
// 1-D / 2-D fused step
// ---------------------------------------------------------------------------
constexpr int PF2 = 3;  // rows in flight per wave

template <typename T, int AX0, int AX1, bool UP>
__device__ __forceinline__ void march2d(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t x0, int lane, int64_t jb, int64_t je) {
  const int64_t nx = a.nx, ny = a.ny;
  const int nit = static_cast<int>(je - jb) + 2;
  const int64_t x = x0 + lane;
  const bool own = x < nx;
  const bool use_v = (a.ph.mode == 2);
  // input row of iteration `it` and the output row it completes
  auto in_row = [&](int it) -> int64_t { return UP ? jb - 1 + it : je - it; };
  auto out_row = [&](int it) -> int64_t { return UP ? jb - 2 + it : je - it + 1; };

  Row<T> ring[PF2];
#pragma unroll
  for (int k = 0; k < PF2; ++k) {
    if (k < nit) {
      load_row(src, nx, ny, a.periodic, x0, lane, in_row(k), ring[k]);
      ring[k].v = (use_v && k >= 2 && own) ? V[out_row(k) * nx + x] : 0.0;
    }
  }
  Mov<T> s1, s2;  // movers of the two previous rows (r when UP, l when down)
  zero(s1);
  zero(s2);
  for (int base = 0; base < nit; base += PF2) {
#pragma unroll
    for (int k = 0; k < PF2; ++k) {
      const int it = base + k;
      if (it < nit) {
        const Row<T> cur = ring[k];
        const int nxt = it + PF2;
        if (nxt < nit) {
          load_row(src, nx, ny, a.periodic, x0, lane, in_row(nxt), ring[k]);
          ring[k].v = (use_v && own) ? V[out_row(nxt) * nx + x] : 0.0;
        }
        Site<T> phi;
        x_transport<T, AX0>(cur, phi);
        Mov<T> ry, ly;
        Axis<AX1, T>::movers(phi, ry, ly);
        if (it >= 2) {
          Site<T> o;
          if (UP)
            Axis<AX1, T>::combine(s2, ly, o);
          else
            Axis<AX1, T>::combine(ry, s2, o);
          local_step(o, cur.v, a.ph);
          if (own) store_site(dst + (out_row(it) * nx + x) * 8, o);
        }
        s2 = s1;
        s1 = UP ? ry : ly;
      }
    }
  }
}

// one step of a 1-D line for the strip starting at x0
template <typename T, int AX>
__device__ __forceinline__ void one_row(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t x0, int lane) {
  Row<T> R;
  load_row(src, a.nx, 1, a.periodic, x0, lane, 0, R);
  const int64_t x = x0 + lane;
  const bool own = x < a.nx;
  R.v = (a.ph.mode == 2 && own) ? V[x] : 0.0;
  Site<T> o;
  x_transport<T, AX>(R, o);
  local_step(o, R.v, a.ph);
  if (own) store_site(dst + x * 8, o);
}

// march a 2-D segment upwards (up = true) or downwards
template <typename T, int AX0, int AX1>
__device__ __forceinline__ void march_dir(const T* __restrict__ src, T* __restrict__ dst,
                                          const double* __restrict__ V, const SweepArgs& a,
                                          int64_t x0, int lane, int64_t jb, int64_t je, bool up) {
  if (up)
    march2d<T, AX0, AX1, true>(src, dst, V, a, x0, lane, jb, je);
  else
    march2d<T, AX0, AX1, false>(src, dst, V, a, x0, lane, jb, je);
}

}  // namespace dirac
