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
//
// Per row the wave issues the loads of the row PF2 iterations ahead, then
// runs one straight-line block: x and y transports of the current row, the
// phase factors of the NEXT row (its potential arrived earlier), and the
// local step of the current row with the factors computed one iteration
// before.  The long dependent chain of the sine/cosine thus overlaps the
// transports of another row instead of stalling its own.  MODE (0: scale
// only, 1: constant mass phases, 2: potential; < 0: read at run time) is a
// template parameter so that the block has no mode branches.
// ---------------------------------------------------------------------------
constexpr int PF2 = 3;  // rows in flight per wave

template <typename T, int AX0, int AX1, bool UP, int MODE>
__device__ __forceinline__ void march2d(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t x0, int lane, int64_t jb, int64_t je) {
  constexpr bool TWO = sizeof(T) == 8;
  const int64_t nx = a.nx, ny = a.ny;
  const int nit = static_cast<int>(je - jb) + 2;  // >= 3 = PF2
  const int64_t x = x0 + lane;
  const bool own = x < nx;
  const int64_t xv = own ? x : nx - 1;            // clamped column for V
  const bool read_v = (MODE == 2) || (MODE < 0 && a.ph.mode == 2);
  // input row of iteration `it` and the output row it completes
  auto in_row = [&](int it) -> int64_t { return UP ? jb - 1 + it : je - it; };
  auto out_row = [&](int it) -> int64_t { return UP ? jb - 2 + it : je - it + 1; };
  auto v_at = [&](int it) -> double {
    int64_t r = out_row(it);
    r = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
    return read_v ? V[r * nx + xv] : 0.0;
  };

  // ring entry k holds the input row of iteration it and the potential of
  // iteration it + 1, so the factors of the next row arrive with the data
  // the current row waits for anyway
  Row<T> ring[PF2];
#pragma unroll
  for (int k = 0; k < PF2; ++k) {
    load_row(src, nx, ny, a.periodic, x0, lane, in_row(k), ring[k]);
    ring[k].v = v_at(k + 1);
  }
  const double v0 = v_at(0);
  Factors fcur = factors_of<MODE, TWO>(v0, a.ph);
  factors_fix<MODE, TWO>(fcur, v0, a.ph);
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
          ring[k].v = v_at(nxt + 1);
        }
        // straight-line part: factors of the next row, transports and local
        // step of this row
        Factors fnext = factors_of<MODE, TWO>(cur.v, a.ph);
        Site<T> phi;
        x_transport<T, AX0>(cur, phi);
        Mov<T> ry, ly;
        Axis<AX1, T>::movers(phi, ry, ly);
        Site<T> o;
        if (UP)
          Axis<AX1, T>::combine(s2, ly, o);
        else
          Axis<AX1, T>::combine(ry, s2, o);
        apply_local<MODE>(o, fcur, a.ph);
        s2 = s1;
        s1 = UP ? ry : ly;
        if (it >= 2 && own) store_site(dst + (out_row(it) * nx + x) * 8, o);
        factors_fix<MODE, TWO>(fnext, cur.v, a.ph);
        fcur = fnext;
      }
    }
  }
}

// one step of a 1-D line for the strip starting at x0
template <typename T, int AX, int MODE>
__device__ __forceinline__ void one_row(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t x0, int lane) {
  constexpr bool TWO = sizeof(T) == 8;
  Row<T> R;
  load_row(src, a.nx, 1, a.periodic, x0, lane, 0, R);
  const int64_t x = x0 + lane;
  const bool own = x < a.nx;
  const bool read_v = (MODE == 2) || (MODE < 0 && a.ph.mode == 2);
  R.v = read_v ? V[own ? x : a.nx - 1] : 0.0;
  Factors f = factors_of<MODE, TWO>(R.v, a.ph);
  Site<T> o;
  x_transport<T, AX>(R, o);
  factors_fix<MODE, TWO>(f, R.v, a.ph);
  apply_local<MODE>(o, f, a.ph);
  if (own) store_site(dst + x * 8, o);
}

// march a 2-D segment upwards (up = true) or downwards
template <typename T, int AX0, int AX1, int MODE>
__device__ __forceinline__ void march_dir(const T* __restrict__ src, T* __restrict__ dst,
                                          const double* __restrict__ V, const SweepArgs& a,
                                          int64_t x0, int lane, int64_t jb, int64_t je, bool up) {
  if (up)
    march2d<T, AX0, AX1, true, MODE>(src, dst, V, a, x0, lane, jb, je);
  else
    march2d<T, AX0, AX1, false, MODE>(src, dst, V, a, x0, lane, jb, je);
}

}  // namespace dirac

namespace dirac {

// ---------------------------------------------------------------------------
// Two steps per pass (temporal blocking).  A wave covers 64 columns starting
// one column left of its 62 output columns; lanes 0 and 63 load the columns
// beside those (the first step needs them), so the first step is valid on
// all 64 lanes and the second on lanes 1..62.  Along y the wave marches one
// row ahead for the first step and keeps the y movers of both steps for the
// two previous rows.  Each cell's phase factors are formed once and applied
// by both steps.  The intermediate state is rounded to T exactly as a stored
// single step, so two steps per pass give the same bits as two passes.
// With zero walls the intermediate state is zero outside the box, as the
// transports of the second step require.
// ---------------------------------------------------------------------------

// load row j for the columns xs .. xs+63 of this wave (lane l: xs + l; lane 0
// also xs - 1 and lane 63 xs + 64), wrapping or zeroing outside the box
template <typename T>
__device__ __forceinline__ void load_row_any(const T* __restrict__ plane, int64_t nx, int64_t ny,
                                             int periodic, int64_t xs, int lane, int64_t j,
                                             Row<T>& R) {
  zero(R.m);
  zero(R.h);
  if (j < 0 || j >= ny) {
    if (!periodic) return;
    j = (j < 0) ? j + ny : j - ny;
  }
  const T* row = plane + j * nx * 8;
  auto col = [&](int64_t x) -> int64_t {
    if (x >= 0 && x < nx) return x;
    if (!periodic) return -1;
    return ((x % nx) + nx) % nx;
  };
  const int64_t xm = col(xs + lane);
  if (xm >= 0) load_site(row + xm * 8, R.m);
  int64_t hx = -1;
  if (lane == 0) hx = col(xs - 1);
  if (lane == 63) hx = col(xs + 64);
  if (hx >= 0) load_site(row + hx * 8, R.h);
}

// x transport of an intermediate row held across the wave (no halo lanes:
// lanes 0 and 63 produce values that are not used)
template <typename T, int AX>
__device__ __forceinline__ void x_transport_inner(const Site<T>& s, Site<T>& phi) {
  Mov<T> r, l, rL, lR;
  Axis<AX, T>::movers(s, r, l);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rL.v[k] = dpp_from_left(r.v[k], r.v[k]);
    lR.v[k] = dpp_from_right(l.v[k], l.v[k]);
  }
  Axis<AX, T>::combine(rL, lR, phi);
}

template <typename T, int AX0, int AX1, bool UP, int MODE>
__device__ __forceinline__ void march2d_x2(const T* __restrict__ src, T* __restrict__ dst,
                                           const double* __restrict__ V, const SweepArgs& a,
                                           int64_t xs, int lane, int64_t jb, int64_t je) {
  constexpr bool TWO = sizeof(T) == 8;
  const int64_t nx = a.nx, ny = a.ny;
  const int nit = static_cast<int>(je - jb) + 4;  // >= 5
  const int64_t x = xs + lane;                    // this lane's column (may lie outside)
  const bool inside_x = x >= 0 && x < nx;
  const bool own = inside_x && lane >= 1 && lane <= 62;
  int64_t xv = x;                                 // column of V (wrapped or clamped)
  if (!inside_x) xv = a.periodic ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
  const bool read_v = (MODE == 2) || (MODE < 0 && a.ph.mode == 2);
  const bool zero_walls = !a.periodic;
  auto in_row = [&](int it) -> int64_t { return UP ? jb - 2 + it : je + 1 - it; };
  auto row1 = [&](int it) -> int64_t { return UP ? jb - 3 + it : je + 2 - it; };  // first-step row
  auto row2 = [&](int it) -> int64_t { return UP ? jb - 4 + it : je + 3 - it; };  // second-step row
  auto v_at = [&](int it) -> double {
    int64_t r = row1(it);
    if (r < 0 || r >= ny) r = a.periodic ? ((r % ny) + ny) % ny : (r < 0 ? 0 : ny - 1);
    return read_v ? V[r * nx + xv] : 0.0;
  };

  // ring entry k: input row of iteration it and the potential of iteration it + 1
  Row<T> ring[PF2];
#pragma unroll
  for (int k = 0; k < PF2; ++k) {
    load_row_any(src, nx, ny, a.periodic, xs, lane, in_row(k), ring[k]);
    ring[k].v = v_at(k + 1);
  }
  const double v0 = v_at(0);
  Factors f1 = factors_of<MODE, TWO>(v0, a.ph);   // first-step factors of iteration it
  factors_fix<MODE, TWO>(f1, v0, a.ph);
  Factors f2 = f1;                                 // second-step factors (previous f1)
  Mov<T> s1, s2, t1, t2;  // y movers of the two previous rows, first and second step
  zero(s1);
  zero(s2);
  zero(t1);
  zero(t2);
  for (int base = 0; base < nit; base += PF2) {
#pragma unroll
    for (int k = 0; k < PF2; ++k) {
      const int it = base + k;
      if (it < nit) {
        const Row<T> cur = ring[k];
        const int nxt = it + PF2;
        if (nxt < nit) {
          load_row_any(src, nx, ny, a.periodic, xs, lane, in_row(nxt), ring[k]);
          ring[k].v = v_at(nxt + 1);
        }
        const double vnext = cur.v;
        Factors fnext = factors_of<MODE, TWO>(vnext, a.ph);
        // first step: row1(it) from input rows row1 - 1 .. row1 + 1
        Site<T> phi;
        x_transport<T, AX0>(cur, phi);
        Mov<T> ry, ly;
        Axis<AX1, T>::movers(phi, ry, ly);
        Site<T> o1;
        if (UP)
          Axis<AX1, T>::combine(s2, ly, o1);
        else
          Axis<AX1, T>::combine(ry, s2, o1);
        apply_local<MODE>(o1, f1, a.ph);
        s2 = s1;
        s1 = UP ? ry : ly;
        if (zero_walls) {
          const int64_t r1 = row1(it);
          if (!inside_x || r1 < 0 || r1 >= ny) zero(o1);
        }
        // second step: row2(it) from first-step rows row2 - 1 .. row2 + 1
        Site<T> phi2;
        x_transport_inner<T, AX0>(o1, phi2);
        Mov<T> ry2, ly2;
        Axis<AX1, T>::movers(phi2, ry2, ly2);
        Site<T> o2;
        if (UP)
          Axis<AX1, T>::combine(t2, ly2, o2);
        else
          Axis<AX1, T>::combine(ry2, t2, o2);
        apply_local<MODE>(o2, f2, a.ph);
        if (it >= 2) {
          t2 = t1;
          t1 = UP ? ry2 : ly2;
        }
        if (it >= 4 && own) store_site(dst + (row2(it) * nx + x) * 8, o2);
        factors_fix<MODE, TWO>(fnext, vnext, a.ph);
        f2 = f1;
        f1 = fnext;
      }
    }
  }
}

// two steps of a 1-D line for the 62 output cells of the wave
template <typename T, int AX, int MODE>
__device__ __forceinline__ void one_row_x2(const T* __restrict__ src, T* __restrict__ dst,
                                           const double* __restrict__ V, const SweepArgs& a,
                                           int64_t xs, int lane) {
  constexpr bool TWO = sizeof(T) == 8;
  const int64_t nx = a.nx;
  Row<T> R;
  load_row_any(src, nx, 1, a.periodic, xs, lane, 0, R);
  const int64_t x = xs + lane;
  const bool inside_x = x >= 0 && x < nx;
  const bool own = inside_x && lane >= 1 && lane <= 62;
  int64_t xv = x;
  if (!inside_x) xv = a.periodic ? ((x % nx) + nx) % nx : (x < 0 ? 0 : nx - 1);
  const bool read_v = (MODE == 2) || (MODE < 0 && a.ph.mode == 2);
  R.v = read_v ? V[xv] : 0.0;
  Factors f = factors_of<MODE, TWO>(R.v, a.ph);
  factors_fix<MODE, TWO>(f, R.v, a.ph);
  Site<T> o1, o2;
  x_transport<T, AX>(R, o1);
  apply_local<MODE>(o1, f, a.ph);
  if (!a.periodic && !inside_x) zero(o1);
  x_transport_inner<T, AX>(o1, o2);
  apply_local<MODE>(o2, f, a.ph);
  if (own) store_site(dst + x * 8, o2);
}

template <typename T, int AX0, int AX1, int MODE>
__device__ __forceinline__ void march_dir_x2(const T* __restrict__ src, T* __restrict__ dst,
                                             const double* __restrict__ V, const SweepArgs& a,
                                             int64_t xs, int lane, int64_t jb, int64_t je,
                                             bool up) {
  if (up)
    march2d_x2<T, AX0, AX1, true, MODE>(src, dst, V, a, xs, lane, jb, je);
  else
    march2d_x2<T, AX0, AX1, false, MODE>(src, dst, V, a, xs, lane, jb, je);
}

}  // namespace dirac
