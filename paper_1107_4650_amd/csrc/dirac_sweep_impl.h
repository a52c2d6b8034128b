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
#include <type_traits>

#include "dirac_device.h"
#include "dirac_launch.h"
#include "dirac_obs.h"

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
// Helpers of the 1-D / 2-D marches
// ---------------------------------------------------------------------------

// wave-uniform row index wrapped around a periodic box, -1 beyond a wall;
// rows with work lie at most 4 cells outside the box and periodic boxes
// marched here have ny >= 4, so one correction suffices (the plan ensures it)
__device__ __forceinline__ int64_t wrap_row(int64_t j, int64_t ny, int periodic) {
  if (j >= 0 && j < ny) return j;
  if (!periodic) return -1;
  return j < 0 ? j + ny : j - ny;
}

// row actually read for row r: wrapped, else the nearest row of the box
// (rows beyond a wall are zeroed where they are used; rows read past the end
// of a segment are not used at all)
__device__ __forceinline__ int64_t read_row(int64_t r, int64_t ny, int periodic) {
  int64_t w = wrap_row(r, ny, periodic);
  if (w < 0) w = r < 0 ? 0 : ny - 1;
  return w < 0 ? 0 : (w >= ny ? ny - 1 : w);
}

// this lane's column x wrapped around a periodic box, -1 beyond a wall
__device__ __forceinline__ int64_t wave_col(int64_t nx, int periodic, int64_t x) {
  if (x >= 0 && x < nx) return x;
  if (!periodic) return -1;
  return ((x % nx) + nx) % nx;
}

// x transport inside the wave (result is 2x the transport); lanes 0 and 63
// lack a neighbour and produce values that are not used
template <typename T, int AX>
__device__ __forceinline__ void x_transport_inner(const Site<T>& s, Site<T>& phi) {
  Mov<T> r, l, rL, lR;
  Axis<AX, T>::movers(s, r, l);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rL.v[k] = dpp_from_left_zero(r.v[k]);
    lR.v[k] = dpp_from_right_zero(l.v[k]);
  }
  Axis<AX, T>::combine(rL, lR, phi);
}

// Columns of one wave: lane l holds column xs + l.  `col` is the column read
// (wrapped, or clamped beyond a wall), `out` says whether the lane's column
// lies beyond a wall (its cells read as zero).
struct Lanes {
  int64_t x;     // this lane's column (may lie outside the box)
  int64_t col;   // column read
  bool inside;   // 0 <= x < nx
  bool out;      // beyond a wall
  bool full;     // wave-uniform: no lane beyond a wall
};

__device__ __forceinline__ Lanes lanes_of(int64_t nx, int periodic, int64_t xs, int lane) {
  Lanes c;
  c.x = xs + lane;
  c.inside = c.x >= 0 && c.x < nx;
  const int64_t w = wave_col(nx, periodic, c.x);
  c.out = w < 0;
  c.col = w >= 0 ? w : (c.x < 0 ? 0 : nx - 1);
  c.full = periodic || (xs >= 0 && xs + 63 < nx);
  return c;
}

// ---------------------------------------------------------------------------
// 1-D / 2-D fused pass of K full steps (temporal blocking).
//
// A step is a sequence of stages, each holding one y transport and row-local
// work before and after it (the scheme, below):
//   Lie (Sec. 2.1):    T_x, T_y, D                 -- one stage per step;
//   Strang (Sec. 2.4): T_x, T_y, D | T_y, T_x      -- two stages per step,
// every transport a one-cell shift.  A pass of K steps runs NS = K * stages
// per step.
//
// A wave holds 64 consecutive columns (lane l: column xs + l) and writes the
// middle 64 - 2X of them, X being the x transports of the pass: each x
// transport is valid one lane further in from both ends, and every x
// neighbour it needs sits in the wave, so the neighbour exchange is a plain
// DPP shift and no lane loads a halo cell.  In 2-D the wave marches along y
// over a segment of H rows.  Iteration it reads input row in_row(it); stage
// st (0-based) then completes the row st + 1 behind it, from the stage-(st-1)
// rows two behind, one behind and current, keeping the y movers of two
// previous rows per stage in registers.  Each row is read once per segment
// (plus NS halo rows at each end) and written once, whatever K.
//
// Each intermediate state is rounded to T exactly as a stored single step, so
// a pass of K steps gives the same bits as K passes of one step.  With zero
// walls the intermediate states are forced to zero outside the box, as the
// transports of the next stage require.
//
// The potential of a row arrives with the row; its phase factors are formed
// once, in the iteration that reads it, and applied by every stage with a
// local step in the following iterations, so the dependent sine/cosine chain
// overlaps the transports of other rows.  MODE (0: scale only, 1: constant
// mass phases, 2: potential; < 0: read at run time) is a template parameter
// so that the block has no mode branches.
//
// Rolling state lives in register slots indexed by the iteration modulo
// their period (row ring: L + 1 slots for L rows in flight, y movers: 2 per
// stage, factors: P) and the loop is unrolled by a common multiple, so no
// register copies are needed to advance it.  Memory accesses sit outside
// branches: rows and columns beyond a wall are read at a clamped address and
// zeroed where they are consumed, rows past the segment end are read and
// ignored, and the only branch that leaves the loop is a wave-uniform exit
// after the last row, so the loads of later rows stay in flight while the
// current row is computed.
// ---------------------------------------------------------------------------
struct LieStep {  // T_x, T_y, D
  static constexpr int kStages = 1;  // stages per step
  static constexpr int kXPerStep = 1;
  static constexpr bool pre_x(int) { return true; }
  static constexpr bool phase(int) { return true; }
  static constexpr bool post_x(int) { return false; }
};
struct StrangStep {  // T_x, T_y, D, T_y, T_x (half-step transports)
  static constexpr int kStages = 2;
  static constexpr int kXPerStep = 2;
  static constexpr bool pre_x(int st) { return st % 2 == 0; }
  static constexpr bool phase(int st) { return st % 2 == 0; }
  static constexpr bool post_x(int st) { return st % 2 == 1; }
};

// x transports of a pass of K steps: lanes lost at each end of the wave
template <class S> __host__ __device__ constexpr int halo_lanes(int K) { return K * S::kXPerStep; }

template <class S, int K> struct MarchShape;  // L: rows in flight; U: unroll
template <> struct MarchShape<LieStep, 1> { static constexpr int L = 3, U = 4; };
template <> struct MarchShape<LieStep, 2> { static constexpr int L = 2, U = 6; };
template <> struct MarchShape<LieStep, 3> { static constexpr int L = 1, U = 4; };
template <> struct MarchShape<LieStep, 4> { static constexpr int L = 1, U = 10; };
template <> struct MarchShape<LieStep, 5> { static constexpr int L = 2, U = 6; };
template <> struct MarchShape<StrangStep, 1> { static constexpr int L = 3, U = 4; };
template <> struct MarchShape<StrangStep, 2> { static constexpr int L = 3, U = 4; };
template <> struct MarchShape<StrangStep, 3> { static constexpr int L = 1, U = 6; };

// factor slots: rows from the newest read to the oldest still to be phased
template <class S> constexpr int factor_slots(int NS) {
  int last = 0;
  for (int st = 0; st < NS; ++st)
    if (S::phase(st)) last = st;
  return last + 2;
}

// OBS: also add the observables of every stored cell to the lane's sums acc
template <typename T, class S, int K, int AX0, int AX1, bool UP, int MODE, bool EDGE,
          bool OBS = false>
__device__ __forceinline__ void march2d(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t xs, int lane, int64_t jb, int64_t je,
                                        int wlane, NSum* acc = nullptr,
                                        const ObsArgs* ob = nullptr) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int NS = K * S::kStages;          // stages of the pass
  constexpr int X = halo_lanes<S>(K);         // x transports of the pass
  constexpr int L = MarchShape<S, K>::L;      // rows in flight
  constexpr int RS = L + 1;                   // ring slots
  constexpr int P = factor_slots<S>(NS);      // factor slots
  constexpr int U = MarchShape<S, K>::U;
  static_assert(U % RS == 0 && U % 2 == 0 && U % P == 0, "unroll must cover every period");
  const int64_t nx = a.nx, ny = a.ny;
  const int nit = static_cast<int>(je - jb) + 2 * NS;  // iterations with work
  const Lanes c = lanes_of(nx, a.periodic, xs, lane);
  const bool own = c.inside && lane >= wlane && lane <= 63 - wlane;  // wlane >= X
  constexpr bool PULSE = MODE == 4;             // ... with a pulse (per-step field integral)
  constexpr bool FIELD = MODE == 3 || PULSE;    // local step with a vector potential
  // factor slots: the field's factors, else the phase factors as kept for T
  using FT = typename std::conditional<FIELD, typename FactorOf<MODE>::type,
                                       typename Stored<T>::type>::type;
  const bool read_v = (MODE == 2) || (FIELD && V != nullptr) || (MODE < 0 && a.ph.mode == 2);
  // pulse: the field integral factor of each step of the pass
  double Fs[PULSE ? K : 1];
#pragma unroll
  for (int s = 0; s < (PULSE ? K : 1); ++s) Fs[s] = PULSE ? pulse_step_integral(a.pulse, s) : 0.0;
  const bool zero_walls = !a.periodic;
  // input row of iteration it; stage st completes row in_row(it) -+ (st + 1)
  auto in_row = [&](int it) -> int64_t { return UP ? jb - NS + it : je - 1 + NS - it; };
  auto out_row = [&](int it, int done) -> int64_t {
    return UP ? in_row(it) - done : in_row(it) + done;
  };
  // Row out_row(it, d) lies in the box iff lo <= it - d < hi.  The bounds
  // are wave-uniform and clamped to 32 bits (it - d spans -NS .. nit + L), so
  // the wall tests of the loop are scalar compares.
  auto clamp_it = [&](int64_t e) -> int {
    return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
  };
  const int64_t lo64 = UP ? NS - jb : je + NS - ny;
  const int lo = clamp_it(lo64), hi = clamp_it(lo64 + ny);
  auto row_in = [&](int e) -> bool { return e >= lo && e < hi; };
  auto load_in = [&](int it, Site<T>& m, double& v, double* at) {
    int64_t r = in_row(it);
    if (!row_in(it)) r = read_row(r, ny, a.periodic);
    load_site(src + (r * nx + c.col) * 8, m);
    v = read_v ? V[r * nx + c.col] : 0.0;
    if constexpr (FIELD) {
      const int64_t q = r * nx + c.col;
      at[0] = a.At[q];
      at[1] = a.At[a.cells + q];
      at[2] = a.At[2 * a.cells + q];
    }
  };

  // ring slot it % RS: input row of iteration it, its potential (and field)
  Site<T> ring[RS];
  double vr[RS];
  double ar[RS][FIELD ? 3 : 1];
#pragma unroll
  for (int k = 0; k < L; ++k) load_in(k, ring[k], vr[k], ar[k]);
  // slot it % P: phase factors of in_row(it); stage st of iteration it uses
  // slot (it - st - 1) % P.  Slots of rows before the first input row feed
  // only results that are not stored.
  FT f[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    if constexpr (FIELD)
      f[q] = FT{};
    else
      f[q] = Stored<T>::of(const_factors(a.ph));
  }
  // y movers of stage st, slot it % 2: the stage's input row two iterations
  // back (r movers when marching up, l movers when down)
  Mov<T> mv[NS][2];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    zero(mv[q][0]);
    zero(mv[q][1]);
  }
  for (int trip = 0;; ++trip) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int it = trip * U + k;
      // wave-uniform exit; the loads issued for later rows are simply dropped
      if (it >= nit) return;
      Site<T> cur = ring[k % RS];
      const double vcur = vr[k % RS];
      double acur[3] = {0.0, 0.0, 0.0};
      if constexpr (FIELD) {
        acur[0] = ar[k % RS][0];
        acur[1] = ar[k % RS][1];
        acur[2] = ar[k % RS][2];
      }
      load_in(it + L, ring[(k + L) % RS], vr[(k + L) % RS], ar[(k + L) % RS]);
      if (zero_walls) {  // cells beyond a wall read as zero
        if (!row_in(it)) zero(cur);
        if (EDGE && !c.full && c.out) zero(cur);
      }
      // this row's factors; stage st reads slot (it - st - 1) % P, never the
      // current one, so the plain phase factors are stored at the end of the
      // iteration, after their far-argument repair
      FT& fnew = f[k % P];
      Factors fd{};
      if constexpr (PULSE)
        fnew = pulse_row<TWO>(vcur, acur[0], acur[1], acur[2], a.ph);
      else if constexpr (FIELD)
        fnew = field_factors<TWO, false>(vcur, acur[0], acur[1], acur[2], a.ph);
      else
        fd = factors_of<MODE, TWO>(vcur, a.ph);
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        // Filling the pipeline: stage st has a valid input from iteration
        // 2 st on (stage st - 1's first valid row) and a valid output from
        // 2 st + 2 on (it needs the y movers of the two rows before).  Earlier
        // iterations would compute values no stored row depends on, so they
        // stop here (wave-uniform scalar tests; the bits are unchanged).
        if (it < 2 * st) break;
        if (S::pre_x(st)) {
          Site<T> phi;
          x_transport_inner<T, AX0>(cur, phi);
          cur = phi;
        }
        Mov<T> ry, ly;
        Axis<AX1, T>::movers(cur, ry, ly);
        const bool live = it >= 2 * st + 2;
        Site<T> o;
        if (live) {
          if (UP)
            Axis<AX1, T>::combine(mv[st][k % 2], ly, o);
          else
            Axis<AX1, T>::combine(ry, mv[st][k % 2], o);
        }
        mv[st][k % 2] = UP ? ry : ly;
        if (!live) break;
        if (S::phase(st)) {
          if constexpr (PULSE)
            apply_field(o, pulse_factors<TWO>(f[((k - st - 1) % P + P) % P],
                                              Fs[st / S::kStages], a.ph));
          else if constexpr (FIELD)
            apply_field(o, f[((k - st - 1) % P + P) % P]);
          else
            apply_local<MODE>(o, f[((k - st - 1) % P + P) % P], a.ph);
        }
        if (S::post_x(st)) {
          Site<T> phi;
          x_transport_inner<T, AX0>(o, phi);
          o = phi;
        }
        if (st < NS - 1 && zero_walls) {
          if (!row_in(it - st - 1)) zero(o);
          if (EDGE && !c.full && !c.inside) zero(o);
        }
        cur = o;
      }
      if (it >= 2 * NS && own) {
        store_site(dst + (out_row(it, NS) * nx + c.x) * 8, cur);
        if constexpr (OBS) obs_add_cell(acc, cur, out_row(it, NS), *ob);
      }
      if constexpr (PULSE) {
        // pulse_row repaired far phase arguments itself
      } else if constexpr (FIELD) {
        field_fix<TWO>(fnew, vcur, acur[0], acur[1], acur[2], a.ph);
      } else {
        factors_fix<MODE, TWO>(fd, vcur, a.ph);
        fnew = Stored<T>::of(fd);
      }
    }
  }
}

// K steps of a 1-D line; the wave writes lanes wlane .. 63 - wlane (the
// 64 - 2X lanes where all K steps are valid, or fewer).  NC: components
// stored per cell (4, or 2 for the two-component line)
template <typename T, class S, int K, int AX, int MODE, int NC = 4>
__device__ __forceinline__ void one_row(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t xs, int lane, int wlane) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int X = halo_lanes<S>(K);
  const Lanes c = lanes_of(a.nx, a.periodic, xs, lane);
  const bool own = c.inside && lane >= wlane && lane <= 63 - wlane;  // wlane >= X
  const bool walls = !a.periodic && !c.inside;  // this lane's cell lies beyond a wall
  Site<T> m;
  load_cell<NC, AX>(src, c.col, m);
  if (c.out) zero(m);
  constexpr bool PULSE = MODE == 4;
  constexpr bool FIELD = MODE == 3 || PULSE;
  const bool read_v = (MODE == 2) || (FIELD && V != nullptr) || (MODE < 0 && a.ph.mode == 2);
  const double v = read_v ? V[c.col] : 0.0;
  typename std::conditional<FIELD, typename FactorOf<MODE>::type,
                            typename Stored<T>::type>::type f;
  if constexpr (PULSE) {
    f = pulse_row<TWO>(v, a.At[c.col], a.At[a.cells + c.col], a.At[2 * a.cells + c.col], a.ph);
  } else if constexpr (FIELD) {
    const double ax = a.At[c.col], ay = a.At[a.cells + c.col], az = a.At[2 * a.cells + c.col];
    f = field_factors<TWO, false>(v, ax, ay, az, a.ph);
    field_fix<TWO>(f, v, ax, ay, az, a.ph);
  } else {
    Factors fd = factors_of<MODE, TWO>(v, a.ph);
    factors_fix<MODE, TWO>(fd, v, a.ph);
    f = Stored<T>::of(fd);
  }
#pragma unroll
  for (int s = 0; s < K * S::kStages; ++s) {
    if (S::pre_x(s)) {
      Site<T> o;
      x_transport_inner<T, AX>(m, o);
      m = o;
      if (walls) zero(m);
    }
    if (S::phase(s)) {
      if constexpr (PULSE)
        apply_field(m, pulse_factors<TWO>(f, pulse_step_integral(a.pulse, s / S::kStages), a.ph));
      else if constexpr (FIELD)
        apply_field(m, f);
      else
        apply_local<MODE>(m, f, a.ph);
    }
    if (S::post_x(s)) {
      Site<T> o;
      x_transport_inner<T, AX>(m, o);
      m = o;
      if (walls) zero(m);
    }
  }
  if (own) store_cell<NC, AX>(dst, c.x, m);
}

// march a 2-D segment upwards (up = true) or downwards, writing lanes
// wlane .. 63 - wlane (wlane >= the pass's x transports).  With FP32 state,
// waves with a lane beyond a zero wall run a variant that zeroes those lanes
// at every stage and the others (nearly all) one without that work.  FP64
// marches keep one variant per direction that tests at run time: their code
// is twice as long and two more variants would crowd the instruction cache.
template <typename T, class S, int K, int AX0, int AX1, int MODE, bool OBS = false>
__device__ __forceinline__ void march_dir(const T* __restrict__ src, T* __restrict__ dst,
                                          const double* __restrict__ V, const SweepArgs& a,
                                          int64_t xs, int lane, int64_t jb, int64_t je, bool up,
                                          int wlane, NSum* acc = nullptr,
                                          const ObsArgs* ob = nullptr) {
  // wave-uniform
  const bool edge = sizeof(T) == 8 || !lanes_of(a.nx, a.periodic, xs, 0).full;
  if (edge) {
    if (up)
      march2d<T, S, K, AX0, AX1, true, MODE, true, OBS>(src, dst, V, a, xs, lane, jb, je,
                                                        wlane, acc, ob);
    else
      march2d<T, S, K, AX0, AX1, false, MODE, true, OBS>(src, dst, V, a, xs, lane, jb, je,
                                                         wlane, acc, ob);
  } else {
    if (up)
      march2d<T, S, K, AX0, AX1, true, MODE, false, OBS>(src, dst, V, a, xs, lane, jb, je,
                                                         wlane, acc, ob);
    else
      march2d<T, S, K, AX0, AX1, false, MODE, false, OBS>(src, dst, V, a, xs, lane, jb, je,
                                                          wlane, acc, ob);
  }
}

}  // namespace dirac
