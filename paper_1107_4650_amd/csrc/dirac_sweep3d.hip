// dirac_sweep3d.hip -- the Dirac sweep on 3-D grids (gfx950).
//
// A full lowest-order step (Sec. 2.1) on a 3-D grid: T_x, T_y, T_z, then the
// local step.  A wave marches along z with a plane tile of 64 x cells by TY y
// rows, the y transport rolling over the rows of the tile and the z
// transport rolling over planes.  With FP32 state a pass advances two steps
// (60 output columns, two halo rows in y and two halo planes in z).
#include "dirac_device.h"
#include "dirac_launch.h"
#include "dirac_sweep_impl.h"

namespace dirac {

// ---------------------------------------------------------------------------
// 3-D fused step: march along z, plane tile 64 x TY per wave.  The potential
// of the TY output rows is loaded one plane ahead, so each plane starts with
// the TY independent phase-factor chains, which run while the plane's rows
// are still in flight.
// ---------------------------------------------------------------------------
template <typename T, int TY, bool UP, int MODE>
__device__ __forceinline__ void march3d(const T* __restrict__ src, T* __restrict__ dst,
                                        const double* __restrict__ V, const SweepArgs& a,
                                        int64_t x0, int lane, int64_t y0, int64_t kb,
                                        int64_t ke) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr bool FIELD = MODE == 3;  // local step with a vector potential
  using FT = typename FactorOf<MODE>::type;
  const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane_cells = nx * ny;
  const int nit = static_cast<int>(ke - kb) + 2;
  const int64_t x = x0 + lane;
  const int64_t xv = x < nx ? x : nx - 1;
  const bool read_v = (MODE == 2) || (FIELD && V != nullptr);
  // under a pulse the array holds the profile P and the step's field integral
  // is F P (a pass is one step; the scale is exactly 1 for a static field)
  double fscale = 1.0;
  if constexpr (FIELD)
    if (a.pulse_on) fscale = pulse_step_integral(a.pulse, 0);
  auto kout_of = [&](int it) -> int64_t { return UP ? kb - 2 + it : ke - it + 1; };
  // the potential (and field integrals) of the TY output rows of iteration it
  auto load_v = [&](int it, double* v, double (*at)[3]) {
    int64_t k = kout_of(it);
    k = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const int64_t y = (y0 + t < ny) ? y0 + t : ny - 1;
      const int64_t q = (k * ny + y) * nx + xv;
      v[t] = read_v ? V[q] : 0.0;
      if constexpr (FIELD) {
        at[t][0] = fscale * a.At[q];
        at[t][1] = fscale * a.At[a.cells + q];
        at[t][2] = fscale * a.At[2 * a.cells + q];
      }
    }
  };
  Mov<T> zs1[TY], zs2[TY];
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    zero(zs1[t]);
    zero(zs2[t]);
  }
  double vcur[TY], acur[TY][3];
  load_v(0, vcur, acur);
  for (int it = 0; it < nit; ++it) {
    const int64_t kin = UP ? kb - 1 + it : ke - it;
    const int64_t kout = kout_of(it);
    const int64_t kr = wrap_or_neg(kin, nz, a.periodic);
    // loads of this plane tile (rows y0-1 .. y0+TY) and of the next plane's potential
    Row<T> rows[TY + 2];
#pragma unroll
    for (int t = 0; t < TY + 2; ++t) {
      if (kr >= 0) {
        load_row(src + kr * plane_cells * 8, nx, ny, a.periodic, x0, lane, y0 - 1 + t, rows[t]);
      } else {
        zero(rows[t].m);
        zero(rows[t].h);
      }
    }
    double vnext[TY], anext[TY][3];
    load_v(it + 1, vnext, anext);
    FT fac[TY];
    if constexpr (FIELD) {
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        fac[t] = field_factors<TWO, false>(vcur[t], acur[t][0], acur[t][1], acur[t][2], a.ph);
        field_fix<TWO>(fac[t], vcur[t], acur[t][0], acur[t][1], acur[t][2], a.ph);
      }
    } else {
#pragma unroll
      for (int t = 0; t < TY; ++t) fac[t] = factors_of<MODE, TWO>(vcur[t], a.ph);
#pragma unroll
      for (int t = 0; t < TY; ++t) factors_fix<MODE, TWO>(fac[t], vcur[t], a.ph);
    }
    // x transport of every row, y transport rolling over the rows
    Mov<T> ry1, ry2;
    zero(ry1);
    zero(ry2);
#pragma unroll
    for (int t = 0; t < TY + 2; ++t) {
      Site<T> phi;
      x_transport<T, 0>(rows[t], phi);
      Mov<T> ry, ly;
      Axis<1, T>::movers(phi, ry, ly);
      if (t >= 2) {
        const int ty = t - 2;  // output row y0 + ty
        Site<T> psi2;
        Axis<1, T>::combine(ry2, ly, psi2);
        Mov<T> rz, lz;
        Axis<2, T>::movers(psi2, rz, lz);
        if (it >= 2) {
          Site<T> o;
          if (UP)
            Axis<2, T>::combine(zs2[ty], lz, o);
          else
            Axis<2, T>::combine(rz, zs2[ty], o);
          if constexpr (FIELD)
            apply_field(o, fac[ty]);
          else
            apply_local<MODE>(o, fac[ty], a.ph);
          const int64_t y = y0 + ty;
          if (x < nx && y < ny) store_site(dst + ((kout * ny + y) * nx + x) * 8, o);
        }
        zs2[ty] = zs1[ty];
        zs1[ty] = UP ? rz : lz;
      }
      ry2 = ry1;
      ry1 = ry;
    }
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      vcur[t] = vnext[t];
      if constexpr (FIELD) {
        acur[t][0] = anext[t][0];
        acur[t][1] = anext[t][1];
        acur[t][2] = anext[t][2];
      }
    }
  }
}

template <typename T, int TY, int MODE>
__global__ __launch_bounds__(256) void k_sweep3d(const T* __restrict__ src, T* __restrict__ dst,
                                                 const double* __restrict__ V, SweepArgs a) {
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  const int64_t tile = blk * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  // tile order: x strips fastest, then y row blocks, then z segments
  const int64_t strip = tile % a.nstrips;
  const int64_t rest = tile / a.nstrips;
  const int64_t yblk = rest % a.nyblk;
  const int64_t seg = rest / a.nyblk;
  const int64_t x0 = strip * 64, y0 = yblk * TY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < a.nz) ? kb + a.H : a.nz;
  if (seg & 1)
    march3d<T, TY, false, MODE>(src, dst, V, a, x0, lane, y0, kb, ke);
  else
    march3d<T, TY, true, MODE>(src, dst, V, a, x0, lane, y0, kb, ke);
}

// ---------------------------------------------------------------------------
// 3-D pass of two fused steps (temporal blocking).  A wave holds 64 x
// columns (writing the middle 60) and a block of TY y rows, and marches along
// z.  Each plane iteration reads TY + 4 rows of the input plane (two halo rows
// on each side); the rows of the next plane and their potential are loaded
// while the current plane computes.  The first step completes, in streaming
// order, the TY + 2 rows y0 - 1 .. y0 + TY of the plane one behind (its own y
// halo for the second step); each of those rows feeds the second step at
// once, which completes the TY output rows of the plane two behind.  The z
// movers of two previous planes are kept per step and row.  The phase
// factors of a row are formed once, by the first step, and kept for the
// second step, which reaches the same row and plane one iteration later.
// Intermediate states are rounded as stored steps and zeroed outside the box
// with zero walls, so the pass gives the bits of two single steps.
// ---------------------------------------------------------------------------
template <typename T, int TY, bool UP, int MODE, bool EDGE>
__device__ __forceinline__ void march3d_x2(const T* __restrict__ src, T* __restrict__ dst,
                                           const double* __restrict__ V, const SweepArgs& a,
                                           int64_t xs, int lane, int64_t y0, int64_t kb,
                                           int64_t ke) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int K = 2;
  constexpr int R0 = TY + 4;  // rows read per plane
  constexpr int R1 = TY + 2;  // rows completed by the first step
  const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane_cells = nx * ny;
  const int nit = static_cast<int>(ke - kb) + 2 * K;
  const Lanes c = lanes_of(nx, a.periodic, xs, lane);
  const bool own = c.inside && lane >= K && lane <= 63 - K;
  // per-lane offsets fit 32 bits (a row holds fewer than 2^28 cells); row and
  // plane bases are wave-uniform
  const uint32_t cell_off = static_cast<uint32_t>(c.col) * 8u;
  const uint32_t v_off = static_cast<uint32_t>(c.col);
  const bool read_v = (MODE == 2);
  const bool zero_walls = !a.periodic;
  auto in_plane = [&](int it) -> int64_t { return UP ? kb - K + it : ke - 1 + K - it; };
  auto plane_of = [&](int it, int st) -> int64_t {
    return UP ? in_plane(it) - st : in_plane(it) + st;
  };
  // wall tests as wave-uniform 32-bit compares: plane plane_of(it, st) lies
  // in the box iff klo <= it - st < khi (it - st spans -K .. nit), and bit t
  // of ymask says whether row y0 - 2 + t does
  auto clamp_it = [&](int64_t e) -> int {
    return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
  };
  const int64_t klo64 = UP ? K - kb : ke + K - nz;
  const int klo = clamp_it(klo64), khi = clamp_it(klo64 + nz);
  auto plane_in = [&](int e) -> bool { return e >= klo && e < khi; };
  uint32_t ymask = 0;
#pragma unroll
  for (int t = 0; t < R0; ++t)
    if (y0 - 2 + t >= 0 && y0 - 2 + t < ny) ymask |= 1u << t;
  ymask = __builtin_amdgcn_readfirstlane(ymask);
  // input rows of iteration it (slot it % 2) and the V of its first-step rows;
  // the plane of iteration it + 1 is loaded while iteration it computes
  Site<T> buf[2][R0];
  double vb[2][R1];
  auto load_plane = [&](int it, Site<T>* rows, double* v) {
    const int64_t kr = read_row(in_plane(it), nz, a.periodic);
    const T* plane = src + kr * plane_cells * 8;
#pragma unroll
    for (int t = 0; t < R0; ++t)
      load_site(plane + read_row(y0 - 2 + t, ny, a.periodic) * nx * 8 + cell_off, rows[t]);
    const int64_t k1r = read_row(plane_of(it, 1), nz, a.periodic);
#pragma unroll
    for (int u = 0; u < R1; ++u)
      v[u] = read_v ? (V + (k1r * ny + read_row(y0 - 1 + u, ny, a.periodic)) * nx)[v_off] : 0.0;
  };
  // z movers of two previous planes, per step and row (slot it % 2)
  Mov<T> zm1[2][R1], zm2[2][TY];
  // factors of the output rows, formed by the first step on plane k1 and used
  // by the second step on the same plane one iteration later
  Factors fc[TY];
#pragma unroll
  for (int w = 0; w < TY; ++w) fc[w] = Factors{};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int u = 0; u < R1; ++u) {
      zero(zm1[q][u]);
      vb[q][u] = 0.0;
    }
#pragma unroll
    for (int w = 0; w < TY; ++w) zero(zm2[q][w]);
  }
  load_plane(0, buf[0], vb[0]);
  for (int pair = 0;; ++pair) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int it = 2 * pair + k;
      if (it >= nit) return;
      const int64_t k2 = plane_of(it, 2);
      load_plane(it + 1, buf[k ^ 1], vb[k ^ 1]);
      Factors pend{};  // factors of the previous first-step row
      // streaming over rows: first step (y movers of two rows back), then second
      Mov<T> ya1, yb1, ya2, yb2;  // r movers of rows t - 1 and t - 2 (first, second step)
      zero(ya1);
      zero(yb1);
      zero(ya2);
      zero(yb2);
#pragma unroll
      for (int t = 0; t < R0; ++t) {
        Site<T> in = buf[k][t];
        if (zero_walls) {
          if (!plane_in(it) || !((ymask >> t) & 1u)) zero(in);
          if (EDGE && c.out) zero(in);
        }
        Site<T> phi;
        x_transport_inner<T, 0>(in, phi);
        Mov<T> ry, ly;
        Axis<1, T>::movers(phi, ry, ly);
        if (t >= 2) {
          const int u = t - 2;  // first-step row y0 - 1 + u of plane k1
          Site<T> py;
          Axis<1, T>::combine(yb1, ly, py);
          Mov<T> rz, lz;
          Axis<2, T>::movers(py, rz, lz);
          Site<T> o1;
          if (UP)
            Axis<2, T>::combine(zm1[k][u], lz, o1);
          else
            Axis<2, T>::combine(rz, zm1[k][u], o1);
          zm1[k][u] = UP ? rz : lz;
          Factors f1 = factors_of<MODE, TWO>(vb[k][u], a.ph);
          factors_fix<MODE, TWO>(f1, vb[k][u], a.ph);
          apply_local<MODE>(o1, f1, a.ph);
          if (zero_walls) {
            if (!plane_in(it - 1) || !((ymask >> (u + 1)) & 1u)) zero(o1);
            if (EDGE && !c.inside) zero(o1);
          }
          // second step on first-step row u
          Site<T> phi2;
          x_transport_inner<T, 0>(o1, phi2);
          Mov<T> ry2, ly2;
          Axis<1, T>::movers(phi2, ry2, ly2);
          if (u >= 2) {
            const int w = u - 2;  // output row y0 + w of plane k2
            Site<T> py2;
            Axis<1, T>::combine(yb2, ly2, py2);
            Mov<T> rz2, lz2;
            Axis<2, T>::movers(py2, rz2, lz2);
            Site<T> o2;
            if (UP)
              Axis<2, T>::combine(zm2[k][w], lz2, o2);
            else
              Axis<2, T>::combine(rz2, zm2[k][w], o2);
            zm2[k][w] = UP ? rz2 : lz2;
            apply_local<MODE>(o2, fc[w], a.ph);
            const int64_t y = y0 + w;
            if (it >= 2 * K && own && y < ny)
              store_site(dst + (k2 * ny + y) * nx * 8 + cell_off, o2);
            // row y0 + w of plane k1 takes these factors in the next iteration
            fc[w] = pend;
          }
          pend = f1;
          yb2 = ya2;
          ya2 = ry2;
        }
        yb1 = ya1;
        ya1 = ry;
      }
    }
  }
}

template <typename T, int TY, int MODE>
__global__ __launch_bounds__(256, kMinBlocks3D2) void k_sweep3d_x2(const T* __restrict__ src,
                                                       T* __restrict__ dst,
                                                       const double* __restrict__ V,
                                                       SweepArgs a) {
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  const int64_t tile = blk * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  // tile order: x strips fastest, then y row blocks, then z segments; with
  // blocks of two rows (FP64), whose halo rows outnumber their own, y row
  // blocks fastest, so that the waves of a workgroup share their halo rows
  constexpr bool kYFast = TY <= 2;
  const int64_t n0 = kYFast ? a.nyblk : a.nstrips;
  const int64_t n1 = kYFast ? a.nstrips : a.nyblk;
  const int64_t i0 = tile % n0;
  const int64_t rest = tile / n0;
  const int64_t i1 = rest % n1;
  const int64_t seg = rest / n1;
  const int64_t strip = kYFast ? i1 : i0;
  const int64_t yblk = kYFast ? i0 : i1;
  const int64_t xs = strip * strip_width(2) - 2, y0 = yblk * TY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < a.nz) ? kb + a.H : a.nz;
  // waves with a lane beyond a zero wall zero those lanes at every step;
  // the others skip that work
  const bool edge = !lanes_of(a.nx, a.periodic, xs, 0).full;
  if (edge) {
    if (seg & 1)
      march3d_x2<T, TY, false, MODE, true>(src, dst, V, a, xs, lane, y0, kb, ke);
    else
      march3d_x2<T, TY, true, MODE, true>(src, dst, V, a, xs, lane, y0, kb, ke);
  } else {
    if (seg & 1)
      march3d_x2<T, TY, false, MODE, false>(src, dst, V, a, xs, lane, y0, kb, ke);
    else
      march3d_x2<T, TY, true, MODE, false>(src, dst, V, a, xs, lane, y0, kb, ke);
  }
}

// ---------------------------------------------------------------------------
// 3-D second-order step (Sec. 2.4): A(dt/4) B(dt/2) A(dt/4) C(dt/2) D(dt)
// C(dt/2) A(dt/4) B(dt/2) A(dt/4), with c dt/4 = a: A is the one-cell x
// shift, B and C the two-cell y and z shifts.  A group of steps runs as one
// pass per step (the x-y transports that open the step, preceded from the
// second step on by those that close the previous one, then C D C along z)
// and a pass with the closing A B A.  The factors 1/2 of the eight transports
// are deferred to the local step (scale 2^-8), so the intermediate states
// carry exact powers of two.
// ---------------------------------------------------------------------------

// r wrapped into [0, n) around a periodic box, else clamped (cells beyond a
// wall are zeroed where they are used)
__device__ __forceinline__ int64_t wrap_or_clamp(int64_t r, int64_t n, int periodic) {
  if (periodic) return ((r % n) + n) % n;
  return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

// A B A on row j of plane k: a wave holds 64 columns and writes the middle 60
template <typename T>
__global__ __launch_bounds__(256) void k_strang3d_aba(const T* __restrict__ src,
                                                      T* __restrict__ dst, SweepArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = int64_t(blockIdx.x) * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  const int64_t nx = a.nx, ny = a.ny;
  const int64_t strip = tile % a.nstrips;
  const int64_t rest = tile / a.nstrips;
  const int64_t j = rest % ny, k = rest / ny;
  const Lanes c = lanes_of(nx, a.periodic, strip * strip_width(2) - 2, lane);
  const bool walls = !a.periodic;
  auto load = [&](int64_t r, Site<T>& s) {
    load_site(src + ((k * ny + wrap_or_clamp(r, ny, a.periodic)) * nx + c.col) * 8, s);
    if (walls && (r < 0 || r >= ny || (!c.full && c.out))) zero(s);
  };
  Site<T> lo, hi, alo, ahi;
  load(j - 2, lo);
  load(j + 2, hi);
  x_transport_inner<T, 0>(lo, alo);
  x_transport_inner<T, 0>(hi, ahi);
  if (walls && !c.full && !c.inside) {
    zero(alo);
    zero(ahi);
  }
  // B: the +1 movers of row j - 2 and the -1 movers of row j + 2 reach row j
  Mov<T> r1, l1, r2, l2;
  Axis<1, T>::movers(alo, r1, l1);
  Axis<1, T>::movers(ahi, r2, l2);
  Site<T> b, o;
  Axis<1, T>::combine(r1, l2, b);
  if (walls && !c.full && !c.inside) zero(b);
  x_transport_inner<T, 0>(b, o);
  if (c.inside && lane >= 2 && lane <= 61) store_site(dst + ((k * ny + j) * nx + c.x) * 8, o);
}

// Wall test of a march: position kb - 4 + it (rows or planes) lies in [0, n)
// iff lo <= it < hi, with lo, hi clamped to 32 bits (it spans 0 .. nit).
struct MarchBounds {
  int lo, hi;
  __device__ MarchBounds(int64_t kb, int64_t n, int nit) {
    auto clamp_it = [&](int64_t e) -> int {
      return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
    };
    lo = clamp_it(4 - kb);
    hi = clamp_it(4 - kb + n);
  }
  __device__ bool in(int it) const { return it >= lo && it < hi; }
};

// rows per wave and resident blocks per CU of the fused second-order pass
template <typename T> struct StrangShape;
template <> struct StrangShape<float> { static constexpr int TY = 2, kMinBlocks = 2; };
template <> struct StrangShape<double> { static constexpr int TY = 2, kMinBlocks = 1; };

// One pass of the 3-D second-order step: the transports along x and y that
// open it (A B A for the first step of a group, else the A B A that closes
// the previous step followed by the one that opens this step), then C D C.
// A wave holds 64 columns and TY rows and marches up a segment [kb, ke) of
// planes.  Reading plane n it applies the x-y transports to its rows (a march
// over the TY + 2 XL rows of the tile with two four-slot rings of right
// movers, XL = 2 or 4 halo rows and lanes on each side) and feeds each output
// row to C D C along z, which completes C at plane n - 2, applies D there
// (phase mode 3: with the field integral of the vector potential) and
// completes the second C at plane n - 4 (rings of the right movers of the last
// four planes per row).  The x-y results are rounded as a stored pass would
// round them, so the bits are those of the separate passes.
template <typename T, int MODE, bool FIRST>
__global__ __launch_bounds__(256, StrangShape<T>::kMinBlocks) void k_strang3d_step(
    const T* __restrict__ src, T* __restrict__ dst, const double* __restrict__ V,
    SweepArgs a) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int TY = StrangShape<T>::TY;
  constexpr int XL = FIRST ? 2 : 4;  // halo lanes and rows
  constexpr int NR = TY + 2 * XL;    // rows read per plane
  const int lane = threadIdx.x & 63;
  const int64_t tile = int64_t(blockIdx.x) * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
  // tile order: row blocks fastest (neighbours share their halo rows), then
  // x strips, then z segments
  const int64_t yblk = tile % a.nyblk;
  const int64_t rest = tile / a.nyblk;
  const int64_t strip = rest % a.nstrips, seg = rest / a.nstrips;
  const int64_t y0 = yblk * TY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < nz) ? kb + a.H : nz;
  const int nit = static_cast<int>(ke - kb) + 8;
  const Lanes c = lanes_of(nx, a.periodic, strip * strip_width(XL) - XL, lane);
  const bool own = c.inside && lane >= XL && lane <= 63 - XL;
  const bool walls = !a.periodic;
  const bool lanes_out = walls && !c.full && !c.inside;
  const MarchBounds planes(kb, nz, nit);
  // phase mode 3: under a pulse the field array holds the profile P and the
  // step's integral is F P (a pass carries one step's D)
  double fscale = 1.0;
  if constexpr (MODE == 3)
    if (a.pulse_on) fscale = pulse_step_integral(a.pulse, 0);
  // the rows read (wrapped or clamped) and, bit t, whether row y0 - XL + t
  // lies in the box
  int64_t rowoff[NR];
  uint32_t rin = 0;
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int64_t y = y0 - XL + t;
    rowoff[t] = wrap_or_clamp(y, ny, a.periodic) * nx + c.col;
    if (y >= 0 && y < ny) rin |= 1u << t;
  }
  rin = __builtin_amdgcn_readfirstlane(rin);
  auto row_in = [&](int t) -> bool { return (rin >> t) & 1u; };
  auto A = [&](const Site<T>& in, Site<T>& out) {
    x_transport_inner<T, 0>(in, out);
    if (lanes_out) zero(out);
  };
  Mov<T> rs[4][TY], rd[4][TY];  // right movers of the input / of C D, slot: plane % 4
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int w = 0; w < TY; ++w) {
      zero(rs[q][w]);
      zero(rd[q][w]);
    }
  }
  for (int base = 0;; base += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int it = base + u;
      if (it >= nit) return;
      const int64_t n = kb - 4 + it;  // plane read
      const bool n_in = planes.in(it);
      const T* plane = src + wrap_or_clamp(n, nz, a.periodic) * ny * nx * 8;
      const int64_t vplane = wrap_or_clamp(n - 2, nz, a.periodic) * ny;
      Mov<T> ra[4], rc[4];  // right movers after the first / second A, slot: row % 4
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        zero(ra[q]);
        zero(rc[q]);
      }
#pragma unroll
      for (int t = 0; t < NR; ++t) {
        Site<T> sv, tt, yb, o;
        load_site(plane + rowoff[t] * 8, sv);
        if (walls && (!row_in(t) || (!c.full && c.out))) zero(sv);
        A(sv, tt);
        Mov<T> r, l;
        Axis<1, T>::movers(tt, r, l);
        if (t < 4) {
          ra[t % 4] = r;
          continue;
        }
        Axis<1, T>::combine(ra[t % 4], l, yb);  // first B at tile row t - 2
        ra[t % 4] = r;
        if (lanes_out) zero(yb);
        int w;  // output row y0 + w of the x-y transports
        if constexpr (FIRST) {
          x_transport_inner<T, 0>(yb, o);
          w = t - 4;
        } else {
          Site<T> t2, cc;
          A(yb, t2);
          if (walls && !row_in(t - 2)) zero(t2);  // row beyond a wall
          A(t2, cc);                              // the next step's A B A starts
          Mov<T> r2, l2;
          Axis<1, T>::movers(cc, r2, l2);
          if (t < 8) {
            rc[t % 4] = r2;
            continue;
          }
          Axis<1, T>::combine(rc[t % 4], l2, yb);  // second B at tile row t - 4
          rc[t % 4] = r2;
          if (lanes_out) zero(yb);
          x_transport_inner<T, 0>(yb, o);
          w = t - 8;
        }
        // C D C along z for row y0 + w
        if (walls && !n_in) zero(o);
        Axis<2, T>::movers(o, r, l);
        Site<T> cd, out;
        Axis<2, T>::combine(rs[u][w], l, cd);  // C at plane n - 2
        rs[u][w] = r;
        const int64_t q = (vplane + wrap_or_clamp(y0 + w, ny, a.periodic)) * nx + c.col;
        if constexpr (MODE == 3) {  // D with the step's field integral
          const double v = V ? V[q] : 0.0;
          const double ax = fscale * a.At[q], ay = fscale * a.At[a.cells + q],
                       az = fscale * a.At[2 * a.cells + q];
          FieldFactors f = field_factors<TWO, false>(v, ax, ay, az, a.ph);
          field_fix<TWO>(f, v, ax, ay, az, a.ph);
          apply_field(cd, f);
        } else {
          const double v = (MODE == 2) ? V[q] : 0.0;
          Factors f = factors_of<MODE, TWO>(v, a.ph);
          factors_fix<MODE, TWO>(f, v, a.ph);
          apply_local<MODE>(cd, f, a.ph);
        }
        if (walls && !planes.in(it - 2)) zero(cd);
        Axis<2, T>::movers(cd, r, l);
        Axis<2, T>::combine(rd[(u + 2) % 4][w], l, out);  // second C at plane n - 4
        rd[(u + 2) % 4][w] = r;
        if (it >= 8 && own && y0 + w < ny)
          store_site(dst + (((n - 4) * ny + y0 + w) * nx + c.x) * 8, out);
      }
    }
  }
}

template <typename T, bool FIRST>
static const void* strang_step_kernel(int mode) {
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_strang3d_step<T, 0, FIRST>);
    case 1: return reinterpret_cast<const void*>(&k_strang3d_step<T, 1, FIRST>);
    case 3: return reinterpret_cast<const void*>(&k_strang3d_step<T, 3, FIRST>);
    default: return reinterpret_cast<const void*>(&k_strang3d_step<T, 2, FIRST>);
  }
}

// waves of a step pass the device holds at once, measured when a plan that
// uses the pass is created (never while a stream is being captured)
template <typename T, bool FIRST>
static int& strang_resident() {
  static int waves = 0;
  return waves;
}

template <typename T, bool FIRST>
static void strang_measure() {
  int occ = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, strang_step_kernel<T, FIRST>(2), 256,
                                                   0) != hipSuccess) {
    (void)hipGetLastError();
    occ = 0;
  }
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 0;
  }
  strang_resident<T, FIRST>() =
      (occ > 0 ? occ : StrangShape<T>::kMinBlocks) * 4 * (cus > 0 ? cus : 256);
}

void strang3d_prepare(bool fp64) {
  if (fp64) {
    strang_measure<double, true>();
    strang_measure<double, false>();
  } else {
    strang_measure<float, true>();
    strang_measure<float, false>();
  }
}

// grid of a fused second-order pass: z segments from a cost model, (rounds of
// resident waves) x (H + 8 plane iterations)
template <typename T, bool FIRST>
static int64_t strang_step_grid(const SweepArgs& a, SweepArgs& t) {
  constexpr int TY = StrangShape<T>::TY;
  constexpr int XL = FIRST ? 2 : 4;
  int resident = strang_resident<T, FIRST>();
  if (resident <= 0) resident = StrangShape<T>::kMinBlocks * 4 * 256;
  t = a;
  t.nstrips = (a.nx + strip_width(XL) - 1) / strip_width(XL);
  t.nyblk = (a.ny + TY - 1) / TY;
  const int64_t per_seg = t.nstrips * t.nyblk;
  int64_t best_H = a.nz, best_cost = -1;
  for (int64_t nseg = 1; nseg <= 64 && nseg <= a.nz; ++nseg) {
    const int64_t H = (a.nz + nseg - 1) / nseg;
    const int64_t segs = (a.nz + H - 1) / H;
    const int64_t cost = ((per_seg * segs + resident - 1) / resident) * (H + 8);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best_H = H;
    }
  }
  if (best_H > INT32_MAX - 64) return int64_t(INT32_MAX) + 1;  // refused by the caller
  t.H = static_cast<int>(best_H);
  t.nseg = (a.nz + best_H - 1) / best_H;
  t.ntiles = per_seg * t.nseg;
  return (t.ntiles + 3) / 4;
}

template <typename T>
static hipError_t strang3d_t(const void* src, void* dst, void* mid, const double* V,
                             const SweepArgs& a, int64_t nsteps, hipStream_t st) {
  const T* s = static_cast<const T*>(src);
  T* d = static_cast<T*>(dst);
  T* m = static_cast<T*>(mid);
  auto plane_grid = [&](int width, SweepArgs& t) {
    t = a;
    t.nstrips = (a.nx + width - 1) / width;
    t.ntiles = t.nstrips * a.ny * a.nz;
    return (t.ntiles + 3) / 4;
  };
  SweepArgs ab, first, next;
  const int64_t bab = plane_grid(strip_width(2), ab);
  const int64_t bfirst = strang_step_grid<T, true>(a, first);
  const int64_t bnext = strang_step_grid<T, false>(a, next);
  if (bab > INT32_MAX || bfirst > INT32_MAX || bnext > INT32_MAX) return hipErrorInvalidValue;
  const int mode = a.ph.mode;
  // A B A + C D C, then per further step the closing A B A of one step and the
  // opening one of the next + C D C, and a closing A B A: nsteps + 1 passes.
  // The first pass writes the buffer that makes the last one land in `mid`.
  auto step_pass = [&](bool first_pass, int64_t step, const T* in, T* out) {
    SweepArgs t = first_pass ? first : next;
    t.pulse.n0 += step;  // the pulse's step index of this pass's D
    const dim3 g(static_cast<unsigned>(first_pass ? bfirst : bnext));
    if (first_pass) {
      switch (mode) {
        case 0: hipLaunchKernelGGL((k_strang3d_step<T, 0, true>), g, dim3(256), 0, st, in, out, V, t); break;
        case 1: hipLaunchKernelGGL((k_strang3d_step<T, 1, true>), g, dim3(256), 0, st, in, out, V, t); break;
        case 3: hipLaunchKernelGGL((k_strang3d_step<T, 3, true>), g, dim3(256), 0, st, in, out, V, t); break;
        default: hipLaunchKernelGGL((k_strang3d_step<T, 2, true>), g, dim3(256), 0, st, in, out, V, t); break;
      }
    } else {
      switch (mode) {
        case 0: hipLaunchKernelGGL((k_strang3d_step<T, 0, false>), g, dim3(256), 0, st, in, out, V, t); break;
        case 1: hipLaunchKernelGGL((k_strang3d_step<T, 1, false>), g, dim3(256), 0, st, in, out, V, t); break;
        case 3: hipLaunchKernelGGL((k_strang3d_step<T, 3, false>), g, dim3(256), 0, st, in, out, V, t); break;
        default: hipLaunchKernelGGL((k_strang3d_step<T, 2, false>), g, dim3(256), 0, st, in, out, V, t); break;
      }
    }
  };
  T* cur = (nsteps % 2 == 1) ? m : d;
  T* other = (cur == m) ? d : m;
  step_pass(true, 0, s, cur);
  for (int64_t n = 1; n < nsteps; ++n) {
    step_pass(false, n, cur, other);
    T* t = cur;
    cur = other;
    other = t;
  }
  // cur == m here: the closing A B A into dst
  hipLaunchKernelGGL((k_strang3d_aba<T>), dim3(static_cast<unsigned>(bab)), dim3(256), 0, st, cur,
                     d, ab);
  return hipGetLastError();
}

hipError_t launch_strang3d(bool fp64, const void* src, void* dst, void* mid, const double* V,
                           const SweepArgs& a, int64_t nsteps, hipStream_t st) {
  if (nsteps < 1) return hipErrorInvalidValue;
  return fp64 ? strang3d_t<double>(src, dst, mid, V, a, nsteps, st)
              : strang3d_t<float>(src, dst, mid, V, a, nsteps, st);
}

// ---- 3-D kernels: one step, or a pass of two fused steps ---------------------
template <typename T>
static const void* kernel3d(int depth, int mode) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int TY1 = F64 ? kTY3D_F64 : kTY3D_F32;
  if (depth == 2) {  // phase modes 0 to 2
    constexpr int TY2 = F64 ? kTY3D2_F64 : kTY3D2_F32;
    switch (mode) {
      case 0: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, TY2, 0>);
      case 1: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, TY2, 1>);
      case 2: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, TY2, 2>);
      default: return nullptr;
    }
  }
  if (depth != 1) return nullptr;
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_sweep3d<T, TY1, 0>);
    case 1: return reinterpret_cast<const void*>(&k_sweep3d<T, TY1, 1>);
    case 2: return reinterpret_cast<const void*>(&k_sweep3d<T, TY1, 2>);
    case 3: return reinterpret_cast<const void*>(&k_sweep3d<T, TY1, 3>);
    default: return nullptr;
  }
}

static int occ_of(const void* kernel) {
  if (!kernel) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int occupancy3d(bool fp64, int mode, int depth) {
  const int m = mode < 0 || mode > 3 ? 2 : mode;
  return occ_of(fp64 ? kernel3d<double>(depth, m) : kernel3d<float>(depth, m));
}

hipError_t launch_sweep3d(bool fp64, int depth, const void* src, void* dst, const double* V,
                          const SweepArgs& a, int blocks, hipStream_t st) {
  const int m = a.ph.mode < 0 || a.ph.mode > 3 ? 2 : a.ph.mode;
  const void* fn = fp64 ? kernel3d<double>(depth, m) : kernel3d<float>(depth, m);
  if (!fn || blocks <= 0) return hipErrorInvalidValue;
  SweepArgs args = a;
  void* kargs[] = {const_cast<void**>(&src), &dst, const_cast<double**>(&V), &args};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
}

}  // namespace dirac
