// dirac_sweep3d.hip -- the Dirac sweep on 3-D grids (gfx950).
//
// A full lowest-order step (Sec. 2.1) on a 3-D grid: T_x, T_y, T_z, then the
// local step.  A wave marches along z with a plane tile of 64 x cells by TY y
// rows, the y transport rolling over the rows of the tile and the z
// transport rolling over planes.  With FP32 state a pass advances two steps
// (60 output columns, two halo rows in y and two halo planes in z).
#include "dirac_device.h"
#include "dirac_launch.h"
#include "dirac_obs.h"
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
// 3-D pass of two fused steps (temporal blocking).  A workgroup of four waves
// holds 64 x columns (writing the middle 60) and WY = 4 TW y rows (TW = 2
// output rows per wave, WY = 8) and marches along z.  Each plane iteration shares the work
// of the tile's rows among the waves through LDS, so no row is transported
// twice:
//  1. each wave reads TW + 1 of the WY + 4 input rows of the plane (two halo
//     rows on each side), applies the x transport and leaves the y movers in
//     LDS;
//  2. after a barrier, each wave completes the first step (y and z transports
//     and D) on its own TW rows of the plane one behind -- waves 0 and 3 also
//     on the halo row y0 - 1 or y0 + WY that the second step needs -- applies
//     the second step's x transport and leaves those y movers in LDS;
//  3. after a second barrier, each wave completes the second step on its own
//     rows of the plane two behind.
// The z movers of two previous planes are kept per step and row.  The phase
// factors of an own row are formed once, by the first step, and kept for the
// second step, which reaches the same row and plane one iteration later.
// Intermediate states are rounded as stored steps and zeroed outside the box
// with zero walls, so the pass gives the bits of two single steps.
// ---------------------------------------------------------------------------
template <typename T> struct X2Tile {
  static constexpr int WY = sizeof(T) == 8 ? kTY3D2_F64 : kTY3D2_F32;  // output rows
  static constexpr int TW = WY / 4;                                  // per wave
  static constexpr int NI = WY + 4;  // input rows per plane
  static constexpr int N1 = NI / 4;  // input rows per wave
  static constexpr int NS = WY + 2;  // first-step rows per plane
  static_assert(NI <= 32, "row mask");
};

// y movers of the input rows (index t: row y0 - 2 + t): right movers of rows
// t < NI - 2 at [t], left movers of rows t >= 2 at [t - 2]; of the
// first-step rows (index u: row y0 - 1 + u): right movers of u < NS - 2 at
// [u], left movers of u >= 2 at [u - 2]
// (16-byte aligned, so that a lane's mover moves as one 128-bit LDS access)
template <typename T> struct alignas(16) X2Lds {
  using S = X2Tile<T>;
  Mov<T> r1[S::NI - 2][64], l1[S::NI - 2][64];
  Mov<T> r2[S::NS - 2][64], l2[S::NS - 2][64];
};

// OBS: also add the observables of every stored cell to the lane's sums acc
template <typename T, bool UP, int MODE, bool EDGE, bool OBS = false>
__device__ __forceinline__ void march3d_x2(const T* __restrict__ src, T* __restrict__ dst,
                                           const double* __restrict__ V, const SweepArgs& a,
                                           X2Lds<T>& sh, int lane, int wv, int64_t xs,
                                           int64_t y0, int64_t kb, int64_t ke,
                                           NSum* acc = nullptr, const ObsArgs* ob = nullptr) {
  using S = X2Tile<T>;
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int K = 2, TW = S::TW, NI = S::NI, N1 = S::N1, NS = S::NS;
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
  // of ymask says whether input row y0 - 2 + t does
  auto clamp_it = [&](int64_t e) -> int {
    return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
  };
  const int64_t klo64 = UP ? K - kb : ke + K - nz;
  const int klo = clamp_it(klo64), khi = clamp_it(klo64 + nz);
  auto plane_in = [&](int e) -> bool { return e >= klo && e < khi; };
  uint32_t ymask = 0;
#pragma unroll
  for (int t = 0; t < NI; ++t)
    if (y0 - 2 + t >= 0 && y0 - 2 + t < ny) ymask |= 1u << t;
  ymask = __builtin_amdgcn_readfirstlane(ymask);
  // first-step rows of this wave: slots j < TW are its own rows u = 1 + wv TW
  // + j (output rows y0 + wv TW + j); slot TW is the halo row u = 0 (wave 0)
  // or u = NS - 1 (wave 3)
  const bool halo = (wv == 0) || (wv == 3);
  const int u_halo = (wv == 0) ? 0 : NS - 1;
  auto srow = [&](int j) -> int { return j < TW ? 1 + wv * TW + j : u_halo; };
  int64_t inrow[N1], srow_off[TW + 1];
#pragma unroll
  for (int j = 0; j < N1; ++j) inrow[j] = read_row(y0 - 2 + wv * N1 + j, ny, a.periodic) * nx * 8;
#pragma unroll
  for (int j = 0; j <= TW; ++j) srow_off[j] = read_row(y0 - 1 + srow(j), ny, a.periodic) * nx;
  Mov<T> zm1[2][TW + 1], zm2[2][TW];  // z movers of two previous planes, slot it % 2
  Factors fc[TW];  // factors of the own rows, formed by the first step one iteration earlier
#pragma unroll
  for (int j = 0; j < TW; ++j) fc[j] = Factors{};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int j = 0; j <= TW; ++j) zero(zm1[q][j]);
#pragma unroll
    for (int j = 0; j < TW; ++j) zero(zm2[q][j]);
  }
  // this wave's input rows of the plane read at iteration it and the V of its
  // first-step rows on the plane one behind, loaded one iteration ahead
  Site<T> in[N1];
  double vn[TW + 1];
  auto load_inputs = [&](int it) {
    const T* plane = src + read_row(in_plane(it), nz, a.periodic) * plane_cells * 8;
#pragma unroll
    for (int j = 0; j < N1; ++j) load_site(plane + inrow[j] + cell_off, in[j]);
    const double* vp = V + read_row(plane_of(it, 1), nz, a.periodic) * plane_cells;
#pragma unroll
    for (int j = 0; j <= TW; ++j)
      vn[j] = (read_v && (j < TW || halo)) ? (vp + srow_off[j])[v_off] : 0.0;
  };
  load_inputs(0);
  for (int pair = 0;; ++pair) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int it = 2 * pair + k;
      if (it >= nit) return;  // uniform over the workgroup
      const int64_t k2 = plane_of(it, 2);
      double vb[TW + 1];
#pragma unroll
      for (int j = 0; j <= TW; ++j) vb[j] = vn[j];
      // 1. x transport of the input rows, y movers to LDS
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const int t = wv * N1 + j;
        Site<T> s0 = in[j], phi;
        if (zero_walls) {
          if (!plane_in(it) || !((ymask >> t) & 1u)) zero(s0);
          if (EDGE && c.out) zero(s0);
        }
        x_transport_inner<T, 0>(s0, phi);
        Mov<T> ry, ly;
        Axis<1, T>::movers(phi, ry, ly);
        if (t < NI - 2) sh.r1[t][lane] = ry;
        if (t >= 2) sh.l1[t - 2][lane] = ly;
      }
      if (it + 1 < nit) load_inputs(it + 1);
      __syncthreads();
      // 2. first step on the first-step rows of the plane one behind, then the
      //    second step's x transport, y movers to LDS
      Factors fnew[TW];
#pragma unroll
      for (int j = 0; j <= TW; ++j) {
        if (j == TW && !halo) break;
        const int u = srow(j);
        Site<T> py, o1;
        Axis<1, T>::combine(sh.r1[u][lane], sh.l1[u][lane], py);
        Mov<T> rz, lz;
        Axis<2, T>::movers(py, rz, lz);
        if (UP)
          Axis<2, T>::combine(zm1[k][j], lz, o1);
        else
          Axis<2, T>::combine(rz, zm1[k][j], o1);
        zm1[k][j] = UP ? rz : lz;
        Factors f1 = factors_of<MODE, TWO>(vb[j], a.ph);
        factors_fix<MODE, TWO>(f1, vb[j], a.ph);
        apply_local<MODE>(o1, f1, a.ph);
        if (zero_walls) {
          if (!plane_in(it - 1) || !((ymask >> (u + 1)) & 1u)) zero(o1);
          if (EDGE && !c.inside) zero(o1);
        }
        Site<T> phi2;
        x_transport_inner<T, 0>(o1, phi2);
        Mov<T> ry2, ly2;
        Axis<1, T>::movers(phi2, ry2, ly2);
        if (u < NS - 2) sh.r2[u][lane] = ry2;
        if (u >= 2) sh.l2[u - 2][lane] = ly2;
        if (j < TW) fnew[j] = f1;
      }
      __syncthreads();
      // 3. second step on the own rows of the plane two behind
#pragma unroll
      for (int j = 0; j < TW; ++j) {
        const int w = wv * TW + j;  // output row y0 + w: first-step rows w and w + 2
        Site<T> py2, o2;
        Axis<1, T>::combine(sh.r2[w][lane], sh.l2[w][lane], py2);
        Mov<T> rz2, lz2;
        Axis<2, T>::movers(py2, rz2, lz2);
        if (UP)
          Axis<2, T>::combine(zm2[k][j], lz2, o2);
        else
          Axis<2, T>::combine(rz2, zm2[k][j], o2);
        zm2[k][j] = UP ? rz2 : lz2;
        apply_local<MODE>(o2, fc[j], a.ph);
        const int64_t y = y0 + w;
        if (it >= 2 * K && own && y < ny) {
          store_site(dst + (k2 * ny + y) * nx * 8 + cell_off, o2);
          if constexpr (OBS) obs_add_cell3(acc, o2, y, k2, *ob);
        }
        fc[j] = fnew[j];
      }
    }
  }
}

// FP32 state: two waves per SIMD; FP64 state (8-row tiles, two rows per
// wave): one, with the accumulation registers holding the rest
template <typename T, int MODE>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 1 : 2) void k_sweep3d_x2(
    const T* __restrict__ src, T* __restrict__ dst, const double* __restrict__ V, SweepArgs a) {
  __shared__ X2Lds<T> sh;
  const int lane = threadIdx.x & 63;
  const int wv = wave_in_block();
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  if (blk >= a.ntiles) return;  // the whole workgroup
  // tile order: y row blocks fastest (neighbouring tiles share their halo
  // rows), then x strips, then z segments
  const int64_t yblk = blk % a.nyblk;
  const int64_t rest = blk / a.nyblk;
  const int64_t strip = rest % a.nstrips;
  const int64_t seg = rest / a.nstrips;
  const int64_t xs = strip * strip_width(2) - 2, y0 = yblk * X2Tile<T>::WY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < a.nz) ? kb + a.H : a.nz;
  // tiles with a lane beyond a zero wall zero those lanes at every step;
  // the others skip that work
  const bool edge = !lanes_of(a.nx, a.periodic, xs, 0).full;
  if (edge) {
    if (seg & 1)
      march3d_x2<T, false, MODE, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke);
    else
      march3d_x2<T, true, MODE, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke);
  } else {
    if (seg & 1)
      march3d_x2<T, false, MODE, false>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke);
    else
      march3d_x2<T, true, MODE, false>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke);
  }
}

// The two-step pass that also sums the observables of the cells it stores:
// each wave's totals (every lane's column sums, merged in a fixed butterfly)
// go to partials[blk * 4 + wave], for the final reduction in that order
template <typename T, int MODE>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 1 : 2) void k_sweep3d_x2_obs(
    const T* __restrict__ src, T* __restrict__ dst, const double* __restrict__ V, SweepArgs a,
    ObsArgs o, double* __restrict__ partials) {
  __shared__ X2Lds<T> sh;
  const int lane = threadIdx.x & 63;
  const int wv = wave_in_block();
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  if (blk >= a.ntiles) return;  // the whole workgroup
  const int64_t yblk = blk % a.nyblk;
  const int64_t rest = blk / a.nyblk;
  const int64_t strip = rest % a.nstrips;
  const int64_t seg = rest / a.nstrips;
  const int64_t xs = strip * strip_width(2) - 2, y0 = yblk * X2Tile<T>::WY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < a.nz) ? kb + a.H : a.nz;
  NSum acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) acc[q] = NSum{0.0, 0.0};
  const bool edge = !lanes_of(a.nx, a.periodic, xs, 0).full;
  if (edge) {
    if (seg & 1)
      march3d_x2<T, false, MODE, true, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke, acc,
                                             &o);
    else
      march3d_x2<T, true, MODE, true, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke, acc,
                                            &o);
  } else {
    if (seg & 1)
      march3d_x2<T, false, MODE, false, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke, acc,
                                              &o);
    else
      march3d_x2<T, true, MODE, false, true>(src, dst, V, a, sh, lane, wv, xs, y0, kb, ke, acc,
                                             &o);
  }
  obs_column_close(acc, xs + lane, o);  // lanes that stored nothing hold zeros
  wave_merge(acc);
  if (lane == 0) {
    const int64_t w = blk * 4 + wv;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      partials[(w * kQ + q) * 2 + 0] = acc[q].s;
      partials[(w * kQ + q) * 2 + 1] = acc[q].c;
    }
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
  if (periodic) {
    // one wrap covers the halos of any box of a few cells or more; the
    // division only runs for smaller boxes
    if (r < 0 && r >= -n) return r + n;
    if (r >= n && r < 2 * n) return r - n;
    if (r >= 0 && r < n) return r;
    return ((r % n) + n) % n;
  }
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

// rows per wave of the fused second-order pass; a workgroup of four waves
// holds 4 TW rows
template <typename T> struct StrangShape;
template <> struct StrangShape<float> { static constexpr int TW = 2; };
template <> struct StrangShape<double> { static constexpr int TW = 1; };
constexpr int kStrangWaves = 4;

// One pass of the 3-D second-order step: the transports along x and y that
// open it (A B A for the first step of a group, else the A B A that closes
// the previous step followed by the one that opens this step), then C D C.
// A workgroup holds 64 columns and WY = 4 TW rows (TW per wave) and marches
// up a segment [kb, ke) of planes.  For plane n the four waves share the x-y
// transports of the tile's WY + 2 XL rows (XL = 2 or 4 halo rows and lanes on
// each side) through LDS: each wave applies A to its share of the rows read
// and leaves their y movers in LDS; after a barrier, B is formed for the
// rows that are still needed (with the second A B A, shares of those rows go
// through LDS once more), so every x-y transport of the tile is computed
// once.  Each wave then feeds its TW output rows to C D C along z, which
// completes C at plane n - 2, applies D there (phase mode 3: with the field
// integral of the vector potential) and completes the second C at plane
// n - 4 (rings of the right movers of the last four planes per row).  The
// x-y results are rounded as a stored pass would round them, so the bits are
// those of the separate passes.
template <typename T, int MODE, bool FIRST>
__global__ __launch_bounds__(256, 2) void k_strang3d_step(const T* __restrict__ src,
                                                          T* __restrict__ dst,
                                                          const double* __restrict__ V,
                                                          SweepArgs a) {
  constexpr bool TWO = sizeof(T) == 8;
  constexpr int TW = StrangShape<T>::TW;
  constexpr int WY = kStrangWaves * TW;  // output rows of the workgroup
  constexpr int XL = FIRST ? 2 : 4;      // halo lanes and rows
  constexpr int NR = WY + 2 * XL;        // rows read per plane
  constexpr int N1 = NR / kStrangWaves;  // rows read per wave
  constexpr int NL = NR - 4;             // rows whose first-B movers are kept
  constexpr int NB = NL / kStrangWaves;  // second A B A: first-B rows per wave
  constexpr int NBUF = FIRST ? 2 : 1;    // one barrier per plane: two buffers
  static_assert(NR <= 32 && NR % kStrangWaves == 0, "row mask and shares");
  // y movers of the rows read: right movers of tile rows t < NR - 4 at [t],
  // left movers of rows t >= 4 at [t - 4]; after the first B (second A B A
  // only) right movers of rows s in [2, WY + 2) at [s - 2], left movers of
  // rows s in [6, WY + 6) at [s - 6]
  __shared__ Mov<T> r1s[NBUF][NL][64], l1s[NBUF][NL][64];
  __shared__ Mov<T> r2s[FIRST ? 1 : WY][64], l2s[FIRST ? 1 : WY][64];
  const int lane = threadIdx.x & 63;
  const int wv = wave_in_block();
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  if (blk >= a.ntiles) return;  // the whole workgroup
  const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
  // tile order: row blocks fastest (neighbours share their halo rows), then
  // x strips, then z segments
  const int64_t yblk = blk % a.nyblk;
  const int64_t rest = blk / a.nyblk;
  const int64_t strip = rest % a.nstrips, seg = rest / a.nstrips;
  const int64_t y0 = yblk * WY;
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
  // bit t: row y0 - XL + t lies in the box
  uint32_t rin = 0;
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int64_t y = y0 - XL + t;
    if (y >= 0 && y < ny) rin |= 1u << t;
  }
  rin = __builtin_amdgcn_readfirstlane(rin);
  auto row_in = [&](int t) -> bool { return (rin >> t) & 1u; };
  // the rows this wave reads (wrapped or clamped): tile rows wv N1 + j
  int64_t rowoff[N1];
#pragma unroll
  for (int j = 0; j < N1; ++j)
    rowoff[j] = wrap_or_clamp(y0 - XL + wv * N1 + j, ny, a.periodic) * nx + c.col;
  // the output rows of this wave: y0 + wv TW + j
  int64_t voff[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j)
    voff[j] = wrap_or_clamp(y0 + wv * TW + j, ny, a.periodic) * nx + c.col;
  auto A = [&](const Site<T>& in, Site<T>& out) {
    x_transport_inner<T, 0>(in, out);
    if (lanes_out) zero(out);
  };
  Site<T> ld[N1];  // this wave's rows of the plane read
  auto load_rows = [&](int it) {
    const T* plane = src + wrap_or_clamp(kb - 4 + it, nz, a.periodic) * ny * nx * 8;
#pragma unroll
    for (int j = 0; j < N1; ++j) load_site(plane + rowoff[j] * 8, ld[j]);
  };
  Mov<T> rs[4][TW], rd[4][TW];  // right movers of the input / of C D, slot: plane % 4
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int w = 0; w < TW; ++w) {
      zero(rs[q][w]);
      zero(rd[q][w]);
    }
  }
  for (int base = 0;; base += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int it = base + u;
      if (it >= nit) return;  // uniform over the workgroup
      const int64_t n = kb - 4 + it;  // plane read
      const bool n_in = planes.in(it);
      const int bf = FIRST ? (u & 1) : 0;
      load_rows(it);
      // A on this wave's rows of plane n, their y movers to LDS
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const int t = wv * N1 + j;
        Site<T> sv = ld[j], tt;
        if (walls && (!row_in(t) || (!c.full && c.out))) zero(sv);
        A(sv, tt);
        Mov<T> r, l;
        Axis<1, T>::movers(tt, r, l);
        if (t < NR - 4) r1s[bf][t][lane] = r;
        if (t >= 4) l1s[bf][t - 4][lane] = l;
      }
      // potential (and field integrals) of the output rows at plane n - 2
      const int64_t vplane = wrap_or_clamp(n - 2, nz, a.periodic) * ny * nx;
      double vv[TW], ax[TW], ay[TW], az[TW];
#pragma unroll
      for (int j = 0; j < TW; ++j) {
        const int64_t q = vplane + voff[j];
        vv[j] = (MODE == 2 || (MODE == 3 && V != nullptr)) ? V[q] : 0.0;
        if constexpr (MODE == 3) {
          ax[j] = fscale * a.At[q];
          ay[j] = fscale * a.At[a.cells + q];
          az[j] = fscale * a.At[2 * a.cells + q];
        }
      }
      __syncthreads();
      Site<T> o[TW];  // output rows of the x-y transports
      if constexpr (FIRST) {
        // B at tile row w + 2 from rows w and w + 4, then A
#pragma unroll
        for (int j = 0; j < TW; ++j) {
          const int w = wv * TW + j;
          Site<T> yb;
          Axis<1, T>::combine(r1s[bf][w][lane], l1s[bf][w][lane], yb);
          if (lanes_out) zero(yb);
          x_transport_inner<T, 0>(yb, o[j]);
        }
      } else {
        // first B at tile rows s in [2, NR - 2), then A A (closing one step,
        // opening the next), their y movers to LDS
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int s = 2 + wv * NB + j;
          Site<T> yb, t2, cc;
          Axis<1, T>::combine(r1s[0][s - 2][lane], l1s[0][s - 2][lane], yb);
          if (lanes_out) zero(yb);
          A(yb, t2);
          if (walls && !row_in(s)) zero(t2);  // row beyond a wall
          A(t2, cc);
          Mov<T> r2, l2;
          Axis<1, T>::movers(cc, r2, l2);
          if (s < WY + 2) r2s[s - 2][lane] = r2;
          if (s >= 6) l2s[s - 6][lane] = l2;
        }
        __syncthreads();
        // second B at tile row w + 4 from first-B rows w + 2 and w + 6, then A
#pragma unroll
        for (int j = 0; j < TW; ++j) {
          const int w = wv * TW + j;
          Site<T> yb;
          Axis<1, T>::combine(r2s[w][lane], l2s[w][lane], yb);
          if (lanes_out) zero(yb);
          x_transport_inner<T, 0>(yb, o[j]);
        }
      }
      // C D C along z for the output rows y0 + wv TW + j
#pragma unroll
      for (int j = 0; j < TW; ++j) {
        Site<T> oz = o[j];
        if (walls && !n_in) zero(oz);
        Mov<T> r, l;
        Axis<2, T>::movers(oz, r, l);
        Site<T> cd, out;
        Axis<2, T>::combine(rs[u][j], l, cd);  // C at plane n - 2
        rs[u][j] = r;
        if constexpr (MODE == 3) {  // D with the step's field integral
          FieldFactors f = field_factors<TWO, false>(vv[j], ax[j], ay[j], az[j], a.ph);
          field_fix<TWO>(f, vv[j], ax[j], ay[j], az[j], a.ph);
          apply_field(cd, f);
        } else {
          Factors f = factors_of<MODE, TWO>(vv[j], a.ph);
          factors_fix<MODE, TWO>(f, vv[j], a.ph);
          apply_local<MODE>(cd, f, a.ph);
        }
        if (walls && !planes.in(it - 2)) zero(cd);
        Axis<2, T>::movers(cd, r, l);
        Axis<2, T>::combine(rd[(u + 2) % 4][j], l, out);  // second C at plane n - 4
        rd[(u + 2) % 4][j] = r;
        const int64_t y = y0 + wv * TW + j;
        if (it >= 8 && own && y < ny)
          store_site(dst + (((n - 4) * ny + y) * nx + c.x) * 8, out);
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

// workgroups of a step pass the device holds at once, measured when a plan
// that uses the pass is created (never while a stream is being captured)
template <typename T, bool FIRST>
static int& strang_resident() {
  static int groups = 0;
  return groups;
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
  strang_resident<T, FIRST>() = (occ > 0 ? occ : 2) * (cus > 0 ? cus : 256);
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

// grid of a fused second-order pass, one workgroup per tile: z segments from
// a cost model, (rounds of resident workgroups) x (H + 8 plane iterations);
// the grid is a multiple of 8 so that each XCD takes a contiguous run of
// tiles (neighbouring row blocks share their halo rows in its L2)
template <typename T, bool FIRST>
static int64_t strang_step_grid(const SweepArgs& a, SweepArgs& t) {
  constexpr int WY = kStrangWaves * StrangShape<T>::TW;
  constexpr int XL = FIRST ? 2 : 4;
  int resident = strang_resident<T, FIRST>();
  if (resident <= 0) resident = 2 * 256;
  t = a;
  t.nstrips = (a.nx + strip_width(XL) - 1) / strip_width(XL);
  t.nyblk = (a.ny + WY - 1) / WY;
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
  t.xcd_remap = 1;
  return (t.ntiles + 7) / 8 * 8;
}

template <typename T>
static hipError_t strang3d_t(const void* src, void* dst, void* mid, void* mid2, const double* V,
                             const SweepArgs& a, int64_t nsteps, hipStream_t st) {
  const T* s = static_cast<const T*>(src);
  T* d = static_cast<T*>(dst);
  T* m = static_cast<T*>(mid);
  T* m2 = mid2 ? static_cast<T*>(mid2) : d;  // the step passes alternate between m and m2
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
  // The first pass writes the buffer that makes the last one land in `mid`;
  // src is only read by the first pass and dst only written by the last, so
  // with a second scratch state (mid2) src and dst may be the same buffer.
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
  T* cur = (nsteps % 2 == 1) ? m : m2;
  T* other = (cur == m) ? m2 : m;
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

hipError_t launch_strang3d(bool fp64, const void* src, void* dst, void* mid, void* mid2,
                           const double* V, const SweepArgs& a, int64_t nsteps, hipStream_t st) {
  if (nsteps < 1) return hipErrorInvalidValue;
  if (!mid2 && src == dst) return hipErrorInvalidValue;
  return fp64 ? strang3d_t<double>(src, dst, mid, mid2, V, a, nsteps, st)
              : strang3d_t<float>(src, dst, mid, mid2, V, a, nsteps, st);
}

// ---- 3-D kernels: one step, or a pass of two fused steps ---------------------
template <typename T>
static const void* kernel3d(int depth, int mode) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int TY1 = F64 ? kTY3D_F64 : kTY3D_F32;
  if (depth == 2) {  // phase modes 0 to 2
    switch (mode) {
      case 0: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, 0>);
      case 1: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, 1>);
      case 2: return reinterpret_cast<const void*>(&k_sweep3d_x2<T, 2>);
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

template <typename T>
static const void* kernel3d_obs(int mode) {
  switch (mode) {
    case 0: return reinterpret_cast<const void*>(&k_sweep3d_x2_obs<T, 0>);
    case 1: return reinterpret_cast<const void*>(&k_sweep3d_x2_obs<T, 1>);
    case 2: return reinterpret_cast<const void*>(&k_sweep3d_x2_obs<T, 2>);
    default: return nullptr;
  }
}

hipError_t launch_sweep3d_obs(bool fp64, const void* src, void* dst, const double* V,
                              const SweepArgs& a, const ObsArgs& o, double* partials, int blocks,
                              hipStream_t st) {
  const void* fn = fp64 ? kernel3d_obs<double>(a.ph.mode) : kernel3d_obs<float>(a.ph.mode);
  if (!fn || blocks <= 0) return hipErrorInvalidValue;
  SweepArgs args = a;
  ObsArgs oargs = o;
  void* kargs[] = {const_cast<void**>(&src), &dst, const_cast<double**>(&V), &args, &oargs,
                   &partials};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
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
