// dirac_device.h -- device building blocks of the MI355X Dirac sweep (gfx950).
//
// Site layout: one cell = 4 complex components (a, b, c, d) = 8 reals of type
// T, stored (a.re, a.im, b.re, b.im, c.re, c.im, d.re, d.im).
//
// Transport along one axis (eq:sol_dis_1-3, App. A):
//     psi'(i) = 1/2 (I + alpha) psi(i - e) + 1/2 (I - alpha) psi(i + e).
// Each site is split into two "right movers" r (the two independent entries
// of (I + alpha) psi, taken from the left neighbour) and two "left movers" l
// (entries of (I - alpha) psi, taken from the right neighbour); the output is
// recombined from r of the left neighbour and l of the right neighbour.
// This is the eigenbasis rotation of App. A without its 1/sqrt(2) factors:
// only additions and exact multiplications by +-i occur, and the factor 1/2
// of every transport is deferred and applied once per step, as an exact
// power of two folded into the phase factor.  The rounding of each output
// component is therefore that of fl(x_L + x_R) with x_L, x_R the rounded
// two-term movers, i.e. the same as the plain projector formula evaluated
// neighbour by neighbour (barring subnormal intermediates).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dirac {

// index of this wave in its workgroup, as a wave-uniform (scalar) value, so
// that everything derived from it (tile, rows, addresses) stays in SGPRs
__device__ __forceinline__ int wave_in_block() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

template <typename T> struct Site { T v[8]; };
template <typename T> struct Mov { T v[4]; };  // two complex numbers

template <typename T> __device__ __forceinline__ void zero(Site<T>& s) {
#pragma unroll
  for (int k = 0; k < 8; ++k) s.v[k] = T(0);
}
template <typename T> __device__ __forceinline__ void zero(Mov<T>& s) {
#pragma unroll
  for (int k = 0; k < 4; ++k) s.v[k] = T(0);
}

// ---------------------------------------------------------------------------
// global memory: 16-byte vector loads/stores of one site
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_site(const float* __restrict__ p, Site<float>& s) {
  const float4 lo = reinterpret_cast<const float4*>(p)[0];
  const float4 hi = reinterpret_cast<const float4*>(p)[1];
  s.v[0] = lo.x; s.v[1] = lo.y; s.v[2] = lo.z; s.v[3] = lo.w;
  s.v[4] = hi.x; s.v[5] = hi.y; s.v[6] = hi.z; s.v[7] = hi.w;
}
__device__ __forceinline__ void load_site(const double* __restrict__ p, Site<double>& s) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 t = q[k];
    s.v[2 * k] = t.x;
    s.v[2 * k + 1] = t.y;
  }
}
__device__ __forceinline__ void store_site(float* __restrict__ p, const Site<float>& s) {
  reinterpret_cast<float4*>(p)[0] = make_float4(s.v[0], s.v[1], s.v[2], s.v[3]);
  reinterpret_cast<float4*>(p)[1] = make_float4(s.v[4], s.v[5], s.v[6], s.v[7]);
}
__device__ __forceinline__ void store_site(double* __restrict__ p, const Site<double>& s) {
  double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = make_double2(s.v[2 * k], s.v[2 * k + 1]);
}

// ---------------------------------------------------------------------------
// Two-component storage of 1-D lines.  With a single transport axis the four
// components pair up -- alpha_x and alpha_y couple a with d (and b with c),
// alpha_z couples a with c (and b with d), beta is diagonal -- and each pair
// evolves on its own (Sec. 2.4 notes the two-component reduction in 1-D).  A
// two-component state (NC = 2) stores the pair that contains a, as two
// complex numbers per cell; the other pair is taken as zero.
// ---------------------------------------------------------------------------
template <int AX> __host__ __device__ constexpr int pair_second() { return AX == 2 ? 2 : 3; }

__device__ __forceinline__ void load_pair(const float* __restrict__ p, float& a0, float& a1,
                                          float& b0, float& b1) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  a0 = q.x; a1 = q.y; b0 = q.z; b1 = q.w;
}
__device__ __forceinline__ void load_pair(const double* __restrict__ p, double& a0, double& a1,
                                          double& b0, double& b1) {
  const double2 q0 = reinterpret_cast<const double2*>(p)[0];
  const double2 q1 = reinterpret_cast<const double2*>(p)[1];
  a0 = q0.x; a1 = q0.y; b0 = q1.x; b1 = q1.y;
}
__device__ __forceinline__ void store_pair(float* __restrict__ p, float a0, float a1, float b0,
                                           float b1) {
  *reinterpret_cast<float4*>(p) = make_float4(a0, a1, b0, b1);
}
__device__ __forceinline__ void store_pair(double* __restrict__ p, double a0, double a1,
                                           double b0, double b1) {
  reinterpret_cast<double2*>(p)[0] = make_double2(a0, a1);
  reinterpret_cast<double2*>(p)[1] = make_double2(b0, b1);
}

// load / store cell `cell` of a state with NC stored components per cell
template <int NC, int AX, typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ base, int64_t cell, Site<T>& s) {
  if constexpr (NC == 4) {
    load_site(base + cell * 8, s);
  } else {
    constexpr int j = pair_second<AX>();
    zero(s);
    load_pair(base + cell * 4, s.v[0], s.v[1], s.v[2 * j], s.v[2 * j + 1]);
  }
}
template <int NC, int AX, typename T>
__device__ __forceinline__ void store_cell(T* __restrict__ base, int64_t cell, const Site<T>& s) {
  if constexpr (NC == 4) {
    store_site(base + cell * 8, s);
  } else {
    constexpr int j = pair_second<AX>();
    store_pair(base + cell * 4, s.v[0], s.v[1], s.v[2 * j], s.v[2 * j + 1]);
  }
}

// ---------------------------------------------------------------------------
// wave64 neighbour exchange with DPP (wave_shr:1 / wave_shl:1).  Lanes whose
// source lies outside the wave (lane 0 for shr, lane 63 for shl) keep `old`.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dpp_from_left(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_from_left(double old, double v) {
  const int2 o = __builtin_bit_cast(int2, old), s = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(o.x, s.x, 0x138, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(o.y, s.y, 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double dpp_from_right(double old, double v) {
  const int2 o = __builtin_bit_cast(int2, old), s = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(o.x, s.x, 0x130, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(o.y, s.y, 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, r);
}

// Same shifts with zero fill: the lane without a source receives 0, and no
// old value is needed, so the shift can fold into the instruction using it.
__device__ __forceinline__ float dpp_from_left_zero(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_from_right_zero(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double dpp_from_left_zero(double v) {
  const int2 s = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, s.x, 0x138, 0xf, 0xf, true);
  r.y = __builtin_amdgcn_update_dpp(0, s.y, 0x138, 0xf, 0xf, true);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double dpp_from_right_zero(double v) {
  const int2 s = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, s.x, 0x130, 0xf, 0xf, true);
  r.y = __builtin_amdgcn_update_dpp(0, s.y, 0x130, 0xf, 0xf, true);
  return __builtin_bit_cast(double, r);
}

// ---------------------------------------------------------------------------
// Per-axis movers and recombination (outputs are 2x the transported value).
// ---------------------------------------------------------------------------
template <int AX, typename T> struct Axis;

// alpha_x: (I+alpha)psi ~ (a+d, b+c, b+c, a+d); (I-alpha)psi ~ (a-d, b-c, c-b, d-a)
template <typename T> struct Axis<0, T> {
  static __device__ __forceinline__ void movers(const Site<T>& s, Mov<T>& r, Mov<T>& l) {
    r.v[0] = s.v[0] + s.v[6]; r.v[1] = s.v[1] + s.v[7];
    r.v[2] = s.v[2] + s.v[4]; r.v[3] = s.v[3] + s.v[5];
    l.v[0] = s.v[0] - s.v[6]; l.v[1] = s.v[1] - s.v[7];
    l.v[2] = s.v[2] - s.v[4]; l.v[3] = s.v[3] - s.v[5];
  }
  static __device__ __forceinline__ void combine(const Mov<T>& r, const Mov<T>& l, Site<T>& o) {
    o.v[0] = r.v[0] + l.v[0]; o.v[1] = r.v[1] + l.v[1];
    o.v[2] = r.v[2] + l.v[2]; o.v[3] = r.v[3] + l.v[3];
    o.v[4] = r.v[2] - l.v[2]; o.v[5] = r.v[3] - l.v[3];
    o.v[6] = r.v[0] - l.v[0]; o.v[7] = r.v[1] - l.v[1];
  }
};

// alpha_y: r = (a - i d, b + i c), l = (a + i d, b - i c);
// out = (r1 + l1, r2 + l2, -i (r2 - l2), i (r1 - l1))
template <typename T> struct Axis<1, T> {
  static __device__ __forceinline__ void movers(const Site<T>& s, Mov<T>& r, Mov<T>& l) {
    r.v[0] = s.v[0] + s.v[7]; r.v[1] = s.v[1] - s.v[6];
    r.v[2] = s.v[2] - s.v[5]; r.v[3] = s.v[3] + s.v[4];
    l.v[0] = s.v[0] - s.v[7]; l.v[1] = s.v[1] + s.v[6];
    l.v[2] = s.v[2] + s.v[5]; l.v[3] = s.v[3] - s.v[4];
  }
  static __device__ __forceinline__ void combine(const Mov<T>& r, const Mov<T>& l, Site<T>& o) {
    o.v[0] = r.v[0] + l.v[0]; o.v[1] = r.v[1] + l.v[1];
    o.v[2] = r.v[2] + l.v[2]; o.v[3] = r.v[3] + l.v[3];
    o.v[4] = r.v[3] - l.v[3]; o.v[5] = l.v[2] - r.v[2];
    o.v[6] = l.v[1] - r.v[1]; o.v[7] = r.v[0] - l.v[0];
  }
};

// alpha_z: r = (a + c, b - d), l = (a - c, b + d); out = (r1 + l1, r2 + l2, r1 - l1, l2 - r2)
template <typename T> struct Axis<2, T> {
  static __device__ __forceinline__ void movers(const Site<T>& s, Mov<T>& r, Mov<T>& l) {
    r.v[0] = s.v[0] + s.v[4]; r.v[1] = s.v[1] + s.v[5];
    r.v[2] = s.v[2] - s.v[6]; r.v[3] = s.v[3] - s.v[7];
    l.v[0] = s.v[0] - s.v[4]; l.v[1] = s.v[1] - s.v[5];
    l.v[2] = s.v[2] + s.v[6]; l.v[3] = s.v[3] + s.v[7];
  }
  static __device__ __forceinline__ void combine(const Mov<T>& r, const Mov<T>& l, Site<T>& o) {
    o.v[0] = r.v[0] + l.v[0]; o.v[1] = r.v[1] + l.v[1];
    o.v[2] = r.v[2] + l.v[2]; o.v[3] = r.v[3] + l.v[3];
    o.v[4] = r.v[0] - l.v[0]; o.v[5] = r.v[1] - l.v[1];
    o.v[6] = l.v[2] - r.v[2]; o.v[7] = l.v[3] - r.v[3];
  }
};

// ---------------------------------------------------------------------------
// FP64 sine and cosine for the local step.  Cody-Waite reduction by pi/2 with
// a three-part constant; Taylor polynomials on [-pi/4, pi/4].
//   ACC = 2 (FP64 storage): terms to r^17 (sin) and r^18 (cos), truncation
//     below 1e-19; the reduced argument is kept as rh + rl and
//     sin(rh + rl) = sin rh + rl cos rh, cos(rh + rl) = cos rh - rl sin rh to
//     first order in rl, with 1 - rh^2/2 carried as an unevaluated sum (its
//     rounding errors recovered exactly by FMA and Sterbenz subtraction).
//     Error below 1 ulp, equal to the correctly rounded value for about
//     98.5 % of arguments in [-12, 12].
//   ACC = 1 (FP32 storage): terms to r^13 and r^14 (truncation below 3e-14),
//     no tail terms; a few ulp, far below the FP32 rounding of the state.
// Valid for |x| < 2^20; far_arg() flags the rest (and NaN), which callers
// route to the library routine outside their hot loops.
// ---------------------------------------------------------------------------
// pi/2 = P1 + P2 + P3: P1, P2 hold 33 significant bits each (so k * P1 and
// k * P2 are exact for |k| < 2^20), P3 the rounded remainder.
#define DIRAC_PIO2_1 0x1.921fb54400000p+0
#define DIRAC_PIO2_2 0x1.0b4611a600000p-34
#define DIRAC_PIO2_3 0x1.3198a2e037073p-69
#define DIRAC_2_OVER_PI 0x1.45f306dc9c883p-1

__device__ __forceinline__ bool far_arg(double x) { return !(fabs(x) < 1048576.0); }

template <int ACC>
__device__ __forceinline__ void sincos_fast(double x, double* s_out, double* c_out) {
  const double k = rint(x * DIRAC_2_OVER_PI);
  // x - k pi/2 = rh + rl: k P1, k P2 are exact and so is x - k P1
  const double a = fma(-k, DIRAC_PIO2_1, x);
  const double b = k * DIRAC_PIO2_2;
  const double rh = a - b;
  const double r2 = rh * rh;
  double sn, cs;
  if constexpr (ACC >= 2) {
    const double rl = ((a - rh) - b) - k * DIRAC_PIO2_3;
    // sin: rh + rh^3 (-1/3! + r^2/5! - ... + r^14/17!) + rl (1 - r^2/2)
    double ps = 1.0 / 355687428096000.0;          // 1/17!
    ps = fma(ps, r2, -1.0 / 1307674368000.0);     // 1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);         // 1/13!
    ps = fma(ps, r2, -1.0 / 39916800.0);          // 1/11!
    ps = fma(ps, r2, 1.0 / 362880.0);             // 1/9!
    ps = fma(ps, r2, -1.0 / 5040.0);              // 1/7!
    ps = fma(ps, r2, 1.0 / 120.0);                // 1/5!
    ps = fma(ps, r2, -1.0 / 6.0);                 // 1/3!
    sn = rh + fma(rh * r2, ps, rl * fma(-0.5, r2, 1.0));
    // cos: (1 - rh^2/2) + rh^4 (1/4! - r^2/6! + ... + r^14/18!) - rh rl
    double pc = -1.0 / 6402373705728000.0;        // 1/18!
    pc = fma(pc, r2, 1.0 / 20922789888000.0);     // 1/16!
    pc = fma(pc, r2, -1.0 / 87178291200.0);       // 1/14!
    pc = fma(pc, r2, 1.0 / 479001600.0);          // 1/12!
    pc = fma(pc, r2, -1.0 / 3628800.0);           // 1/10!
    pc = fma(pc, r2, 1.0 / 40320.0);              // 1/8!
    pc = fma(pc, r2, -1.0 / 720.0);               // 1/6!
    pc = fma(pc, r2, 1.0 / 24.0);                 // 1/4!
    const double e2 = fma(rh, rh, -r2);           // rh^2 = r2 + e2 exactly
    const double hz = 0.5 * r2;
    const double w = 1.0 - hz;
    const double tail = ((1.0 - w) - hz) - 0.5 * e2;
    cs = w + (fma(r2 * r2, pc, tail) - rh * rl);
  } else {
    const double r = fma(-k, DIRAC_PIO2_3, rh);
    const double q2 = r * r;
    double ps = 1.0 / 6227020800.0;               // 1/13!
    ps = fma(ps, q2, -1.0 / 39916800.0);          // 1/11!
    ps = fma(ps, q2, 1.0 / 362880.0);             // 1/9!
    ps = fma(ps, q2, -1.0 / 5040.0);              // 1/7!
    ps = fma(ps, q2, 1.0 / 120.0);                // 1/5!
    ps = fma(ps, q2, -1.0 / 6.0);                 // 1/3!
    sn = fma(r * q2, ps, r);
    double pc = 1.0 / 87178291200.0;              // 1/14!
    pc = fma(pc, q2, -1.0 / 479001600.0);         // 1/12!
    pc = fma(pc, q2, 1.0 / 3628800.0);            // 1/10!
    pc = fma(pc, q2, -1.0 / 40320.0);             // 1/8!
    pc = fma(pc, q2, 1.0 / 720.0);                // 1/6!
    pc = fma(pc, q2, -1.0 / 24.0);                // 1/4!
    pc = fma(pc, q2, 0.5);                        // 1/2!
    cs = fma(-pc, q2, 1.0);
    (void)r2;
  }
  const int q = static_cast<int>(static_cast<long long>(k) & 3);
  const double s1 = (q & 1) ? cs : sn;
  const double c1 = (q & 1) ? sn : cs;
  *s_out = (q & 2) ? -s1 : s1;
  *c_out = ((q + 1) & 2) ? -c1 : c1;
}

// Arguments beyond the reduction range go to the library routine, kept out of
// line so that its large-argument reduction does not occupy the hot loop.
__device__ __attribute__((noinline)) double2 sincos_far(double x) {
  double2 r;
  sincos(x, &r.x, &r.y);
  return r;
}

template <int ACC>
__device__ __forceinline__ void sincos_any(double x, double* s_out, double* c_out) {
  if (far_arg(x)) {
    const double2 r = sincos_far(x);
    *s_out = r.x;
    *c_out = r.y;
  } else {
    sincos_fast<ACC>(x, s_out, c_out);
  }
}

// ---------------------------------------------------------------------------
// Local step D.  The two distinct phase factors per cell,
//   f_up = s exp(-i (V + m c^2) dt)   (components a, b)
//   f_dn = s exp(-i (V - m c^2) dt)   (components c, d),
// are formed in FP64, where s = 2^-(number of transports) undoes the deferred
// factors 1/2 exactly.  The components are promoted to FP64, multiplied and
// rounded once to T.
// ---------------------------------------------------------------------------
struct PhaseK {
  double eu_re, eu_im, ed_re, ed_im;  // s exp(-+ i m c^2 dt)
  double dt;
  double mc2;                         // m c^2 (rounded as (m c) c)
  double scale;                       // s = 2^-(number of transports)
  float scale_f;                      // s (pure-streaming mode)
  int mode;                           // 0: scale only, 1: mass only, 2: mass + V
  int two_angles;                     // mode 2: theta = (V +- m c^2) dt per pair
};

struct Factors { double ur, ui, dr, di; };

// Phase factors of one cell in mode 2.  TWO (FP64 storage): the angles are
// formed as (V + m c^2) dt and (V - m c^2) dt, each with its own sine and
// cosine (ACC 2).  Otherwise (FP32 storage) exp(-i V dt) (ACC 1) is multiplied
// by the FP64 constants eu, ed: one sine/cosine pair per cell.
template <bool TWO, bool ANY>
__device__ __forceinline__ Factors factors_v(double V, const PhaseK& k) {
  Factors f;
  if constexpr (TWO) {
    double su, cu, sd, cd;
    const double tu = (V + k.mc2) * k.dt, td = (V - k.mc2) * k.dt;
    if constexpr (ANY) {
      sincos_any<2>(tu, &su, &cu);
      sincos_any<2>(td, &sd, &cd);
    } else {
      sincos_fast<2>(tu, &su, &cu);
      sincos_fast<2>(td, &sd, &cd);
    }
    f.ur = k.scale * cu;
    f.ui = -k.scale * su;
    f.dr = k.scale * cd;
    f.di = -k.scale * sd;
  } else {
    double sn, cs;
    if constexpr (ANY)
      sincos_any<1>(V * k.dt, &sn, &cs);
    else
      sincos_fast<1>(V * k.dt, &sn, &cs);
    // (cs - i sn) (x + i y) = (cs x + sn y) + i (cs y - sn x)
    f.ur = fma(cs, k.eu_re, sn * k.eu_im);
    f.ui = fma(cs, k.eu_im, -sn * k.eu_re);
    f.dr = fma(cs, k.ed_re, sn * k.ed_im);
    f.di = fma(cs, k.ed_im, -sn * k.ed_re);
  }
  return f;
}

// true if a phase angle of this cell lies outside the fast reduction range
template <bool TWO>
__device__ __forceinline__ bool factors_far(double V, const PhaseK& k) {
  if constexpr (TWO)
    return far_arg((V + k.mc2) * k.dt) || far_arg((V - k.mc2) * k.dt);
  else
    return far_arg(V * k.dt);
}

__device__ __forceinline__ Factors const_factors(const PhaseK& k) {
  Factors f;
  f.ur = k.eu_re; f.ui = k.eu_im; f.dr = k.ed_re; f.di = k.ed_im;
  return f;
}

// Generic factors for any mode and argument (same values as the fast path).
__device__ __forceinline__ Factors phase_factors(double V, const PhaseK& k) {
  if (k.mode == 2) {
    if (k.two_angles) return factors_v<true, true>(V, k);
    return factors_v<false, true>(V, k);
  }
  return const_factors(k);
}

template <typename T>
__device__ __forceinline__ void cmul_round(T& re, T& im, double fr, double fi) {
  const double x = static_cast<double>(re), y = static_cast<double>(im);
  re = static_cast<T>(fma(fr, x, -fi * y));
  im = static_cast<T>(fma(fr, y, fi * x));
}

template <typename T>
__device__ __forceinline__ void apply_factors(Site<T>& s, const Factors& f) {
  cmul_round(s.v[0], s.v[1], f.ur, f.ui);
  cmul_round(s.v[2], s.v[3], f.ur, f.ui);
  cmul_round(s.v[4], s.v[5], f.dr, f.di);
  cmul_round(s.v[6], s.v[7], f.dr, f.di);
}

// FP32 storage, the form kept in the 1-D / 2-D passes: every FP64 factor f is
// held as an unevaluated pair of floats, f = hi + lo with hi = fl32(f) and
// lo = fl32(f - hi) (split once per row, when the factors are formed), and
// applied with FP32 fused multiply-adds, the small lo products first:
//   re' = fma(-y, fi, fma(x, fr, fma(-y, fi_lo, x fr_lo)))   and likewise im'.
// The pair carries the factor to about 2^-48 relative, so the modulus and
// phase of the applied factor do not drift (what an FP32-rounded factor
// would do, by about 1e-8 per step, coherently over the steps of a run); each
// product is rounded at most twice in FP32.  No FP64 operation or conversion
// remains in the stages.
struct FactorsHL {
  float ur, ui, dr, di;      // hi parts
  float urL, uiL, drL, diL;  // lo parts
};

__device__ __forceinline__ void split_pair(double v, float& hi, float& lo) {
  hi = static_cast<float>(v);
  lo = static_cast<float>(v - static_cast<double>(hi));
}

__device__ __forceinline__ FactorsHL split_factors(const Factors& f) {
  FactorsHL h;
  split_pair(f.ur, h.ur, h.urL);
  split_pair(f.ui, h.ui, h.uiL);
  split_pair(f.dr, h.dr, h.drL);
  split_pair(f.di, h.di, h.diL);
  return h;
}

__device__ __forceinline__ void cmul_hl(float& re, float& im, float fr, float fi, float frL,
                                        float fiL) {
  const float x = re, y = im;
  re = fmaf(-y, fi, fmaf(x, fr, fmaf(-y, fiL, x * frL)));
  im = fmaf(y, fr, fmaf(x, fi, fmaf(y, frL, x * fiL)));
}

__device__ __forceinline__ void apply_factors(Site<float>& s, const FactorsHL& f) {
  cmul_hl(s.v[0], s.v[1], f.ur, f.ui, f.urL, f.uiL);
  cmul_hl(s.v[2], s.v[3], f.ur, f.ui, f.urL, f.uiL);
  cmul_hl(s.v[4], s.v[5], f.dr, f.di, f.drL, f.diL);
  cmul_hl(s.v[6], s.v[7], f.dr, f.di, f.drL, f.diL);
}

// the factors as a 1-D / 2-D pass keeps them for state type T
template <typename T> struct Stored {
  using type = Factors;
  static __device__ __forceinline__ Factors of(const Factors& f) { return f; }
};
template <> struct Stored<float> {
  using type = FactorsHL;
  static __device__ __forceinline__ FactorsHL of(const Factors& f) { return split_factors(f); }
};

template <typename T> __device__ __forceinline__ T scale_of(const PhaseK& k);
template <> __device__ __forceinline__ float scale_of<float>(const PhaseK& k) { return k.scale_f; }
template <> __device__ __forceinline__ double scale_of<double>(const PhaseK& k) {
  return static_cast<double>(k.scale_f);
}

template <typename T>
__device__ __forceinline__ void scale_site(Site<T>& s, const PhaseK& k) {
  const T sc = scale_of<T>(k);
#pragma unroll
  for (int j = 0; j < 8; ++j) s.v[j] *= sc;
}

// Local step with the phase mode fixed at compile time (MODE < 0: read it
// from k at run time); f holds the cell's factors for modes 1 and 2 (as FP64
// factors, or as FP32 hi + lo pairs).
template <int MODE, typename T, typename F>
__device__ __forceinline__ void apply_local(Site<T>& s, const F& f, const PhaseK& k) {
  if constexpr (MODE == 0) {
    scale_site(s, k);
  } else if constexpr (MODE > 0) {
    apply_factors(s, f);
  } else {
    if (k.mode == 0)
      scale_site(s, k);
    else
      apply_factors(s, f);
  }
}

// Factors of a cell for the given mode, fast path only for mode 2 (callers
// repair far arguments with factors_fix).
template <int MODE, bool TWO>
__device__ __forceinline__ Factors factors_of(double V, const PhaseK& k) {
  if constexpr (MODE == 2) return factors_v<TWO, false>(V, k);
  else if constexpr (MODE == 1 || MODE == 0) return const_factors(k);
  else return (k.mode == 2) ? factors_v<TWO, false>(V, k) : const_factors(k);
}

// After factors_of: if any lane of the wave had an angle outside the fast
// range, recompute that wave's factors with the library fallback (the values
// of in-range lanes are unchanged).  A wave-uniform, rarely taken branch.
template <int MODE, bool TWO>
__device__ __forceinline__ void factors_fix(Factors& f, double V, const PhaseK& k) {
  if constexpr (MODE == 2 || MODE < 0) {
    const bool need = (MODE == 2 || k.mode == 2) && factors_far<TWO>(V, k);
    if (__any(need)) f = factors_v<TWO, true>(V, k);
  }
}

// ---------------------------------------------------------------------------
// Local step with a vector potential (eq:sol_dis_4 with the closed-form
// exponential of Dirac matrices, Sec. 2.3):
//   D = U exp(-i V dt),  U = cos(A) + i (-beta mu + alpha . At) sin(A) / A,
//   mu = m c^2 dt, A = sqrt(mu^2 + At . At), At the field integral of the
//   step at the cell.
// In the Dirac representation U has the blocks
//   [[ (cos A - i mu sA) I,   i sA sigma.At ],
//    [ i sA sigma.At,         (cos A + i mu sA) I ]],   sA = sin(A) / A,
// so per cell three complex numbers (times s exp(-i V dt)) and At suffice.
// ---------------------------------------------------------------------------
struct FieldFactors {
  double ur, ui;      // s e^{-iVdt} (cos A - i mu sA): components a, b
  double dr, di;      // s e^{-iVdt} (cos A + i mu sA): components c, d
  double qr, qi;      // s e^{-iVdt} i sA: both off-diagonal blocks
  double ax, ay, az;  // At
};

template <bool TWO>
__device__ __forceinline__ bool field_far(double V, double ax, double ay, double az,
                                          const PhaseK& k) {
  const double mu = k.mc2 * k.dt;
  return far_arg(sqrt(mu * mu + ax * ax + ay * ay + az * az)) || far_arg(V * k.dt);
}

// ph = s e^{-i V dt}, the scalar part of the local step
template <bool TWO, bool ANY>
__device__ __forceinline__ void scalar_phase(double V, const PhaseK& k, double& pr, double& pi) {
  constexpr int ACC = TWO ? 2 : 1;
  double sv, cv;
  if constexpr (ANY)
    sincos_any<ACC>(V * k.dt, &sv, &cv);
  else
    sincos_fast<ACC>(V * k.dt, &sv, &cv);
  pr = k.scale * cv;
  pi = -k.scale * sv;
}

// U ph for the field integral At = (ax, ay, az) of the step, given ph
template <bool TWO, bool ANY>
__device__ __forceinline__ FieldFactors field_with(double pr, double pi, double ax, double ay,
                                                   double az, const PhaseK& k) {
  constexpr int ACC = TWO ? 2 : 1;
  const double mu = k.mc2 * k.dt;
  const double A = sqrt(mu * mu + ax * ax + ay * ay + az * az);
  double sA, cA;
  if constexpr (ANY)
    sincos_any<ACC>(A, &sA, &cA);
  else
    sincos_fast<ACC>(A, &sA, &cA);
  const double sa = (A > 0.0) ? sA / A : 1.0;
  const double ms = mu * sa;
  FieldFactors f;
  f.ur = fma(pr, cA, pi * ms);   // ph * (cA - i ms)
  f.ui = fma(pi, cA, -pr * ms);
  f.dr = fma(pr, cA, -pi * ms);  // ph * (cA + i ms)
  f.di = fma(pi, cA, pr * ms);
  f.qr = -pi * sa;               // ph * (i sa)
  f.qi = pr * sa;
  f.ax = ax;
  f.ay = ay;
  f.az = az;
  return f;
}

template <bool TWO, bool ANY>
__device__ __forceinline__ FieldFactors field_factors(double V, double ax, double ay, double az,
                                                      const PhaseK& k) {
  double pr, pi;
  scalar_phase<TWO, ANY>(V, k, pr, pi);
  return field_with<TWO, ANY>(pr, pi, ax, ay, az, k);
}

// if any lane of the wave has an angle outside the fast reduction range,
// recompute the wave's factors with the library fallback (a rare branch)
template <bool TWO>
__device__ __forceinline__ void field_fix(FieldFactors& f, double V, double ax, double ay,
                                          double az, const PhaseK& k) {
  if (__any(field_far<TWO>(V, ax, ay, az, k))) f = field_factors<TWO, true>(V, ax, ay, az, k);
}

// psi <- U e^{-i V dt} psi (with the deferred scale), promoted to FP64 and
// rounded once per component
template <typename T>
__device__ __forceinline__ void apply_field(Site<T>& s, const FieldFactors& f) {
  const double ar = s.v[0], ai = s.v[1], br = s.v[2], bi = s.v[3];
  const double cr = s.v[4], ci = s.v[5], dr = s.v[6], di = s.v[7];
  // sigma.At (x, y):  (az x0 + (ax - i ay) x1,  (ax + i ay) x0 - az x1)
  auto sig = [&](double x0r, double x0i, double x1r, double x1i, double& o0r, double& o0i,
                 double& o1r, double& o1i) {
    o0r = fma(f.az, x0r, fma(f.ax, x1r, f.ay * x1i));
    o0i = fma(f.az, x0i, fma(f.ax, x1i, -f.ay * x1r));
    o1r = fma(f.ax, x0r, fma(-f.ay, x0i, -f.az * x1r));
    o1i = fma(f.ax, x0i, fma(f.ay, x0r, -f.az * x1i));
  };
  double t1r, t1i, t2r, t2i, t3r, t3i, t4r, t4i;
  sig(cr, ci, dr, di, t1r, t1i, t2r, t2i);  // acts on the lower pair
  sig(ar, ai, br, bi, t3r, t3i, t4r, t4i);  // acts on the upper pair
  // x' = diag * x + q * t
  auto mix = [&](double xr, double xi, double gr, double gi, double tr, double ti, T& oR, T& oI) {
    oR = static_cast<T>(fma(gr, xr, fma(-gi, xi, fma(f.qr, tr, -f.qi * ti))));
    oI = static_cast<T>(fma(gr, xi, fma(gi, xr, fma(f.qr, ti, f.qi * tr))));
  };
  mix(ar, ai, f.ur, f.ui, t1r, t1i, s.v[0], s.v[1]);
  mix(br, bi, f.ur, f.ui, t2r, t2i, s.v[2], s.v[3]);
  mix(cr, ci, f.dr, f.di, t3r, t3i, s.v[4], s.v[5]);
  mix(dr, di, f.dr, f.di, t4r, t4i, s.v[6], s.v[7]);
}

// ---------------------------------------------------------------------------
// A time-dependent vector potential A(t, x) = f(t) P(x): a laser pulse with a
// linear turn-on ramp, the kind of field whose integral Sec. 2.3 notes can be
// found analytically.  f(t) = w(t) sin(omega t + phase) with the trapezoid
// envelope w: 0 before t = 0, t / t_on on [0, t_on), 1 for t_flat, a linear
// fall to 0 over t_off, 0 afterwards.  The local step of step n carries the
// field integral At^n(x) = P(x) F_n, F_n = int f over [t0 + n dt,
// t0 + (n + 1) dt] (eq:field_dis1), evaluated here in closed form per step.
// ---------------------------------------------------------------------------
struct PulseK {
  double omega, phase;           // carrier
  double t_on, t_flat, t_off;    // envelope
  double t0, dt;                 // step n starts at t0 + n dt
  int64_t n0;                    // first step of the pass
};

// sin(u) / u
__device__ __forceinline__ double sinc_d(double u) {
  const double u2 = u * u;
  if (fabs(u) < 1e-3) return 1.0 - u2 * (1.0 / 6.0 - u2 * (1.0 / 120.0));
  return sin(u) / u;
}

// (sin u - u cos u) / u^2: a series below |u| = 1/4 (terms to u^11, the next
// below 2e-19 relative), the direct form above (cancellation costs at most
// 3 eps / u^2 < 5e-15 relative there)
__device__ __forceinline__ double j1_d(double u) {
  if (fabs(u) < 0.25) {
    const double u2 = u * u;
    double p = -1.0 / 518918400.0;          // -12 / 13!
    p = fma(p, u2, 1.0 / 3991680.0);        //  10 / 11!
    p = fma(p, u2, -1.0 / 45360.0);         //  -8 / 9!
    p = fma(p, u2, 1.0 / 840.0);            //   6 / 7!
    p = fma(p, u2, -1.0 / 30.0);            //  -4 / 5!
    p = fma(p, u2, 1.0 / 3.0);              //   2 / 3!
    return u * p;
  }
  double s, c;
  sincos(u, &s, &c);
  return (s - u * c) / (u * u);
}

// int_a^b (w_m + beta (t - m)) sin(omega t + phase) dt with m = (a + b) / 2,
// h = (b - a) / 2, psi = omega m + phase:
//   int sin(omega t + phase)        = 2 h sin(psi) sinc(omega h)
//   int (t - m) sin(omega t + phase) = 2 h^2 cos(psi) j1(omega h)
// (the product forms avoid the cancellation of a difference of cosines)
__device__ __forceinline__ double lin_sin_integral(double a, double b, double w_m, double beta,
                                                   double omega, double phase) {
  const double h = 0.5 * (b - a), m = 0.5 * (a + b);
  const double u = omega * h;
  double sp, cp;
  sincos(fma(omega, m, phase), &sp, &cp);
  const double i0 = 2.0 * h * sp * sinc_d(u);
  const double i1 = 2.0 * h * h * cp * j1_d(u);
  return fma(w_m, i0, beta * i1);
}

// F = int_ta^tb f(t) dt, over the pieces of [ta, tb] on which w is linear
__device__ __forceinline__ double pulse_integral(const PulseK& p, double ta, double tb) {
  const double t1 = p.t_on + p.t_flat, t2 = t1 + p.t_off;
  double sum = 0.0;
  if (p.t_on > 0.0) {  // rise: w = t / t_on
    const double a = fmax(ta, 0.0), b = fmin(tb, p.t_on);
    if (a < b) sum += lin_sin_integral(a, b, 0.5 * (a + b) / p.t_on, 1.0 / p.t_on, p.omega, p.phase);
  }
  {  // flat top: w = 1
    const double a = fmax(ta, p.t_on), b = fmin(tb, t1);
    if (a < b) sum += lin_sin_integral(a, b, 1.0, 0.0, p.omega, p.phase);
  }
  if (p.t_off > 0.0) {  // fall: w = (t2 - t) / t_off
    const double a = fmax(ta, t1), b = fmin(tb, t2);
    if (a < b)
      sum += lin_sin_integral(a, b, (t2 - 0.5 * (a + b)) / p.t_off, -1.0 / p.t_off, p.omega,
                              p.phase);
  }
  return sum;
}

// F of step n0 + s of the pass (the time of a step is formed from its global
// index, so a pass of K steps and K passes of one step see the same values)
__device__ __forceinline__ double pulse_step_integral(const PulseK& p, int s) {
  const double n = static_cast<double>(p.n0 + s);
  return pulse_integral(p, fma(n, p.dt, p.t0), fma(n + 1.0, p.dt, p.t0));
}

// what a row carries between its read and its local steps under a pulse:
// ph = s e^{-i V dt} and the field profile P
struct PulseRow {
  double pr, pi;
  double px, py, pz;
};

template <bool TWO>
__device__ __forceinline__ PulseRow pulse_row(double V, double px, double py, double pz,
                                              const PhaseK& k) {
  PulseRow r;
  scalar_phase<TWO, false>(V, k, r.pr, r.pi);
  if (__any(far_arg(V * k.dt))) scalar_phase<TWO, true>(V, k, r.pr, r.pi);
  r.px = px;
  r.py = py;
  r.pz = pz;
  return r;
}

// U ph of the step whose field integral factor is F
template <bool TWO>
__device__ __forceinline__ FieldFactors pulse_factors(const PulseRow& r, double F,
                                                      const PhaseK& k) {
  return field_with<TWO, true>(r.pr, r.pi, F * r.px, F * r.py, F * r.pz, k);
}

// Phase factors of a cell for phase mode MODE (3: with a static vector
// potential; 4: with a pulse, formed per step from the row's PulseRow)
template <int MODE> struct FactorOf { using type = Factors; };
template <> struct FactorOf<3> { using type = FieldFactors; };
template <> struct FactorOf<4> { using type = PulseRow; };

// Full local step on one site (V ignored unless mode == 2).
template <typename T>
__device__ __forceinline__ void local_step(Site<T>& s, double V, const PhaseK& k) {
  if (k.mode == 0) {
    const T sc = scale_of<T>(k);
#pragma unroll
    for (int j = 0; j < 8; ++j) s.v[j] *= sc;
  } else {
    apply_factors(s, phase_factors(V, k));
  }
}

}  // namespace dirac
