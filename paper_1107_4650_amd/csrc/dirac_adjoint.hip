// dirac_adjoint.hip -- discrete adjoint of the sweep: reverse steps that
// recompute psi backwards and carry the adjoint field lambda, the seed of the
// transmitted-probability loss, and the projection of dL/dV on parameters.
//
// One forward step is S = D W with W = T_last ... T_first (transports,
// eq:sol_dis_1-3) and D the local phase step (eq:sol_dis_4).  Its adjoint is
// S^H = W^H D^H = T_first^H ... T_last^H D^H, with
//     T_d^H lam (i) = 1/2 (I + alpha) lam(i + e) + 1/2 (I - alpha) lam(i - e)
// (the transport run backwards: right movers come from the right neighbour,
// left movers from the left one; cells outside a zero wall are zero) and
// D^H = exp(+i theta).  With periodic cells every T_d is unitary and
// S^{-1} = S^H, so the same fused operator rebuilds psi_{n-1} from psi_n.
//
// For L = dV sum_{x0 > x_b} |psi_N|^2 and lambda_N = M psi_N, the gradient
// with respect to the potential at every cell is
//     dL/dV = 2 dt dV sum_{n=1..N} Im(lambda_n^H psi_n),
// accumulated in FP64 at the start of every reverse step.
//
// Work decomposition: a pass of K reverse steps gives each wave 64 columns
// and writes the middle 64 - 2K (every backward x transport, the last
// transport of a reverse step, narrows the valid lanes by one on each side),
// and marches along y as the forward passes do.
#include "dirac_device.h"
#include "dirac_plan.h"
#include "dirac_sweep_impl.h"
#include "dirac_trace.h"

#include <utility>

namespace dirac {

struct RevArgs {
  int64_t nx, ny;
  int periodic;
  int H;
  int64_t nstrips;  // ceil(nx / 62)
  int64_t nseg;
  int64_t ntiles;
  int xcd_remap;
  int axes_code;
  double qscale;    // 2 dt dV
  PhaseK ph;        // forward phase constants (conjugated here)
};

// conjugate factors: D^H = s exp(+i theta).  The phase mode is read at run
// time; the fast sine/cosine serves every lane unless some lane of the wave
// has an angle beyond its range (a wave-uniform, rarely taken repair).
template <bool TWO>
__device__ __forceinline__ Factors adjoint_factors(double V, const PhaseK& k) {
  Factors f = factors_of<-1, TWO>(V, k);
  factors_fix<-1, TWO>(f, V, k);
  f.ui = -f.ui;
  f.di = -f.di;
  return f;
}

// D^H on one site (scale folded in); mode 0 is the bare scale
template <typename T>
__device__ __forceinline__ void adjoint_local(Site<T>& s, const Factors& f, const PhaseK& k) {
  if (k.mode == 0)
    scale_site(s, k);
  else
    apply_factors(s, f);
}

template <typename T>
__device__ __forceinline__ double im_dot(const Site<T>& l, const Site<T>& p) {
  // Im(sum_c conj(l_c) p_c) = sum_c (l.re p.im - l.im p.re)
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double lr = static_cast<double>(l.v[2 * c]), li = static_cast<double>(l.v[2 * c + 1]);
    const double pr = static_cast<double>(p.v[2 * c]), pi = static_cast<double>(p.v[2 * c + 1]);
    acc = fma(lr, pi, acc);
    acc = fma(-li, pr, acc);
  }
  return acc;
}

// backward x transport inside the wave: right movers from the right lane,
// left movers from the left lane (lanes 0 and 63 lack a neighbour and give
// values that are not used)
template <typename T, int AX>
__device__ __forceinline__ void x_transport_adj(const Site<T>& in, Site<T>& out) {
  Mov<T> r, l, rR, lL;
  Axis<AX, T>::movers(in, r, l);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rR.v[k] = dpp_from_right_zero(r.v[k]);
    lL.v[k] = dpp_from_left_zero(l.v[k]);
  }
  Axis<AX, T>::combine(rR, lL, out);
}

// resident 256-thread blocks per CU the reverse kernel is compiled for: a
// single reverse step fits two waves per SIMD; fused passes carry two fields
// through every stage and run one wave per SIMD, the compiler parking part of
// the working set in the accumulation registers
__host__ __device__ constexpr int rev_min_blocks(bool fp64, int depth) {
  return (fp64 || depth > 1) ? 1 : 2;
}

// one input row of the reverse march: psi, lambda, V and Q at this lane's
// (wrapped or clamped) column
template <typename T> struct RevIn {
  Site<T> p, l;
  double v, q;
};

// ---------------------------------------------------------------------------
// K reverse steps per launch (temporal blocking of the adjoint).  Stage s
// takes the row of time level n - s + 1 (psi and lambda): it adds that level's
// term to dL/dV, applies D^H to both fields, and completes the row one behind
// with T_y^H then T_x^H; that row is the input of stage s + 1.  The wave
// holds 64 columns and writes the 64 - 2K middle ones (every stage narrows
// the valid lanes by one on each side).  A row's factors and its dL/dV
// accumulator are formed when the row is read and move one slot on per
// iteration until the last stage has taken the row; the accumulator then goes back to
// Q once per pass.  The K terms of a cell are added in the order of the
// single steps, and intermediate rows are rounded and zeroed beyond walls
// as stored steps are, so a pass gives the bits of K single reverse steps.
// ---------------------------------------------------------------------------

template <typename T, int K, int AX0, int AX1, bool UP, bool EDGE>
__device__ __forceinline__ void rev_march(T* __restrict__ psi_out, T* __restrict__ lam_out,
                                          const T* __restrict__ psi, const T* __restrict__ lam,
                                          const double* __restrict__ V, double* __restrict__ Q,
                                          const RevArgs& a, const Lanes& c, bool own,
                                          int64_t jb, int64_t je) {
  constexpr int L = 2;  // rows in flight; the loop is unrolled by the same 2
  const int64_t nx = a.nx, ny = a.ny;
  const int nit = static_cast<int>(je - jb) + 2 * K;
  const bool zero_walls = !a.periodic;
  const bool read_v = (a.ph.mode == 2);
  auto in_row = [&](int it) -> int64_t { return UP ? jb - K + it : je - 1 + K - it; };
  // row in_row(it) -+ s lies in the box iff lo <= it - s < hi: wave-uniform
  // bounds clamped to 32 bits (it - s spans -K .. nit + L), so the wall tests
  // of the loop are scalar compares
  auto clamp_it = [&](int64_t e) -> int {
    return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
  };
  const int64_t lo64 = UP ? K - jb : je + K - ny;
  const int lo = clamp_it(lo64), hi = clamp_it(lo64 + ny);
  auto row_in = [&](int e) -> bool { return e >= lo && e < hi; };
  auto load = [&](int it, RevIn<T>& R) {
    int64_t r = in_row(it);
    if (!row_in(it)) r = read_row(r, ny, a.periodic);
    const int64_t q = r * nx + c.col;
    load_site(psi + q * 8, R.p);
    load_site(lam + q * 8, R.l);
    R.v = read_v ? V[q] : 0.0;
    R.q = Q[q];
  };
  RevIn<T> ring[L];
#pragma unroll
  for (int k = 0; k < L; ++k) load(k, ring[k]);
  static_assert(L == 2, "the y mover slots alternate with the iteration");
  Mov<T> mp[K][2], ml[K][2];  // stored y movers per stage (psi, lambda), slot it % 2
  Factors fr[K];              // factors of the rows in flight: fr[s - 1] for stage s
  double qa[K];               // their dL/dV accumulators
#pragma unroll
  for (int s = 0; s < K; ++s) {
    zero(mp[s][0]);
    zero(mp[s][1]);
    zero(ml[s][0]);
    zero(ml[s][1]);
    qa[s] = 0.0;
  }
  for (int base = 0;; base += L) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int it = base + k;
      if (it >= nit) return;
      RevIn<T> cur = ring[k % L];
      load(it + L, ring[k % L]);  // rows past the segment are read and dropped
      const int64_t jin = in_row(it);
      if (zero_walls) {
        if (!row_in(it)) {
          zero(cur.p);
          zero(cur.l);
        }
        if (EDGE && !c.full && c.out) {
          zero(cur.p);
          zero(cur.l);
        }
      }
      // the rows in flight move one stage on; the new row enters stage 1
#pragma unroll
      for (int s = K - 1; s >= 1; --s) {
        fr[s] = fr[s - 1];
        qa[s] = qa[s - 1];
      }
      fr[0] = adjoint_factors<sizeof(T) == 8>(cur.v, a.ph);
      qa[0] = cur.q;
      Site<T> p = cur.p, l = cur.l;
#pragma unroll
      for (int s = 1; s <= K; ++s) {
        const int slot = s - 1;  // the input row's factors and accumulator
        const int64_t j = UP ? jin - (s - 1) : jin + (s - 1);  // input row of stage s
        qa[slot] = fma(a.qscale, im_dot(l, p), qa[slot]);
        adjoint_local(p, fr[slot], a.ph);
        adjoint_local(l, fr[slot], a.ph);
        Mov<T> rp, lp, rl, ll;
        Axis<AX1, T>::movers(p, rp, lp);
        Axis<AX1, T>::movers(l, rl, ll);
        // T_y^H: right movers from the row above, left movers from the row below
        Site<T> yp, yl;
        if (UP) {
          Axis<AX1, T>::combine(rp, mp[s - 1][k % 2], yp);
          Axis<AX1, T>::combine(rl, ml[s - 1][k % 2], yl);
        } else {
          Axis<AX1, T>::combine(mp[s - 1][k % 2], lp, yp);
          Axis<AX1, T>::combine(ml[s - 1][k % 2], ll, yl);
        }
        mp[s - 1][k % 2] = UP ? lp : rp;
        ml[s - 1][k % 2] = UP ? ll : rl;
        const int64_t jo = UP ? j - 1 : j + 1;  // output row of stage s: in_row(it) -+ s
        x_transport_adj<T, AX0>(yp, p);
        x_transport_adj<T, AX0>(yl, l);
        if (s < K) {
          if (zero_walls) {
            if (!row_in(it - s)) {
              zero(p);
              zero(l);
            }
            if (EDGE && !c.full && !c.inside) {
              zero(p);
              zero(l);
            }
          }
        } else {
          if (it >= 2 * K && own) {
            const int64_t off = (jo * nx + c.col) * 8;
            store_site(psi_out + off, p);
            store_site(lam_out + off, l);
          }
          // the last stage has added its term to row j, which lies in the
          // segment [jb, je) exactly for 2K - 1 <= it < nit - 1
          if (own && it >= 2 * K - 1 && it < nit - 1) Q[j * nx + c.col] = qa[slot];
        }
      }
    }
  }
}

// K reverse steps on a 1-D line: every stage in place on the one row
template <typename T, int K, int AX0>
__device__ __forceinline__ void rev_line(T* __restrict__ psi_out, T* __restrict__ lam_out,
                                         const T* __restrict__ psi, const T* __restrict__ lam,
                                         const double* __restrict__ V, double* __restrict__ Q,
                                         const RevArgs& a, const Lanes& c, bool own) {
  Site<T> p, l;
  load_site(psi + c.col * 8, p);
  load_site(lam + c.col * 8, l);
  const bool zero_walls = !a.periodic;
  if (zero_walls && !c.full && c.out) {
    zero(p);
    zero(l);
  }
  const double v = (a.ph.mode == 2) ? V[c.col] : 0.0;
  double q = Q[c.col];
  const Factors f = adjoint_factors<sizeof(T) == 8>(v, a.ph);
#pragma unroll
  for (int s = 1; s <= K; ++s) {
    q = fma(a.qscale, im_dot(l, p), q);
    adjoint_local(p, f, a.ph);
    adjoint_local(l, f, a.ph);
    Site<T> op, ol;
    x_transport_adj<T, AX0>(p, op);
    x_transport_adj<T, AX0>(l, ol);
    p = op;
    l = ol;
    if (s < K && zero_walls && !c.full && !c.inside) {
      zero(p);
      zero(l);
    }
  }
  if (own) {
    store_site(psi_out + c.col * 8, p);
    store_site(lam_out + c.col * 8, l);
    Q[c.col] = q;
  }
}

template <typename T, int K, int AX0, int AX1>
__global__ __launch_bounds__(256, rev_min_blocks(sizeof(T) == 8, K)) void k_reverse(T* __restrict__ psi_out,
                                                    T* __restrict__ lam_out,
                                                    const T* __restrict__ psi,
                                                    const T* __restrict__ lam,
                                                    const double* __restrict__ V,
                                                    double* __restrict__ Q, RevArgs a) {
  const int lane = threadIdx.x & 63;
  int64_t blk = blockIdx.x;
  if (a.xcd_remap) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  const int64_t tile = blk * 4 + wave_in_block();
  if (tile >= a.ntiles) return;
  const int64_t strip = tile % a.nstrips;
  const int64_t seg = tile / a.nstrips;
  const int64_t xs = strip * strip_width(K) - K;  // lanes K .. 63 - K are written
  const Lanes c = lanes_of(a.nx, a.periodic, xs, lane);
  const bool own = c.inside && lane >= K && lane <= 63 - K;
  if constexpr (AX1 < 0) {
    rev_line<T, K, AX0>(psi_out, lam_out, psi, lam, V, Q, a, c, own);
  } else {
    const int64_t jb = seg * a.H;
    const int64_t je = (jb + a.H < a.ny) ? jb + a.H : a.ny;
    // FP32: waves with a lane beyond a zero wall run a variant that zeroes
    // those lanes at every stage, the others one without that work; FP64
    // keeps one variant per direction (its code is twice as long)
    if (sizeof(T) == 8 || !c.full) {
      if (seg & 1)
        rev_march<T, K, AX0, AX1, false, true>(psi_out, lam_out, psi, lam, V, Q, a, c, own, jb, je);
      else
        rev_march<T, K, AX0, AX1, true, true>(psi_out, lam_out, psi, lam, V, Q, a, c, own, jb, je);
    } else {
      if (seg & 1)
        rev_march<T, K, AX0, AX1, false, false>(psi_out, lam_out, psi, lam, V, Q, a, c, own, jb,
                                                je);
      else
        rev_march<T, K, AX0, AX1, true, false>(psi_out, lam_out, psi, lam, V, Q, a, c, own, jb,
                                               je);
    }
  }
}

// lam = [x0 > x_b] psi, Q = 0
template <typename T>
__global__ __launch_bounds__(256) void k_seed(const T* __restrict__ psi, T* __restrict__ lam,
                                              double* __restrict__ Q, int64_t ncell, int64_t n0,
                                              double xmin0, double dx, double x_b) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const double x0 = xmin0 + (static_cast<double>(c % n0) + 0.5) * dx;
  Site<T> s;
  if (x0 > x_b)
    load_site(psi + c * 8, s);
  else
    zero(s);
  store_site(lam + c * 8, s);
  Q[c] = 0.0;
}

// ---------------------------------------------------------------------------
// out[j] = sum_c G[j][c] Q[c]: per-block compensated partials in a fixed
// order, then one pass per j over the partials.
// ---------------------------------------------------------------------------
struct NS {
  double s, c;
};
__device__ __forceinline__ void ns_add(NS& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ void ns_merge(NS& a, const NS& b) {
  const double t = a.s + b.s;
  const double bb = t - a.s;
  const double err = (a.s - (t - bb)) + (b.s - bb);
  a.c = a.c + b.c + err;
  a.s = t;
}

constexpr int kProjBlocks = 256;

__device__ NS block_ns(NS v, NS* lds) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    NS o;
    o.s = __shfl_xor(v.s, m, 64);
    o.c = __shfl_xor(v.c, m, 64);
    ns_merge(v, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  NS t = lds[0];
  for (int k = 1; k < 4; ++k) ns_merge(t, lds[k]);
  return t;
}

__global__ __launch_bounds__(256) void k_project_partial(const double* __restrict__ Q,
                                                         const double* __restrict__ G,
                                                         int64_t ncell,
                                                         double* __restrict__ partials) {
  __shared__ NS lds[4];
  const int j = blockIdx.y;
  const double* g = G + static_cast<int64_t>(j) * ncell;
  NS acc{0.0, 0.0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell;
       c += stride)
    ns_add(acc, g[c] * Q[c]);
  const NS t = block_ns(acc, lds);
  if (threadIdx.x == 0) {
    partials[(static_cast<int64_t>(j) * gridDim.x + blockIdx.x) * 2] = t.s;
    partials[(static_cast<int64_t>(j) * gridDim.x + blockIdx.x) * 2 + 1] = t.c;
  }
}

__global__ __launch_bounds__(256) void k_project_final(const double* __restrict__ partials,
                                                       int nblk, double* __restrict__ out) {
  __shared__ NS lds[4];
  const int j = blockIdx.x;
  NS acc{0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const NS p{partials[(static_cast<int64_t>(j) * nblk + b) * 2],
               partials[(static_cast<int64_t>(j) * nblk + b) * 2 + 1]};
    ns_merge(acc, p);
  }
  const NS t = block_ns(acc, lds);
  if (threadIdx.x == 0) out[j] = t.s + t.c;
}

// V = sum_j theta[j] G[j] (the transpose of the projection), FP64, fixed order
__global__ __launch_bounds__(256) void k_expand(const double* __restrict__ G,
                                                const double* __restrict__ theta, int nb,
                                                int64_t ncell, double* __restrict__ V) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  double acc = 0.0;
  for (int j = 0; j < nb; ++j) acc = fma(theta[j], G[static_cast<int64_t>(j) * ncell + c], acc);
  V[c] = acc;
}

template <typename T, int K>
static const void* rev_kernel_k(int axes_code) {
  switch (axes_code) {
    case 0: return reinterpret_cast<const void*>(&k_reverse<T, K, 0, -1>);
    case 1: return reinterpret_cast<const void*>(&k_reverse<T, K, 1, -1>);
    case 2: return reinterpret_cast<const void*>(&k_reverse<T, K, 2, -1>);
    case 10: return reinterpret_cast<const void*>(&k_reverse<T, K, 0, 1>);
    case 20: return reinterpret_cast<const void*>(&k_reverse<T, K, 0, 2>);
    case 21: return reinterpret_cast<const void*>(&k_reverse<T, K, 1, 2>);
    default: return nullptr;
  }
}

// the reverse kernel of `depth` fused steps for this layout (nullptr if not built)
static const void* rev_kernel(bool fp64, int depth, int axes_code) {
  if (fp64) {
    switch (depth) {
      case 1: return rev_kernel_k<double, 1>(axes_code);
      case 2: return rev_kernel_k<double, 2>(axes_code);
      default: return nullptr;
    }
  }
  switch (depth) {
    case 1: return rev_kernel_k<float, 1>(axes_code);
    case 2: return rev_kernel_k<float, 2>(axes_code);
    case 3: return rev_kernel_k<float, 3>(axes_code);
    default: return nullptr;
  }
}

static hipError_t launch_rev(bool fp64, int depth, void* po, void* lo, const void* pi,
                             const void* li, const double* V, double* Q, const RevArgs& a,
                             int blocks, hipStream_t st) {
  const void* fn = rev_kernel(fp64, depth, a.axes_code);
  if (!fn || blocks <= 0) return hipErrorInvalidValue;
  RevArgs args = a;
  void* kargs[] = {&po, &lo, const_cast<void**>(&pi), const_cast<void**>(&li),
                   const_cast<double**>(&V), &Q, &args};
  return hipLaunchKernel(fn, dim3(blocks), dim3(256), kargs, 0, st);
}

static int rev_occ(bool fp64, int depth, int axes_code) {
  const void* k = rev_kernel(fp64, depth, axes_code);
  if (!k) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// ---------------------------------------------------------------------------
// 3-D reverse step in one pass.  A workgroup holds 64 columns (writing the
// middle 62) and a block of WY rows, and marches up a segment [kb, ke) of
// planes.  Reading plane n it adds the step's term to dL/dV at its own cells
// of that plane, applies D^H to the rows y0 - 1 .. y0 + WY of the plane and
// completes T_z^H at plane n - 1 for those rows (right movers of plane n, left
// movers of plane n - 2 kept in a two-slot ring); then T_y^H and T_x^H give
// the WY own rows of plane n - 1.  The T_z^H results are rounded as the stored
// state of a pass would be, so the bits are those of transports applied one by
// one.
// ---------------------------------------------------------------------------
struct Rev3Args {
  int64_t nx, ny, nz;
  int periodic;
  int64_t nstrips, nyblk, nseg, ntiles;
  int H;  // planes per segment
  double qscale;
  PhaseK ph;
};

// resident blocks per CU the 3-D reverse pass is compiled for
template <typename T> struct Rev3Shape;
template <> struct Rev3Shape<float> { static constexpr int kMinBlocks = 2; };
template <> struct Rev3Shape<double> { static constexpr int kMinBlocks = 1; };

__device__ __forceinline__ int64_t rev_wrap(int64_t r, int64_t n, int periodic) {
  if (periodic) return ((r % n) + n) % n;
  return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

// The tile of a workgroup: four waves own TW rows each (WY = 4 TW rows), and
// the WY + 2 rows of a plane are read once, D^H and T_z^H applied by the wave
// that reads them (wave w takes rows w, w + 4, ...), their y movers left in
// LDS; after a barrier each wave completes T_y^H and T_x^H on its own rows (a
// second barrier frees the LDS for the next plane).  Per cell the arithmetic
// and its order are those of a wave that reads its own halo rows, so the bits
// do not depend on the tile.
template <typename T> struct Rev3Tile {
  static constexpr int TW = 4;  // 16-row tiles (8: 3 % slower at 512^3 FP32)
  static constexpr int WY = 4 * TW;       // rows written per workgroup
  static constexpr int R = WY + 2;        // rows read: y0 - 1 .. y0 + WY
  static constexpr int NL = (R + 3) / 4;  // rows read per wave (the last waves fewer)
  static_assert(R <= 32, "row mask");
};

template <typename T> struct alignas(16) Rev3Lds {
  // y movers of T_z^H psi (p) and lambda (l) of every row read: right (r) and
  // left (l) movers
  Mov<T> rp[Rev3Tile<T>::R][64], lp[Rev3Tile<T>::R][64];
  Mov<T> rl[Rev3Tile<T>::R][64], ll[Rev3Tile<T>::R][64];
};

template <typename T>
__global__ __launch_bounds__(256, Rev3Shape<T>::kMinBlocks) void k_reverse3d_wg(
    T* __restrict__ psi_out, T* __restrict__ lam_out, const T* __restrict__ psi,
    const T* __restrict__ lam, const double* __restrict__ V, double* __restrict__ Q,
    Rev3Args a) {
  using S = Rev3Tile<T>;
  constexpr int TW = S::TW, WY = S::WY, R = S::R, NL = S::NL;
  constexpr bool TWO = sizeof(T) == 8;
  __shared__ Rev3Lds<T> sh;
  const int lane = threadIdx.x & 63;
  const int wv = wave_in_block();
  const int64_t tile = blockIdx.x;
  if (tile >= a.ntiles) return;  // the whole workgroup
  const int64_t nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t strip = tile % a.nstrips;
  const int64_t rest = tile / a.nstrips;
  const int64_t yblk = rest % a.nyblk, seg = rest / a.nyblk;
  const int64_t y0 = yblk * WY;
  const int64_t kb = seg * a.H;
  const int64_t ke = (kb + a.H < nz) ? kb + a.H : nz;
  const int nit = static_cast<int>(ke - kb) + 2;  // planes kb - 1 .. ke
  const Lanes c = lanes_of(nx, a.periodic, strip * strip_width(1) - 1, lane);
  const bool own = c.inside && lane >= 1 && lane <= 62;
  const bool walls = !a.periodic;
  const bool read_v = (a.ph.mode == 2);
  auto clamp_it = [&](int64_t e) -> int {
    return static_cast<int>(e < -64 ? -64 : (e > nit + 64 ? nit + 64 : e));
  };
  const int klo = clamp_it(1 - kb), khi = clamp_it(1 - kb + nz);
  uint32_t rin = 0;  // bit t: row y0 - 1 + t lies in the box
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int64_t y = y0 - 1 + t;
    if (y >= 0 && y < ny) rin |= 1u << t;
  }
  rin = __builtin_amdgcn_readfirstlane(rin);
  int64_t rowoff[NL];  // this wave's rows t = wv + 4 j
#pragma unroll
  for (int j = 0; j < NL; ++j) rowoff[j] = rev_wrap(y0 - 1 + wv + 4 * j, ny, a.periodic) * nx;
  Mov<T> lpr[2][NL], llr[2][NL];  // left z movers of D^H psi, lambda; slot: plane % 2
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      zero(lpr[q][j]);
      zero(llr[q][j]);
    }
  }
  for (int base = 0;; base += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int it = base + u;
      if (it >= nit) return;  // uniform over the workgroup
      const int64_t n = kb - 1 + it;  // plane read
      const bool n_in = it >= klo && it < khi;
      const bool n_own = it >= 1 && it < nit - 1;  // kb <= n < ke
      const int64_t pbase = rev_wrap(n, nz, a.periodic) * ny * nx + c.col;
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int t = wv + 4 * j;
        if (t >= R) break;  // wave-uniform
        const int64_t q = pbase + rowoff[j];
        Site<T> ps, ls;
        load_site(psi + q * 8, ps);
        load_site(lam + q * 8, ls);
        const double v = read_v ? V[q] : 0.0;
        // the step's term of dL/dV, once per cell: own rows, lanes and planes
        if (t >= 1 && t <= WY && n_own && ((rin >> t) & 1u) && own)
          Q[q] = fma(a.qscale, im_dot(ls, ps), Q[q]);
        const Factors f = adjoint_factors<TWO>(v, a.ph);
        adjoint_local(ps, f, a.ph);
        adjoint_local(ls, f, a.ph);
        if (walls && !n_in) {
          zero(ps);
          zero(ls);
        }
        Mov<T> rp, lp, rl, ll;
        Site<T> zp, zl;  // T_z^H of psi and lambda at plane n - 1, row t
        Axis<2, T>::movers(ps, rp, lp);
        Axis<2, T>::movers(ls, rl, ll);
        Axis<2, T>::combine(rp, lpr[u][j], zp);
        Axis<2, T>::combine(rl, llr[u][j], zl);
        lpr[u][j] = lp;
        llr[u][j] = ll;
        if (it < 2) continue;  // plane n - 1 lies before the segment
        // rows beyond a wall and lanes beyond a side wall read as zero
        if (walls && (!((rin >> t) & 1u) || (!c.full && c.out))) {
          zero(zp);
          zero(zl);
        }
        Axis<1, T>::movers(zp, sh.rp[t][lane], sh.lp[t][lane]);
        Axis<1, T>::movers(zl, sh.rl[t][lane], sh.ll[t][lane]);
      }
      if (it < 2) continue;  // uniform
      __syncthreads();
      const int64_t obase = ((n - 1) * ny + y0) * nx + c.x;
#pragma unroll
      for (int k = 0; k < TW; ++k) {
        // T_y^H at row y0 + w: right movers from the row above, left from below
        const int w = wv * TW + k;
        Site<T> yp, yl, op, ol;
        Axis<1, T>::combine(sh.rp[w + 2][lane], sh.lp[w][lane], yp);
        Axis<1, T>::combine(sh.rl[w + 2][lane], sh.ll[w][lane], yl);
        if (walls && !c.full && !c.inside) {
          zero(yp);
          zero(yl);
        }
        x_transport_adj<T, 0>(yp, op);
        x_transport_adj<T, 0>(yl, ol);
        if (own && y0 + w < ny) {
          store_site(psi_out + (obase + w * nx) * 8, op);
          store_site(lam_out + (obase + w * nx) * 8, ol);
        }
      }
      __syncthreads();  // the next plane's movers overwrite these
    }
  }
}

template <typename T>
static int rev3_occupancy() {
  static int occ = -1;
  if (occ < 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_reverse3d_wg<T>, 256, 0) !=
        hipSuccess) {
      (void)hipGetLastError();
      n = 0;
    }
    occ = n > 0 ? n : Rev3Shape<T>::kMinBlocks;
  }
  return occ;
}

// one reverse step on a 3-D grid, (pi, li) -> (po, lo).  Segments along z
// from a cost model: (rounds of resident waves) x (H + 2 plane iterations).
template <typename T>
static hipError_t rev3d_t(const void* pi, const void* li, void* po, void* lo, const double* V,
                          double* Q, Rev3Args a, int cu_count, hipStream_t st) {
  constexpr int WY = Rev3Tile<T>::WY;
  a.nstrips = (a.nx + strip_width(1) - 1) / strip_width(1);
  a.nyblk = (a.ny + WY - 1) / WY;
  const int64_t per_seg = a.nstrips * a.nyblk;
  // workgroup tiles: resident workgroups are the target
  const int64_t resident = int64_t(rev3_occupancy<T>()) * (cu_count > 0 ? cu_count : 256);
  int64_t best_H = a.nz, best_cost = -1;
  for (int64_t nseg = 1; nseg <= 64 && nseg <= a.nz; ++nseg) {
    const int64_t H = (a.nz + nseg - 1) / nseg;
    const int64_t segs = (a.nz + H - 1) / H;
    const int64_t rounds = (per_seg * segs + resident - 1) / resident;
    const int64_t cost = rounds * (H + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best_H = H;
    }
  }
  if (best_H > INT32_MAX - 64) return hipErrorInvalidValue;
  a.H = static_cast<int>(best_H);
  a.nseg = (a.nz + best_H - 1) / best_H;
  a.ntiles = per_seg * a.nseg;
  const int64_t blocks = a.ntiles;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reverse3d_wg<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     static_cast<T*>(po), static_cast<T*>(lo), static_cast<const T*>(pi),
                     static_cast<const T*>(li), V, Q, a);
  return hipGetLastError();
}

static hipError_t launch_rev3d(bool fp64, const void* pi, const void* li, void* po, void* lo,
                               const double* V, double* Q, const Rev3Args& a, int cu_count,
                               hipStream_t st) {
  return fp64 ? rev3d_t<double>(pi, li, po, lo, V, Q, a, cu_count, st)
              : rev3d_t<float>(pi, li, po, lo, V, Q, a, cu_count, st);
}

}  // namespace dirac

using namespace dirac;

// reverse steps fused per pass: FP32 up to 3, FP64 up to 2, within the plan's
// depth cap; a periodic 2-D box needs at least 2 rows per fused step
int dirac::reverse_depth(dl_plan p) {
  if (p->g.ndim > 2 || p->strang || p->nc != 4) return 1;
  int d = std::min(p->depth_limit, p->fp64 ? kMaxRevDepthF64 : kMaxRevDepthF32);
  if (p->g.ndim == 2 && p->bc == DL_BC_PERIODIC)
    while (d > 1 && p->g.n[1] < 2 * d) --d;
  return d < 1 ? 1 : d;
}

static void rev_tiling(dl_plan p, int depth, RevArgs& a, int& blocks) {
  a.nx = p->g.n[0];
  a.ny = p->g.ndim > 1 ? p->g.n[1] : 1;
  a.periodic = (p->bc == DL_BC_PERIODIC);
  const int w = strip_width(depth);
  a.nstrips = (a.nx + w - 1) / w;
  a.axes_code = axes_code(p->g);
  int64_t target;
  if (p->waves_per_cu > 0) {
    target = int64_t(p->cu_count) * p->waves_per_cu;
  } else {
    int occ = rev_occ(p->fp64, depth, a.axes_code);
    if (occ <= 0) occ = 2;
    target = int64_t(occ) * 4 * p->cu_count;
  }
  if (p->g.ndim == 1) {
    a.nseg = 1;
    a.H = 1;
  } else {
    int64_t H = p->seg_override;
    if (H <= 0) {
      int64_t nseg = target / a.nstrips;
      if (nseg < 1) nseg = 1;
      H = (a.ny + nseg - 1) / nseg;
      if (H < 8) H = 8;
    }
    if (H > a.ny) H = a.ny;
    a.H = static_cast<int>(H);
    a.nseg = (a.ny + H - 1) / H;
  }
  a.ntiles = a.nstrips * a.nseg;
  blocks = static_cast<int>((a.ntiles + 3) / 4);
  a.xcd_remap = (blocks % 8 == 0) ? 1 : 0;
  double dV = p->dx;
  for (int d = 1; d < p->g.ndim; ++d) dV *= p->dx;
  a.qscale = 2.0 * p->dt * dV;
}

static int check_adjoint_plan(dl_plan p) {
  int rc = check_live(p);
  if (rc) return rc;
  if (p->strang) return set_error(DL_ERR_ARG, "the adjoint is built for lowest-order steps only");
  if (p->nc != 4) return set_error(DL_ERR_ARG, "the adjoint is built for four-component states");
  return DL_OK;
}

extern "C" int dl_seed_adjoint(dl_plan p, const void* psi, double x_b, void* lam, double* Q,
                               void* stream) {
  dirac::TraceRange trace_range("dl_seed_adjoint");
  int rc = check_adjoint_plan(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi")) || (rc = check_state_ptr(lam, "lam")) ||
      (rc = check_f64_ptr(Q, "Q", false)))
    return rc;
  if (psi == lam) return set_error(DL_ERR_ARG, "psi and lam must differ");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int blocks = static_cast<int>((p->cells + 255) / 256);
  if (p->fp64)
    hipLaunchKernelGGL(k_seed<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const double*>(psi), static_cast<double*>(lam), Q, p->cells,
                       p->g.n[0], p->g.xmin[0], p->dx, x_b);
  else
    hipLaunchKernelGGL(k_seed<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const float*>(psi), static_cast<float*>(lam), Q, p->cells,
                       p->g.n[0], p->g.xmin[0], p->dx, x_b);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DL_OK : set_hip_error(e, "seed launch");
}

extern "C" int dl_grad_step(dl_plan p, void* psi, void* lam, const double* V, double* Q,
                            int64_t nsteps, void* stream) {
  dirac::TraceRange trace_range("dl_grad_step");
  int rc = check_adjoint_plan(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi")) || (rc = check_state_ptr(lam, "lam")) ||
      (rc = check_f64_ptr(V, "V", true)) || (rc = check_f64_ptr(Q, "Q", false)))
    return rc;
  if (psi == lam) return set_error(DL_ERR_ARG, "psi and lam must differ");
  if (nsteps < 0) return set_error(DL_ERR_ARG, "nsteps < 0");
  if (nsteps == 0) return DL_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!p->tmp2) {
    hipError_t e = hipMalloc(&p->tmp2, p->state_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->tmp2 = nullptr;
      return set_error(DL_ERR_NOMEM, "allocation of the second adjoint buffer failed");
    }
  }
  const PhaseK ph = make_phase(p->g.ndim, p->dt, p->c, p->m, phase_mode(p->m, V), p->fp64);
  if (p->g.ndim == 3) {  // one pass per reverse step, alternating buffers, ending in psi and lam
    Rev3Args a{};
    a.nx = p->g.n[0];
    a.ny = p->g.n[1];
    a.nz = p->g.n[2];
    a.periodic = (p->bc == DL_BC_PERIODIC);
    a.qscale = 2.0 * p->dt * p->dx * p->dx * p->dx;
    a.ph = ph;
    void* pa = psi;
    void* la = lam;
    void* pb = p->tmp;
    void* lb = p->tmp2;
    for (int64_t s = 0; s < nsteps; ++s) {
      hipError_t e = launch_rev3d(p->fp64, pa, la, pb, lb, V, Q, a, p->cu_count, st);
      if (e != hipSuccess) return set_hip_error(e, "reverse sweep launch");
      std::swap(pa, pb);
      std::swap(la, lb);
    }
    if (pa != psi) {  // odd step count: the result sits in the plan's buffers
      hipError_t e = hipMemcpyAsync(psi, pa, p->state_bytes, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(lam, la, p->state_bytes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return set_hip_error(e, "reverse sweep copy");
    }
    return DL_OK;
  }
  const int dmax = reverse_depth(p);
  void* pa = psi;
  void* la = lam;
  void* pb = p->tmp;
  void* lb = p->tmp2;
  int64_t left = nsteps;
  for (int d = dmax; d >= 1; --d) {
    if (left < d) continue;
    RevArgs a{};
    int blocks = 0;
    rev_tiling(p, d, a, blocks);
    a.ph = ph;
    for (; left >= d; left -= d) {
      hipError_t e = launch_rev(p->fp64, d, pb, lb, pa, la, V, Q, a, blocks, st);
      if (e != hipSuccess) return set_hip_error(e, "reverse sweep launch");
      void* t = pa; pa = pb; pb = t;
      t = la; la = lb; lb = t;
    }
  }
  if (pa != psi) {
    hipError_t e = hipMemcpyAsync(psi, pa, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(lam, la, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return set_hip_error(e, "hipMemcpyAsync");
  }
  return DL_OK;
}

extern "C" int dl_project(dl_plan p, const double* Q, const double* G, int nb, double* out,
                          void* stream) {
  dirac::TraceRange trace_range("dl_project");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_f64_ptr(Q, "Q", false)) || (rc = check_f64_ptr(G, "G", false)) ||
      (rc = check_f64_ptr(out, "out", false)))
    return rc;
  if (nb < 1 || nb > 65535) return set_error(DL_ERR_ARG, "nb must be in 1..65535");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t need = sizeof(double) * 2 * kProjBlocks * static_cast<size_t>(nb);
  if (need > p->proj_bytes) {
    if (p->proj) (void)hipFree(p->proj);
    p->proj = nullptr;
    p->proj_bytes = 0;
    if (hipMalloc(&p->proj, need) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(DL_ERR_NOMEM, "allocation of projection partials failed");
    }
    p->proj_bytes = need;
  }
  hipLaunchKernelGGL(k_project_partial, dim3(kProjBlocks, nb), dim3(256), 0, st, Q, G, p->cells,
                     p->proj);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_error(e, "projection launch");
  hipLaunchKernelGGL(k_project_final, dim3(nb), dim3(256), 0, st, p->proj, kProjBlocks, out);
  e = hipGetLastError();
  return e == hipSuccess ? DL_OK : set_hip_error(e, "projection launch");
}

extern "C" int dl_expand(dl_plan p, const double* G, const double* theta, int nb, double* V,
                         void* stream) {
  dirac::TraceRange trace_range("dl_expand");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_f64_ptr(G, "G", false)) || (rc = check_f64_ptr(theta, "theta", false)) ||
      (rc = check_f64_ptr(V, "V", false)))
    return rc;
  if (nb < 1) return set_error(DL_ERR_ARG, "nb must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int blocks = static_cast<int>((p->cells + 255) / 256);
  hipLaunchKernelGGL(k_expand, dim3(blocks), dim3(256), 0, st, G, theta, nb, p->cells, V);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DL_OK : set_hip_error(e, "expand launch");
}
