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
// Work decomposition of the reverse step: the y transport precedes the x
// transport, so a strip's edge columns need the y-transported values of the
// columns beside the strip.  A wave therefore covers 64 columns starting one
// column left of its 62 output columns; lanes 0 and 63 compute the halo
// columns in full and do not store.
#include "dirac_device.h"
#include "dirac_plan.h"

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

// conjugate factors: D^H = s exp(+i theta)
__device__ __forceinline__ Factors adjoint_factors(double V, const PhaseK& k) {
  Factors f = phase_factors(V, k);
  f.ui = -f.ui;
  f.di = -f.di;
  return f;
}

// load the cell at column x of row j (walls / wrap-around), zeros outside
template <typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ f, int64_t nx, int64_t ny,
                                          int periodic, int64_t x, int64_t j, Site<T>& s,
                                          bool& inside) {
  zero(s);
  inside = false;
  if (j < 0 || j >= ny) {
    if (!periodic) return;
    j = (j < 0) ? j + ny : j - ny;
  }
  if (x < 0 || x >= nx) {
    if (!periodic) return;
    x = (x < 0) ? x + nx : x - nx;
  }
  inside = true;
  load_site(f + (j * nx + x) * 8, s);
}

template <typename T> struct RevRow {
  Site<T> p, l;  // psi and lambda at this lane's column
  double v;      // potential at this lane's (possibly wrapped) column
  bool inside;
};

template <typename T>
__device__ __forceinline__ void load_rev_row(const T* psi, const T* lam, const double* V,
                                             const RevArgs& a, int64_t x, int64_t j,
                                             RevRow<T>& R) {
  bool in2;
  load_cell(psi, a.nx, a.ny, a.periodic, x, j, R.p, R.inside);
  load_cell(lam, a.nx, a.ny, a.periodic, x, j, R.l, in2);
  R.v = 0.0;
  if (R.inside && a.ph.mode == 2) {
    int64_t jj = j, xx = x;
    if (jj < 0) jj += a.ny;
    if (jj >= a.ny) jj -= a.ny;
    if (xx < 0) xx += a.nx;
    if (xx >= a.nx) xx -= a.nx;
    R.v = V[jj * a.nx + xx];
  }
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

// backward x transport of a row held across the wave: right movers from the
// right lane, left movers from the left lane (lanes 0 and 63 are halo lanes)
template <typename T, int AX>
__device__ __forceinline__ void x_transport_adj(const Site<T>& in, Site<T>& out) {
  Mov<T> r, l, rR, lL;
  Axis<AX, T>::movers(in, r, l);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rR.v[k] = dpp_from_right(r.v[k], r.v[k]);
    lL.v[k] = dpp_from_left(l.v[k], l.v[k]);
  }
  Axis<AX, T>::combine(rR, lL, out);
}

constexpr int PFR = 2;

template <typename T, int AX0, int AX1, bool UP>
__device__ __forceinline__ void rev_march(T* __restrict__ psi_out, T* __restrict__ lam_out,
                                          const T* __restrict__ psi, const T* __restrict__ lam,
                                          const double* __restrict__ V, double* __restrict__ Q,
                                          const RevArgs& a, int64_t x, bool own, int64_t jb,
                                          int64_t je) {
  const int nit = static_cast<int>(je - jb) + 2;
  auto in_row = [&](int it) -> int64_t { return UP ? jb - 1 + it : je - it; };
  auto out_row = [&](int it) -> int64_t { return UP ? jb - 2 + it : je - it + 1; };
  RevRow<T> ring[PFR];
#pragma unroll
  for (int k = 0; k < PFR; ++k)
    if (k < nit) load_rev_row(psi, lam, V, a, x, in_row(k), ring[k]);
  Mov<T> sp1, sp2, sl1, sl2;  // y movers of the two previous rows (psi, lambda)
  zero(sp1); zero(sp2); zero(sl1); zero(sl2);
  for (int base = 0; base < nit; base += PFR) {
#pragma unroll
    for (int k = 0; k < PFR; ++k) {
      const int it = base + k;
      if (it < nit) {
        const RevRow<T> cur = ring[k];
        if (it + PFR < nit) load_rev_row(psi, lam, V, a, x, in_row(it + PFR), ring[k]);
        const int64_t jin = in_row(it);
        // gradient accumulation at the input time level, owned cells only
        if (own && jin >= jb && jin < je) {
          double* q = Q + jin * a.nx + x;
          *q = fma(a.qscale, im_dot(cur.l, cur.p), *q);
        }
        // D^H on both fields
        Site<T> p = cur.p, l = cur.l;
        const Factors f = adjoint_factors(cur.v, a.ph);
        adjoint_local(p, f, a.ph);
        adjoint_local(l, f, a.ph);
        Mov<T> rp, lp, rl, ll;
        Axis<AX1, T>::movers(p, rp, lp);
        Axis<AX1, T>::movers(l, rl, ll);
        if (it >= 2) {
          // T_y^H: right movers from row j+1, left movers from row j-1
          Site<T> yp, yl;
          if (UP) {
            Axis<AX1, T>::combine(rp, sp2, yp);
            Axis<AX1, T>::combine(rl, sl2, yl);
          } else {
            Axis<AX1, T>::combine(sp2, lp, yp);
            Axis<AX1, T>::combine(sl2, ll, yl);
          }
          Site<T> op, ol;
          x_transport_adj<T, AX0>(yp, op);
          x_transport_adj<T, AX0>(yl, ol);
          if (own) {
            const int64_t off = (out_row(it) * a.nx + x) * 8;
            store_site(psi_out + off, op);
            store_site(lam_out + off, ol);
          }
        }
        sp2 = sp1;
        sl2 = sl1;
        sp1 = UP ? lp : rp;
        sl1 = UP ? ll : rl;
      }
    }
  }
}

template <typename T, int AX0, int AX1>
__global__ __launch_bounds__(256) void k_reverse(T* __restrict__ psi_out, T* __restrict__ lam_out,
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
  const int64_t x = strip * 62 - 1 + lane;
  const bool own = lane >= 1 && lane <= 62 && x >= 0 && x < a.nx;
  if constexpr (AX1 < 0) {
    RevRow<T> R;
    load_rev_row(psi, lam, V, a, x, 0, R);
    if (own) Q[x] = fma(a.qscale, im_dot(R.l, R.p), Q[x]);
    const Factors f = adjoint_factors(R.v, a.ph);
    adjoint_local(R.p, f, a.ph);
    adjoint_local(R.l, f, a.ph);
    Site<T> op, ol;
    x_transport_adj<T, AX0>(R.p, op);
    x_transport_adj<T, AX0>(R.l, ol);
    if (own) {
      store_site(psi_out + x * 8, op);
      store_site(lam_out + x * 8, ol);
    }
  } else {
    const int64_t jb = seg * a.H;
    const int64_t je = (jb + a.H < a.ny) ? jb + a.H : a.ny;
    if (seg & 1)
      rev_march<T, AX0, AX1, false>(psi_out, lam_out, psi, lam, V, Q, a, x, own, jb, je);
    else
      rev_march<T, AX0, AX1, true>(psi_out, lam_out, psi, lam, V, Q, a, x, own, jb, je);
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

template <typename T, int AX0, int AX1>
static hipError_t launch_rev_t(void* po, void* lo, const void* pi, const void* li,
                               const double* V, double* Q, const RevArgs& a, int blocks,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_reverse<T, AX0, AX1>), dim3(blocks), dim3(256), 0, st,
                     static_cast<T*>(po), static_cast<T*>(lo), static_cast<const T*>(pi),
                     static_cast<const T*>(li), V, Q, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_rev(void* po, void* lo, const void* pi, const void* li, const double* V,
                             double* Q, const RevArgs& a, int blocks, hipStream_t st) {
  switch (a.axes_code) {
    case 0: return launch_rev_t<T, 0, -1>(po, lo, pi, li, V, Q, a, blocks, st);
    case 1: return launch_rev_t<T, 1, -1>(po, lo, pi, li, V, Q, a, blocks, st);
    case 2: return launch_rev_t<T, 2, -1>(po, lo, pi, li, V, Q, a, blocks, st);
    case 10: return launch_rev_t<T, 0, 1>(po, lo, pi, li, V, Q, a, blocks, st);
    case 20: return launch_rev_t<T, 0, 2>(po, lo, pi, li, V, Q, a, blocks, st);
    case 21: return launch_rev_t<T, 1, 2>(po, lo, pi, li, V, Q, a, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static int rev_occ(int axes_code) {
  const void* k;
  switch (axes_code) {
    case 0: k = reinterpret_cast<const void*>(&k_reverse<T, 0, -1>); break;
    case 1: k = reinterpret_cast<const void*>(&k_reverse<T, 1, -1>); break;
    case 2: k = reinterpret_cast<const void*>(&k_reverse<T, 2, -1>); break;
    case 10: k = reinterpret_cast<const void*>(&k_reverse<T, 0, 1>); break;
    case 20: k = reinterpret_cast<const void*>(&k_reverse<T, 0, 2>); break;
    case 21: k = reinterpret_cast<const void*>(&k_reverse<T, 1, 2>); break;
    default: return 0;
  }
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

}  // namespace dirac

using namespace dirac;

static void rev_tiling(dl_plan p, RevArgs& a, int& blocks) {
  a.nx = p->g.n[0];
  a.ny = p->g.ndim > 1 ? p->g.n[1] : 1;
  a.periodic = (p->bc == DL_BC_PERIODIC);
  a.nstrips = (a.nx + 61) / 62;
  int64_t target;
  if (p->waves_per_cu > 0) {
    target = int64_t(p->cu_count) * p->waves_per_cu;
  } else {
    int occ = p->fp64 ? rev_occ<double>(axes_code(p->g)) : rev_occ<float>(axes_code(p->g));
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
  a.axes_code = axes_code(p->g);
  double dV = p->dx;
  for (int d = 1; d < p->g.ndim; ++d) dV *= p->dx;
  a.qscale = 2.0 * p->dt * dV;
}

static int check_adjoint_plan(dl_plan p) {
  int rc = check_live(p);
  if (rc) return rc;
  if (p->g.ndim > 2) return set_error(DL_ERR_ARG, "the adjoint supports 1-D and 2-D grids");
  if (p->strang) return set_error(DL_ERR_ARG, "the adjoint is built for lowest-order steps only");
  if (p->nc != 4) return set_error(DL_ERR_ARG, "the adjoint is built for four-component states");
  return DL_OK;
}

extern "C" int dl_seed_adjoint(dl_plan p, const void* psi, double x_b, void* lam, double* Q,
                               void* stream) {
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
  RevArgs a{};
  int blocks = 0;
  rev_tiling(p, a, blocks);
  a.ph = make_phase(p->g.ndim, p->dt, p->c, p->m, phase_mode(p->m, V), p->fp64);
  void* pa = psi;
  void* la = lam;
  void* pb = p->tmp;
  void* lb = p->tmp2;
  for (int64_t s = 0; s < nsteps; ++s) {
    hipError_t e = p->fp64 ? launch_rev<double>(pb, lb, pa, la, V, Q, a, blocks, st)
                           : launch_rev<float>(pb, lb, pa, la, V, Q, a, blocks, st);
    if (e != hipSuccess) return set_hip_error(e, "reverse sweep launch");
    void* t = pa; pa = pb; pb = t;
    t = la; la = lb; lb = t;
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
