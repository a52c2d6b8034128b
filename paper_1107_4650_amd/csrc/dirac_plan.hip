// dirac_plan.hip -- plans, argument checking and the C ABI of libdirac.
// The operations are defined in include/libdirac.h; this file validates
// arguments, owns the scratch memory and sequences kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/libdirac.h"
#include "dirac_launch.h"
#include "dirac_trace.h"
#include "dirac_plan.h"

using namespace dirac;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

namespace dirac {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
int set_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }

int validate_grid(const dl_grid* g, double dx, double dt, double c, double m, int dtype, int bc,
                  int max_ndim, int shift) {
  if (!g) return fail(DL_ERR_ARG, "grid is NULL");
  if (g->ndim < 1 || g->ndim > max_ndim) return fail(DL_ERR_ARG, "ndim must be 1..%d", max_ndim);
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < 2) return fail(DL_ERR_ARG, "n[%d] = %lld: need at least 2 cells", d,
                                 static_cast<long long>(g->n[d]));
    if (g->n[d] > (int64_t(1) << 31)) return fail(DL_ERR_ARG, "n[%d] too large", d);
    if (g->axis[d] < 0 || g->axis[d] > 2) return fail(DL_ERR_ARG, "axis[%d] must be 0, 1 or 2", d);
    if (d > 0 && g->axis[d] <= g->axis[d - 1])
      return fail(DL_ERR_ARG, "axis[] must increase with the grid dimension");
    if (!std::isfinite(g->xmin[d])) return fail(DL_ERR_ARG, "xmin[%d] not finite", d);
  }
  int64_t cells = 1;
  for (int d = 0; d < g->ndim; ++d) {
    if (cells > (int64_t(1) << 40) / g->n[d]) return fail(DL_ERR_ARG, "grid too large");
    cells *= g->n[d];
  }
  if (!finite_pos(dx) || !finite_pos(dt) || !finite_pos(c))
    return fail(DL_ERR_ARG, "dx, dt and c must be finite and positive");
  if (!std::isfinite(m) || m < 0.0) return fail(DL_ERR_ARG, "m must be finite and >= 0");
  if (dtype != DL_C64 && dtype != DL_C128) return fail(DL_ERR_DTYPE, "unknown dtype %d", dtype);
  if (bc != DL_BC_ZERO && bc != DL_BC_PERIODIC) return fail(DL_ERR_ARG, "unknown bc %d", bc);
  const double K = c * dt / dx;
  if (!(std::fabs(K - shift) <= 1e-12 * shift))
    return fail(DL_ERR_CFL, "c*dt/dx = %.17g: the characteristic shift needs c*dt = %d dx", K,
                shift);
  return DL_OK;
}

PhaseK make_phase(int ntransports, double dt, double c, double m, int mode, bool two_angles) {
  PhaseK k{};
  const double s = std::ldexp(1.0, -ntransports);
  const double mc2 = m * c * c;
  const double mu = mc2 * dt;
  k.eu_re = s * std::cos(mu);
  k.eu_im = -s * std::sin(mu);
  k.ed_re = s * std::cos(mu);
  k.ed_im = s * std::sin(mu);
  k.dt = dt;
  k.mc2 = mc2;
  k.scale = s;
  k.scale_f = static_cast<float>(s);
  k.mode = mode;
  k.two_angles = two_angles ? 1 : 0;
  return k;
}

int phase_mode(double m, const double* V) {
  if (V) return 2;
  return (m != 0.0) ? 1 : 0;
}

int axes_code(const dl_grid& g) {
  if (g.ndim == 1) return g.axis[0];
  if (g.ndim == 2) return 10 * g.axis[1] + g.axis[0];  // 10: (x,y) 20: (x,z) 21: (y,z)
  return 210;
}

// Tiling of the one-pass sweep: strips of `strip_width` x cells, march
// segments sized so that at most `target` waves (one full round of resident
// waves) are created, avoiding a partial second round.
void make_tiling(const dl_grid& g, int64_t target, int seg_override, SweepArgs& a, int& blocks,
                 int strip_width) {
  a.nx = g.n[0];
  a.ny = g.ndim > 1 ? g.n[1] : 1;
  a.nz = g.ndim > 2 ? g.n[2] : 1;
  a.nstrips = (a.nx + strip_width - 1) / strip_width;
  if (g.ndim == 1) {
    a.nseg = 1;
    a.H = 1;
    a.nyblk = 1;
    a.ntiles = a.nstrips;
  } else if (g.ndim == 2) {
    const int64_t ny = a.ny;
    int64_t H;
    if (seg_override > 0) {
      H = seg_override;
    } else {
      int64_t nseg = target / a.nstrips;
      if (nseg < 1) nseg = 1;
      H = (ny + nseg - 1) / nseg;
      if (H < 8) H = 8;
    }
    if (H > ny) H = ny;
    a.H = static_cast<int>(H);
    a.nseg = (ny + H - 1) / H;
    a.nyblk = 1;
    a.ntiles = a.nstrips * a.nseg;
  } else {
    const int TY = kTY3D_F32;  // overwritten by the caller for FP64
    (void)TY;
    a.ntiles = 0;
  }
  blocks = static_cast<int>((a.ntiles + 3) / 4);
  a.xcd_remap = (blocks % 8 == 0) ? 1 : 0;
  a.axes_code = axes_code(g);
}

// 3-D tiling: strips of `strip_width` x cells by blocks of `ty` y rows, march
// segments along z.  A tile (a wave, or with per_block = 1 a workgroup) of a
// segment of H planes runs H + halo plane iterations; with `target` tiles
// resident at once, the segment count is the one that minimises (rounds of
// resident tiles) x (H + halo).  per_block: tiles per workgroup (4 or 1).
void make_tiling3d(const dl_grid& g, int ty, int strip_width, int halo, int64_t target,
                   int seg_override, SweepArgs& a, int& blocks, int per_block) {
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.nstrips = (a.nx + strip_width - 1) / strip_width;
  a.nyblk = (a.ny + ty - 1) / ty;
  const int64_t per_seg = a.nstrips * a.nyblk;
  int64_t H;
  if (seg_override > 0) {
    H = seg_override;
  } else {
    if (target < 1) target = 1;
    H = a.nz;
    int64_t best = -1;
    for (int64_t ns = 1; ns <= 4096 && ns <= a.nz; ++ns) {
      const int64_t h = (a.nz + ns - 1) / ns;
      if (h < 4 && ns > 1) break;
      const int64_t nseg = (a.nz + h - 1) / h;
      const int64_t rounds = (per_seg * nseg + target - 1) / target;
      const int64_t cost = rounds * (h + halo);
      if (best < 0 || cost < best) {
        best = cost;
        H = h;
      }
    }
  }
  if (H > a.nz) H = a.nz;
  a.H = static_cast<int>(H);
  a.nseg = (a.nz + H - 1) / H;
  a.ntiles = per_seg * a.nseg;
  if (per_block == 1) {  // one workgroup per tile, XCD-contiguous runs of tiles
    blocks = static_cast<int>((a.ntiles + 7) / 8 * 8);
    a.xcd_remap = 1;
  } else {
    blocks = static_cast<int>((a.ntiles + 3) / 4);
    a.xcd_remap = (blocks % 8 == 0) ? 1 : 0;
  }
  a.axes_code = 210;
}

}  // namespace dirac

// ===========================================================================
// plan
// ===========================================================================

// one-cell transports per step: one per axis (Sec. 2.1), or two per axis for
// the second-order step (Sec. 2.4)
int dirac::transports_per_step(dl_plan p) {
  if (p->strang && p->g.ndim == 3) return 8;  // A four times, B and C twice
  return (p->strang ? 2 : 1) * p->g.ndim;
}

// make the tilings of phase mode `mode` current
static void select_tiling(dl_plan p, int mode) {
  const PlanTiling& t = p->tiling[mode < 0 || mode > 4 ? 2 : mode];
  for (int d = 0; d < kMaxDepth; ++d) {
    p->sw[d] = t.a[d];
    p->bl[d] = t.b[d];
  }
  p->sw_deep = t.deep;
  p->bl_deep = t.deep_b;
}

// waves that can be resident at once for the sweep kernel of this plan
static int64_t resident_waves(dl_plan p, int mode, int depth) {
  if (p->waves_per_cu > 0) return int64_t(p->cu_count) * p->waves_per_cu;
  int occ = p->dry ? 0
                   : sweep_occupancy(p->fp64, p->strang, p->g.ndim, axes_code(p->g), mode, depth,
                                     p->nc);
  if (occ <= 0) occ = 2;
  return int64_t(occ) * 4 * p->cu_count;
}

static int plan_tiling(dl_plan p) {
  // fused steps per pass.  A periodic 2-D pass reaches one row per stage (one
  // per lowest-order step, two per second-order step) beyond a segment on each
  // side and wraps once, so the box needs at least twice that many rows.  A
  // 3-D pass fuses at most two steps; the rows and planes its stored cells
  // depend on lie at most two beyond the box, which one wrap reaches for any
  // box of two or more cells per axis.
  int depth = 1;
  if (p->g.ndim == 3) {
    if (p->strang)
      depth = p->depth_limit;  // second-order groups: a capped depth, else the whole call
    else if (p->g.n[0] < kMaxRow3DFused)
      depth = std::min(p->depth_limit, max_depth3d(p->fp64));
  } else {
    depth = std::min(p->depth_limit, max_depth(p->fp64, p->strang));
    const int stages_per_step = p->strang ? 2 : 1;
    if (p->g.ndim == 2 && p->bc == DL_BC_PERIODIC)
      while (depth > 1 && p->g.n[1] < 2 * stages_per_step * depth) --depth;
  }
  p->depth = depth;
  // with a vector potential: 3-D lowest-order passes carry one step; the 3-D
  // second-order passes carry one D each and group steps as without a field
  p->depth_field = (p->g.ndim == 3) ? (p->strang ? depth : 1)
                                    : std::min(depth, field_max_depth(p->fp64, p->strang));
  for (int mode = 0; mode < 5; ++mode) {
    PlanTiling& t = p->tiling[mode];
    if (p->g.ndim == 3) {
      if (mode >= 3) {  // with a vector potential (static or pulsed): one step per pass
        make_tiling3d(p->g, p->fp64 ? kTY3D_F64 : kTY3D_F32, 64, 2, resident_waves(p, 3, 1),
                      p->seg_override, t.a[0], t.b[0], 4);
        for (int d = 0; d < kMaxDepth; ++d) t.a[d].periodic = (p->bc == DL_BC_PERIODIC);
        continue;
      }
      make_tiling3d(p->g, p->fp64 ? kTY3D_F64 : kTY3D_F32, 64, 2, resident_waves(p, mode, 1),
                    p->seg_override, t.a[0], t.b[0], 4);
      if (depth >= 2)  // workgroup tiles: resident workgroups are the target
        make_tiling3d(p->g, p->fp64 ? kTY3D2_F64 : kTY3D2_F32, strip_width(2), 4,
                      resident_waves(p, mode, 2) / 4, p->seg_override, t.a[1], t.b[1], 1);
    } else {
      for (int d = 1; d <= (mode >= 3 ? p->depth_field : depth); ++d)
        make_tiling(p->g, resident_waves(p, mode, d), p->seg_override, t.a[d - 1], t.b[d - 1],
                    strip_width(pass_xlanes(p->strang, d)));
      if (p->g.ndim == 1 && !p->strang && mode <= 2 && p->g.n[0] <= kDeep1DMaxCells) {
        make_tiling(p->g, resident_waves(p, mode, 1), p->seg_override, t.deep, t.deep_b,
                    strip_width(kDeep1D));
        t.deep.periodic = (p->bc == DL_BC_PERIODIC);
      }
    }
    for (int d = 0; d < kMaxDepth; ++d) t.a[d].periodic = (p->bc == DL_BC_PERIODIC);
  }
  select_tiling(p, 2);
  // resident 1-D path: the whole line in one workgroup (4 cells per thread)
  // for all steps of a call.  One workgroup issues every step, so it only
  // beats the tiled passes when those pay a launch for every one or two
  // steps: it is used for plans that fuse at most 2 steps per pass.
  p->resident = false;
  if (p->g.ndim == 1 && p->allow_resident && !p->strang && depth <= 2) {
    const int64_t n = p->g.n[0];
    const int64_t threads = ((n + 4 * 64 - 1) / (4 * 64)) * 64;
    if (threads <= 1024 && (p->bc == DL_BC_ZERO || threads * 4 == n)) {
      p->resident = true;
      p->res_threads = static_cast<int>(threads);
    }
  }
  return DL_OK;
}

extern "C" int dl_plan_create(dl_plan* out, const dl_grid* g, double dx, double dt, double c,
                              double m, dl_dtype dtype, dl_bc bc, unsigned flags) {
  dirac::TraceRange trace_range("dl_plan_create");
  if (!out) return fail(DL_ERR_ARG, "out is NULL");
  *out = nullptr;
  const bool strang = (flags & DL_STRANG) != 0;
  // characteristic shift per step: one cell (lowest order), two cells (the
  // half steps of the 1-D / 2-D second-order step), four cells (the quarter
  // steps of A in the 3-D second-order step)
  const int shift = strang ? ((g && g->ndim == 3) ? 4 : 2) : 1;
  int rc = validate_grid(g, dx, dt, c, m, dtype, bc, 3, shift);
  if (rc) return rc;
  if (g->ndim == 3 && !(g->axis[0] == 0 && g->axis[1] == 1 && g->axis[2] == 2))
    return fail(DL_ERR_ARG, "3-D grids carry alpha_x, alpha_y, alpha_z in order");
  const bool pair = (flags & DL_BISPINOR) != 0;
  if (pair && g->ndim != 1) return fail(DL_ERR_ARG, "two-component states are 1-D lines");
  dl_plan p = new (std::nothrow) dl_plan_s();
  if (!p) return fail(DL_ERR_NOMEM, "host allocation failed");
  p->g = *g;
  for (int d = g->ndim; d < 3; ++d) {
    p->g.n[d] = 1;
    p->g.axis[d] = -1;
    p->g.xmin[d] = 0.0;
  }
  p->dx = dx;
  p->dt = dt;
  p->c = c;
  p->m = m;
  p->dtype = dtype;
  p->bc = bc;
  p->flags = flags;
  p->fp64 = (dtype == DL_C128);
  p->cells = 1;
  for (int d = 0; d < g->ndim; ++d) p->cells *= g->n[d];
  p->nc = pair ? 2 : 4;
  p->state_bytes = static_cast<size_t>(p->cells) * p->nc * (p->fp64 ? 16 : 8);
  p->dry = (flags & DL_DRY) != 0;
  p->use_graph = (flags & DL_GRAPH) != 0;
  p->strang = strang;
  plan_tiling(p);
  if (p->dry) {
    *out = p;
    return DL_OK;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
      ncu > 0)
    p->cu_count = ncu;
  plan_tiling(p);
  const bool mid = strang && g->ndim == 3;  // the 3-D second-order step runs through a third buffer
  if (mid) dirac::strang3d_prepare(p->fp64);
  if (hipMalloc(&p->tmp, p->state_bytes) != hipSuccess ||
      (mid && hipMalloc(&p->tmp2, p->state_bytes) != hipSuccess) ||
      hipMalloc(&p->partials, sizeof(double) * 2 * 8 * kObsBlocks) != hipSuccess ||
      hipMalloc(&p->dres, sizeof(double) * 64) != hipSuccess ||
      hipHostMalloc(&p->hres, sizeof(double) * 64, hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&p->hres_dev), p->hres, 0) !=
          hipSuccess) {
    (void)hipGetLastError();
    dl_plan_destroy(p);
    return fail(DL_ERR_NOMEM, "device allocation of %zu bytes of scratch failed", p->state_bytes);
  }
  *out = p;
  return DL_OK;
}

void dl_plan_s::drop_graphs() {
  for (auto& ge : graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
  }
  graphs.clear();
}

extern "C" int dl_plan_destroy(dl_plan p) {
  if (!p) return DL_OK;
  if (p->is_batch) {
    if (!p->dry) (void)hipDeviceSynchronize();
    destroy_batch(p);
    delete p;
    return DL_OK;
  }
  if (!p->dry) {
    (void)hipDeviceSynchronize();
    p->drop_graphs();
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->tmp) (void)hipFree(p->tmp);
    if (p->tmp2) (void)hipFree(p->tmp2);
    if (p->proj) (void)hipFree(p->proj);
    if (p->partials) (void)hipFree(p->partials);
    if (p->dres) (void)hipFree(p->dres);
    if (p->hres) (void)hipHostFree(p->hres);
    if (p->tile_partials) (void)hipFree(p->tile_partials);
    if (p->alt) (void)hipFree(p->alt);
    (void)hipGetLastError();
  }
  delete p;
  return DL_OK;
}

namespace dirac {

int check_live(dl_plan p) {
  if (!p) return fail(DL_ERR_ARG, "plan is NULL");
  if (p->is_batch) return fail(DL_ERR_STATE, "a batch handle: use dl_batch_step");
  if (p->dry) return fail(DL_ERR_STATE, "dry plan: created with DL_DRY, no device work allowed");
  return DL_OK;
}

int check_state_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(DL_ERR_ARG, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(ptr) % 16) return fail(DL_ERR_ALIGN, "%s not 16-byte aligned", name);
  return DL_OK;
}

int check_f64_ptr(const void* ptr, const char* name, bool nullable) {
  if (!ptr) return nullable ? DL_OK : fail(DL_ERR_ARG, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(ptr) % 8) return fail(DL_ERR_ALIGN, "%s not 8-byte aligned", name);
  return DL_OK;
}

// one pass of `depth` fused steps src -> dst with the current phase and tiling
hipError_t launch_pass(dl_plan p, int depth, const void* src, void* dst, const double* V,
                       hipStream_t st) {
  if (p->g.ndim == 3) {
    SweepArgs a = p->sw[p->strang ? 0 : depth - 1];  // second-order passes size their own grids
    a.ph = p->ph;
    a.At = p->field;
    a.pulse = p->pulse;
    a.pulse_on = p->pulse_on ? 1 : 0;
    a.cells = p->cells;
    if (p->strang) return launch_strang3d(p->fp64, src, dst, p->tmp2, nullptr, V, a, depth, st);
    return launch_sweep3d(p->fp64, depth, src, dst, V, a, p->bl[depth - 1], st);
  }
  SweepArgs a = p->sw[depth - 1];
  a.ph = p->ph;
  a.At = p->field;
  a.pulse = p->pulse;
  a.pulse_on = p->pulse_on ? 1 : 0;
  a.cells = p->cells;
  a.nc = p->nc;
  return launch_sweep2d(p->fp64, p->strang, depth, src, dst, V, a, p->bl[depth - 1], st);
}

// the last pass of a dl_step_observables call: a lowest-order pass (2-D, or
// the two-step 3-D pass) that also leaves the observables sums of every wave
// in p->tile_partials
static hipError_t launch_pass_obs(dl_plan p, int depth, const void* src, void* dst,
                                  const double* V, const ObsArgs& o, hipStream_t st,
                                  int64_t* waves) {
  if (p->g.ndim == 3) {
    if (depth != 2) return hipErrorInvalidValue;
    SweepArgs a = p->sw[1];
    a.ph = p->ph;
    a.At = nullptr;
    a.pulse = p->pulse;
    a.pulse_on = 0;
    a.cells = p->cells;
    *waves = a.ntiles * 4;  // four waves per workgroup tile
    return launch_sweep3d_obs(p->fp64, src, dst, V, a, o, p->tile_partials, p->bl[1], st);
  }
  SweepArgs a = p->sw[depth - 1];
  a.ph = p->ph;
  a.At = nullptr;
  a.pulse = p->pulse;
  a.pulse_on = 0;
  a.cells = p->cells;
  a.nc = p->nc;
  *waves = a.ntiles;
  return launch_sweep2d_obs(p->fp64, depth, src, dst, V, a, o, p->tile_partials,
                            p->bl[depth - 1], st);
}

// 1-D lines of lowest-order steps without a vector potential (and no cap on
// the depth) run passes of kDeep1D steps first
static bool deep1d(dl_plan p) {
  return p->g.ndim == 1 && !p->strang && p->ph.mode <= 2 && p->depth_limit >= kMaxDepth &&
         p->bl_deep > 0;
}

// one pass of kDeep1D steps src -> dst on a 1-D line
static hipError_t launch_pass_deep(dl_plan p, const void* src, void* dst, const double* V,
                                   hipStream_t st) {
  SweepArgs a = p->sw_deep;
  a.ph = p->ph;
  a.At = nullptr;
  a.pulse = p->pulse;
  a.pulse_on = 0;
  a.cells = p->cells;
  a.nc = p->nc;
  return launch_sweep1d_deep(p->fp64, src, dst, V, a, p->bl_deep, st);
}

// passes of `nsteps` steps at the plan's current depth (deepest first)
static int64_t pass_count(dl_plan p, int64_t nsteps) {
  const int dmax = (p->ph.mode >= 3) ? p->depth_field : p->depth;
  int64_t n = 0, left = nsteps;
  if (deep1d(p)) {
    n += left / kDeep1D;
    left %= kDeep1D;
  }
  for (int d = dmax; d >= 1; --d) {
    n += left / d;
    left %= d;
  }
  return n;
}

// The plan's third state buffer: with it, an odd number (>= 3) of passes
// ends in psi (psi -> tmp -> alt -> tmp ... -> psi) instead of in tmp with a
// copy back.  Allocated once, by the first call that needs it, and never
// while the stream is being captured; without it the copy stays.
static void want_alt(dl_plan p, int64_t nsteps, hipStream_t st) {
  if (p->alt || p->alt_failed) return;
  if (p->g.ndim == 3 && p->strang) return;  // second-order 3-D groups end in psi by themselves
  const int64_t n = pass_count(p, nsteps);
  if (n < 3 || n % 2 == 0) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return;
  }
  if (hipMalloc(&p->alt, p->state_bytes) != hipSuccess) {
    (void)hipGetLastError();
    p->alt = nullptr;
    p->alt_failed = true;
  }
}

// enqueue `nsteps` steps starting from psi, in passes of the plan's depth
// (the remainder in shallower passes), alternating between psi and the plan's
// tmp buffer, or, for an odd number (>= 3) of passes when the plan holds its
// third buffer, through tmp and that buffer so that the last pass writes psi;
// returns the buffer that holds the result.  With `obs`, the last pass also
// sums the observables (launch_pass_obs; `obs_waves` receives the number of
// partials it writes).
hipError_t enqueue_steps(dl_plan p, void* psi, const double* V, int64_t nsteps, hipStream_t st,
                         void** result, const ObsArgs* obs = nullptr,
                         int64_t* obs_waves = nullptr) {
  if (p->g.ndim == 3 && p->strang && p->depth_limit >= kMaxDepth && nsteps > 0 && !obs) {
    // second-order 3-D steps: the whole call is one group, nsteps + 1 passes
    // in place through the plan's two scratch states (a cap on the depth
    // keeps groups of that many steps instead)
    SweepArgs a = p->sw[0];
    a.ph = p->ph;
    a.At = p->field;
    a.pulse = p->pulse;
    a.pulse_on = p->pulse_on ? 1 : 0;
    a.cells = p->cells;
    hipError_t e = launch_strang3d(p->fp64, psi, psi, p->tmp2, p->tmp, V, a, nsteps, st);
    if (e != hipSuccess) return e;
    p->pulse.n0 += nsteps;
    *result = psi;
    return hipSuccess;
  }
  want_alt(p, nsteps, st);
  const int64_t passes = pass_count(p, nsteps);
  void* third = (passes >= 3 && passes % 2 == 1) ? p->alt : nullptr;
  void* in = psi;
  int64_t i = 0, left = nsteps;
  if (obs && p->g.ndim == 3 && p->depth == 2 && left % 2 == 1 && left > 1) {
    // the single step first, so that the last pass is a two-step one, the
    // pass that sums the observables
    void* out = third ? ((i == passes - 1) ? psi : (i % 2 == 0 ? p->tmp : third))
                      : (in == psi ? p->tmp : psi);
    hipError_t e = launch_pass(p, 1, in, out, V, st);
    if (e != hipSuccess) return e;
    p->pulse.n0 += 1;
    in = out;
    ++i;
    --left;
  }
  if (deep1d(p)) {
    for (; left >= kDeep1D; left -= kDeep1D, ++i) {
      void* out = third ? ((i == passes - 1) ? psi : (i % 2 == 0 ? p->tmp : third))
                        : (in == psi ? p->tmp : psi);
      hipError_t e = launch_pass_deep(p, in, out, V, st);
      if (e != hipSuccess) return e;
      p->pulse.n0 += kDeep1D;
      in = out;
    }
  }
  const int dmax = (p->ph.mode >= 3) ? p->depth_field : p->depth;
  for (int d = dmax; d >= 1; --d) {
    for (; left >= d; left -= d, ++i) {
      void* out = third ? ((i == passes - 1) ? psi : (i % 2 == 0 ? p->tmp : third))
                        : (in == psi ? p->tmp : psi);
      hipError_t e = (obs && left == d) ? launch_pass_obs(p, d, in, out, V, *obs, st, obs_waves)
                                        : launch_pass(p, d, in, out, V, st);
      if (e != hipSuccess) return e;
      p->pulse.n0 += d;  // the pulse's step index of the next pass
      in = out;
    }
  }
  *result = in;
  return hipSuccess;
}

}  // namespace dirac

// dst = src for n 16-byte words: a plain kernel rather than a copy node, so a
// captured graph holds kernels only
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

static hipError_t graph_for(dl_plan p, void* psi, const double* V, int64_t pairs,
                            hipGraphExec_t* exec) {
  for (auto& ge : p->graphs) {
    if (ge.psi == psi && ge.V == V && ge.pairs == pairs && ge.mode == p->ph.mode) {
      *exec = ge.exec;
      return hipSuccess;
    }
  }
  if (!p->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  want_alt(p, 2 * pairs, p->cap_stream);  // before the capture begins
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  void* res = nullptr;
  hipError_t e2 = enqueue_steps(p, psi, V, 2 * pairs, p->cap_stream, &res);
  if (e2 == hipSuccess && res != psi) {
    // an odd number of passes ends in the plan's buffer: every replay must
    // leave the state in psi, where the next one starts
    const int64_t words = static_cast<int64_t>(p->state_bytes / 16);
    const int64_t blocks = std::min<int64_t>((words + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       p->cap_stream, static_cast<const uint4*>(res), static_cast<uint4*>(psi),
                       words);
    e2 = hipGetLastError();
  }
  e = hipStreamEndCapture(p->cap_stream, &graph);
  if (e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return e2;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if (p->graphs.size() >= 8) p->drop_graphs();
  p->graphs.push_back(GraphEntry{psi, V, pairs, p->ph.mode, ex});
  *exec = ex;
  return hipSuccess;
}

extern "C" int dl_step(dl_plan p, void* psi, const double* V, int64_t nsteps, void* stream) {
  dirac::TraceRange trace_range("dl_step");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  if (nsteps < 0) return fail(DL_ERR_ARG, "nsteps = %lld < 0", static_cast<long long>(nsteps));
  if (nsteps == 0) return DL_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int mode = phase_mode(p->m, V);
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, mode, p->fp64);
  p->field = nullptr;
  select_tiling(p, mode);
  if (p->resident) {
    ResidentArgs ra{};
    ra.n = p->g.n[0];
    ra.nsteps = nsteps;
    ra.periodic = (p->bc == DL_BC_PERIODIC);
    ra.ph = p->ph;
    ra.nc = p->nc;
    hipError_t e = launch_resident1d(p->fp64, p->g.axis[0], psi, V, ra, 4, p->res_threads, st);
    return e == hipSuccess ? DL_OK : hip_fail(e, "resident 1-D sweep launch");
  }
  int64_t done = 0;
  if (p->use_graph && nsteps >= 2 * p->graph_pairs) {
    hipGraphExec_t ex = nullptr;
    hipError_t e = graph_for(p, psi, V, p->graph_pairs, &ex);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    const int64_t reps = nsteps / (2 * p->graph_pairs);
    for (int64_t r = 0; r < reps; ++r) {
      e = hipGraphLaunch(ex, st);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    done = reps * 2 * p->graph_pairs;
  }
  void* res = nullptr;
  hipError_t e = enqueue_steps(p, psi, V, nsteps - done, st, &res);
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  if (res != psi) {
    e = hipMemcpyAsync(psi, res, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return DL_OK;
}

extern "C" int dl_step_field(dl_plan p, void* psi, const double* V, const double* A,
                             int64_t nsteps, void* stream) {
  dirac::TraceRange trace_range("dl_step_field");
  int rc = check_live(p);
  if (rc) return rc;
  if (!A) return dl_step(p, psi, V, nsteps, stream);
  if ((rc = check_state_ptr(psi, "psi"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  if ((rc = check_f64_ptr(A, "A", false))) return rc;
  if (p->nc != 4) return fail(DL_ERR_ARG, "a vector potential couples all four components");
  if (nsteps < 0) return fail(DL_ERR_ARG, "nsteps = %lld < 0", static_cast<long long>(nsteps));
  if (nsteps == 0) return DL_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, 3, p->fp64);
  p->field = A;
  select_tiling(p, 3);
  void* res = nullptr;
  hipError_t e = enqueue_steps(p, psi, V, nsteps, st, &res);
  p->field = nullptr;
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  if (res != psi) {
    e = hipMemcpyAsync(psi, res, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return DL_OK;
}

extern "C" int dl_step_pulse(dl_plan p, void* psi, const double* V, const double* P,
                             const dl_pulse* pulse, double t0, int64_t nsteps, void* stream) {
  dirac::TraceRange trace_range("dl_step_pulse");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  if ((rc = check_f64_ptr(P, "P", false))) return rc;
  if (!pulse) return fail(DL_ERR_ARG, "pulse is NULL");
  const double pv[5] = {pulse->omega, pulse->phase, pulse->t_on, pulse->t_flat, pulse->t_off};
  for (double v : pv)
    if (!std::isfinite(v)) return fail(DL_ERR_ARG, "pulse parameters must be finite");
  if (pulse->t_on < 0.0 || pulse->t_flat < 0.0 || pulse->t_off < 0.0)
    return fail(DL_ERR_ARG, "pulse durations must be >= 0");
  if (!std::isfinite(t0)) return fail(DL_ERR_ARG, "t0 must be finite");
  if (p->nc != 4) return fail(DL_ERR_ARG, "a vector potential couples all four components");
  if (nsteps < 0) return fail(DL_ERR_ARG, "nsteps = %lld < 0", static_cast<long long>(nsteps));
  if (nsteps == 0) return DL_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // 1-D / 2-D: phase mode 4 forms each step's field integral in the pass; 3-D
  // passes (one D each) run the static-field kernels with At = F P
  const int mode = (p->g.ndim == 3) ? 3 : 4;
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, mode, p->fp64);
  p->field = P;
  p->pulse = PulseK{pulse->omega, pulse->phase, pulse->t_on, pulse->t_flat, pulse->t_off,
                    t0, p->dt, 0};
  p->pulse_on = true;
  select_tiling(p, mode);
  void* res = nullptr;
  hipError_t e = enqueue_steps(p, psi, V, nsteps, st, &res);
  p->field = nullptr;
  p->pulse_on = false;
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  if (res != psi) {
    e = hipMemcpyAsync(psi, res, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return DL_OK;
}

extern "C" int dl_step_out(dl_plan p, const void* src, void* dst, const double* V,
                           void* stream) {
  dirac::TraceRange trace_range("dl_step_out");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(src, "src"))) return rc;
  if ((rc = check_state_ptr(dst, "dst"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + p->state_bytes && b < a + p->state_bytes)
    return fail(DL_ERR_ARG, "src and dst overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, phase_mode(p->m, V), p->fp64);
  p->field = nullptr;
  select_tiling(p, p->ph.mode);
  hipError_t e = launch_pass(p, 1, src, dst, V, st);
  return e == hipSuccess ? DL_OK : hip_fail(e, "sweep launch");
}

extern "C" int dl_step_fused_out(dl_plan p, const void* src, void* dst, const double* V,
                                 int64_t nsteps, void* stream) {
  dirac::TraceRange trace_range("dl_step_fused_out");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(src, "src"))) return rc;
  if ((rc = check_state_ptr(dst, "dst"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  if (nsteps < 1) return fail(DL_ERR_ARG, "nsteps = %lld < 1", static_cast<long long>(nsteps));
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + p->state_bytes && b < a + p->state_bytes)
    return fail(DL_ERR_ARG, "src and dst overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, phase_mode(p->m, V), p->fp64);
  p->field = nullptr;
  select_tiling(p, p->ph.mode);
  // passes deepest first; they alternate between dst and the plan's buffer
  // so that the last one writes dst
  int64_t passes = 0;
  {
    int64_t left = nsteps;
    for (int d = p->depth; d >= 1; --d) {
      passes += left / d;
      left %= d;
    }
  }
  const void* in = src;
  int64_t i = 0, left = nsteps;
  for (int d = p->depth; d >= 1; --d) {
    for (; left >= d; left -= d, ++i) {
      void* out = ((passes - 1 - i) % 2 == 0) ? dst : p->tmp;
      hipError_t e = launch_pass(p, d, in, out, V, st);
      if (e != hipSuccess) return hip_fail(e, "sweep launch");
      in = out;
    }
  }
  return DL_OK;
}

// status of an observables result: a non-finite sum means a non-finite cell
// (|psi|^2 of finite FP32 / FP64 values cannot overflow a double sum of fewer
// than 2^40 cells); then the norm watchdog
static int observables_status(dl_plan p, const double* out) {
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(out[i]))
      return fail(DL_ERR_NONFINITE, "the state holds a NaN or an infinity (observable %d = %g)",
                  i, out[i]);
  if (p->norm_tol > 0.0) {
    const double N = out[0], hi = p->norm_ref * (1.0 + p->norm_tol),
                 lo = p->norm_ref * (1.0 - p->norm_tol);
    if (N > hi)
      return fail(DL_WARN_NORM, "norm %.17g exceeds the reference %.17g by more than %g", N,
                  p->norm_ref, p->norm_tol);
    if (p->bc == DL_BC_PERIODIC && N < lo)
      return fail(DL_WARN_NORM, "norm %.17g fell below the reference %.17g by more than %g "
                  "on a periodic box", N, p->norm_ref, p->norm_tol);
  }
  return DL_OK;
}

static ObsArgs obs_args(dl_plan p, double x_b) {
  ObsArgs a{};
  a.n0 = p->g.n[0];
  a.n1 = p->g.n[1];
  a.n2 = p->g.n[2];
  a.ndim = p->g.ndim;
  a.dx = p->dx;
  a.xmin0 = p->g.xmin[0];
  a.xmin1 = p->g.xmin[1];
  a.xmin2 = p->g.xmin[2];
  a.x_b = x_b;
  a.nc = p->nc;
  return a;
}

// wait for the final reduction, which wrote the five values straight into
// the plan's mapped pinned buffer (no copy back), and check them
static int finish_observables(dl_plan p, hipStream_t st, double out[5]) {
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int i = 0; i < 5; ++i) out[i] = p->hres[i];
  return observables_status(p, out);
}

extern "C" int dl_observables(dl_plan p, const void* psi, double x_b, double out[5],
                              void* stream) {
  dirac::TraceRange trace_range("dl_observables");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi"))) return rc;
  if (!out) return fail(DL_ERR_ARG, "out is NULL");
  if (!std::isfinite(x_b) && !std::isinf(x_b)) return fail(DL_ERR_ARG, "x_b is NaN");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_observables(p->fp64, psi, obs_args(p, x_b), p->partials, p->hres_dev, st);
  if (e != hipSuccess) return hip_fail(e, "observables launch");
  return finish_observables(p, st, out);
}

extern "C" int dl_step_observables(dl_plan p, void* psi, const double* V, int64_t nsteps,
                                   double x_b, double out[5], void* stream) {
  dirac::TraceRange trace_range("dl_step_observables");
  int rc = check_live(p);
  if (rc) return rc;
  if ((rc = check_state_ptr(psi, "psi"))) return rc;
  if ((rc = check_f64_ptr(V, "V", true))) return rc;
  if (nsteps < 0) return fail(DL_ERR_ARG, "nsteps = %lld < 0", static_cast<long long>(nsteps));
  if (!out) return fail(DL_ERR_ARG, "out is NULL");
  if (std::isnan(x_b)) return fail(DL_ERR_ARG, "x_b is NaN");
  const int mode = phase_mode(p->m, V);
  // the fused last pass exists for 2-D lowest-order plans of four-component
  // states on grid axes (x, y) and for 3-D lowest-order plans of two-step
  // passes (then at least two steps); every other plan steps, then reduces
  const bool fused2 = nsteps > 0 && p->g.ndim == 2 && !p->strang && p->nc == 4 &&
                      axes_code(p->g) == 10 && mode <= 2;
  const bool fused3 = nsteps > 1 && p->g.ndim == 3 && !p->strang && p->depth == 2 && mode <= 2;
  const bool fused = fused2 || fused3;
  if (!fused) {
    rc = dl_step(p, psi, V, nsteps, stream);
    if (rc) return rc;
    return dl_observables(p, psi, x_b, out, stream);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  p->ph = make_phase(transports_per_step(p), p->dt, p->c, p->m, mode, p->fp64);
  p->field = nullptr;
  select_tiling(p, mode);
  if (fused2)
    for (int d = 1; d <= p->depth; ++d)
      if (!sweep2d_obs_available(p->fp64, d, mode))
        return fail(DL_ERR_STATE, "no fused observables pass of depth %d", d);
  int64_t need = 0;
  if (fused3)
    need = p->sw[1].ntiles * 4;
  else
    for (int d = 1; d <= p->depth; ++d) need = std::max<int64_t>(need, p->sw[d - 1].ntiles);
  if (need > p->tile_partials_n) {
    if (p->tile_partials) (void)hipFree(p->tile_partials);
    p->tile_partials = nullptr;
    p->tile_partials_n = 0;
    hipError_t e = hipMalloc(&p->tile_partials, sizeof(double) * kObsDoubles * need);
    if (e != hipSuccess) {
      p->tile_partials = nullptr;
      return hip_fail(e, "hipMalloc (observables partials)");
    }
    p->tile_partials_n = need;
  }
  // whole graphs for all but the steps of the fused pass (at least one step,
  // two on 3-D grids)
  int64_t done = 0;
  const int64_t keep = fused3 ? 2 : 1;
  if (p->use_graph && nsteps - keep >= 2 * p->graph_pairs) {
    hipGraphExec_t ex = nullptr;
    hipError_t e = graph_for(p, psi, V, p->graph_pairs, &ex);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    const int64_t reps = (nsteps - keep) / (2 * p->graph_pairs);
    for (int64_t r = 0; r < reps; ++r) {
      e = hipGraphLaunch(ex, st);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    done = reps * 2 * p->graph_pairs;
  }
  const ObsArgs o = obs_args(p, x_b);
  void* res = nullptr;
  int64_t waves = 0;
  hipError_t e = enqueue_steps(p, psi, V, nsteps - done, st, &res, &o, &waves);
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  if (res != psi) {
    e = hipMemcpyAsync(psi, res, p->state_bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  e = launch_obs_final(p->tile_partials, waves, o, p->hres_dev, st);
  if (e != hipSuccess) return hip_fail(e, "observables launch");
  return finish_observables(p, st, out);
}

extern "C" int dl_plan_set_norm_check(dl_plan p, double N_ref, double tol) {
  if (!p) return fail(DL_ERR_ARG, "plan is NULL");
  if (p->is_batch) return fail(DL_ERR_STATE, "a batch handle has no observables");
  if (!finite_pos(N_ref) || !std::isfinite(tol) || tol < 0.0)
    return fail(DL_ERR_ARG, "need N_ref > 0 and tol >= 0, both finite");
  p->norm_ref = N_ref;
  p->norm_tol = tol;
  return DL_OK;
}

extern "C" const char* dl_last_error(void) { return g_err; }
extern "C" int dl_version(void) { return LIBDIRAC_VERSION; }

// ---- tuning: tiling, fusion depth, plan description ----
extern "C" int dl_plan_set_tiling(dl_plan p, int waves_per_cu, int seg_len, int allow_resident,
                                  int graph_pairs) {
  if (!p) return fail(DL_ERR_ARG, "plan is NULL");
  if (waves_per_cu < 0 || waves_per_cu > 32) return fail(DL_ERR_ARG, "waves_per_cu out of range");
  if (seg_len < 0 || graph_pairs < 1) return fail(DL_ERR_ARG, "bad seg_len / graph_pairs");
  p->waves_per_cu = waves_per_cu;
  p->seg_override = seg_len;
  p->allow_resident = allow_resident != 0;
  p->graph_pairs = graph_pairs;
  if (!p->dry) p->drop_graphs();
  return plan_tiling(p);
}

extern "C" int dl_plan_set_depth(dl_plan p, int depth) {
  if (!p) return fail(DL_ERR_ARG, "plan is NULL");
  if (depth < 1 || depth > kMaxDepth) return fail(DL_ERR_ARG, "depth %d not in 1..%d", depth, kMaxDepth);
  p->depth_limit = depth;
  if (!p->dry) p->drop_graphs();
  return plan_tiling(p);
}

extern "C" int dl_plan_info(dl_plan p, int64_t* info, int n) {
  if (!p || !info) return fail(DL_ERR_ARG, "NULL argument");
  if (p->is_batch) {
    batch_info(p, info, n);
    return DL_OK;
  }
  const SweepArgs& t = p->sw[p->depth - 1];  // tiling of the deepest pass in use
  const int64_t vals[] = {p->bl[p->depth - 1], t.H,          t.nseg,         t.nstrips,
                          t.ntiles,            p->resident,  p->res_threads, p->waves_per_cu,
                          t.xcd_remap,         p->graph_pairs, p->depth,     p->bl[0],
                          reverse_depth(p),    p->depth_field,
                          (p->g.ndim == 1 && !p->strang && p->depth_limit >= kMaxDepth &&
                           p->bl_deep > 0) ? kDeep1D : 0};
  const int nv = static_cast<int>(sizeof vals / sizeof vals[0]);
  for (int i = 0; i < n && i < nv; ++i) info[i] = vals[i];
  return DL_OK;
}
