// dirac_batch.hip -- many independent 1-D / 2-D instances advanced together.
//
// One launch performs one pass of D fused steps (then, for the remainder of
// each instance's count, single steps) of every active instance: the grid is
// a flat table of tiles (instance, strip of 64 - 2D cells, march segment),
// ordered longest first (2-D segments of H rows before single 1-D rows) so
// that the workgroup dispatcher's in-order assignment is a
// longest-processing-time list schedule.  Each tile runs exactly the per-cell
// code of the single-plan sweep (x transport / y march / local step, the
// phase mode read at run time), so every instance ends bit-identical to
// dl_step on its own plan.  Consecutive passes are ordered by the launch
// boundary (no cross-workgroup waits inside a kernel); long runs are replayed
// from a captured hipGraph.  The segment length is chosen by timing
// candidates on the batch itself (dl_batch_autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dirac_plan.h"
#include "dirac_sweep_impl.h"

namespace dirac {

struct BatchInst {
  void* a;            // caller's state (set per call)
  void* b;            // batch-owned second buffer
  const double* V;    // per call
  int64_t nx, ny;
  int64_t nsteps;     // per call
  int64_t passes;     // per call: passes of the batch's depth ...
  int64_t rem;        // ... then this many single steps
  int periodic;
  int axes_code;
  PhaseK ph;          // per call (mode depends on V)
};

struct BatchTile {
  int inst;
  int strip;
  int jb, je;         // 2-D: rows [jb, je); 1-D: 0, 1
  int up;             // march direction (alternates between segments)
};

// One launch advances every instance still due by one pass of K steps.
// phase 0: the index-th pass of the batch's depth D = K (instances with more
// passes skip); phase 1: the index-th single step (K = 1) of the remainder.
// Tiles are strips of 64 - 2D columns (lanes D .. 63 - D are written), valid
// for every K <= D.  An instance's buffers alternate with the passes it has
// done, so its parity is computed here from its own counts.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_batch(const BatchInst* __restrict__ insts,
                                               const BatchTile* __restrict__ tiles, int ntiles,
                                               int phase, int64_t index, int depth) {
  const int lane = threadIdx.x & 63;
  const int tile = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x) * 4 +
                                                  static_cast<int>(threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const BatchTile t = tiles[tile];
  const BatchInst& I = insts[t.inst];
  int64_t done;  // passes this instance has completed before this launch
  if (phase == 0) {
    if (index >= I.passes) return;
    done = index;
  } else {
    if (index >= I.rem) return;
    done = I.passes + index;
  }
  const int parity = static_cast<int>(done & 1);
  const T* src = static_cast<const T*>(parity ? I.b : I.a);
  T* dst = static_cast<T*>(parity ? I.a : I.b);
  SweepArgs a{};
  a.nx = I.nx;
  a.ny = I.ny;
  a.nz = 1;
  a.periodic = I.periodic;
  a.ph = I.ph;
  const int64_t xs = static_cast<int64_t>(t.strip) * strip_width(depth) - depth;
  const bool up = t.up != 0;
  switch (I.axes_code) {
    case 0: one_row<T, LieStep, K, 0, -1>(src, dst, I.V, a, xs, lane, depth); break;
    case 1: one_row<T, LieStep, K, 1, -1>(src, dst, I.V, a, xs, lane, depth); break;
    case 2: one_row<T, LieStep, K, 2, -1>(src, dst, I.V, a, xs, lane, depth); break;
    case 10:
      march_dir<T, LieStep, K, 0, 1, -1>(src, dst, I.V, a, xs, lane, t.jb, t.je, up, depth);
      break;
    case 20:
      march_dir<T, LieStep, K, 0, 2, -1>(src, dst, I.V, a, xs, lane, t.jb, t.je, up, depth);
      break;
    case 21:
      march_dir<T, LieStep, K, 1, 2, -1>(src, dst, I.V, a, xs, lane, t.jb, t.je, up, depth);
      break;
    default: break;
  }
}

// depth of the batch's passes (steps fused per launch); a periodic batch
// lowers it until every 2-D instance has at least 2 * depth rows
constexpr int kBatchDepthF32 = 5;
constexpr int kBatchDepthF64 = 5;  // passes of 3 or more run one wave per SIMD

}  // namespace dirac

using namespace dirac;

namespace {

struct Batch {
  std::vector<dl_grid> grids;
  std::vector<double> dx, dt, c, m;
  int count = 0;
  bool fp64 = false;
  int bc = DL_BC_ZERO;
  bool use_graph = true;
  int seg_len = 32;                 // 2-D march segment length (autotuned)
  int depth = 1;                    // steps fused per pass
  int64_t graph_pairs = 16;
  std::vector<size_t> bytes;        // state bytes per instance
  void* scratch = nullptr;          // second buffers of all instances
  BatchInst* d_insts = nullptr;
  BatchTile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  int ntiles = 0;
  std::vector<BatchInst> h_insts;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_seg = -1;
  int graph_tiles = -1;
};

Batch* as_batch(dl_plan p) { return static_cast<Batch*>(p->batch); }

int64_t segs_of(int64_t ny, int H, int64_t* Hout) {
  int64_t h = std::min<int64_t>(H, ny);
  if (h < 1) h = 1;
  *Hout = h;
  return (ny + h - 1) / h;
}

// tile table, 2-D segments first (longest first), 1-D rows last
std::vector<BatchTile> make_tiles(const Batch& B) {
  std::vector<BatchTile> two, one;
  for (int k = 0; k < B.count; ++k) {
    const dl_grid& g = B.grids[k];
    const int64_t nstrips = (g.n[0] + strip_width(B.depth) - 1) / strip_width(B.depth);
    if (g.ndim == 1) {
      for (int64_t s = 0; s < nstrips; ++s)
        one.push_back(BatchTile{k, static_cast<int>(s), 0, 1, 1});
    } else {
      int64_t H;
      const int64_t nseg = segs_of(g.n[1], B.seg_len, &H);
      for (int64_t q = 0; q < nseg; ++q) {
        const int64_t jb = q * H;
        const int64_t je = std::min<int64_t>(jb + H, g.n[1]);
        for (int64_t s = 0; s < nstrips; ++s)
          two.push_back(BatchTile{k, static_cast<int>(s), static_cast<int>(jb),
                                  static_cast<int>(je), (q & 1) == 0 ? 1 : 0});
      }
    }
  }
  std::stable_sort(two.begin(), two.end(), [](const BatchTile& x, const BatchTile& y) {
    return (x.je - x.jb) > (y.je - y.jb);
  });
  two.insert(two.end(), one.begin(), one.end());
  return two;
}

int upload_tiles(Batch& B) {
  std::vector<BatchTile> t = make_tiles(B);
  if (t.size() > B.tiles_cap) {
    if (B.d_tiles) (void)hipFree(B.d_tiles);
    B.d_tiles = nullptr;
    if (hipMalloc(&B.d_tiles, t.size() * sizeof(BatchTile)) != hipSuccess) {
      (void)hipGetLastError();
      B.tiles_cap = 0;
      return set_error(DL_ERR_NOMEM, "tile table allocation failed");
    }
    B.tiles_cap = t.size();
  }
  hipError_t e = hipMemcpy(B.d_tiles, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e != hipSuccess) return set_hip_error(e, "tile table upload");
  B.ntiles = static_cast<int>(t.size());
  return DL_OK;
}

void drop_graph(Batch& B) {
  if (B.graph) (void)hipGraphExecDestroy(B.graph);
  B.graph = nullptr;
  B.graph_seg = -1;
  B.graph_tiles = -1;
}

template <typename T, int K>
static void launch_k(const Batch& B, int phase, int64_t index, hipStream_t st) {
  hipLaunchKernelGGL((k_batch<T, K>), dim3((B.ntiles + 3) / 4), dim3(256), 0, st, B.d_insts,
                     B.d_tiles, B.ntiles, phase, index, B.depth);
}

template <typename T>
hipError_t launch_pass_t(const Batch& B, int K, int phase, int64_t index, hipStream_t st) {
  if (K < 1 || K > (sizeof(T) == 8 ? kBatchDepthF64 : kBatchDepthF32)) return hipErrorInvalidValue;
  switch (K) {
    case 1: launch_k<T, 1>(B, phase, index, st); break;
    case 2: launch_k<T, 2>(B, phase, index, st); break;
    case 3: launch_k<T, 3>(B, phase, index, st); break;
    case 4: launch_k<T, 4>(B, phase, index, st); break;
    case 5: launch_k<T, 5>(B, phase, index, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// phase 0: the index-th pass of the batch's depth; phase 1: the index-th
// single step of the remainder
hipError_t launch_pass(const Batch& B, int phase, int64_t index, hipStream_t st) {
  const int K = phase == 0 ? B.depth : 1;
  return B.fp64 ? launch_pass_t<double>(B, K, phase, index, st)
                : launch_pass_t<float>(B, K, phase, index, st);
}

// fill per-call descriptors (pointers, step counts, phase mode) and upload
int prepare(Batch& B, void* const* psi, const double* const* V, const int64_t* nsteps,
            hipStream_t st) {
  // the previous upload from h_insts must have completed before it is rewritten
  hipError_t es = hipStreamSynchronize(st);
  if (es != hipSuccess) return set_hip_error(es, "hipStreamSynchronize");
  for (int k = 0; k < B.count; ++k) {
    BatchInst& I = B.h_insts[k];
    I.a = psi[k];
    I.V = V ? V[k] : nullptr;
    I.nsteps = nsteps[k];
    I.passes = nsteps[k] / B.depth;
    I.rem = nsteps[k] % B.depth;
    I.ph = make_phase(B.grids[k].ndim, B.dt[k], B.c[k], B.m[k], phase_mode(B.m[k], I.V), B.fp64);
  }
  hipError_t e = hipMemcpyAsync(B.d_insts, B.h_insts.data(), B.count * sizeof(BatchInst),
                                hipMemcpyHostToDevice, st);
  return e == hipSuccess ? DL_OK : set_hip_error(e, "descriptor upload");
}

// run every instance's passes of the batch's depth, then its remaining
// single steps; the kernel skips instances whose count is reached
int run(Batch& B, const int64_t* nsteps, hipStream_t st) {
  int64_t pmax = 0, pmin = INT64_MAX, rmax = 0;
  for (int k = 0; k < B.count; ++k) {
    pmax = std::max(pmax, nsteps[k] / B.depth);
    pmin = std::min(pmin, nsteps[k] / B.depth);
    rmax = std::max(rmax, nsteps[k] % B.depth);
  }
  int64_t q = 0;
  // passes [0, pmin) have every instance active: replay a graph of 2*pairs passes
  if (B.use_graph && pmin >= 2 * B.graph_pairs) {
    // the launches read pointers and counts from the device descriptor table,
    // so one captured graph serves every call with the same tile table
    if (!B.graph || B.graph_seg != B.seg_len || B.graph_tiles != B.ntiles) {
      drop_graph(B);
      if (!B.cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return set_hip_error(e, "stream create");
      }
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return set_hip_error(e, "begin capture");
      hipError_t e2 = hipSuccess;
      // pass indices 0 .. 2*pairs-1: the parity of an all-active pass is its index's
      for (int64_t i = 0; i < 2 * B.graph_pairs && e2 == hipSuccess; ++i)
        e2 = launch_pass(B, 0, i, B.cap_stream);
      e = hipStreamEndCapture(B.cap_stream, &g);
      if (e2 != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_hip_error(e2 != hipSuccess ? e2 : e, "batch graph capture");
      }
      e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return set_hip_error(e, "graph instantiate");
      B.graph_seg = B.seg_len;
      B.graph_tiles = B.ntiles;
    }
    const int64_t reps = pmin / (2 * B.graph_pairs);
    for (int64_t r = 0; r < reps; ++r) {
      hipError_t e = hipGraphLaunch(B.graph, st);
      if (e != hipSuccess) return set_hip_error(e, "graph launch");
    }
    q = reps * 2 * B.graph_pairs;
  }
  for (; q < pmax; ++q) {
    hipError_t e = launch_pass(B, 0, q, st);
    if (e != hipSuccess) return set_hip_error(e, "batch pass launch");
  }
  for (int64_t r = 0; r < rmax; ++r) {
    hipError_t e = launch_pass(B, 1, r, st);
    if (e != hipSuccess) return set_hip_error(e, "batch step launch");
  }
  // an odd number of passes ends in the second buffer
  for (int k = 0; k < B.count; ++k) {
    if ((nsteps[k] / B.depth + nsteps[k] % B.depth) & 1) {
      hipError_t e = hipMemcpyAsync(B.h_insts[k].a, B.h_insts[k].b, B.bytes[k],
                                    hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return set_hip_error(e, "hipMemcpyAsync");
    }
  }
  return DL_OK;
}

void free_batch(Batch* B) {
  if (!B) return;
  drop_graph(*B);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->scratch) (void)hipFree(B->scratch);
  if (B->d_insts) (void)hipFree(B->d_insts);
  if (B->d_tiles) (void)hipFree(B->d_tiles);
  (void)hipGetLastError();
  delete B;
}

}  // namespace

int dirac::batch_depth(dl_plan b) { return as_batch(b)->depth; }

namespace dirac {
void destroy_batch(dl_plan p) {
  free_batch(as_batch(p));
  p->batch = nullptr;
}
}  // namespace dirac

extern "C" int dl_batch_create(dl_plan* out, const dl_grid* grids, const double* dx,
                               const double* dt, const double* c, const double* m, int count,
                               dl_dtype dtype, dl_bc bc, unsigned flags) {
  if (!out) return set_error(DL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!grids || !dx || !dt || !c || !m) return set_error(DL_ERR_ARG, "NULL parameter array");
  if (count < 1 || count > (1 << 20)) return set_error(DL_ERR_ARG, "count out of range");
  for (int k = 0; k < count; ++k) {
    int rc = validate_grid(&grids[k], dx[k], dt[k], c[k], m[k], dtype, bc, 2, 1);
    if (rc) return rc;
    if (grids[k].n[0] > (int64_t(1) << 30) || (grids[k].ndim > 1 && grids[k].n[1] > (1 << 30)))
      return set_error(DL_ERR_ARG, "instance too large for a batch");
  }
  dl_plan p = new (std::nothrow) dl_plan_s();
  Batch* B = new (std::nothrow) Batch();
  if (!p || !B) {
    delete p;
    delete B;
    return set_error(DL_ERR_NOMEM, "host allocation failed");
  }
  p->is_batch = true;
  p->batch = B;
  p->dtype = dtype;
  p->bc = bc;
  p->fp64 = (dtype == DL_C128);
  p->dry = (flags & DL_DRY) != 0;
  B->depth = p->fp64 ? kBatchDepthF64 : kBatchDepthF32;
  if (bc == DL_BC_PERIODIC)
    for (int k = 0; k < count; ++k)
      while (grids[k].ndim == 2 && B->depth > 1 && grids[k].n[1] < 2 * B->depth) --B->depth;
  B->count = count;
  B->fp64 = p->fp64;
  B->bc = bc;
  B->use_graph = (flags & DL_GRAPH) != 0;
  B->grids.assign(grids, grids + count);
  B->dx.assign(dx, dx + count);
  B->dt.assign(dt, dt + count);
  B->c.assign(c, c + count);
  B->m.assign(m, m + count);
  B->h_insts.resize(count);
  size_t total = 0;
  for (int k = 0; k < count; ++k) {
    int64_t cells = grids[k].n[0] * (grids[k].ndim > 1 ? grids[k].n[1] : 1);
    B->bytes.push_back(static_cast<size_t>(cells) * 4 * (p->fp64 ? 16 : 8));
    total += (B->bytes.back() + 255) / 256 * 256;
  }
  if (p->dry) {
    *out = p;
    return DL_OK;
  }
  if (hipMalloc(&B->scratch, total) != hipSuccess ||
      hipMalloc(&B->d_insts, count * sizeof(BatchInst)) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(B);
    delete p;
    return set_error(DL_ERR_NOMEM, "batch scratch allocation failed");
  }
  size_t off = 0;
  for (int k = 0; k < count; ++k) {
    BatchInst& I = B->h_insts[k];
    I.b = static_cast<char*>(B->scratch) + off;
    off += (B->bytes[k] + 255) / 256 * 256;
    I.nx = grids[k].n[0];
    I.ny = grids[k].ndim > 1 ? grids[k].n[1] : 1;
    I.periodic = (bc == DL_BC_PERIODIC);
    I.axes_code = axes_code(grids[k]);
  }
  // a tuned segment length from the cache file, if one is configured
  if (const char* path = std::getenv("LIBDIRAC_TUNE_CACHE")) {
    FILE* f = std::fopen(path, "r");
    if (f) {
      char line[256];
      const std::string key = std::string(p->fp64 ? "f64" : "f32") + ":" + std::to_string(count);
      while (std::fgets(line, sizeof line, f)) {
        char k2[128];
        int v = 0;
        if (std::sscanf(line, "%127s %d", k2, &v) == 2 && key == k2 && v > 0) B->seg_len = v;
      }
      std::fclose(f);
    }
  }
  int rc = upload_tiles(*B);
  if (rc) {
    free_batch(B);
    delete p;
    return rc;
  }
  *out = p;
  return DL_OK;
}

extern "C" int dl_batch_step(dl_plan b, void* const* psi, const double* const* V,
                             const int64_t* nsteps, void* stream) {
  if (!b) return set_error(DL_ERR_ARG, "batch is NULL");
  if (!b->is_batch) return set_error(DL_ERR_STATE, "not a batch (use dl_step)");
  if (b->dry) return set_error(DL_ERR_STATE, "dry batch: no device work allowed");
  Batch& B = *as_batch(b);
  if (!psi || !nsteps) return set_error(DL_ERR_ARG, "psi and nsteps are required");
  for (int k = 0; k < B.count; ++k) {
    int rc = check_state_ptr(psi[k], "psi[k]");
    if (rc) return rc;
    if (V && (rc = check_f64_ptr(V[k], "V[k]", true))) return rc;
    if (nsteps[k] < 0) return set_error(DL_ERR_ARG, "nsteps[k] < 0");
    for (int j = 0; j < k; ++j)
      if (psi[j] == psi[k]) return set_error(DL_ERR_ARG, "two instances share a state buffer");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = prepare(B, psi, V, nsteps, st);
  if (rc) return rc;
  return run(B, nsteps, st);
}

// Time each candidate segment length on a scratch copy of the batch's states
// (the caller's arrays are not modified) and keep the fastest.  The result is
// appended to LIBDIRAC_TUNE_CACHE when that variable names a file.
extern "C" int dl_batch_autotune(dl_plan b, void* const* psi, const double* const* V, int trials,
                                 int* chosen, void* stream) {
  if (!b || !b->is_batch) return set_error(DL_ERR_ARG, "not a batch");
  if (b->dry) return set_error(DL_ERR_STATE, "dry batch");
  if (!psi || trials < 1) return set_error(DL_ERR_ARG, "bad arguments");
  Batch& B = *as_batch(b);
  hipStream_t st = static_cast<hipStream_t>(stream);
  size_t total = 0;
  for (int k = 0; k < B.count; ++k) total += (B.bytes[k] + 255) / 256 * 256;
  void* copy = nullptr;
  if (hipMalloc(&copy, total) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(DL_ERR_NOMEM, "autotune scratch allocation failed");
  }
  std::vector<void*> cp(B.count);
  size_t off = 0;
  for (int k = 0; k < B.count; ++k) {
    cp[k] = static_cast<char*>(copy) + off;
    off += (B.bytes[k] + 255) / 256 * 256;
    if (hipMemcpyAsync(cp[k], psi[k], B.bytes[k], hipMemcpyDeviceToDevice, st) != hipSuccess) {
      (void)hipFree(copy);
      return set_error(DL_ERR_HIP, "autotune copy failed");
    }
  }
  std::vector<int64_t> ns(B.count, 2 * trials);
  const bool graph_was = B.use_graph;
  B.use_graph = false;
  const int saved = B.seg_len;
  const int cands[] = {8, 16, 32, 64, 128};
  int best = saved;
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int rc = DL_OK;
  for (int H : cands) {
    B.seg_len = H;
    if ((rc = upload_tiles(B))) break;
    if ((rc = prepare(B, cp.data(), V, ns.data(), st))) break;
    if ((rc = run(B, ns.data(), st))) break;  // warm-up
    (void)hipEventRecord(e0, st);
    if ((rc = run(B, ns.data(), st))) break;
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = H;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(copy);
  B.use_graph = graph_was;
  B.seg_len = (rc == DL_OK) ? best : saved;
  drop_graph(B);
  int rc2 = upload_tiles(B);
  if (rc) return rc;
  if (rc2) return rc2;
  if (chosen) *chosen = B.seg_len;
  if (const char* path = std::getenv("LIBDIRAC_TUNE_CACHE")) {
    FILE* f = std::fopen(path, "a");
    if (f) {
      std::fprintf(f, "%s:%d %d\n", B.fp64 ? "f64" : "f32", B.count, B.seg_len);
      std::fclose(f);
    }
  }
  return DL_OK;
}

extern "C" int dl_batch_set(dl_plan b, int seg_len, int graph_pairs) {
  if (!b || !b->is_batch) return set_error(DL_ERR_ARG, "not a batch");
  if (seg_len < 1 || graph_pairs < 1) return set_error(DL_ERR_ARG, "bad tiling");
  Batch& B = *as_batch(b);
  B.seg_len = seg_len;
  B.graph_pairs = graph_pairs;
  if (b->dry) return DL_OK;
  drop_graph(B);
  return upload_tiles(B);
}
