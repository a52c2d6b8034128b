// dirac_batch.hip -- many independent 1-D / 2-D instances advanced together.
//
// One dl_batch_step call runs every instance through all of its steps:
//   * 1-D instances up to a work share ("lines") run in a persistent kernel,
//     k_batch_lines: each workgroup owns a bin of whole lines (packed longest
//     first by cell count) and advances each line through all of its steps,
//     pass by pass -- the waves split the line's strips, a barrier separates
//     the passes, and the line's two buffers (at most a few MiB) stay in the
//     caches, so HBM sees a line at the start and at the end only;
//   * 2-D instances (and 1-D instances too long for a bin) advance pass by
//     pass: one launch per pass of D fused steps over a flat table of tiles
//     (instance, strip of 64 - 2D columns, march segment), longest first, so
//     that the in-order workgroup dispatch is a longest-processing-time list
//     schedule;
//   * the two run concurrently: the lines kernel on a second stream forked
//     from the caller's and joined before a last kernel that moves every state
//     whose pass count was odd from the batch's buffer back to the caller's.
// With DL_GRAPH the whole sequence is captured once per shape of the call
// (passes, remainders, tiling) and a call is one graph launch.  Every tile
// and every line runs the per-cell code of the single-plan sweep (x
// transport, y march, local step; the phase mode read at run time), so each
// instance ends bit-identical to dl_step on its own plan.
//
// Tile shapes come from dl_batch_autotune: the pass depth D (which sets the
// strip width), the march segment length of each 2-D size class (the power
// of two of the row count) and the lines kernel's workgroup size, each kept
// per (dtype, ndim, size class) in a cache file.
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
#include "dirac_trace.h"

namespace dirac {

struct BatchInst {
  void* a;            // caller's state (set per call)
  void* b;            // batch-owned second buffer
  const double* V;    // per call
  int64_t nx, ny;
  int64_t nsteps;     // per call
  int64_t passes;     // per call: passes of the batch's depth ...
  int64_t rem;        // ... then this many single steps
  int64_t words;      // state size in 16-byte words
  int periodic;
  int axes_code;
  int line;           // 1: advanced by the lines kernel
  int pad;
  PhaseK ph;          // per call (mode depends on V)
};

struct BatchTile {
  int inst;
  int strip;
  int jb, je;         // 2-D: rows [jb, je); 1-D: 0, 1
  int up;             // march direction (alternates between segments)
};

// the K-step pass of one strip of a 1-D instance, for its axis
template <typename T, int K>
__device__ __forceinline__ void line_strip(int axes_code, const T* src, T* dst, const double* V,
                                           const SweepArgs& a, int64_t xs, int lane, int depth) {
  switch (axes_code) {
    case 0: one_row<T, LieStep, K, 0, -1>(src, dst, V, a, xs, lane, depth); break;
    case 1: one_row<T, LieStep, K, 1, -1>(src, dst, V, a, xs, lane, depth); break;
    case 2: one_row<T, LieStep, K, 2, -1>(src, dst, V, a, xs, lane, depth); break;
    default: break;
  }
}

// One launch advances every tiled instance still due by one pass of K steps.
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
    case 0:
    case 1:
    case 2: line_strip<T, K>(I.axes_code, src, dst, I.V, a, xs, lane, depth); break;
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

// Whole 1-D instances in one workgroup each, all steps in one launch.
// Workgroup b advances the lines ids[bin_start[b] .. bin_start[b + 1]) one
// after the other; for each line it runs the line's passes of the batch's
// depth K and then its single-step remainder, the waves of the workgroup
// taking the line's strips in turn.  A barrier (a workgroup-scope release and
// acquire) ends each pass, so the next pass reads what every wave of the
// workgroup wrote; no other workgroup touches the line.  The strips and the
// per-cell code are those of k_batch, so the bits are the same.
// workgroup size limit of the lines kernel: FP64 strips hold twice the
// registers, so their workgroups stop at 512 threads (two waves per SIMD)
template <typename T> constexpr int line_threads_max() { return sizeof(T) == 8 ? 512 : 1024; }

template <typename T, int K>
__global__ __launch_bounds__(line_threads_max<T>()) void k_batch_lines(const BatchInst* __restrict__ insts,
                                                      const int* __restrict__ ids,
                                                      const int* __restrict__ bin_start,
                                                      int depth) {
  const int lane = threadIdx.x & 63;
  const int wave = wave_in_block();
  const int nw = static_cast<int>(blockDim.x >> 6);
  const int64_t sw = strip_width(depth);
  for (int q = bin_start[blockIdx.x]; q < bin_start[blockIdx.x + 1]; ++q) {
    const BatchInst& I = insts[ids[q]];
    SweepArgs a{};
    a.nx = I.nx;
    a.ny = 1;
    a.nz = 1;
    a.periodic = I.periodic;
    a.ph = I.ph;
    const int64_t nstrips = (I.nx + sw - 1) / sw;
    const int64_t total = I.passes + I.rem;
    for (int64_t pass = 0; pass < total; ++pass) {
      const int parity = static_cast<int>(pass & 1);
      const T* src = static_cast<const T*>(parity ? I.b : I.a);
      T* dst = static_cast<T*>(parity ? I.a : I.b);
      if (pass < I.passes) {
        for (int64_t s = wave; s < nstrips; s += nw)
          line_strip<T, K>(I.axes_code, src, dst, I.V, a, s * sw - depth, lane, depth);
      } else {
        for (int64_t s = wave; s < nstrips; s += nw)
          line_strip<T, 1>(I.axes_code, src, dst, I.V, a, s * sw - depth, lane, depth);
      }
      __syncthreads();
    }
  }
}

// States whose pass count was odd end in the batch's buffer: copy them back.
// Block k * kFixBlocks + j copies part j of instance k (16-byte words).
constexpr int kFixBlocks = 32;
__global__ __launch_bounds__(256) void k_batch_fix(const BatchInst* __restrict__ insts) {
  const int k = static_cast<int>(blockIdx.x / kFixBlocks);
  const int j = static_cast<int>(blockIdx.x % kFixBlocks);
  const BatchInst& I = insts[k];
  if (((I.passes + I.rem) & 1) == 0) return;
  const uint4* __restrict__ src = static_cast<const uint4*>(I.b);
  uint4* __restrict__ dst = static_cast<uint4*>(I.a);
  for (int64_t w = int64_t(j) * 256 + threadIdx.x; w < I.words; w += int64_t(kFixBlocks) * 256)
    dst[w] = src[w];
}

// passes of the batch: up to 5 fused steps for both state types (FP64
// passes of 3 or more run one wave per SIMD); a periodic batch lowers the
// depth until every 2-D instance has at least twice as many rows
constexpr int kBatchDepthF32 = 5;
constexpr int kBatchDepthF64 = 5;
constexpr int kSegDefault = 64;           // rows per march segment before tuning
constexpr int kLineThreadsDefault = 1024;  // FP32; FP64: line_threads_max
constexpr int kMaxClass = 32;             // 2-D size classes: floor(log2(rows))

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
  int depth = 1;                    // steps fused per pass
  int depth_cap = 5;                // largest depth the instances allow
  int seg_of[kMaxClass] = {};       // march segment length per 2-D size class
  int line_threads = kLineThreadsDefault;
  int cu_count = 256;
  std::vector<size_t> bytes;        // state bytes per instance
  void* scratch = nullptr;          // second buffers of all instances
  BatchInst* d_insts = nullptr;
  BatchTile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  int ntiles = 0;
  int* d_lines = nullptr;           // line ids by bin, then bin starts
  int nlines = 0, nbins = 0;
  std::vector<BatchInst> h_insts;
  hipStream_t side = nullptr;       // the lines kernel's stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int64_t gkey[4] = {-1, -1, -1, -1};
  int64_t version = 0;              // bumped whenever tiles or bins change
};

Batch* as_batch(dl_plan p) { return static_cast<Batch*>(p->batch); }

int size_class(int64_t rows) {
  int c = 0;
  while (c + 1 < kMaxClass && (int64_t(1) << (c + 1)) <= rows) ++c;
  return c;
}

int64_t cells_of(const dl_grid& g) { return g.n[0] * (g.ndim > 1 ? g.n[1] : 1); }

// instances advanced whole by the lines kernel: 1-D instances whose cell
// count is at most four times an even share of the batch per compute unit
// (and at most 2^20 cells), so that no bin outlasts the tiled passes
void choose_lines(Batch& B) {
  int64_t total = 0;
  for (int k = 0; k < B.count; ++k) total += cells_of(B.grids[k]);
  const int64_t limit =
      std::min<int64_t>(int64_t(1) << 20, std::max<int64_t>(4096, 4 * total / B.cu_count));
  for (int k = 0; k < B.count; ++k) {
    const dl_grid& g = B.grids[k];
    B.h_insts[k].line = (g.ndim == 1 && g.n[0] <= limit) ? 1 : 0;
  }
}

// tile table of the non-line instances, 2-D segments first (longest first),
// 1-D rows last
std::vector<BatchTile> make_tiles(const Batch& B) {
  std::vector<BatchTile> two, one;
  for (int k = 0; k < B.count; ++k) {
    if (B.h_insts[k].line) continue;
    const dl_grid& g = B.grids[k];
    const int64_t nstrips = (g.n[0] + strip_width(B.depth) - 1) / strip_width(B.depth);
    if (g.ndim == 1) {
      for (int64_t s = 0; s < nstrips; ++s)
        one.push_back(BatchTile{k, static_cast<int>(s), 0, 1, 1});
    } else {
      const int64_t ny = g.n[1];
      int64_t H = std::min<int64_t>(B.seg_of[size_class(ny)], ny);
      if (H < 1) H = 1;
      const int64_t nseg = (ny + H - 1) / H;
      for (int64_t q = 0; q < nseg; ++q) {
        const int64_t jb = q * H;
        const int64_t je = std::min<int64_t>(jb + H, ny);
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

// bins of lines: as many as the lines' share of the cells asks for (twice
// their share of the compute units, a line pass being lighter per cell than
// a march), filled longest first onto the emptiest bin
void make_bins(const Batch& B, std::vector<int>& ids, std::vector<int>& start, int* nbins) {
  std::vector<int> lines;
  int64_t all = 0, lw = 0;
  for (int k = 0; k < B.count; ++k) {
    all += cells_of(B.grids[k]);
    if (B.h_insts[k].line) {
      lines.push_back(k);
      lw += cells_of(B.grids[k]);
    }
  }
  ids.clear();
  start.assign(1, 0);
  *nbins = 0;
  if (lines.empty()) return;
  const bool only_lines = (lw == all);
  int64_t nb = only_lines ? int64_t(2) * B.cu_count
                          : (2 * int64_t(B.cu_count) * lw + all - 1) / all;
  nb = std::max<int64_t>(1, std::min<int64_t>(nb, static_cast<int64_t>(lines.size())));
  std::stable_sort(lines.begin(), lines.end(), [&](int x, int y) {
    return cells_of(B.grids[x]) > cells_of(B.grids[y]);
  });
  std::vector<std::vector<int>> bins(static_cast<size_t>(nb));
  std::vector<int64_t> load(static_cast<size_t>(nb), 0);
  for (int k : lines) {
    const size_t b = static_cast<size_t>(std::min_element(load.begin(), load.end()) - load.begin());
    bins[b].push_back(k);
    load[b] += cells_of(B.grids[k]);
  }
  for (const auto& v : bins) {
    ids.insert(ids.end(), v.begin(), v.end());
    start.push_back(static_cast<int>(ids.size()));
  }
  *nbins = static_cast<int>(nb);
}

void drop_graph(Batch& B) {
  if (B.graph) (void)hipGraphExecDestroy(B.graph);
  B.graph = nullptr;
  for (auto& v : B.gkey) v = -1;
}

// rebuild the tile table and the line bins for the current tuning
int upload_layout(Batch& B) {
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
  if (!t.empty()) {
    hipError_t e =
        hipMemcpy(B.d_tiles, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return set_hip_error(e, "tile table upload");
  }
  B.ntiles = static_cast<int>(t.size());
  std::vector<int> ids, start;
  make_bins(B, ids, start, &B.nbins);
  B.nlines = static_cast<int>(ids.size());
  if (B.d_lines) (void)hipFree(B.d_lines);
  B.d_lines = nullptr;
  if (B.nbins > 0) {
    std::vector<int> all(ids);
    all.insert(all.end(), start.begin(), start.end());
    if (hipMalloc(&B.d_lines, all.size() * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(DL_ERR_NOMEM, "line table allocation failed");
    }
    hipError_t e = hipMemcpy(B.d_lines, all.data(), all.size() * sizeof(int),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return set_hip_error(e, "line table upload");
  }
  ++B.version;
  drop_graph(B);
  return DL_OK;
}

template <typename T, int K>
void launch_k(const Batch& B, int phase, int64_t index, hipStream_t st) {
  hipLaunchKernelGGL((k_batch<T, K>), dim3((B.ntiles + 3) / 4), dim3(256), 0, st, B.d_insts,
                     B.d_tiles, B.ntiles, phase, index, B.depth);
}

template <typename T, int K>
void launch_lines_k(const Batch& B, hipStream_t st) {
  const int threads = std::min(B.line_threads, line_threads_max<T>());
  hipLaunchKernelGGL((k_batch_lines<T, K>), dim3(B.nbins), dim3(threads), 0, st, B.d_insts,
                     B.d_lines, B.d_lines + B.nlines, B.depth);
}

template <typename T>
hipError_t launch_pass_t(const Batch& B, int K, int phase, int64_t index, hipStream_t st) {
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

template <typename T>
hipError_t launch_lines_t(const Batch& B, hipStream_t st) {
  switch (B.depth) {
    case 1: launch_lines_k<T, 1>(B, st); break;
    case 2: launch_lines_k<T, 2>(B, st); break;
    case 3: launch_lines_k<T, 3>(B, st); break;
    case 4: launch_lines_k<T, 4>(B, st); break;
    case 5: launch_lines_k<T, 5>(B, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// phase 0: the index-th pass of the batch's depth; phase 1: the index-th
// single step of the remainder
hipError_t launch_pass(const Batch& B, int phase, int64_t index, hipStream_t st) {
  if (B.ntiles == 0) return hipSuccess;
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

// the launches of one call on stream cs: the lines kernel on the side stream
// (forked from cs and joined back), the tiled passes on cs, then the copy of
// odd-parity states
hipError_t enqueue_call(Batch& B, int64_t pmax, int64_t rmax, bool lines, hipStream_t cs) {
  hipError_t e = hipSuccess;
  if (lines) {
    if ((e = hipEventRecord(B.ev_fork, cs)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(B.side, B.ev_fork, 0)) != hipSuccess) return e;
    e = B.fp64 ? launch_lines_t<double>(B, B.side) : launch_lines_t<float>(B, B.side);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(B.ev_join, B.side)) != hipSuccess) return e;
  }
  for (int64_t q = 0; q < pmax && e == hipSuccess; ++q) e = launch_pass(B, 0, q, cs);
  for (int64_t r = 0; r < rmax && e == hipSuccess; ++r) e = launch_pass(B, 1, r, cs);
  if (e != hipSuccess) return e;
  if (lines && (e = hipStreamWaitEvent(cs, B.ev_join, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_fix, dim3(static_cast<unsigned>(B.count) * kFixBlocks), dim3(256), 0,
                     cs, B.d_insts);
  return hipGetLastError();
}

// run every instance through its steps (descriptors already uploaded)
int run(Batch& B, const int64_t* nsteps, hipStream_t st) {
  int64_t pmax = 0, rmax = 0;
  bool lines = false;
  for (int k = 0; k < B.count; ++k) {
    if (B.h_insts[k].line) {
      lines = lines || nsteps[k] > 0;
    } else {
      pmax = std::max(pmax, nsteps[k] / B.depth);
      rmax = std::max(rmax, nsteps[k] % B.depth);
    }
  }
  if (!B.use_graph) {
    hipError_t e = enqueue_call(B, pmax, rmax, lines, st);
    return e == hipSuccess ? DL_OK : set_hip_error(e, "batch launch");
  }
  // the kernels read pointers and counts from the device descriptor table, so
  // one captured graph serves every call of the same shape
  const int64_t key[4] = {pmax, rmax, lines ? 1 : 0, B.version};
  if (!B.graph || !std::equal(key, key + 4, B.gkey)) {
    drop_graph(B);
    if (!B.cap_stream) {
      hipError_t e = hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return set_hip_error(e, "stream create");
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return set_hip_error(e, "begin capture");
    hipError_t e2 = enqueue_call(B, pmax, rmax, lines, B.cap_stream);
    e = hipStreamEndCapture(B.cap_stream, &g);
    if (e2 != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return set_hip_error(e2 != hipSuccess ? e2 : e, "batch graph capture");
    }
    e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B.graph = nullptr;
      return set_hip_error(e, "graph instantiate");
    }
    std::copy(key, key + 4, B.gkey);
  }
  hipError_t e = hipGraphLaunch(B.graph, st);
  return e == hipSuccess ? DL_OK : set_hip_error(e, "graph launch");
}

void free_batch(Batch* B) {
  if (!B) return;
  drop_graph(*B);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->side) (void)hipStreamDestroy(B->side);
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->ev_join) (void)hipEventDestroy(B->ev_join);
  if (B->scratch) (void)hipFree(B->scratch);
  if (B->d_insts) (void)hipFree(B->d_insts);
  if (B->d_tiles) (void)hipFree(B->d_tiles);
  if (B->d_lines) (void)hipFree(B->d_lines);
  (void)hipGetLastError();
  delete B;
}

// ---- tuning cache: one "dirac-batch <dtype> <key> <value>" line per setting
// keys: "2d-depth" (steps per pass), "2d-rows<class>-seg" (segment length of
// the 2-D size class), "1d-threads" (lines kernel workgroup size)
const char* dtype_name(const Batch& B) { return B.fp64 ? "c128" : "c64"; }

void apply_cache(Batch& B) {
  const char* path = std::getenv("LIBDIRAC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    char tag[32], dt[16], key[48];
    int v = 0;
    if (std::sscanf(line, "%31s %15s %47s %d", tag, dt, key, &v) != 4) continue;
    if (std::strcmp(tag, "dirac-batch") != 0 || std::strcmp(dt, dtype_name(B)) != 0 || v <= 0)
      continue;
    int cls = -1;
    if (std::strcmp(key, "2d-depth") == 0) {
      B.depth = std::min(v, B.depth_cap);
    } else if (std::strcmp(key, "1d-threads") == 0) {
      if (v % 64 == 0 && v <= 1024) B.line_threads = v;
    } else if (std::sscanf(key, "2d-rows%d-seg", &cls) == 1 && cls >= 0 && cls < kMaxClass) {
      B.seg_of[cls] = v;
    }
  }
  std::fclose(f);
}

void append_cache(const Batch& B, const std::vector<int>& classes) {
  const char* path = std::getenv("LIBDIRAC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "dirac-batch %s 2d-depth %d\n", dtype_name(B), B.depth);
  for (int cls : classes)
    std::fprintf(f, "dirac-batch %s 2d-rows%d-seg %d\n", dtype_name(B), cls, B.seg_of[cls]);
  std::fprintf(f, "dirac-batch %s 1d-threads %d\n", dtype_name(B), B.line_threads);
  std::fclose(f);
}

}  // namespace

int dirac::batch_depth(dl_plan b) { return as_batch(b)->depth; }

namespace dirac {
void destroy_batch(dl_plan p) {
  free_batch(as_batch(p));
  p->batch = nullptr;
}

// [10] steps per pass, [14] instances run whole by the lines kernel,
// [15] its workgroups, [16] their threads
void batch_info(dl_plan b, int64_t* info, int n) {
  const Batch& B = *as_batch(b);
  for (int i = 0; i < n; ++i) {
    int64_t v = 0;
    if (i == 10) v = B.depth;
    if (i == 14) v = B.nlines;
    if (i == 15) v = B.nbins;
    if (i == 16) v = B.line_threads;
    info[i] = v;
  }
}
}  // namespace dirac

extern "C" int dl_batch_create(dl_plan* out, const dl_grid* grids, const double* dx,
                               const double* dt, const double* c, const double* m, int count,
                               dl_dtype dtype, dl_bc bc, unsigned flags) {
  dirac::TraceRange trace_range("dl_batch_create");
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
  B->depth_cap = p->fp64 ? kBatchDepthF64 : kBatchDepthF32;
  if (bc == DL_BC_PERIODIC)
    for (int k = 0; k < count; ++k)
      while (grids[k].ndim == 2 && B->depth_cap > 1 && grids[k].n[1] < 2 * B->depth_cap)
        --B->depth_cap;
  B->depth = B->depth_cap;
  for (int& s : B->seg_of) s = kSegDefault;
  B->line_threads = p->fp64 ? line_threads_max<double>() : line_threads_max<float>();
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
    B->bytes.push_back(static_cast<size_t>(cells_of(grids[k])) * 4 * (p->fp64 ? 16 : 8));
    total += (B->bytes.back() + 255) / 256 * 256;
  }
  apply_cache(*B);
  if (p->dry) {
    choose_lines(*B);
    *out = p;
    return DL_OK;
  }
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      ncu > 0)
    B->cu_count = ncu;
  if (hipMalloc(&B->scratch, total) != hipSuccess ||
      hipMalloc(&B->d_insts, count * sizeof(BatchInst)) != hipSuccess ||
      hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming) != hipSuccess) {
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
    I.words = static_cast<int64_t>(B->bytes[k] / 16);
    I.periodic = (bc == DL_BC_PERIODIC);
    I.axes_code = axes_code(grids[k]);
  }
  choose_lines(*B);
  int rc = upload_layout(*B);
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
  dirac::TraceRange trace_range("dl_batch_step");
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

// Coordinate search over the batch's tile shapes, timed on a scratch copy of
// the states (the caller's arrays are not modified): first the pass depth
// (steps per pass: the strip width 64 - 2D follows), then the march segment
// length of each 2-D size class present (largest class first), then the lines
// kernel's workgroup size.  Each candidate runs `trials` passes after one
// warm-up run, without graphs, and is scored by its time per step.
extern "C" int dl_batch_autotune(dl_plan b, void* const* psi, const double* const* V, int trials,
                                 int* chosen, void* stream) {
  dirac::TraceRange trace_range("dl_batch_autotune");
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
  const bool graph_was = B.use_graph;
  B.use_graph = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int rc = DL_OK;
  // time per step of `trials` passes at the current settings
  auto score = [&](double* ms_per_step) -> int {
    std::vector<int64_t> ns(B.count, int64_t(trials) * B.depth);
    int r = upload_layout(B);
    if (!r) r = prepare(B, cp.data(), V, ns.data(), st);
    if (!r) r = run(B, ns.data(), st);  // warm-up
    if (r) return r;
    (void)hipEventRecord(e0, st);
    if ((r = run(B, ns.data(), st))) return r;
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_per_step = ms / (double(trials) * B.depth);
    return DL_OK;
  };
  // 1. the pass depth
  {
    int best = B.depth;
    double best_t = 1e300;
    for (int d = std::min(3, B.depth_cap); d <= B.depth_cap && rc == DL_OK; ++d) {
      B.depth = d;
      double t = 0;
      if ((rc = score(&t))) break;
      if (t < best_t) {
        best_t = t;
        best = d;
      }
    }
    B.depth = best;
  }
  // 2. the segment length of each 2-D size class, largest class first
  std::vector<int> classes;
  for (int k = 0; k < B.count; ++k)
    if (B.grids[k].ndim == 2) classes.push_back(size_class(B.grids[k].n[1]));
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  std::reverse(classes.begin(), classes.end());
  for (int cls : classes) {
    if (rc) break;
    const int rows = 1 << cls;
    int best = B.seg_of[cls];
    double best_t = 1e300;
    for (int H : {16, 32, 64, 128, 256, 512}) {
      if (H > 2 * rows) break;
      B.seg_of[cls] = H;
      double t = 0;
      if ((rc = score(&t))) break;
      if (t < best_t) {
        best_t = t;
        best = H;
      }
    }
    B.seg_of[cls] = best;
  }
  // 3. the lines kernel's workgroup size
  bool any_line = false;
  for (const BatchInst& I : B.h_insts) any_line = any_line || I.line;
  if (any_line && rc == DL_OK) {
    int best = B.line_threads;
    double best_t = 1e300;
    for (int th : {256, 512, 1024}) {
      if (th > (B.fp64 ? line_threads_max<double>() : line_threads_max<float>())) break;
      B.line_threads = th;
      double t = 0;
      if ((rc = score(&t))) break;
      if (t < best_t) {
        best_t = t;
        best = th;
      }
    }
    B.line_threads = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(copy);
  B.use_graph = graph_was;
  int rc2 = upload_layout(B);
  if (rc) return rc;
  if (rc2) return rc2;
  if (chosen) {
    chosen[0] = B.depth;
    chosen[1] = B.line_threads;
    chosen[2] = classes.empty() ? 0 : B.seg_of[classes.front()];
  }
  append_cache(B, classes);
  return DL_OK;
}

extern "C" int dl_batch_set(dl_plan b, int seg_len, int depth) {
  if (!b || !b->is_batch) return set_error(DL_ERR_ARG, "not a batch");
  Batch& B = *as_batch(b);
  if (seg_len < 1) return set_error(DL_ERR_ARG, "seg_len must be >= 1");
  if (depth < 1 || depth > B.depth_cap)
    return set_error(DL_ERR_ARG, "depth outside 1 .. the batch's largest depth");
  for (int& s : B.seg_of) s = seg_len;
  B.depth = depth;
  if (b->dry) return DL_OK;
  return upload_layout(B);
}
