// dirac_plan.h -- the plan object behind the opaque dl_plan handle, and the
// helpers shared by the plan, adjoint and batch translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/libdirac.h"
#include "dirac_launch.h"

namespace dirac {

struct PlanTiling {
  SweepArgs a[kMaxDepth]{};  // index depth - 1 (3-D grids: depth 1 only)
  int b[kMaxDepth] = {};     // blocks
  SweepArgs deep{};          // 1-D lines: passes of kDeep1D steps
  int deep_b = 0;
};

struct GraphEntry {
  void* psi;
  const double* V;
  int64_t pairs;
  int mode;
  hipGraphExec_t exec;
};

}  // namespace dirac

struct dl_plan_s {
  dl_grid g{};
  double dx = 0, dt = 0, c = 0, m = 0;
  int dtype = DL_C64;
  int bc = DL_BC_ZERO;
  unsigned flags = 0;
  bool fp64 = false;
  bool dry = false;
  bool use_graph = false;
  bool strang = false;         // second-order steps (Sec. 2.4)
  int nc = 4;                  // components stored per cell (2: two-component 1-D line)
  int64_t cells = 0;
  size_t state_bytes = 0;
  int device = 0;
  dirac::PhaseK ph{};          // phase constants of the current call
  // tilings of the passes of 1 .. kMaxDepth fused steps (index depth - 1),
  // for the phase mode of the current call
  dirac::SweepArgs sw[dirac::kMaxDepth]{};
  int bl[dirac::kMaxDepth] = {};
  dirac::SweepArgs sw_deep{};  // 1-D lines: passes of kDeep1D steps
  int bl_deep = 0;
  int depth_limit = dirac::kMaxDepth;  // caller's cap on fused steps per pass
  int depth = 1;                        // fused steps per pass in use
  int waves_per_cu = 0;        // 0: size the grid from the kernels' occupancy
  int cu_count = 256;
  dirac::PlanTiling tiling[5];  // per phase mode (3: a vector potential, 4: a pulse)
  int depth_field = 1;          // fused steps per pass with a vector potential
  const double* field = nullptr;  // field integrals (mode 3) or profile (mode 4) of the call
  dirac::PulseK pulse{};          // mode 4: the pulse; pulse.n0 counts the call's steps
  bool pulse_on = false;
  int seg_override = 0;
  bool allow_resident = true;
  bool resident = false;
  int res_threads = 0;
  int64_t graph_pairs = 32;  // a captured graph holds 2 * graph_pairs steps
  double norm_ref = 0.0;     // norm watchdog of dl_observables (off while norm_tol == 0)
  double norm_tol = 0.0;
  // scratch
  void* tmp = nullptr;         // second state buffer
  void* tmp2 = nullptr;        // second state buffer for the adjoint field
  void* alt = nullptr;         // third state buffer (odd pass counts end in psi)
  bool alt_failed = false;     // its allocation failed once: keep copying back
  double* partials = nullptr;  // reduction partials
  double* dres = nullptr;      // device results
  double* hres = nullptr;      // pinned host results (mapped)
  double* hres_dev = nullptr;  // their device address
  double* proj = nullptr;      // projection partials (grown on demand)
  size_t proj_bytes = 0;
  double* tile_partials = nullptr;  // per-wave observables sums of a fused last pass
  int64_t tile_partials_n = 0;      // (grown on demand: waves of the deepest tiling)
  hipStream_t cap_stream = nullptr;
  std::vector<dirac::GraphEntry> graphs;
  // batches
  bool is_batch = false;
  void* batch = nullptr;
  void drop_graphs();
};

namespace dirac {

int set_error(int code, const char* msg);
int set_hip_error(hipError_t e, const char* what);
int transports_per_step(dl_plan p);
// shift: cells per one-cell-transport step, c dt = shift * dx (2 for the
// second-order step, whose transports run over dt / 2)
int validate_grid(const dl_grid* g, double dx, double dt, double c, double m, int dtype, int bc,
                  int max_ndim, int shift);
PhaseK make_phase(int ntransports, double dt, double c, double m, int mode, bool two_angles);
int phase_mode(double m, const double* V);
int axes_code(const dl_grid& g);
void make_tiling(const dl_grid& g, int64_t target, int seg_override, SweepArgs& a, int& blocks,
                 int strip_width);
int check_live(dl_plan p);
int check_state_ptr(const void* ptr, const char* name);
int check_f64_ptr(const void* ptr, const char* name, bool nullable);
void destroy_batch(dl_plan p);
// reverse steps fused per pass of dl_grad_step (1 where the adjoint is refused)
int reverse_depth(dl_plan p);
// steps fused per pass of a batch
int batch_depth(dl_plan b);
// dl_plan_info of a batch handle
void batch_info(dl_plan b, int64_t* info, int n);
// measures the occupancy of the 3-D second-order passes (called when such a
// plan is created, outside any stream capture)
void strang3d_prepare(bool fp64);

}  // namespace dirac
