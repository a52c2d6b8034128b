/*
 * libdirac.h -- C ABI of the MI355X split-operator Dirac sweep.
 *
 * The library advances a four-component complex spinor field on a regular
 * grid with the lowest-order operator splitting of the time-dependent Dirac
 * equation in coordinate space (Fillion-Gourdeau, Lorin, Bandrauk, Sec. 2;
 * the second-order splitting of Sec. 2.4 with DL_STRANG, a vector potential
 * with dl_step_field, two-component 1-D lines with DL_BISPINOR):
 * per time step, for every active grid axis d in the order x, y, z, the exact
 * characteristic transport
 *
 *     psi'(i) = 1/2 (I + alpha_d) psi(i - e_d) + 1/2 (I - alpha_d) psi(i + e_d)
 *
 * (eq:sol_dis_1-3, valid because c dt equals the cell size a), then the local
 * step D (eq:sol_dis_4 without vector potential, static V so Vtilde = V dt):
 *
 *     psi_c(i) <- exp(-i (beta_cc m c^2 + V(i)) dt) psi_c(i).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All calls return a dl_status; none throws or aborts.  On a non-OK
 *    status, dl_last_error() returns a message for the calling thread.
 *  - Pointers named psi, lam, V, Q, G are DEVICE pointers owned by the caller;
 *    the library never frees them.  Arrays are C-contiguous with grid
 *    dimension 0 (x) fastest and the spinor component last:
 *    psi[((k * n1 + j) * n0 + i) * 4 + comp] (a DL_BISPINOR plan: 2 stored
 *    components per cell), each component an interleaved (re, im) pair of
 *    float (DL_C64) or double (DL_C128).  V, Q and G hold
 *    one double per cell in the same cell order.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it and the call returns without waiting, except where noted.
 *    Kernel faults surface at the next synchronising call as DL_ERR_HIP.
 *  - A plan owns its scratch (a second state buffer, reduction partials),
 *    allocated in dl_plan_create.  Steps run in passes over memory that
 *    alternate between psi and that buffer; a call that takes an odd number
 *    of passes ends in the buffer and copies the result back into psi, except
 *    that for three or more passes the plan allocates (once, on the first
 *    such call outside stream capture) a third state buffer through which
 *    the last pass writes psi directly.  One plan must not be used from two
 *    streams or threads at once.
 *  - psi and lam must be 16-byte aligned, V, Q and G 8-byte aligned.
 *  - The plan, step, observables, adjoint and batch calls each open a named
 *    roctx range (the call's name) for rocprofv3 --marker-trace, so a trace
 *    shows every call on the host timeline beside the kernels it enqueued.
 */
#ifndef LIBDIRAC_H
#define LIBDIRAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LIBDIRAC_VERSION 1

typedef struct dl_plan_s *dl_plan;

typedef enum {
    DL_OK = 0,
    DL_ERR_ARG = -1,    /* null pointer, bad size, bad enum, nsteps < 0 ... */
    DL_ERR_CFL = -2,    /* c dt differs from the cell size (with DL_STRANG: twice it, four
                           times on 3-D grids), relative 1e-12 */
    DL_ERR_DTYPE = -3,  /* unknown dtype, or call not valid for the plan's dtype */
    DL_ERR_ALIGN = -4,  /* a pointer is not aligned as required */
    DL_ERR_NOMEM = -5,  /* device allocation failed */
    DL_ERR_HIP = -6,    /* a HIP runtime call or kernel failed */
    DL_ERR_STATE = -7,  /* call not allowed on this plan (e.g. a dry plan) */
    DL_ERR_NONFINITE = -8, /* dl_observables: the state holds a NaN or an infinity
                              (out[] is still written; its sums are then not finite) */
    DL_WARN_NORM = 1    /* dl_observables: the norm left the band set with
                           dl_plan_set_norm_check (out[] is written; a warning) */
} dl_status;

typedef enum { DL_C64 = 0, DL_C128 = 1 } dl_dtype;

/* Cells outside the box: DL_BC_ZERO = zero (the Dirichlet wall of Sec. 5);
 * DL_BC_PERIODIC = the box wraps around (exactly unitary steps). */
typedef enum { DL_BC_ZERO = 0, DL_BC_PERIODIC = 1 } dl_bc;

/* Plan flags */
#define DL_DRY 1u    /* validate only: no HIP call, no allocation; every other
                        entry point then returns DL_ERR_STATE */
#define DL_GRAPH 2u  /* replay long step sequences from captured hipGraphs */
#define DL_STRANG 4u /* second-order steps (Sec. 2.4).  1-D and 2-D grids: each
                        step applies the transports over dt/2 in the order
                        A, B, C, the local step over dt, then the transports
                        over dt/2 in the reverse order; every transport is the
                        one-cell shift, so the plan needs c*dt = 2*dx.  3-D
                        grids: A(dt/4) B(dt/2) A(dt/4) C(dt/2) D(dt) C(dt/2)
                        A(dt/4) B(dt/2) A(dt/4) with c*dt = 4*dx: A shifts one
                        cell, B and C two (a call of N steps takes N + 1
                        passes over memory, in place through two scratch
                        states of the plan, one of them an extra buffer; with
                        dl_plan_set_depth(K < 5) groups of K steps take K + 1
                        passes each).  DL_ERR_CFL on any other c*dt.  The adjoint entry points refuse such a
                        plan (DL_ERR_ARG). */
#define DL_BISPINOR 8u /* two-component state, 1-D grids only (Sec. 2.4): with
                        one transport axis the pair of components that contains
                        psi_1 -- (psi_1, psi_4) for alpha_x and alpha_y,
                        (psi_1, psi_3) for alpha_z -- evolves on its own; the
                        state then holds that pair, 2 complex numbers per cell
                        (layout (n, 2)), and the other pair is taken as zero.
                        Results equal those components of the four-component
                        step.  dl_step_field and the adjoint refuse such a plan
                        (DL_ERR_ARG); the observables read the pair. */

/* Grid of P0 cells (Sec. 2.3).  n[d] cells along grid dimension d, n[0]
 * fastest.  axis[d] is the Dirac matrix carried by dimension d (0 = alpha_x,
 * 1 = alpha_y, 2 = alpha_z); it must increase with d, so the transports run
 * in the paper's order A, B, C.  Cell centres are
 * xmin[d] + (i + 1/2) dx; xmin only enters the observables. */
typedef struct {
    int ndim;        /* 1, 2 or 3 */
    int64_t n[3];    /* each >= 2 for d < ndim */
    int axis[3];
    double xmin[3];
} dl_grid;

/* Create a plan for grid g with cell size dx, time step dt, speed of light c
 * and mass m (atomic units in the paper).  Requires c dt = dx to relative
 * 1e-12 (the characteristic condition with K = 1, Sec. 2.3), dx, dt, c > 0 and
 * m >= 0.  On success *out holds the plan; on failure *out is NULL. */
int dl_plan_create(dl_plan *out, const dl_grid *g, double dx, double dt, double c,
                   double m, dl_dtype dtype, dl_bc bc, unsigned flags);

/* Release the plan and its scratch.  Waits for the plan's own work. */
int dl_plan_destroy(dl_plan p);

/* Advance psi in place by nsteps full steps (transports in the order x, y, z,
 * then D).  V: potential energy per cell (FP64) or NULL for V = 0.  With m = 0
 * and V = NULL the step is pure streaming and D is skipped.
 * In the complex64 plan the state is stored in FP32 while the phase
 * exp(-i theta) is formed in FP64 from the FP64 V and applied as an FP32
 * hi + lo pair (1-D, 2-D) or in FP64 (3-D), the product rounded to FP32.
 * nsteps = 0 is a no-op. */
int dl_step(dl_plan p, void *psi, const double *V, int64_t nsteps, void *stream);
/* (Several steps are fused into one pass over memory: up to 5 on 1-D and
 * 2-D grids (1-D lines of at most 65536 cells without a vector potential
 * first run passes of 24 steps, each wave writing 16 cells, unless the depth
 * is capped), fewer on
 * periodic 2-D boxes of fewer than twice that many rows,
 * and 2 on 3-D grids with rows of fewer than 2^28 cells; the remainder of
 * nsteps runs in shallower passes.  Second-order steps on 3-D grids take one
 * pass each plus one closing pass per call (see DL_STRANG).  The bits do not
 * depend on this grouping; dl_plan_set_depth caps it.) */

/* dl_step with a vector potential in the local step (eq:sol_dis_4 and the
 * closed-form exponential of Dirac matrices of Sec. 2.3):
 *     D psi = U exp(-i V dt) psi,
 *     U = cos(A) + i (-beta m c^2 dt + alpha . At) sin(A) / A,
 *     A = sqrt((m c^2 dt)^2 + At . At)   (sin(A)/A -> 1 as A -> 0).
 * A: device array of 3 * cells doubles, planar: the x, y and z components of
 * the field integral At = e int A dtau over one step (eq:field_dis1) at the
 * cell centres, each block in psi's cell order; held fixed for the nsteps
 * steps of the call (a time-dependent field is applied by calls over shorter
 * spans).  A = NULL is dl_step.  1-D and 2-D grids, both splittings, passes
 * of at most 3 steps (1 with DL_STRANG) with the bits of single steps; 3-D
 * grids: lowest-order steps one per pass, second-order steps with U in the
 * middle D of each step and the same grouping of steps as dl_step.  Same
 * buffers and copy rule as dl_step. */
int dl_step_field(dl_plan p, void *psi, const double *V, const double *A, int64_t nsteps,
                  void *stream);

/* A time-dependent vector potential A(t, x) = f(t) P(x): a laser pulse with a
 * linear turn-on ramp, the kind of field whose integral Sec. 2.3 notes is
 * known in closed form.  f(t) = w(t) sin(omega t + phase), with the
 * trapezoid envelope w: 0 for t < 0, t / t_on on [0, t_on), 1 on
 * [t_on, t_on + t_flat), falling linearly to 0 over t_off, 0 afterwards (a
 * zero t_on or t_off is a step).  All in atomic units. */
typedef struct {
    double omega;   /* carrier angular frequency */
    double phase;   /* carrier phase at t = 0 */
    double t_on;    /* rise time of the envelope (>= 0) */
    double t_flat;  /* duration of the plateau (>= 0) */
    double t_off;   /* fall time (>= 0) */
} dl_pulse;

/* nsteps steps whose local step carries the pulse (eq:sol_dis_4 with the U of
 * Sec. 2.3, as dl_step_field): step n = 0 .. nsteps - 1 covers
 * [t0 + n dt, t0 + (n + 1) dt] and uses the field integral (eq:field_dis1)
 *     At^n(x) = P(x) F_n,  F_n = int_{t0 + n dt}^{t0 + (n + 1) dt} f(t) dt,
 * F_n evaluated on the device in closed form for every step (so passes still
 * fuse up to 3 lowest-order steps, each with its own F_n; 1-D and 2-D grids,
 * both splittings).  3-D grids: lowest-order steps one per pass, second-order
 * steps grouped as in dl_step, each D with its own F_n.  P: device array of 3 * cells doubles, planar
 * (x, y, z blocks in psi's cell order): e times the amplitude of A at the
 * cell centres.  pulse: HOST struct; finite values, durations >= 0 (DL_ERR_ARG
 * otherwise).  V as in dl_step.  The bits do not depend on how the steps are
 * grouped into passes (a step's time is formed from its index).  Same buffers
 * and copy rule as dl_step. */
int dl_step_pulse(dl_plan p, void *psi, const double *V, const double *P,
                  const dl_pulse *pulse, double t0, int64_t nsteps, void *stream);

/* One step out of place: dst = S src (same step as dl_step with nsteps = 1).
 * src and dst must not overlap; src is left unchanged.  Lets a caller keep
 * both time levels, or alternate two buffers without the copy dl_step makes
 * when its passes end in the plan's buffer. */
int dl_step_out(dl_plan p, const void *src, void *dst, const double *V, void *stream);

/* nsteps >= 1 steps out of place, dst = S^nsteps src, with the same bits as
 * nsteps single steps.  Up to the plan's fusion depth (see dl_step) this is
 * one pass over memory; larger counts run several passes through the plan's
 * buffer, the last one writing dst.  src and dst must not overlap. */
int dl_step_fused_out(dl_plan p, const void *src, void *dst, const double *V, int64_t nsteps,
                      void *stream);

/* Observables of psi (Sec. 5.2.1 R/T integrals on the cell grid), as FP64
 * compensated sums, written to the HOST array out[5]:
 *   out[0] = N    = dV sum |psi|^2            (dV = dx^ndim)
 *   out[1..3]     = sum x_d |psi|^2 / sum |psi|^2 along grid dims 0..2 (0 if absent)
 *   out[4] = P_T  = dV sum_{x_0 > x_b} |psi|^2 (cell centres, strict >)
 * Synchronises `stream`.  Returns DL_ERR_NONFINITE when a cell holds a NaN or
 * an infinity (the sums then are not finite: no finite state gives an
 * infinite N), and DL_WARN_NORM when the plan's norm check is set and N left
 * its band (below); out[] is written in both cases. */
int dl_observables(dl_plan p, const void *psi, double x_b, double out[5], void *stream);

/* dl_step(p, psi, V, nsteps) followed by dl_observables(p, psi, x_b, out):
 * the same state bits, and the observables of the stepped state (the
 * definitions and status codes of dl_observables; the sums are taken in
 * another order, so they agree with dl_observables' to rounding, ~1e-15
 * relative).  On 2-D lowest-order plans of four-component states on grid
 * axes (x, y), and on 3-D lowest-order plans whose passes fuse two steps
 * (then nsteps >= 2; an odd count runs its single step first), without a
 * vector potential, the last pass sums the observables of the cells as it
 * stores them (Sec. 5.2.1 R/T integrals taken in the epilogue of the last
 * step), so the state is not read again; other plans, and nsteps = 0, step
 * and then reduce.  The first fused call (and one after a retiling that adds
 * waves) allocates the plan's per-wave partials (80 B per wave of the pass).
 * Synchronises `stream`. */
int dl_step_observables(dl_plan p, void *psi, const double *V, int64_t nsteps, double x_b,
                        double out[5], void *stream);

/* dl_observables for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no plan, no
 * allocation, no synchronisation.  The state psi (device, layout of the
 * conventions above; flags = DL_BISPINOR for a two-component 1-D line, else 0)
 * on grid g with cell size dx; out is a DEVICE array of 5 doubles, written
 * with the values of dl_observables (same kernels, same bits), stream-ordered.
 * The per-block partial sums live in a static device array of the library
 * (40 KiB per GPU, held until the process ends) that every call on that GPU
 * shares: calls that overlap on one GPU (two streams, or two threads) race,
 * so serialise them.  Each call writes every partial it reads, so nothing
 * needs clearing.  Grids of any valid size fit (the reduction always uses the
 * same 512 partials); grids beyond 2^40 cells, a NULL or misaligned pointer,
 * or a bad dtype / flag are refused (DL_ERR_ARG, DL_ERR_ALIGN, DL_ERR_DTYPE).
 * The first call on a device looks up the array's device address. */
int dl_observables_noalloc(const dl_grid *g, double dx, dl_dtype dtype, unsigned flags,
                           const void *psi, double x_b, double *out, void *stream);

/* Norm watchdog of dl_observables.  The transports of eq:sol_dis_1-3 are
 * unitary on a periodic box and, with the zero wall of Sec. 5, only lose the
 * probability that crosses the wall; the local step D of eq:sol_dis_4 (and the
 * U of Sec. 2.3) is unitary.  So N = dV sum |psi|^2 never grows beyond its
 * value at the start of a run except by rounding (about 1e-7 relative per
 * 1e4 steps in FP32), and on a periodic box it does not shrink either.  With
 * tol > 0, dl_observables returns DL_WARN_NORM when N > N_ref (1 + tol), or,
 * on a periodic plan, when N < N_ref (1 - tol).  tol = 0 (the default) turns
 * the check off.  N_ref > 0 and tol >= 0, both finite (DL_ERR_ARG otherwise).
 * Works on DL_DRY plans (it only records the values). */
int dl_plan_set_norm_check(dl_plan p, double N_ref, double tol);

/* Seed the adjoint of L = P_T(psi_N): lam = M psi with M the indicator of
 * x_0 > x_b, and Q = 0.  lam has psi's layout, Q one double per cell. */
int dl_seed_adjoint(dl_plan p, const void *psi, double x_b, void *lam, double *Q,
                    void *stream);

/* nsteps reverse steps of the discrete adjoint (derived from eq:sol_dis_1-4).
 * Each step first accumulates, per cell,
 *     Q += 2 dt dV Im(lam^H psi),
 * then replaces psi by S^{-1} psi and lam by S^H lam, where S is one forward
 * step.  S^H lam is exact for both boundary conditions; S^{-1} = S^H holds
 * exactly with DL_BC_PERIODIC (with zero walls it holds only while nothing has
 * left the box).  After N steps from (psi_N, lam_N = M psi_N, Q = 0), Q is
 * dL/dV and psi is the reconstructed psi_0.  Up to 3 reverse steps (2 with
 * complex128 state) are fused into one pass over psi, lam, V and Q, with the
 * bits of single reverse steps (the terms of Q added in the same order).
 * 3-D grids: one pass per reverse step (Q, D^H, T_z^H, T_y^H, T_x^H) through
 * the plan's scratch states, the result copied back to psi and lam after an
 * odd count.  Lowest-order four-component plans only (DL_ERR_ARG else). */
int dl_grad_step(dl_plan p, void *psi, void *lam, const double *V, double *Q,
                 int64_t nsteps, void *stream);

/* out[j] = sum_cells G[j][cell] * Q[cell] for j < nb (deterministic FP64
 * reduction).  G: nb rows of one double per cell (device); out: nb doubles
 * (device).  Gives dL/dtheta_j from dL/dV when G holds dV/dtheta_j. */
int dl_project(dl_plan p, const double *Q, const double *G, int nb, double *out,
               void *stream);

/* V[cell] = sum_j theta[j] G[j][cell] (FP64; the transpose of dl_project).
 * G: nb rows of one double per cell, theta: nb doubles, V: one double per
 * cell, all device pointers.  Builds a parametrised potential on the device. */
int dl_expand(dl_plan p, const double *G, const double *theta, int nb, double *V,
              void *stream);

/* ---- batches: many independent plans advanced by shared launches ------- */

/* Build a batch of `count` instances; grids[k], dx[k], dt[k], c[k], m[k] as in
 * dl_plan_create, one dtype and bc for all.  Instances must be 1-D or 2-D.
 * Flags: DL_GRAPH (each call of one shape is captured once and replayed as
 * one graph), DL_DRY.  The batch owns a second state buffer per instance, a
 * second stream and two events. */
int dl_batch_create(dl_plan *out, const dl_grid *grids, const double *dx,
                    const double *dt, const double *c, const double *m, int count,
                    dl_dtype dtype, dl_bc bc, unsigned flags);

/* Advance instance k in place by nsteps[k] steps: psi[k] (device), V[k]
 * (device or NULL).  The arrays psi, V and nsteps are HOST arrays of length
 * count.  Each instance's result is bit-identical to dl_step on a plan with
 * the same parameters.  1-D instances of up to 4096 cells, or of up to four
 * times an even share of the batch's cells per compute unit if that is more
 * (at most 2^20 cells), run whole in a
 * persistent kernel (a workgroup carries a bin of such lines through all of
 * their steps); the others advance by one launch per pass of fused steps over
 * a table of tiles; the two run concurrently (a second stream forked from and
 * joined to `stream`).  Synchronises `stream` before it rewrites the
 * descriptors of the previous call. */
int dl_batch_step(dl_plan b, void *const *psi, const double *const *V,
                  const int64_t *nsteps, void *stream);

/* ---- tuning: tile shapes, fusion depth, and the batch autotuner -------- */

/* Tiling of the plan's kernels.  waves_per_cu in 0..32: 0 sizes each launch
 * from the kernel's occupancy (all march segments in one round of resident
 * waves), otherwise that many waves per compute unit; seg_len >= 0: rows (or
 * z planes) per march segment, 0 derives it from the grid size; allow_resident
 * (0/1): let 1-D lines of up to 4096 cells run in one workgroup for all steps
 * when the plan fuses at most 2 steps per pass (dl_plan_set_depth); graph_pairs
 * >= 1: a captured graph (DL_GRAPH) holds 2 * graph_pairs steps.  Drops the
 * plan's captured graphs.  The bits of every result are independent of these
 * settings.  DL_ERR_ARG on values out of range. */
int dl_plan_set_tiling(dl_plan p, int waves_per_cu, int seg_len, int allow_resident,
                       int graph_pairs);

/* Cap on the steps fused into one pass over memory, depth in 1..5: forward
 * passes (dl_step and friends) and reverse passes (dl_grad_step) use at most
 * this many steps, and never more than the kernels are built for (2-D and
 * 1-D: 5; 3-D: 2; second-order steps: 3; vector potential: 3,
 * second-order 1; reverse steps: 3, complex128 2).  On 3-D second-order
 * plans a cap below 5 groups the steps of a call by that many, each group
 * with its own closing pass.  The bits are independent of the grouping.
 * DL_ERR_ARG outside 1..5. */
int dl_plan_set_depth(dl_plan p, int depth);

/* Up to n values describing the deepest forward pass in use, written to the
 * HOST array info: [0] workgroups, [1] rows per march segment, [2] segments,
 * [3] x strips, [4] wave tiles, [5] resident 1-D path (0/1), [6] its threads,
 * [7] waves_per_cu setting, [8] XCD-contiguous block order (0/1),
 * [9] graph_pairs, [10] fused steps per pass, [11] workgroups of a
 * single-step pass, [12] reverse steps per pass of dl_grad_step, [13] steps
 * per pass of dl_step_field, [14] steps per pass of the deep passes that 1-D
 * lines run first (0 if the plan has none).  Works on DL_DRY plans.  On a
 * batch handle every
 * value is 0 but [10], the steps fused per pass of the batch, [14] the
 * instances run whole by the lines kernel, [15] its workgroups (0 on a dry
 * batch) and [16] their threads. */
int dl_plan_info(dl_plan p, int64_t *info, int n);

/* Batch tiling: seg_len >= 1 rows per 2-D march segment of every size class,
 * depth in 1 .. the batch's largest (5, less on periodic boxes of few rows)
 * fused steps per pass.  Results stay bit-identical. */
int dl_batch_set(dl_plan b, int seg_len, int depth);

/* Autotuner of the batch's tile shapes: a coordinate search, timed on a
 * device copy of the states psi[k] (HOST array of count device pointers; V as
 * in dl_batch_step; the caller's states are not modified), over the steps
 * fused per pass (3 .. the largest; the strip width 64 - 2 depth follows),
 * then the march segment length (16 .. 512 rows) of each 2-D size class
 * present (class = floor(log2(rows))), then the workgroup size of the lines
 * kernel (256 .. 1024 threads, 512 with complex128).  Each candidate runs
 * `trials` passes after a warm-up and is scored by its time per step.
 * chosen (HOST, may be NULL) receives 3 ints: the depth, the lines workgroup
 * size and the segment length of the largest size class (0 if none).
 * Allocates a scratch copy of all states for the call; synchronises
 * `stream`.  When the environment variable LIBDIRAC_TUNE_CACHE names a file,
 * appends one line per setting, "dirac-batch <c64|c128> <key> <value>" with
 * key 2d-depth, 2d-rows<class>-seg or 1d-threads; dl_batch_create reads that
 * file and applies the settings whose dtype (and size class) match. */
int dl_batch_autotune(dl_plan b, void *const *psi, const double *const *V, int trials,
                      int *chosen, void *stream);

/* Thread-local message for the last non-OK status ("" if none). */
const char *dl_last_error(void);

/* LIBDIRAC_VERSION of the built library. */
int dl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBDIRAC_H */
