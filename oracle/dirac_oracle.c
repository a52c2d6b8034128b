/*
 * dirac_oracle.c -- plain, slow, CPU reference of the split-operator /
 * method-of-characteristics Dirac sweep (Fillion-Gourdeau, Lorin, Bandrauk,
 * "Numerical Solution of the Time-Dependent Dirac Equation in Coordinate
 * Space without Fermion-Doubling").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header or table with
 * the GPU library and includes nothing from it.
 *
 * What it computes, in the paper's order and notation:
 *   - Dirac representation alpha_x, alpha_y, alpha_z, beta built from the
 *     Pauli matrices (Sec. 2, eq:dirac_mat).
 *   - One time step of the lowest-order (Lie) splitting (Sec. 2.1,
 *     eq:split1-4): the transport sub-steps A (x), B (y), C (z) in that order,
 *     then the local step D.
 *   - Each transport sub-step is the exact characteristic solution on the P0
 *     grid with c*dt = a (Sec. 2.3, eq:sol_dis_1-3; App. A):
 *         psi'(i) = 1/2 (I + alpha_d) psi(i - e_d) + 1/2 (I - alpha_d) psi(i + e_d)
 *     written as two literal 4x4 complex matrix-vector products accumulated
 *     in column order, then added.  Cells outside the box are zero
 *     (Dirichlet wall, Sec. 5) or wrap around (periodic, a test option).
 *   - D with no vector potential (eq:sol_dis_4, field integrals
 *     eq:field_dis2 with a static V so that Vtilde = V dt):
 *         psi_c <- psi_c * (cos th_c - i sin th_c),
 *         th_c = (V + beta_cc m c^2) dt,
 *     with V the potential energy sampled at cell centres.
 *   - One time step of the second-order (Strang) splitting of Sec. 2.4 with
 *     the simplifications that section states for 1-D and 2-D grids: the
 *     transports over dt/2 in the order A, B, C, the local step D over dt,
 *     then the transports over dt/2 in the reverse order.  Each half-step
 *     transport is the same one-cell characteristic shift, i.e. the grid
 *     obeys c*(dt/2) = a.  On a 3-D grid, the printed nine-part sequence
 *     A(dt/4) B(dt/2) A(dt/4) C(dt/2) D C(dt/2) A(dt/4) B(dt/2) A(dt/4) with
 *     c*(dt/4) = a: A shifts one cell, B and C two cells.
 *   - D with a vector potential (eq:sol_dis_4 with the closed form of the
 *     exponential of Dirac matrices, Sec. 2.3): psi <- U exp(-i Vtilde) psi,
 *     U = cos(A) + i (-beta m c^2 dt + alpha . Atilde) sin(A) / A,
 *     A = sqrt((m c^2 dt)^2 + Atilde . Atilde), written as the printed 4x4
 *     matrix; Atilde (the field integral e int A dtau over the step,
 *     eq:field_dis1) is given per cell.
 *   - A time-dependent vector potential A(t, x) = f(t) P(x) of the kind
 *     Sec. 2.3 names (a laser pulse with a linear turn-on ramp):
 *     f(t) = w(t) sin(omega t + phase) with a trapezoid envelope w.  The
 *     field integral of each step, Atilde^n(x) = P(x) int_{t_n}^{t_{n+1}} f
 *     (eq:field_dis1), is evaluated by Gauss-Legendre quadrature on the
 *     pieces of the step between the envelope's corners; D is then the field
 *     step above with that Atilde.
 *   - Observables: norm, mean coordinates and the probability beyond x_b
 *     (Sec. 5.2.1, R/T integrals), as sequential Neumaier sums in FP64.
 *   - The discrete adjoint of the step (derived from eq:sol_dis_1-4) by
 *     checkpoint-and-recompute: lambda_{n-1} = S^dagger lambda_n with the
 *     literal conjugate transposes of every factor.
 *
 * Floating point: double everywhere; a float instance of the transport
 * sub-steps exists only so that pure streaming can be compared bit for bit.
 * Build with -O2 -ffp-contract=off and without -ffast-math.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zd;
typedef float complex zf;

/* ------------------------------------------------------------------ */
/* Dirac matrices (Sec. 2, eq:dirac_mat) and the projectors 1/2(I +- a) */
/* ------------------------------------------------------------------ */

static zd ALPHA[3][4][4];
static zd BETA[4][4];
/* PROJ[d][0] = 1/2 (I + alpha_d), PROJ[d][1] = 1/2 (I - alpha_d) */
static zd PROJ[3][2][4][4];
static zf PROJF[3][2][4][4];
/* conjugate transposes of PROJ, used by the adjoint */
static zd PROJ_H[3][2][4][4];
static int matrices_ready = 0;

static void build_matrices(void)
{
    if (matrices_ready) return;
    const zd sigma[3][2][2] = {
        {{0, 1}, {1, 0}},   /* sigma_x */
        {{0, -I}, {I, 0}},  /* sigma_y */
        {{1, 0}, {0, -1}},  /* sigma_z */
    };
    memset(ALPHA, 0, sizeof ALPHA);
    memset(BETA, 0, sizeof BETA);
    for (int d = 0; d < 3; ++d)
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s) {
                /* alpha_d = [[0, sigma_d], [sigma_d, 0]] */
                ALPHA[d][r][2 + s] = sigma[d][r][s];
                ALPHA[d][2 + r][s] = sigma[d][r][s];
            }
    /* beta = diag(I_2, -I_2) */
    BETA[0][0] = 1; BETA[1][1] = 1; BETA[2][2] = -1; BETA[3][3] = -1;

    for (int d = 0; d < 3; ++d)
        for (int r = 0; r < 4; ++r)
            for (int s = 0; s < 4; ++s) {
                zd id = (r == s) ? 1.0 : 0.0;
                PROJ[d][0][r][s] = 0.5 * (id + ALPHA[d][r][s]);
                PROJ[d][1][r][s] = 0.5 * (id - ALPHA[d][r][s]);
            }
    for (int d = 0; d < 3; ++d)
        for (int p = 0; p < 2; ++p)
            for (int r = 0; r < 4; ++r)
                for (int s = 0; s < 4; ++s) {
                    PROJF[d][p][r][s] = (zf)PROJ[d][p][r][s];
                    PROJ_H[d][p][r][s] = conj(PROJ[d][p][s][r]);
                }
    matrices_ready = 1;
}

/* Export the matrices so tests can check the Clifford algebra:
 * out = [alpha_x, alpha_y, alpha_z, beta], each 4x4 complex, row-major,
 * interleaved re/im (4 * 16 * 2 doubles). */
void oracle_dirac_matrices(double *out)
{
    build_matrices();
    for (int m = 0; m < 4; ++m)
        for (int r = 0; r < 4; ++r)
            for (int s = 0; s < 4; ++s) {
                zd v = (m < 3) ? ALPHA[m][r][s] : BETA[r][s];
                out[((m * 4 + r) * 4 + s) * 2 + 0] = creal(v);
                out[((m * 4 + r) * 4 + s) * 2 + 1] = cimag(v);
            }
}

/* ------------------------------------------------------------------ */
/* Grid (Sec. 2.3: P0 cells of edge a, centres x_min + (i + 1/2) a)      */
/* ------------------------------------------------------------------ */

typedef struct {
    int ndim;
    int64_t n[3];   /* n[0] fastest (x) */
    int axis[3];    /* Dirac matrix used along grid dimension d */
    int periodic;   /* 0: zero cells outside the box, 1: wrap around */
} grid_t;

static int grid_from_args(grid_t *g, int ndim, const int64_t *n, const int *axis, int bc)
{
    if (ndim < 1 || ndim > 3) return -1;
    g->ndim = ndim;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = (d < ndim) ? n[d] : 1;
        g->axis[d] = (d < ndim) ? axis[d] : -1;
        if (g->n[d] < 1) return -1;
    }
    for (int d = 0; d < ndim; ++d)
        if (g->axis[d] < 0 || g->axis[d] > 2) return -1;
    g->periodic = (bc == 1);
    return 0;
}

static int64_t nsites(const grid_t *g) { return g->n[0] * g->n[1] * g->n[2]; }

/* Site index of cell (i0, i1, i2); returns -1 for a cell outside a
 * non-periodic box. */
static int64_t site_at(const grid_t *g, int64_t i0, int64_t i1, int64_t i2)
{
    int64_t c[3] = {i0, i1, i2};
    for (int d = 0; d < 3; ++d) {
        if (c[d] < 0 || c[d] >= g->n[d]) {
            if (!g->periodic) return -1;
            c[d] = ((c[d] % g->n[d]) + g->n[d]) % g->n[d];
        }
    }
    return (c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
}

/* Order of the transport sub-steps: A (alpha_x), B (alpha_y), C (alpha_z),
 * i.e. grid dimensions sorted by the Dirac matrix they carry. */
static int transport_order(const grid_t *g, int order[3])
{
    int k = 0;
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < g->ndim; ++d)
            if (g->axis[d] == a) order[k++] = d;
    return k;
}

/* ------------------------------------------------------------------ */
/* Transport sub-step along one grid dimension (eq:sol_dis_1-3)         */
/* ------------------------------------------------------------------ */

/* out = P v, accumulated in column order (s = P[r][0] v0 + P[r][1] v1 ...) */
static void matvec_d(zd P[4][4], const zd *v, zd *out)
{
    for (int r = 0; r < 4; ++r) {
        zd s = 0;
        for (int k = 0; k < 4; ++k) s += P[r][k] * v[k];
        out[r] = s;
    }
}

static void matvec_f(zf P[4][4], const zf *v, zf *out)
{
    for (int r = 0; r < 4; ++r) {
        zf s = 0;
        for (int k = 0; k < 4; ++k) s += P[r][k] * v[k];
        out[r] = s;
    }
}

/* psi'(i) = Pm psi(i - s e_d) + Pp psi(i + s e_d): the characteristic
 * solution over a time with c t = s a (s = 1 for every sub-step except the
 * half-step y and z transports of the 3-D second-order step, s = 2).
 * Forward sub-step: Pm = 1/2(I + alpha), Pp = 1/2(I - alpha).
 * Its adjoint:      Pm = (1/2(I - alpha))^H, Pp = (1/2(I + alpha))^H. */
static void transport_d(const grid_t *g, int d, int shift, zd Pm[4][4], zd Pp[4][4],
                        const zd *in, zd *out)
{
    const int64_t rows = g->n[1] * g->n[2];
    #pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < rows; ++row) {
        const int64_t i1 = row % g->n[1], i2 = row / g->n[1];
        for (int64_t i0 = 0; i0 < g->n[0]; ++i0) {
            int64_t c[3] = {i0, i1, i2};
            int64_t cm[3] = {i0, i1, i2}, cp[3] = {i0, i1, i2};
            cm[d] -= shift;
            cp[d] += shift;
            const int64_t sm = site_at(g, cm[0], cm[1], cm[2]);
            const int64_t sp = site_at(g, cp[0], cp[1], cp[2]);
            const zd zero4[4] = {0, 0, 0, 0};
            const zd *vm = (sm < 0) ? zero4 : in + 4 * sm;
            const zd *vp = (sp < 0) ? zero4 : in + 4 * sp;
            zd wm[4], wp[4];
            matvec_d(Pm, vm, wm);
            matvec_d(Pp, vp, wp);
            zd *o = out + 4 * site_at(g, c[0], c[1], c[2]);
            for (int r = 0; r < 4; ++r) o[r] = wm[r] + wp[r];
        }
    }
}

static void transport_f(const grid_t *g, int d, zf Pm[4][4], zf Pp[4][4],
                        const zf *in, zf *out)
{
    const int64_t rows = g->n[1] * g->n[2];
    #pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < rows; ++row) {
        const int64_t i1 = row % g->n[1], i2 = row / g->n[1];
        for (int64_t i0 = 0; i0 < g->n[0]; ++i0) {
            int64_t cm[3] = {i0, i1, i2}, cp[3] = {i0, i1, i2};
            cm[d] -= 1;
            cp[d] += 1;
            const int64_t sm = site_at(g, cm[0], cm[1], cm[2]);
            const int64_t sp = site_at(g, cp[0], cp[1], cp[2]);
            const zf zero4[4] = {0, 0, 0, 0};
            const zf *vm = (sm < 0) ? zero4 : in + 4 * sm;
            const zf *vp = (sp < 0) ? zero4 : in + 4 * sp;
            zf wm[4], wp[4];
            matvec_f(Pm, vm, wm);
            matvec_f(Pp, vp, wp);
            zf *o = out + 4 * site_at(g, i0, i1, i2);
            for (int r = 0; r < 4; ++r) o[r] = wm[r] + wp[r];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Local step D without vector potential (eq:sol_dis_4, static V)       */
/* ------------------------------------------------------------------ */

/* sign = -1: forward exp(-i th); sign = +1: its adjoint exp(+i th). */
static void local_step(const grid_t *g, zd *psi, const double *V,
                       double dt, double c, double m, double sign)
{
    const int64_t ns = nsites(g);
    const double mc2 = m * c * c;
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        const double v = V ? V[s] : 0.0;
        for (int k = 0; k < 4; ++k) {
            const double th = (v + creal(BETA[k][k]) * mc2) * dt;
            psi[4 * s + k] *= CMPLX(cos(th), sign * sin(th));
        }
    }
}

/* D with a vector potential: psi <- U(i) exp(-i V(i) dt) psi with U the
 * printed 4x4 matrix of Sec. 2.3 (entries in terms of c(A), s(A), m c^2 dt
 * and the components of Atilde).  Atil is planar: Atil[d * ns + s] is the
 * component d (x, y, z) at site s, or NULL for no field.  For A = 0
 * (massless, no field) sin(A)/A is its limit 1. */
static void local_step_field(const grid_t *g, zd *psi, const double *V, const double *Atil,
                             double dt, double c, double m)
{
    const int64_t ns = nsites(g);
    const double mu = m * c * c * dt;
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        const double ax = Atil ? Atil[s] : 0.0;
        const double ay = Atil ? Atil[ns + s] : 0.0;
        const double az = Atil ? Atil[2 * ns + s] : 0.0;
        const double A = sqrt(mu * mu + ax * ax + ay * ay + az * az);
        const double cA = cos(A);
        const double sA = (A > 0.0) ? sin(A) / A : 1.0;  /* s(A) / A */
        zd U[4][4];
        memset(U, 0, sizeof U);
        U[0][0] = CMPLX(cA, -mu * sA);
        U[1][1] = CMPLX(cA, -mu * sA);
        U[2][2] = CMPLX(cA, mu * sA);
        U[3][3] = CMPLX(cA, mu * sA);
        U[0][2] = CMPLX(0.0, az * sA);
        U[0][3] = CMPLX(ay * sA, ax * sA);
        U[1][2] = CMPLX(-ay * sA, ax * sA);
        U[1][3] = CMPLX(0.0, -az * sA);
        U[2][0] = CMPLX(0.0, az * sA);
        U[2][1] = CMPLX(ay * sA, ax * sA);
        U[3][0] = CMPLX(-ay * sA, ax * sA);
        U[3][1] = CMPLX(0.0, -az * sA);
        const double th = (V ? V[s] : 0.0) * dt;
        const zd ph = CMPLX(cos(th), -sin(th));
        zd v[4], out[4];
        for (int k = 0; k < 4; ++k) v[k] = psi[4 * s + k] * ph;
        matvec_d(U, v, out);
        for (int k = 0; k < 4; ++k) psi[4 * s + k] = out[k];
    }
}

/* ------------------------------------------------------------------ */
/* Public entry points (called through ctypes by the tests)             */
/* ------------------------------------------------------------------ */

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One forward step S = D * T_{last} ... T_{first}: transports in the order
 * A, B, C then D.  psi and tmp are 4*nsites complex each. */
static void step_once(const grid_t *g, zd *psi, zd *tmp, const double *V,
                      double dt, double c, double m)
{
    int order[3];
    const int k = transport_order(g, order);
    const int64_t bytes = nsites(g) * 4 * (int64_t)sizeof(zd);
    for (int t = 0; t < k; ++t) {
        const int d = order[t];
        const int a = g->axis[d];
        transport_d(g, d, 1, PROJ[a][0], PROJ[a][1], psi, tmp);
        memcpy(psi, tmp, (size_t)bytes);
    }
    local_step(g, psi, V, dt, c, m, -1.0);
}

/* One second-order step (Sec. 2.4, 1-D and 2-D):
 *   T_first(dt/2) ... T_last(dt/2), D(dt), T_last(dt/2) ... T_first(dt/2),
 * each T over dt/2 being the one-cell shift of eq:sol_dis_1-3 (c dt/2 = a). */
static void step_once_strang(const grid_t *g, zd *psi, zd *tmp, const double *V,
                             double dt, double c, double m)
{
    int order[3];
    const int k = transport_order(g, order);
    const int64_t bytes = nsites(g) * 4 * (int64_t)sizeof(zd);
    for (int t = 0; t < k; ++t) {
        const int a = g->axis[order[t]];
        transport_d(g, order[t], 1, PROJ[a][0], PROJ[a][1], psi, tmp);
        memcpy(psi, tmp, (size_t)bytes);
    }
    local_step(g, psi, V, dt, c, m, -1.0);
    for (int t = k - 1; t >= 0; --t) {
        const int a = g->axis[order[t]];
        transport_d(g, order[t], 1, PROJ[a][0], PROJ[a][1], psi, tmp);
        memcpy(psi, tmp, (size_t)bytes);
    }
}

/* One second-order step on a 3-D grid, the sequence printed in Sec. 2.4:
 *   A(dt/4) B(dt/2) A(dt/4) C(dt/2) D(dt) C(dt/2) A(dt/4) B(dt/2) A(dt/4).
 * With c dt/4 = a every A is the one-cell shift and every B and C the
 * two-cell shift of eq:sol_dis_1-3 (c dt/2 = 2a).  D is local_step, or
 * local_step_field with the field integral Atil when `field` is set. */
static void step_once_strang3(const grid_t *g, zd *psi, zd *tmp, const double *V,
                              const double *Atil, int field, double dt, double c, double m)
{
    int order[3];
    transport_order(g, order);
    const int64_t bytes = nsites(g) * 4 * (int64_t)sizeof(zd);
    /* the sub-steps in order: (grid dimension of A, B or C, cells), -1 for D */
    const int seq[9][2] = {{order[0], 1}, {order[1], 2}, {order[0], 1}, {order[2], 2}, {-1, 0},
                           {order[2], 2}, {order[0], 1}, {order[1], 2}, {order[0], 1}};
    for (int t = 0; t < 9; ++t) {
        const int d = seq[t][0];
        if (d < 0) {
            if (field)
                local_step_field(g, psi, V, Atil, dt, c, m);
            else
                local_step(g, psi, V, dt, c, m, -1.0);
            continue;
        }
        const int a = g->axis[d];
        transport_d(g, d, seq[t][1], PROJ[a][0], PROJ[a][1], psi, tmp);
        memcpy(psi, tmp, (size_t)bytes);
    }
}

/* One step whose D carries the field integral Atil: the lowest-order step
 * (scheme 0) or the second-order step of Sec. 2.4 (scheme 1; on 3-D grids
 * its nine-part sequence). */
static void field_step_once(const grid_t *g, zd *psi, zd *tmp, const double *V,
                            const double *Atil, int scheme, double dt, double c, double m)
{
    if (scheme == 1 && g->ndim == 3) {
        step_once_strang3(g, psi, tmp, V, Atil, 1, dt, c, m);
        return;
    }
    int order[3];
    const int k = transport_order(g, order);
    const int64_t bytes = nsites(g) * 4 * (int64_t)sizeof(zd);
    for (int t = 0; t < k; ++t) {
        const int a = g->axis[order[t]];
        transport_d(g, order[t], 1, PROJ[a][0], PROJ[a][1], psi, tmp);
        memcpy(psi, tmp, (size_t)bytes);
    }
    local_step_field(g, psi, V, Atil, dt, c, m);
    if (scheme == 1) {
        for (int t = k - 1; t >= 0; --t) {
            const int a = g->axis[order[t]];
            transport_d(g, order[t], 1, PROJ[a][0], PROJ[a][1], psi, tmp);
            memcpy(psi, tmp, (size_t)bytes);
        }
    }
}

/* One adjoint step S^H = T_first^H ... T_last^H D^H (D^H applied first). */
static void adjoint_once(const grid_t *g, zd *lam, zd *tmp, const double *V,
                         double dt, double c, double m)
{
    int order[3];
    const int k = transport_order(g, order);
    const int64_t bytes = nsites(g) * 4 * (int64_t)sizeof(zd);
    local_step(g, lam, V, dt, c, m, +1.0);
    for (int t = k - 1; t >= 0; --t) {
        const int d = order[t];
        const int a = g->axis[d];
        /* adjoint of psi'(i) = P+ psi(i-1) + P- psi(i+1) is
         * lam'(i) = (P-)^H lam(i-1) + (P+)^H lam(i+1) */
        transport_d(g, d, 1, PROJ_H[a][1], PROJ_H[a][0], lam, tmp);
        memcpy(lam, tmp, (size_t)bytes);
    }
}

/* psi: interleaved complex128, 4 components per site, in/out.
 * V: potential energy per site (FP64) or NULL for V = 0.
 * Returns 0, or -1 on bad arguments / -2 on allocation failure. */
int oracle_step(int ndim, const int64_t *n, const int *axis, int bc,
                double dt, double c, double m, const double *V,
                double *psi, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, bc) || nsteps < 0) return -1;
    build_matrices();
    set_threads(nthreads);
    zd *tmp = (zd *)malloc((size_t)nsites(&g) * 4 * sizeof(zd));
    if (!tmp) return -2;
    for (int64_t s = 0; s < nsteps; ++s) step_once(&g, (zd *)psi, tmp, V, dt, c, m);
    free(tmp);
    return 0;
}

/* nsteps second-order steps; dt is the full step (1-D, 2-D: c dt = 2a;
 * 3-D: c dt = 4a). */
int oracle_step_strang(int ndim, const int64_t *n, const int *axis, int bc,
                       double dt, double c, double m, const double *V,
                       double *psi, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, bc) || nsteps < 0) return -1;
    build_matrices();
    set_threads(nthreads);
    zd *tmp = (zd *)malloc((size_t)nsites(&g) * 4 * sizeof(zd));
    if (!tmp) return -2;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (ndim == 3)
            step_once_strang3(&g, (zd *)psi, tmp, V, NULL, 0, dt, c, m);
        else
            step_once_strang(&g, (zd *)psi, tmp, V, dt, c, m);
    }
    free(tmp);
    return 0;
}

/* nsteps steps with a vector potential: the lowest-order step (scheme 0) or
 * the second-order step of Sec. 2.4 (scheme 1), with D replaced by
 * local_step_field. */
int oracle_step_field(int ndim, const int64_t *n, const int *axis, int bc, int scheme,
                      double dt, double c, double m, const double *V, const double *Atil,
                      double *psi, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (scheme < 0 || scheme > 1 || grid_from_args(&g, ndim, n, axis, bc) || nsteps < 0)
        return -1;
    build_matrices();
    set_threads(nthreads);
    zd *tmp = (zd *)malloc((size_t)nsites(&g) * 4 * sizeof(zd));
    if (!tmp) return -2;
    for (int64_t st = 0; st < nsteps; ++st)
        field_step_once(&g, (zd *)psi, tmp, V, Atil, scheme, dt, c, m);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* A laser pulse with a linear turn-on ramp (Sec. 2.3)                  */
/* ------------------------------------------------------------------ */

/* params: omega, phase, t_on, t_flat, t_off.  The envelope w(t) is 0 for
 * t < 0, rises linearly to 1 over [0, t_on), stays 1 for t_flat, falls
 * linearly to 0 over t_off and is 0 afterwards (a zero t_on or t_off is a
 * step). */
static double pulse_envelope(const double *pp, double t)
{
    const double t_on = pp[2], t1 = pp[2] + pp[3], t2 = pp[2] + pp[3] + pp[4];
    if (t < 0.0 || t >= t2) return 0.0;
    if (t < t_on) return t / t_on;
    if (t < t1) return 1.0;
    return (t2 - t) / pp[4];
}

static double pulse_f(const double *pp, double t)
{
    return pulse_envelope(pp, t) * sin(pp[0] * t + pp[1]);
}

/* Gauss-Legendre rule of order n on [-1, 1]: the roots of the Legendre
 * polynomial P_n found by Newton's method from cos(pi (k + 3/4) / (n + 1/2)),
 * with P_n and P_n' from the three-term recurrence; weights
 * 2 / ((1 - x^2) P_n'(x)^2). */
#define GL_N 16
static void gauss_legendre(int n, double *x, double *w)
{
    for (int k = 0; k < n; ++k) {
        double z = cos(3.14159265358979323846 * (k + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void oracle_gauss_legendre(double *x, double *w) { gauss_legendre(GL_N, x, w); }

/* int_a^b f(t) dt for a piece on which w is linear: Gauss-Legendre on
 * sub-intervals short enough that omega * length <= 1 */
static double pulse_piece(const double *pp, double a, double b, const double *gx,
                          const double *gw)
{
    int nsub = (int)ceil(fabs(pp[0]) * (b - a));
    if (nsub < 1) nsub = 1;
    double sum = 0.0;
    for (int q = 0; q < nsub; ++q) {
        const double lo = a + (b - a) * q / nsub, hi = a + (b - a) * (q + 1) / nsub;
        const double h = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
        double part = 0.0;
        for (int k = 0; k < GL_N; ++k) part += gw[k] * pulse_f(pp, mid + h * gx[k]);
        sum += h * part;
    }
    return sum;
}

/* The field-integral factor of one step, int_{ta}^{tb} f(t) dt: the interval
 * is cut at the envelope's corners 0, t_on, t_on + t_flat, t_on + t_flat +
 * t_off, where w has a kink, and each piece integrated as above. */
double oracle_pulse_integral(const double *pp, double ta, double tb)
{
    double gx[GL_N], gw[GL_N];
    gauss_legendre(GL_N, gx, gw);
    const double corners[4] = {0.0, pp[2], pp[2] + pp[3], pp[2] + pp[3] + pp[4]};
    double cuts[6];
    int nc = 0;
    cuts[nc++] = ta;
    for (int k = 0; k < 4; ++k)
        if (corners[k] > ta && corners[k] < tb) cuts[nc++] = corners[k];
    cuts[nc++] = tb;
    double sum = 0.0;
    for (int k = 0; k + 1 < nc; ++k) sum += pulse_piece(pp, cuts[k], cuts[k + 1], gx, gw);
    return sum;
}

/* nsteps steps with the pulse: step st covers [t0 + st dt, t0 + (st + 1) dt]
 * and its local step carries Atilde = P * oracle_pulse_integral over that
 * interval (P planar, 3 * sites); scheme as in oracle_step_field. */
int oracle_step_pulse(int ndim, const int64_t *n, const int *axis, int bc, int scheme,
                      double dt, double c, double m, const double *V, const double *P,
                      const double *pp, double t0, double *psi, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (scheme < 0 || scheme > 1 || !P || !pp || grid_from_args(&g, ndim, n, axis, bc) ||
        nsteps < 0)
        return -1;
    build_matrices();
    set_threads(nthreads);
    const int64_t ns = nsites(&g);
    zd *tmp = (zd *)malloc((size_t)ns * 4 * sizeof(zd));
    double *At = (double *)malloc((size_t)ns * 3 * sizeof(double));
    if (!tmp || !At) {
        free(tmp);
        free(At);
        return -2;
    }
    for (int64_t st = 0; st < nsteps; ++st) {
        const double F = oracle_pulse_integral(pp, t0 + (double)st * dt, t0 + (double)(st + 1) * dt);
        for (int64_t q = 0; q < 3 * ns; ++q) At[q] = F * P[q];
        field_step_once(&g, (zd *)psi, tmp, V, At, scheme, dt, c, m);
    }
    free(tmp);
    free(At);
    return 0;
}

/* nsteps adjoint steps lam <- S^H lam. */
int oracle_adjoint_step(int ndim, const int64_t *n, const int *axis, int bc,
                        double dt, double c, double m, const double *V,
                        double *lam, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, bc) || nsteps < 0) return -1;
    build_matrices();
    set_threads(nthreads);
    zd *tmp = (zd *)malloc((size_t)nsites(&g) * 4 * sizeof(zd));
    if (!tmp) return -2;
    for (int64_t s = 0; s < nsteps; ++s) adjoint_once(&g, (zd *)lam, tmp, V, dt, c, m);
    free(tmp);
    return 0;
}

/* Float instance of the transport sub-steps only (no D): pure streaming. */
int oracle_stream_f32(int ndim, const int64_t *n, const int *axis, int bc,
                      float *psi, int64_t nsteps, int nthreads)
{
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, bc) || nsteps < 0) return -1;
    build_matrices();
    set_threads(nthreads);
    const int64_t count = nsites(&g) * 4;
    zf *tmp = (zf *)malloc((size_t)count * sizeof(zf));
    if (!tmp) return -2;
    int order[3];
    const int k = transport_order(&g, order);
    for (int64_t s = 0; s < nsteps; ++s)
        for (int t = 0; t < k; ++t) {
            const int d = order[t];
            const int a = g.axis[d];
            transport_f(&g, d, PROJF[a][0], PROJF[a][1], (const zf *)psi, tmp);
            memcpy(psi, tmp, (size_t)count * sizeof(zf));
        }
    free(tmp);
    return 0;
}

/* Neumaier (compensated) accumulation */
typedef struct { double s, comp; } nsum_t;

static void nsum_add(nsum_t *a, double x)
{
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->comp += (a->s - t) + x;
    else a->comp += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum_t *a) { return a->s + a->comp; }

/* out[0] = N = dV sum |psi|^2
 * out[1..3] = <x_d> = sum x_d |psi|^2 / sum |psi|^2 along grid dims 0..2
 *             (0 for dimensions the grid does not have)
 * out[4] = P_T = dV sum_{x_0 > x_b} |psi|^2 (cell centres, strict >)
 * dV = dx^ndim, cell centres x_d = xmin[d] + (i_d + 1/2) dx. */
int oracle_observables(int ndim, const int64_t *n, double dx, const double *xmin,
                       const double *psi, double x_b, double *out)
{
    const int axis[3] = {0, 1, 2};
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, 0)) return -1;
    nsum_t tot = {0, 0}, mom[3] = {{0, 0}, {0, 0}, {0, 0}}, tr = {0, 0};
    const zd *p = (const zd *)psi;
    for (int64_t i2 = 0; i2 < g.n[2]; ++i2)
        for (int64_t i1 = 0; i1 < g.n[1]; ++i1)
            for (int64_t i0 = 0; i0 < g.n[0]; ++i0) {
                const int64_t s = site_at(&g, i0, i1, i2);
                double rho = 0.0;
                for (int k = 0; k < 4; ++k) {
                    const double re = creal(p[4 * s + k]), im = cimag(p[4 * s + k]);
                    rho += re * re + im * im;
                }
                const int64_t ic[3] = {i0, i1, i2};
                nsum_add(&tot, rho);
                for (int d = 0; d < ndim; ++d) {
                    const double xd = xmin[d] + ((double)ic[d] + 0.5) * dx;
                    nsum_add(&mom[d], xd * rho);
                }
                const double x0 = xmin[0] + ((double)i0 + 0.5) * dx;
                if (x0 > x_b) nsum_add(&tr, rho);
            }
    const double dV = pow(dx, ndim);
    const double S = nsum_get(&tot);
    out[0] = dV * S;
    for (int d = 0; d < 3; ++d) out[1 + d] = (d < ndim && S != 0.0) ? nsum_get(&mom[d]) / S : 0.0;
    out[4] = dV * nsum_get(&tr);
    return 0;
}

/* Gradient of L = P_T(psi_N) = dV sum_{x_0 > x_b} |psi_N|^2 with respect to
 * the potential V at every cell:
 *     dL/dV(x) = 2 dt dV sum_{n=1..N} Im(lambda_n(x)^H psi_n(x)),
 *     lambda_N = M psi_N (M = indicator of x_0 > x_b),
 *     lambda_{n-1} = S^H lambda_n.
 * psi_n are recomputed forward from checkpoints stored every `ckpt` steps.
 * Outputs: dLdV (nsites), psiN (4 nsites complex, may be NULL), loss. */
int oracle_grad(int ndim, const int64_t *n, const int *axis, int bc,
                double dx, const double *xmin, double dt, double c, double m,
                const double *V, const double *psi0, int64_t nsteps, double x_b,
                int64_t ckpt, double *dLdV, double *psiN, double *loss, int nthreads)
{
    grid_t g;
    if (grid_from_args(&g, ndim, n, axis, bc) || nsteps < 1 || ckpt < 1) return -1;
    build_matrices();
    set_threads(nthreads);
    const int64_t ns = nsites(&g);
    const size_t sbytes = (size_t)ns * 4 * sizeof(zd);
    const int64_t nck = (nsteps + ckpt - 1) / ckpt;
    zd *cks = (zd *)malloc(sbytes * (size_t)nck);
    zd *seg = (zd *)malloc(sbytes * (size_t)(ckpt + 1));
    zd *cur = (zd *)malloc(sbytes);
    zd *lam = (zd *)malloc(sbytes);
    zd *tmp = (zd *)malloc(sbytes);
    double *Q = (double *)calloc((size_t)ns, sizeof(double));
    if (!cks || !seg || !cur || !lam || !tmp || !Q) {
        free(cks); free(seg); free(cur); free(lam); free(tmp); free(Q);
        return -2;
    }
    /* forward pass with checkpoints psi_{k ckpt} */
    memcpy(cur, psi0, sbytes);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (s % ckpt == 0) memcpy(cks + (size_t)(s / ckpt) * ns * 4, cur, sbytes);
        step_once(&g, cur, tmp, V, dt, c, m);
    }
    if (psiN) memcpy(psiN, cur, sbytes);
    /* loss and seed lambda_N = M psi_N */
    const double dV = pow(dx, ndim);
    nsum_t L = {0, 0};
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t i0 = s % g.n[0];
        const double x0 = xmin[0] + ((double)i0 + 0.5) * dx;
        const int inside = x0 > x_b;
        for (int k = 0; k < 4; ++k) {
            lam[4 * s + k] = inside ? cur[4 * s + k] : 0.0;
            if (inside) {
                const double re = creal(cur[4 * s + k]), im = cimag(cur[4 * s + k]);
                nsum_add(&L, re * re + im * im);
            }
        }
    }
    *loss = dV * nsum_get(&L);
    /* backward over segments [k ckpt, min((k+1) ckpt, N)] */
    for (int64_t k = nck - 1; k >= 0; --k) {
        const int64_t n0 = k * ckpt;
        const int64_t n1 = (n0 + ckpt < nsteps) ? n0 + ckpt : nsteps;
        memcpy(seg, cks + (size_t)k * ns * 4, sbytes);             /* psi_{n0} */
        for (int64_t j = 1; j <= n1 - n0; ++j) {                   /* psi_{n0+j} */
            memcpy(seg + (size_t)j * ns * 4, seg + (size_t)(j - 1) * ns * 4, sbytes);
            step_once(&g, seg + (size_t)j * ns * 4, tmp, V, dt, c, m);
        }
        for (int64_t nn = n1; nn > n0; --nn) {
            const zd *pn = seg + (size_t)(nn - n0) * ns * 4;
            #pragma omp parallel for schedule(static)
            for (int64_t s = 0; s < ns; ++s) {
                zd acc = 0;
                for (int kk = 0; kk < 4; ++kk) acc += conj(lam[4 * s + kk]) * pn[4 * s + kk];
                Q[s] += cimag(acc);
            }
            adjoint_once(&g, lam, tmp, V, dt, c, m);               /* lambda_{nn-1} */
        }
    }
    for (int64_t s = 0; s < ns; ++s) dLdV[s] = 2.0 * dt * dV * Q[s];
    free(cks); free(seg); free(cur); free(lam); free(tmp); free(Q);
    return 0;
}
