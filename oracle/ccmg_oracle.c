/*
 * ccmg_oracle.c -- plain, slow CPU oracle for the cell-centered geometric
 * multigrid solver of the electric-potential Poisson problem in
 * D. Bartuschat and U. Ruede, "Parallel Multiphysics Simulations of Charged
 * Particles in Microfluidic Flows" (arXiv:1410.6609).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation; the two meet only
 * through seeded inputs.
 *
 * What it computes (FP64 unless noted; arrays [nz][ny][nx], x fastest; cell
 * (i,j,k) has centre ((i+1/2)h, (j+1/2)h, (k+1/2)h)):
 *   - Poisson's equation -Lap(phi) = rho/eps (Sec. 2.4, Eq. Poisson), finite
 *     volume 7-point stencil (1/h^2)[6; -1 per face neighbour] (Sec. 2.4).
 *   - Dirichlet and Neumann boundary conditions folded into stencil and RHS
 *     at near-boundary cells (Sec. 2.4, "Boundary conditions"), applied
 *     independently per direction (Sec. 5.3): a Dirichlet face adds +1 to the
 *     stencil centre and 2 g_d / h^2 to the RHS, a Neumann face (g_n = outward
 *     normal derivative) adds -1 to the centre and g_n / h to the RHS.
 *   - Naive volume-mapped charge deposition (Sec. 2.4, "Subsampling"): a cell
 *     belongs to a sphere if its centre lies in the closed ball; the sphere's
 *     charge is spread evenly over its cells, rho = q / (n_s h^3).
 *   - Cell-centered multigrid (Sec. 3, Sec. 5.3): 2x2x2 coarsening, averaging
 *     restriction, nearest-neighbour prolongation with the coarse correction
 *     magnified by omega (about 2, Sec. 3), Galerkin coarse operators, which
 *     for this stencil equal s_l * (integer stencil with the same per-face
 *     centre entries), s_l = 1/(2^l h^2); red-black Gauss-Seidel smoothing;
 *     conjugate gradients on the coarsest grid; V(nu1,nu2) cycles repeated
 *     while the residual L2 norm is not below the tolerance (Alg. 1).
 *   - FP32-in-FP64 iterative refinement and the adjoint solve with the gradient
 *     with respect to the sphere charges (extensions of the method; the
 *     operator is symmetric because folding only changes diagonal entries).
 *
 * Parity pins: see the oracle tests.  Per-cycle multigrid iterates are not
 * printed in the paper, so the cycle itself is pinned only by independent
 * cross-checks (dense solves, explicit sparse Galerkin cycles, closed forms).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no contraction, so
 * every operation rounds exactly as written).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_DIRICHLET 0
#define OR_NEUMANN 1
#define OR_PERIODIC 2   /* both faces of an axis; only the variable-permittivity
                           operator and the gradient/force functions take it */
#define OR_MAXLEVELS 16

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_NONFINITE (-5)
#define OR_E_NOCONV (-6)

typedef struct {
    int nx, ny, nz;
    double s;      /* operator scale 1/(2^l h0^2) */
    int kind[6];   /* x-, x+, y-, y+, z-, z+ */
    double k2;     /* reaction coefficient kappa^2 of the linearised Poisson-Boltzmann
                      operator (0: Poisson); the same on every level, see below */
} or_level;

#define IDX(L, i, j, k) ((((size_t)(k)) * (size_t)(L)->ny + (size_t)(j)) * (size_t)(L)->nx + (size_t)(i))

static size_t or_cells(const or_level* L) { return (size_t)L->nx * L->ny * L->nz; }

/* centre entry of the integer stencil: 6, +1 per Dirichlet face of the cell,
 * -1 per Neumann face (Sec. 2.4: Dirichlet gives beta - alpha, Neumann
 * beta + alpha with alpha = -1). */
static int face_shift(int kind) { return kind == OR_DIRICHLET ? 1 : -1; }

static int or_diag(const or_level* L, int i, int j, int k)
{
    int d = 6;
    if (i == 0)         d += face_shift(L->kind[0]);
    if (i == L->nx - 1) d += face_shift(L->kind[1]);
    if (j == 0)         d += face_shift(L->kind[2]);
    if (j == L->ny - 1) d += face_shift(L->kind[3]);
    if (k == 0)         d += face_shift(L->kind[4]);
    if (k == L->nz - 1) d += face_shift(L->kind[5]);
    return d;
}

static or_level make_level(int nx, int ny, int nz, double h, int level, const int* kinds)
{
    or_level L;
    L.nx = nx; L.ny = ny; L.nz = nz;
    L.s = 1.0 / (ldexp(1.0, level) * h * h);
    for (int f = 0; f < 6; ++f) L.kind[f] = kinds[f];
    L.k2 = 0.0;
    return L;
}

/* ---- the level operations, for double and for float ---------------------- */
#define REAL double
#define FN(name) name##_d
#include "levelops.inc"
#undef REAL
#undef FN
#define REAL float
#define FN(name) name##_f
#include "levelops.inc"
#undef REAL
#undef FN

static double norm2_d(size_t n, const double* v)
{
    double acc = 0.0;
    for (size_t c = 0; c < n; ++c) acc += v[c] * v[c];
    return sqrt(acc);
}

static double dot_d(size_t n, const double* a, const double* b)
{
    double acc = 0.0;
    for (size_t c = 0; c < n; ++c) acc += a[c] * b[c];
    return acc;
}

/* Unpreconditioned conjugate gradients on A_l x = b (Sec. 5.3: the coarsest
 * grid is solved by CG), started from x = 0, stopped when the recursively
 * updated residual satisfies ||r|| <= rtol ||b|| or after maxit iterations.
 * Returns the iteration count. */
static int cg_d(const or_level* L, const double* b, double* x, double rtol, int maxit)
{
    const size_t n = or_cells(L);
    double* r = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    for (size_t c = 0; c < n; ++c) { x[c] = 0.0; r[c] = b[c]; p[c] = b[c]; }
    const double bnorm = norm2_d(n, b);
    double rr = dot_d(n, r, r);
    int it = 0;
    if (bnorm > 0.0) {
        while (it < maxit) {
            apply_d(L, p, q);
            const double alpha = rr / dot_d(n, p, q);
            for (size_t c = 0; c < n; ++c) x[c] += alpha * p[c];
            for (size_t c = 0; c < n; ++c) r[c] -= alpha * q[c];
            const double rr_new = dot_d(n, r, r);
            ++it;
            if (sqrt(rr_new) <= rtol * bnorm) break;
            const double beta = rr_new / rr;
            for (size_t c = 0; c < n; ++c) p[c] = r[c] + beta * p[c];
            rr = rr_new;
        }
    }
    free(r); free(p); free(q);
    return it;
}

/* ---- multigrid hierarchy ---------------------------------------------------- */
typedef struct {
    int nlev;
    or_level lev[OR_MAXLEVELS];
    int nu1, nu2;
    double omega;
    double cg_rtol;
    int cg_maxit;
    /* per-level storage; level 0 of phi/b belongs to the caller */
    double* phi[OR_MAXLEVELS];
    double* b[OR_MAXLEVELS];
    double* r[OR_MAXLEVELS];
    float* phif[OR_MAXLEVELS];
    float* bf[OR_MAXLEVELS];
    float* rf[OR_MAXLEVELS];
    int cg_iters_last;
} or_hier;

static int hier_init(or_hier* H, int nx, int ny, int nz, double h, const int* kinds, int levels,
                     int nu1, int nu2, double omega, double cg_rtol, int cg_maxit, int want_f32)
{
    memset(H, 0, sizeof(*H));
    if (levels < 1 || levels > OR_MAXLEVELS) return OR_E_ARG;
    const int div = 1 << (levels - 1);
    if (nx % div || ny % div || nz % div) return OR_E_ARG;
    H->nlev = levels; H->nu1 = nu1; H->nu2 = nu2; H->omega = omega;
    H->cg_rtol = cg_rtol; H->cg_maxit = cg_maxit;
    for (int l = 0; l < levels; ++l) {
        H->lev[l] = make_level(nx >> l, ny >> l, nz >> l, h, l, kinds);
        const size_t n = or_cells(&H->lev[l]);
        H->r[l] = (double*)calloc(n, sizeof(double));
        if (l > 0) {
            H->phi[l] = (double*)calloc(n, sizeof(double));
            H->b[l] = (double*)calloc(n, sizeof(double));
        }
        if (want_f32) {
            H->phif[l] = (float*)calloc(n, sizeof(float));
            H->bf[l] = (float*)calloc(n, sizeof(float));
            H->rf[l] = (float*)calloc(n, sizeof(float));
        }
    }
    return OR_OK;
}

static void hier_free(or_hier* H)
{
    for (int l = 0; l < H->nlev; ++l) {
        free(H->r[l]);
        if (l > 0) { free(H->phi[l]); free(H->b[l]); }
        free(H->phif[l]); free(H->bf[l]); free(H->rf[l]);
    }
}

/* Coarsest-level solve: CG for the correction e of the current iterate, i.e.
 * A e = b - A phi from e = 0, then phi += e.  On coarse levels phi is zero on
 * entry, so this is CG on A phi = b. */
static void coarse_solve_d(or_hier* H, int l)
{
    const or_level* L = &H->lev[l];
    const size_t n = or_cells(L);
    double* e = (double*)calloc(n, sizeof(double));
    residual_d(L, H->phi[l], H->b[l], H->r[l]);
    H->cg_iters_last = cg_d(L, H->r[l], e, H->cg_rtol, H->cg_maxit);
    for (size_t c = 0; c < n; ++c) H->phi[l][c] += e[c];
    free(e);
}

/* V(nu1,nu2)-cycle on level l (Sec. 3): pre-smooth, restrict the residual,
 * recurse from a zero coarse guess, prolongate with the magnified correction,
 * post-smooth.  The coarsest level is solved by CG. */
static void vcycle_d(or_hier* H, int l)
{
    const or_level* L = &H->lev[l];
    if (l == H->nlev - 1) { coarse_solve_d(H, l); return; }
    for (int s = 0; s < H->nu1; ++s) rbgs_sweep_d(L, H->phi[l], H->b[l]);
    residual_d(L, H->phi[l], H->b[l], H->r[l]);
    restrict_avg_d(L, H->r[l], H->b[l + 1]);
    memset(H->phi[l + 1], 0, or_cells(&H->lev[l + 1]) * sizeof(double));
    vcycle_d(H, l + 1);
    prolong_add_d(L, H->phi[l + 1], H->omega, H->phi[l]);
    for (int s = 0; s < H->nu2; ++s) rbgs_sweep_d(L, H->phi[l], H->b[l]);
}

/* FP32 cycle: the same steps in float arithmetic; the coarsest level is still
 * solved by FP64 CG on the float right-hand side. */
static void vcycle_f(or_hier* H, int l)
{
    const or_level* L = &H->lev[l];
    const size_t n = or_cells(L);
    if (l == H->nlev - 1) {
        double* bd = (double*)malloc(n * sizeof(double));
        double* x = (double*)malloc(n * sizeof(double));
        /* correction of the current float iterate, computed in FP64 */
        for (size_t c = 0; c < n; ++c) bd[c] = (double)H->bf[l][c];
        double* pd = (double*)malloc(n * sizeof(double));
        for (size_t c = 0; c < n; ++c) pd[c] = (double)H->phif[l][c];
        residual_d(L, pd, bd, H->r[l]);
        H->cg_iters_last = cg_d(L, H->r[l], x, H->cg_rtol, H->cg_maxit);
        for (size_t c = 0; c < n; ++c) H->phif[l][c] = (float)(pd[c] + x[c]);
        free(bd); free(x); free(pd);
        return;
    }
    for (int s = 0; s < H->nu1; ++s) rbgs_sweep_f(L, H->phif[l], H->bf[l]);
    residual_f(L, H->phif[l], H->bf[l], H->rf[l]);
    restrict_avg_f(L, H->rf[l], H->bf[l + 1]);
    memset(H->phif[l + 1], 0, or_cells(&H->lev[l + 1]) * sizeof(float));
    vcycle_f(H, l + 1);
    prolong_add_f(L, H->phif[l + 1], (float)H->omega, H->phif[l]);
    for (int s = 0; s < H->nu2; ++s) rbgs_sweep_f(L, H->phif[l], H->bf[l]);
}

/* ============================ exported API ==================================== */

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_diag_at(int nx, int ny, int nz, const int* kinds, int i, int j, int k)
{
    or_level L = make_level(nx, ny, nz, 1.0, 0, kinds);
    return or_diag(&L, i, j, k);
}

void or_apply(int nx, int ny, int nz, double h, int level, const int* kinds,
              const double* phi, double* out)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    apply_d(&L, phi, out);
}

void or_residual(int nx, int ny, int nz, double h, int level, const int* kinds,
                 const double* phi, const double* b, double* r)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    residual_d(&L, phi, b, r);
}

double or_norm2(long long n, const double* v) { return norm2_d((size_t)n, v); }

void or_rbgs_sweep(int nx, int ny, int nz, double h, int level, const int* kinds,
                   double* phi, const double* b)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    rbgs_sweep_d(&L, phi, b);
}

void or_restrict(int nx, int ny, int nz, const double* r, double* bc)
{
    static const int k0[6] = {0, 0, 0, 0, 0, 0};
    or_level L = make_level(nx, ny, nz, 1.0, 0, k0);
    restrict_avg_d(&L, r, bc);
}

void or_prolong_add(int nx, int ny, int nz, const double* ec, double omega, double* phi)
{
    static const int k0[6] = {0, 0, 0, 0, 0, 0};
    or_level L = make_level(nx, ny, nz, 1.0, 0, k0);
    prolong_add_d(&L, ec, omega, phi);
}

int or_cg(int nx, int ny, int nz, double h, int level, const int* kinds,
          const double* b, double* x, double rtol, int maxit)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    return cg_d(&L, b, x, rtol, maxit);
}

/* RHS adaptation to the boundary conditions on the finest level (Sec. 2.4 and
 * Sec. 5.3): b = f plus, for every boundary face a cell touches, 2 g_d / h^2
 * (Dirichlet, value on the face) or g_n / h (Neumann, outward derivative). */
void or_fold(int nx, int ny, int nz, double h, const int* kinds, const double* values,
             const double* f, double* b)
{
    or_level L = make_level(nx, ny, nz, h, 0, kinds);
    double term[6];
    for (int fc = 0; fc < 6; ++fc)
        term[fc] = kinds[fc] == OR_DIRICHLET ? 2.0 * values[fc] / (h * h) : values[fc] / h;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = IDX(&L, i, j, k);
                double v = f[c];
                if (i == 0)      v += term[0];
                if (i == nx - 1) v += term[1];
                if (j == 0)      v += term[2];
                if (j == ny - 1) v += term[3];
                if (k == 0)      v += term[4];
                if (k == nz - 1) v += term[5];
                b[c] = v;
            }
}

/* Boundary folding with per-cell boundary values (Sec. 2.4, "Boundary
 * conditions"; Sec. 6.3 sets the Dirichlet values of the validation domain to
 * the analytic potential at the boundary).  face[fc] == NULL uses the
 * constant values[fc]; otherwise it holds one value per boundary face of the
 * cells on that side: x faces [nz][ny], y faces [nz][nx], z faces [ny][nx]
 * (the first index slowest).  The value is the boundary value g at the face
 * centre (Dirichlet) or the outward normal derivative there (Neumann). */
void or_fold_field(int nx, int ny, int nz, double h, const int* kinds, const double* values,
                   const double* const* face, const double* f, double* b)
{
    or_level L = make_level(nx, ny, nz, h, 0, kinds);
    for (size_t c = 0; c < or_cells(&L); ++c) b[c] = f[c];
    for (int fc = 0; fc < 6; ++fc) {
        const int ax = fc / 2, hi = fc % 2;
        const int n0 = ax == 0 ? ny : nx;          /* fastest index on the face */
        const int n1 = ax == 2 ? ny : nz;
        for (int v = 0; v < n1; ++v)
            for (int u = 0; u < n0; ++u) {
                const double g = face[fc] ? face[fc][(size_t)v * n0 + u] : values[fc];
                const double t = kinds[fc] == OR_DIRICHLET ? 2.0 * g / (h * h) : g / h;
                int i, j, k;
                if (ax == 0)      { i = hi ? nx - 1 : 0; j = u; k = v; }
                else if (ax == 1) { j = hi ? ny - 1 : 0; i = u; k = v; }
                else              { k = hi ? nz - 1 : 0; i = u; j = v; }
                b[IDX(&L, i, j, k)] += t;
            }
    }
}

/* Is the centre of cell (i,j,k) inside the closed ball (c, R)?  Evaluated as
 * dx*dx + dy*dy + dz*dz <= R*R, left to right, no contraction. */
static int inside_ball(int i, int j, int k, double h, const double* c, double R)
{
    const double dx = ((double)i + 0.5) * h - c[0];
    const double dy = ((double)j + 0.5) * h - c[1];
    const double dz = ((double)k + 0.5) * h - c[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    return d2 <= R * R;
}

/* candidate index range of one axis: every cell whose centre can be within R
 * of c, widened by one cell, clipped to the grid */
static void axis_range(double c, double R, double h, int n, int* lo, int* hi)
{
    int a = (int)floor((c - R) / h - 0.5) - 1;
    int b = (int)ceil((c + R) / h - 0.5) + 1;
    *lo = a < 0 ? 0 : a;
    *hi = b > n - 1 ? n - 1 : b;
}

static long long sphere_count(int nx, int ny, int nz, double h, const double* c, double R)
{
    int ilo, ihi, jlo, jhi, klo, khi;
    axis_range(c[0], R, h, nx, &ilo, &ihi);
    axis_range(c[1], R, h, ny, &jlo, &jhi);
    axis_range(c[2], R, h, nz, &klo, &khi);
    long long cnt = 0;
    for (int k = klo; k <= khi; ++k)
        for (int j = jlo; j <= jhi; ++j)
            for (int i = ilo; i <= ihi; ++i)
                cnt += inside_ball(i, j, k, h, c, R);
    return cnt;
}

/* Charge deposition (Sec. 2.4, naive volume mapping with the charge spread
 * evenly over the covered cells): f = rho/eps, f_c = sum over spheres s that
 * cover cell c of q_s / (eps n_s h^3).  Spheres are added in index order.
 * counts[s] receives n_s (may be NULL).  A sphere that covers no cell centre
 * deposits nothing. */
void or_deposit(int nx, int ny, int nz, double h, int n, const double* centers,
                const double* radii, const double* q, double eps, double* f, long long* counts)
{
    const or_level L = make_level(nx, ny, nz, h, 0, (const int[6]){0, 0, 0, 0, 0, 0});
    memset(f, 0, or_cells(&L) * sizeof(double));
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        const long long ns = sphere_count(nx, ny, nz, h, c, R);
        if (counts) counts[s] = ns;
        if (ns == 0) continue;
        const double val = q[s] / (eps * (double)ns * h * h * h);
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i)
                    if (inside_ball(i, j, k, h, c, R)) f[IDX(&L, i, j, k)] += val;
    }
}

/* Gradient of a loss with respect to the sphere charges, given the adjoint
 * lambda = dL/df:  dL/dq_s = sum over covered cells of lambda_c / (eps n_s h^3). */
void or_dq(int nx, int ny, int nz, double h, int n, const double* centers, const double* radii,
           double eps, const double* lambda, double* dq)
{
    const or_level L = make_level(nx, ny, nz, h, 0, (const int[6]){0, 0, 0, 0, 0, 0});
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        const long long ns = sphere_count(nx, ny, nz, h, c, R);
        if (ns == 0) { dq[s] = 0.0; continue; }
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        double acc = 0.0;
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i)
                    if (inside_ball(i, j, k, h, c, R)) acc += lambda[IDX(&L, i, j, k)];
        dq[s] = acc / (eps * (double)ns * h * h * h);
    }
}

/* Sub-sampled deposition (Sec. 2.4, "Subsampling"): each cell is divided
 * equidistantly into sf^3 sub-cells, and its overlap ratio w_{s,c} with
 * sphere s is the fraction of sub-cell centres inside the closed ball
 * (sub-cell centre ((i + (a + 1/2)/sf) h, ...), a = 0..sf-1; same
 * left-to-right, uncontracted distance test as above).
 *   mode 0 (spread):  f_c += q_s w_{s,c} / (eps W_s h^3), W_s = sum_c w_{s,c}
 *                     (the charge is conserved exactly);
 *   mode 1 (volume):  f_c += q_s w_{s,c} / (eps V_s), V_s = 4/3 pi R_s^3
 *                     (the paper's density charge/volume times the ratio).
 * weight_sum[s] receives W_s (may be NULL).  Spheres are added in index
 * order; a sphere with W_s = 0 deposits nothing in mode 0. */
static int sub_inside(int i, int j, int k, int a, int b, int c, int sf, double h, const double* ctr, double R)
{
    const double dx = ((double)i + ((double)a + 0.5) / (double)sf) * h - ctr[0];
    const double dy = ((double)j + ((double)b + 0.5) / (double)sf) * h - ctr[1];
    const double dz = ((double)k + ((double)c + 0.5) / (double)sf) * h - ctr[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    return d2 <= R * R;
}

static int sub_count(int i, int j, int k, int sf, double h, const double* ctr, double R)
{
    int cnt = 0;
    for (int c = 0; c < sf; ++c)
        for (int b = 0; b < sf; ++b)
            for (int a = 0; a < sf; ++a) cnt += sub_inside(i, j, k, a, b, c, sf, h, ctr, R);
    return cnt;
}

static double cell_ratio(int i, int j, int k, int sf, double h, const double* ctr, double R)
{
    return (double)sub_count(i, j, k, sf, h, ctr, R) / (double)(sf * sf * sf);
}

/* W_s = sum_c w_{s,c}, formed as (total sub-cell count) / sf^3: the same sum
 * with a single rounding, independent of the summation order. */
static double sphere_weight(int nx, int ny, int nz, double h, const double* ctr, double R, int sf)
{
    int ilo, ihi, jlo, jhi, klo, khi;
    axis_range(ctr[0], R, h, nx, &ilo, &ihi);
    axis_range(ctr[1], R, h, ny, &jlo, &jhi);
    axis_range(ctr[2], R, h, nz, &klo, &khi);
    long long total = 0;
    for (int k = klo; k <= khi; ++k)
        for (int j = jlo; j <= jhi; ++j)
            for (int i = ilo; i <= ihi; ++i) total += sub_count(i, j, k, sf, h, ctr, R);
    return (double)total / (double)(sf * sf * sf);
}

static double sphere_norm(int mode, double eps, double W, double R, double h)
{
    if (mode == 0) return eps * W * h * h * h;
    return eps * ((4.0 / 3.0) * M_PI * R * R * R);
}

void or_deposit_sub(int nx, int ny, int nz, double h, int n, const double* centers, const double* radii,
                    const double* q, double eps, int sf, int mode, double* f, double* weight_sum)
{
    const or_level L = make_level(nx, ny, nz, h, 0, (const int[6]){0, 0, 0, 0, 0, 0});
    memset(f, 0, or_cells(&L) * sizeof(double));
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        const double W = sphere_weight(nx, ny, nz, h, c, R, sf);
        if (weight_sum) weight_sum[s] = W;
        if (W == 0.0) continue;
        const double norm = sphere_norm(mode, eps, W, R, h);
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i) {
                    const double w = cell_ratio(i, j, k, sf, h, c, R);
                    if (w > 0.0) f[IDX(&L, i, j, k)] += q[s] * w / norm;
                }
    }
}

/* Gradient of a loss with respect to the charges for the sub-sampled
 * deposition: dL/dq_s = sum_c lambda_c w_{s,c} / norm_s. */
void or_dq_sub(int nx, int ny, int nz, double h, int n, const double* centers, const double* radii, double eps,
               int sf, int mode, const double* lambda, double* dq)
{
    const or_level L = make_level(nx, ny, nz, h, 0, (const int[6]){0, 0, 0, 0, 0, 0});
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        const double W = sphere_weight(nx, ny, nz, h, c, R, sf);
        if (W == 0.0 && mode == 0) { dq[s] = 0.0; continue; }
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        double acc = 0.0;
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i) {
                    const double w = cell_ratio(i, j, k, sf, h, c, R);
                    if (w > 0.0) acc += lambda[IDX(&L, i, j, k)] * w;
                }
        dq[s] = acc / sphere_norm(mode, eps, W, R, h);
    }
}

/* ---- electrostatic force on the spheres (Sec. 2.4, "Coulomb force") ------- */

/* Potential at (i,j,k), or the ghost value the boundary treatment implies
 * when the cell lies one layer outside the domain across one face (Sec. 2.4:
 * Dirichlet extrapolates phi_0 = 2 g - phi_1, Neumann takes
 * phi_0 - phi_1 = h g_n with g_n the outward normal derivative).  The face
 * value comes from face[fc] (per cell) when given, else values[fc]. */
static int axis_periodic(const int* kinds, int a) { return kinds[2 * a] == OR_PERIODIC; }

/* indices on periodic axes taken modulo the extent (Sec. 2.4: periodic
 * boundaries cyclically extend the domain) */
static void wrap_periodic(const or_level* L, const int* kinds, int* i, int* j, int* k)
{
    if (axis_periodic(kinds, 0)) *i = (*i + L->nx) % L->nx;
    if (axis_periodic(kinds, 1)) *j = (*j + L->ny) % L->ny;
    if (axis_periodic(kinds, 2)) *k = (*k + L->nz) % L->nz;
}

static double phi_or_ghost(const or_level* L, const double* phi, const int* kinds, const double* values,
                           const double* const* face, double h, int i, int j, int k)
{
    wrap_periodic(L, kinds, &i, &j, &k);
    int fc = -1, ii = i, jj = j, kk = k;
    if (i < 0)             { fc = 0; ii = 0; }
    else if (i >= L->nx)   { fc = 1; ii = L->nx - 1; }
    else if (j < 0)        { fc = 2; jj = 0; }
    else if (j >= L->ny)   { fc = 3; jj = L->ny - 1; }
    else if (k < 0)        { fc = 4; kk = 0; }
    else if (k >= L->nz)   { fc = 5; kk = L->nz - 1; }
    const double in = phi[IDX(L, ii, jj, kk)];
    if (fc < 0) return in;
    double g;
    if (face && face[fc]) {
        const size_t at = fc < 2 ? (size_t)kk * L->ny + jj : fc < 4 ? (size_t)kk * L->nx + ii : (size_t)jj * L->nx + ii;
        g = face[fc][at];
    } else {
        g = values[fc];
    }
    return kinds[fc] == OR_DIRICHLET ? 2.0 * g - in : in + h * g;
}

/* all 18 D3Q19 neighbours exist: away from every non-periodic boundary */
static int d3q19_inside(const or_level* L, const int* kinds, int i, int j, int k)
{
    return (axis_periodic(kinds, 0) || (i > 0 && i < L->nx - 1)) &&
           (axis_periodic(kinds, 1) || (j > 0 && j < L->ny - 1)) &&
           (axis_periodic(kinds, 2) || (k > 0 && k < L->nz - 1));
}

/* Gradient of phi at cell (i,j,k), second order: the isotropic D3Q19 lattice
 * gradient grad = (1/w_1) sum_q w_q phi(x + h c_q) c_q / h over the 18
 * non-rest directions (w_1 = 1/3 the rest weight, w = 1/18 along the axes,
 * 1/36 along the face diagonals) where all 18 neighbours are inside the
 * domain; elsewhere the D3Q7 central differences with the boundary ghost
 * values. */
static void gradient_at(const or_level* L, const double* phi, const int* kinds, const double* values,
                        const double* const* face, double h, int i, int j, int k, double g[3])
{
    const int inner = d3q19_inside(L, kinds, i, j, k);
    g[0] = g[1] = g[2] = 0.0;
    if (inner) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nnz == 0 || nnz == 3) continue;   /* rest and cube-corner directions are not in D3Q19 */
                    const double w = nnz == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                    int a = i + dx, b = j + dy, c = k + dz;
                    wrap_periodic(L, kinds, &a, &b, &c);
                    const double v = phi[IDX(L, a, b, c)];
                    g[0] += w * v * (double)dx;
                    g[1] += w * v * (double)dy;
                    g[2] += w * v * (double)dz;
                }
        for (int a = 0; a < 3; ++a) g[a] = 3.0 * g[a] / h;
        return;
    }
    g[0] = (phi_or_ghost(L, phi, kinds, values, face, h, i + 1, j, k) -
            phi_or_ghost(L, phi, kinds, values, face, h, i - 1, j, k)) / (2.0 * h);
    g[1] = (phi_or_ghost(L, phi, kinds, values, face, h, i, j + 1, k) -
            phi_or_ghost(L, phi, kinds, values, face, h, i, j - 1, k)) / (2.0 * h);
    g[2] = (phi_or_ghost(L, phi, kinds, values, face, h, i, j, k + 1) -
            phi_or_ghost(L, phi, kinds, values, face, h, i, j, k - 1)) / (2.0 * h);
}

void or_gradient(int nx, int ny, int nz, double h, const int* kinds, const double* values,
                 const double* const* face, const double* phi, double* grad /* [3][nz][ny][nx] */)
{
    const or_level L = make_level(nx, ny, nz, h, 0, kinds);
    const size_t n = or_cells(&L);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double g[3];
                gradient_at(&L, phi, kinds, values, face, h, i, j, k, g);
                const size_t c = IDX(&L, i, j, k);
                grad[c] = g[0];
                grad[n + c] = g[1];
                grad[2 * n + c] = g[2];
            }
}

/* F_s = -h^3 sum_b grad(phi)(x_b) rho_s(x_b) (Eq. ElectrostatForce), with the
 * sphere's own charge density of the sub-sampled deposition:
 * rho_s = q_s w_{s,b} / (W_s h^3) (mode 0) or q_s w_{s,b} / (4/3 pi R^3)
 * (mode 1).  force[3s..3s+2] = F_s; 0 for a sphere covering no sub-cell. */
void or_coulomb(int nx, int ny, int nz, double h, const int* kinds, const double* values,
                const double* const* face, const double* phi, int n, const double* centers, const double* radii,
                const double* q, int sf, int mode, double* force)
{
    const or_level L = make_level(nx, ny, nz, h, 0, kinds);
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        double* F = force + 3 * (size_t)s;
        F[0] = F[1] = F[2] = 0.0;
        const double W = sphere_weight(nx, ny, nz, h, c, R, sf);
        if (W == 0.0) continue;
        const double norm = sphere_norm(mode, 1.0, W, R, h);
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i) {
                    const double w = cell_ratio(i, j, k, sf, h, c, R);
                    if (w == 0.0) continue;
                    double g[3];
                    gradient_at(&L, phi, kinds, values, face, h, i, j, k, g);
                    for (int a = 0; a < 3; ++a) acc[a] += g[a] * w;
                }
        for (int a = 0; a < 3; ++a) F[a] = -(h * h * h) * acc[a] * q[s] / norm;
    }
}

/* Adjoint of the force for a loss L(F) with gF[3s..3s+2] = dL/dF_s.  The force
 * is affine in phi: F_s = -h^3 (q_s / norm_s) sum_b w_{s,b} (G phi)_b, G the
 * gradient above (its boundary ghosts add constants).  Outputs:
 *   mu = dL/dphi = sum_s -h^3 (q_s / norm_s) G_lin^T (w_s (x) gF_s), a field
 *        (G_lin: G without the boundary constants);
 *   direct[s] = gF_s . F_s / q_s computed without dividing, i.e. the
 *        derivative of L through the prefactor q_s at fixed phi.
 * dL/dq then adds the charge gradient of the deposition for lambda = A^-1 mu. */
static void scatter_gradient_transpose(const or_level* L, const int* kinds, double h, int i, int j, int k,
                                       const double v[3], double* mu)
{
    if (d3q19_inside(L, kinds, i, j, k)) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nnz == 0 || nnz == 3) continue;
                    const double w = nnz == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                    const double cv = (double)dx * v[0] + (double)dy * v[1] + (double)dz * v[2];
                    int a = i + dx, b = j + dy, c = k + dz;
                    wrap_periodic(L, kinds, &a, &b, &c);
                    mu[IDX(L, a, b, c)] += 3.0 * w * cv / h;
                }
        return;
    }
    /* D3Q7: component a is (phi(+) - phi(-)) / (2h); a ghost is a phi_b + const
     * with a = -1 (Dirichlet) or +1 (Neumann) */
    const int n[3] = {L->nx, L->ny, L->nz};
    const int c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        for (int side = -1; side <= 1; side += 2) {
            int p[3] = {i, j, k};
            p[a] += side;
            wrap_periodic(L, kinds, &p[0], &p[1], &p[2]);
            const double coef = (double)side * v[a] / (2.0 * h);
            if (p[a] >= 0 && p[a] < n[a]) {
                mu[IDX(L, p[0], p[1], p[2])] += coef;
            } else {
                const int fc = 2 * a + (side > 0 ? 1 : 0);
                const double ga = kinds[fc] == OR_DIRICHLET ? -1.0 : 1.0;
                mu[IDX(L, c[0], c[1], c[2])] += coef * ga;
            }
        }
    }
}

void or_coulomb_adjoint(int nx, int ny, int nz, double h, const int* kinds, const double* values,
                        const double* const* face, const double* phi, int n, const double* centers,
                        const double* radii, const double* q, int sf, int mode, const double* gF, double* mu,
                        double* direct)
{
    const or_level L = make_level(nx, ny, nz, h, 0, kinds);
    memset(mu, 0, or_cells(&L) * sizeof(double));
    for (int s = 0; s < n; ++s) {
        const double* c = centers + 3 * (size_t)s;
        const double R = radii[s];
        direct[s] = 0.0;
        const double W = sphere_weight(nx, ny, nz, h, c, R, sf);
        if (W == 0.0) continue;
        const double norm = sphere_norm(mode, 1.0, W, R, h);
        const double pre = -(h * h * h) / norm;
        int ilo, ihi, jlo, jhi, klo, khi;
        axis_range(c[0], R, h, nx, &ilo, &ihi);
        axis_range(c[1], R, h, ny, &jlo, &jhi);
        axis_range(c[2], R, h, nz, &klo, &khi);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int k = klo; k <= khi; ++k)
            for (int j = jlo; j <= jhi; ++j)
                for (int i = ilo; i <= ihi; ++i) {
                    const double w = cell_ratio(i, j, k, sf, h, c, R);
                    if (w == 0.0) continue;
                    double g[3];
                    gradient_at(&L, phi, kinds, values, face, h, i, j, k, g);
                    for (int a = 0; a < 3; ++a) acc[a] += g[a] * w;
                    const double v[3] = {pre * q[s] * w * gF[3 * s], pre * q[s] * w * gF[3 * s + 1],
                                         pre * q[s] * w * gF[3 * s + 2]};
                    scatter_gradient_transpose(&L, kinds, h, i, j, k, v, mu);
                }
        direct[s] = pre * (acc[0] * gF[3 * s] + acc[1] * gF[3 * s + 1] + acc[2] * gF[3 * s + 2]);
    }
}

/* Multigrid solve (Alg. 1): with rho_k = ||b - A phi_k||_2 / ||b||_2, perform
 * V-cycles while rho_k >= rtol, at most max_cycles.  b is the folded finest
 * right-hand side; phi holds the initial guess on entry.  hist[0..cycles]
 * receives rho_0..rho_cycles.  If ||b|| = 0, phi is set to 0 and no cycle is
 * run.  Returns OR_OK, OR_E_NOCONV or OR_E_NONFINITE. */
int or_solve(int nx, int ny, int nz, double h, const int* kinds, int levels, int nu1, int nu2,
             double omega, double cg_rtol, int cg_maxit, const double* b, double* phi,
             double rtol, int max_cycles, double* hist, int* cycles_out)
{
    or_hier H;
    if (hier_init(&H, nx, ny, nz, h, kinds, levels, nu1, nu2, omega, cg_rtol, cg_maxit, 0))
        return OR_E_ARG;
    const or_level* L0 = &H.lev[0];
    const size_t n = or_cells(L0);
    H.phi[0] = phi;
    H.b[0] = (double*)b;
    const double bnorm = norm2_d(n, b);
    int k = 0, status = OR_OK;
    if (bnorm == 0.0) {
        memset(phi, 0, n * sizeof(double));
        if (hist) hist[0] = 0.0;
    } else {
        residual_d(L0, phi, b, H.r[0]);
        double rho = norm2_d(n, H.r[0]) / bnorm;
        if (hist) hist[0] = rho;
        while (isfinite(rho) && rho >= rtol && k < max_cycles) {
            vcycle_d(&H, 0);
            ++k;
            residual_d(L0, phi, b, H.r[0]);
            rho = norm2_d(n, H.r[0]) / bnorm;
            if (hist) hist[k] = rho;
        }
        if (!isfinite(rho)) status = OR_E_NONFINITE;
        else if (rho >= rtol) status = OR_E_NOCONV;
    }
    if (cycles_out) *cycles_out = k;
    H.phi[0] = NULL; H.b[0] = NULL;
    hier_free(&H);
    return status;
}

/* Power of two nearest below |x| (x > 0): scaling by it is exact. */
static double pow2_floor(double x)
{
    int e;
    frexp(x, &e);
    return ldexp(1.0, e - 1);
}

/* FP32-in-FP64 iterative refinement.  The outer loop is FP64: residual
 * r = b - A phi, its norm, and the update.  Each outer step scales r by a
 * power of two sigma (the one just below ||r||), rounds it to float, runs
 * `inner` FP32 V-cycles on A c = r/sigma from c = 0 (coarsest level in FP64),
 * and adds sigma * c to phi.  Stops when ||b - A phi|| / ||b|| < rtol or after
 * max_outer steps.  hist[0..outer] receives the relative residuals. */
int or_solve_ir(int nx, int ny, int nz, double h, const int* kinds, int levels, int nu1, int nu2,
                double omega, double cg_rtol, int cg_maxit, int inner, const double* b, double* phi,
                double rtol, int max_outer, double* hist, int* outer_out)
{
    or_hier H;
    if (hier_init(&H, nx, ny, nz, h, kinds, levels, nu1, nu2, omega, cg_rtol, cg_maxit, 1))
        return OR_E_ARG;
    const or_level* L0 = &H.lev[0];
    const size_t n = or_cells(L0);
    const double bnorm = norm2_d(n, b);
    int k = 0, status = OR_OK;
    if (bnorm == 0.0) {
        memset(phi, 0, n * sizeof(double));
        if (hist) hist[0] = 0.0;
    } else {
        double* r = H.r[0];
        residual_d(L0, phi, b, r);
        double rnorm = norm2_d(n, r);
        double rho = rnorm / bnorm;
        if (hist) hist[0] = rho;
        while (isfinite(rho) && rho >= rtol && k < max_outer) {
            const double sigma = pow2_floor(rnorm);
            for (size_t c = 0; c < n; ++c) H.bf[0][c] = (float)(r[c] / sigma);
            memset(H.phif[0], 0, n * sizeof(float));
            for (int m = 0; m < inner; ++m) vcycle_f(&H, 0);
            for (size_t c = 0; c < n; ++c) phi[c] += sigma * (double)H.phif[0][c];
            ++k;
            residual_d(L0, phi, b, r);
            rnorm = norm2_d(n, r);
            rho = rnorm / bnorm;
            if (hist) hist[k] = rho;
        }
        if (!isfinite(rho)) status = OR_E_NONFINITE;
        else if (rho >= rtol) status = OR_E_NOCONV;
    }
    if (outer_out) *outer_out = k;
    hier_free(&H);
    return status;
}


/* ==================== variable permittivity (extension) =====================
 * -div(eps grad phi) = rho with a cell-wise permittivity (the solver is meant
 * to be extensible to discontinuous dielectricity by Galerkin coarsening,
 * Sec. 3; stored per-unknown stencils, Sec. 5.3).  Finite volumes: the flux
 * across the face between cells a and b is eps_f (phi_b - phi_a) / h with the
 * harmonic mean eps_f = 2 eps_a eps_b / (eps_a + eps_b); a boundary face takes
 * the permittivity of its cell.  Level l's operator is s_l times a 7-point
 * stencil with normalised face coefficients k (s_l = 1/(2^l h^2), k = eps_f on
 * the finest level):
 *     (A_l phi)_c = s_l (d_c phi_c - sum over in-domain faces k_f phi_n),
 *     d_c = sum over in-domain faces k_f + sum over Dirichlet faces 2 k_f
 * (Neumann faces add nothing).  Galerkin coarsening A_{l+1} = R A_l P with the
 * cell-centred transfers of Sec. 3 (P copies a coarse value to its 8 children,
 * R = P^T / 8) keeps this form, with every coarse face coefficient the mean of
 * the 4 fine face coefficients on that face (derivation: P^T (e_i - e_j)
 * vanishes for siblings and is e_I - e_J otherwise, so the coarse coupling is
 * (sum of 4 fine couplings) / 8 = s_{l+1} (sum of 4 k) / 4).  For constant eps
 * this is eps times the constant-coefficient operator above.
 * Face arrays: x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces
 * [nz+1][ny][nx] (face i lies between cells i-1 and i). */
typedef struct {
    int nx, ny, nz;
    double s;
    int kind[6];
    double *kx, *ky, *kz;
} vc_level;

#define VKX(L, i, j, k) ((L)->kx[((size_t)(k) * (L)->ny + (size_t)(j)) * (size_t)((L)->nx + 1) + (size_t)(i)])
#define VKY(L, i, j, k) ((L)->ky[((size_t)(k) * (size_t)((L)->ny + 1) + (size_t)(j)) * (size_t)(L)->nx + (size_t)(i)])
#define VKZ(L, i, j, k) ((L)->kz[((size_t)(k) * (L)->ny + (size_t)(j)) * (size_t)(L)->nx + (size_t)(i)])

static size_t vc_nkx(int nx, int ny, int nz) { return (size_t)(nx + 1) * ny * nz; }
static size_t vc_nky(int nx, int ny, int nz) { return (size_t)nx * (ny + 1) * nz; }
static size_t vc_nkz(int nx, int ny, int nz) { return (size_t)nx * ny * (nz + 1); }

static double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

static void vc_faces_from_eps(vc_level* L, const double* eps)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
#define EPS(i, j, k) eps[((size_t)(k) * ny + (j)) * nx + (i)]
    /* a periodic axis's boundary face joins cell n-1 and cell 0 (stored at 0 and n) */
    const int px = L->kind[0] == OR_PERIODIC, py = L->kind[2] == OR_PERIODIC, pz = L->kind[4] == OR_PERIODIC;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i)
                VKX(L, i, j, k) = (i == 0 || i == nx) ? (px ? harmonic(EPS(nx - 1, j, k), EPS(0, j, k))
                                                            : EPS(i == 0 ? 0 : nx - 1, j, k))
                                                      : harmonic(EPS(i - 1, j, k), EPS(i, j, k));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                VKY(L, i, j, k) = (j == 0 || j == ny) ? (py ? harmonic(EPS(i, ny - 1, k), EPS(i, 0, k))
                                                            : EPS(i, j == 0 ? 0 : ny - 1, k))
                                                      : harmonic(EPS(i, j - 1, k), EPS(i, j, k));
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                VKZ(L, i, j, k) = (k == 0 || k == nz) ? (pz ? harmonic(EPS(i, j, nz - 1), EPS(i, j, 0))
                                                            : EPS(i, j, k == 0 ? 0 : nz - 1))
                                                      : harmonic(EPS(i, j, k - 1), EPS(i, j, k));
#undef EPS
}

/* coarse face coefficient = mean of the 4 fine face coefficients on that face */
static void vc_coarsen(const vc_level* F, vc_level* C)
{
    for (int K = 0; K < C->nz; ++K)
        for (int J = 0; J < C->ny; ++J)
            for (int I = 0; I <= C->nx; ++I)
                VKX(C, I, J, K) = (VKX(F, 2 * I, 2 * J, 2 * K) + VKX(F, 2 * I, 2 * J + 1, 2 * K) +
                                   VKX(F, 2 * I, 2 * J, 2 * K + 1) + VKX(F, 2 * I, 2 * J + 1, 2 * K + 1)) / 4.0;
    for (int K = 0; K < C->nz; ++K)
        for (int J = 0; J <= C->ny; ++J)
            for (int I = 0; I < C->nx; ++I)
                VKY(C, I, J, K) = (VKY(F, 2 * I, 2 * J, 2 * K) + VKY(F, 2 * I + 1, 2 * J, 2 * K) +
                                   VKY(F, 2 * I, 2 * J, 2 * K + 1) + VKY(F, 2 * I + 1, 2 * J, 2 * K + 1)) / 4.0;
    for (int K = 0; K <= C->nz; ++K)
        for (int J = 0; J < C->ny; ++J)
            for (int I = 0; I < C->nx; ++I)
                VKZ(C, I, J, K) = (VKZ(F, 2 * I, 2 * J, 2 * K) + VKZ(F, 2 * I + 1, 2 * J, 2 * K) +
                                   VKZ(F, 2 * I, 2 * J + 1, 2 * K) + VKZ(F, 2 * I + 1, 2 * J + 1, 2 * K)) / 4.0;
}

/* contribution of a boundary face to the diagonal: Dirichlet 2k, Neumann 0,
 * periodic k (an interior face to the cell on the opposite side) */
static double vc_bdiag(int kind, double kf)
{
    return kind == OR_DIRICHLET ? 2.0 * kf : kind == OR_PERIODIC ? kf : 0.0;
}

static double vc_diag(const vc_level* L, int i, int j, int k)
{
    double d = 0.0;
    d += i > 0 ? VKX(L, i, j, k) : vc_bdiag(L->kind[0], VKX(L, 0, j, k));
    d += i < L->nx - 1 ? VKX(L, i + 1, j, k) : vc_bdiag(L->kind[1], VKX(L, L->nx, j, k));
    d += j > 0 ? VKY(L, i, j, k) : vc_bdiag(L->kind[2], VKY(L, i, 0, k));
    d += j < L->ny - 1 ? VKY(L, i, j + 1, k) : vc_bdiag(L->kind[3], VKY(L, i, L->ny, k));
    d += k > 0 ? VKZ(L, i, j, k) : vc_bdiag(L->kind[4], VKZ(L, i, j, 0));
    d += k < L->nz - 1 ? VKZ(L, i, j, k + 1) : vc_bdiag(L->kind[5], VKZ(L, i, j, L->nz));
    return d;
}

/* sum over in-domain faces of k_f phi_n (periodic faces reach the cell on the
 * opposite side), order x-, x+, y-, y+, z-, z+ */
static double vc_nbsum(const vc_level* L, const double* phi, int i, int j, int k)
{
    const size_t nx = L->nx, ny = L->ny, nz = L->nz;
    const size_t c = ((size_t)k * ny + j) * nx + i;
    double sum = 0.0;
    if (i > 0) sum += VKX(L, i, j, k) * phi[c - 1];
    else if (L->kind[0] == OR_PERIODIC) sum += VKX(L, 0, j, k) * phi[c + nx - 1];
    if (i < L->nx - 1) sum += VKX(L, i + 1, j, k) * phi[c + 1];
    else if (L->kind[1] == OR_PERIODIC) sum += VKX(L, L->nx, j, k) * phi[c - (nx - 1)];
    if (j > 0) sum += VKY(L, i, j, k) * phi[c - nx];
    else if (L->kind[2] == OR_PERIODIC) sum += VKY(L, i, 0, k) * phi[c + (ny - 1) * nx];
    if (j < L->ny - 1) sum += VKY(L, i, j + 1, k) * phi[c + nx];
    else if (L->kind[3] == OR_PERIODIC) sum += VKY(L, i, L->ny, k) * phi[c - (ny - 1) * nx];
    if (k > 0) sum += VKZ(L, i, j, k) * phi[c - nx * ny];
    else if (L->kind[4] == OR_PERIODIC) sum += VKZ(L, i, j, 0) * phi[c + (nz - 1) * nx * ny];
    if (k < L->nz - 1) sum += VKZ(L, i, j, k + 1) * phi[c + nx * ny];
    else if (L->kind[5] == OR_PERIODIC) sum += VKZ(L, i, j, L->nz) * phi[c - (nz - 1) * nx * ny];
    return sum;
}

static size_t vc_cells(const vc_level* L) { return (size_t)L->nx * L->ny * L->nz; }

static void vc_apply(const vc_level* L, const double* phi, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                const size_t c = ((size_t)k * L->ny + j) * L->nx + i;
                out[c] = L->s * (vc_diag(L, i, j, k) * phi[c] - vc_nbsum(L, phi, i, j, k));
            }
}

static void vc_residual(const vc_level* L, const double* phi, const double* b, double* r)
{
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                const size_t c = ((size_t)k * L->ny + j) * L->nx + i;
                r[c] = b[c] - L->s * (vc_diag(L, i, j, k) * phi[c] - vc_nbsum(L, phi, i, j, k));
            }
}

/* red-black Gauss-Seidel, red ((i+j+k) even) first: phi_c <- (b_c/s + sum k phi_n) / d_c */
static void vc_rbgs_sweep(const vc_level* L, double* phi, const double* b)
{
    for (int colour = 0; colour < 2; ++colour) {
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < L->nz; ++k)
            for (int j = 0; j < L->ny; ++j)
                for (int i = 0; i < L->nx; ++i) {
                    if (((i + j + k) & 1) != colour) continue;
                    const size_t c = ((size_t)k * L->ny + j) * L->nx + i;
                    phi[c] = (b[c] / L->s + vc_nbsum(L, phi, i, j, k)) / vc_diag(L, i, j, k);
                }
    }
}

static int vc_cg(const vc_level* L, const double* b, double* x, double rtol, int maxit)
{
    const size_t n = vc_cells(L);
    double* r = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    for (size_t c = 0; c < n; ++c) { x[c] = 0.0; r[c] = b[c]; p[c] = b[c]; }
    const double bnorm = norm2_d(n, b);
    double rr = dot_d(n, r, r);
    int it = 0;
    if (bnorm > 0.0) {
        while (it < maxit) {
            vc_apply(L, p, q);
            const double alpha = rr / dot_d(n, p, q);
            for (size_t c = 0; c < n; ++c) x[c] += alpha * p[c];
            for (size_t c = 0; c < n; ++c) r[c] -= alpha * q[c];
            const double rr_new = dot_d(n, r, r);
            ++it;
            if (sqrt(rr_new) <= rtol * bnorm) break;
            const double beta = rr_new / rr;
            for (size_t c = 0; c < n; ++c) p[c] = r[c] + beta * p[c];
            rr = rr_new;
        }
    }
    free(r); free(p); free(q);
    return it;
}

static vc_level vc_make(int nx, int ny, int nz, double h, int level, const int* kinds, double* kx, double* ky,
                        double* kz)
{
    vc_level L;
    L.nx = nx; L.ny = ny; L.nz = nz;
    L.s = 1.0 / (ldexp(1.0, level) * h * h);
    for (int f = 0; f < 6; ++f) L.kind[f] = kinds[f];
    L.kx = kx; L.ky = ky; L.kz = kz;
    return L;
}

void or_vc_faces(int nx, int ny, int nz, const int* kinds, const double* eps, double* kx, double* ky, double* kz)
{
    vc_level L = vc_make(nx, ny, nz, 1.0, 0, kinds, kx, ky, kz);
    vc_faces_from_eps(&L, eps);
}

/* coarse face arrays of the (nx/2, ny/2, nz/2) level from the fine ones */
void or_vc_coarsen(int nx, int ny, int nz, const double* kx, const double* ky, const double* kz, double* ckx,
                   double* cky, double* ckz)
{
    const int kinds[6] = {0, 0, 0, 0, 0, 0};
    vc_level F = vc_make(nx, ny, nz, 1.0, 0, kinds, (double*)kx, (double*)ky, (double*)kz);
    vc_level C = vc_make(nx / 2, ny / 2, nz / 2, 1.0, 1, kinds, ckx, cky, ckz);
    vc_coarsen(&F, &C);
}

void or_vc_apply(int nx, int ny, int nz, double h, int level, const int* kinds, const double* kx, const double* ky,
                 const double* kz, const double* phi, double* out)
{
    vc_level L = vc_make(nx, ny, nz, h, level, kinds, (double*)kx, (double*)ky, (double*)kz);
    vc_apply(&L, phi, out);
}

void or_vc_rbgs_sweep(int nx, int ny, int nz, double h, int level, const int* kinds, const double* kx,
                      const double* ky, const double* kz, double* phi, const double* b, int sweeps)
{
    vc_level L = vc_make(nx, ny, nz, h, level, kinds, (double*)kx, (double*)ky, (double*)kz);
    for (int s = 0; s < sweeps; ++s) vc_rbgs_sweep(&L, phi, b);
}

/* b = f + boundary terms with the boundary face coefficients: Dirichlet
 * 2 k_f g / h^2, Neumann k_f g_n / h (the flux eps dphi/dn = eps g_n), faces in
 * the order x-, x+, y-, y+, z-, z+; face[fc] (nullable) gives per-cell values
 * as in or_fold_field. */
void or_vc_fold(int nx, int ny, int nz, double h, const int* kinds, const double* values, const double* const* face,
                const double* kx, const double* ky, const double* kz, const double* f, double* b)
{
    vc_level L = vc_make(nx, ny, nz, h, 0, kinds, (double*)kx, (double*)ky, (double*)kz);
    const size_t n = vc_cells(&L);
    for (size_t c = 0; c < n; ++c) b[c] = f[c];
    for (int fc = 0; fc < 6; ++fc) {
        const int ax = fc / 2, hi = fc % 2;
        const int n0 = ax == 0 ? ny : nx;
        const int n1 = ax == 2 ? ny : nz;
        for (int v = 0; v < n1; ++v)
            for (int u = 0; u < n0; ++u) {
                const double g = (face && face[fc]) ? face[fc][(size_t)v * n0 + u] : values[fc];
                int i, j, k;
                double kf;
                if (ax == 0)      { i = hi ? nx - 1 : 0; j = u; k = v; kf = VKX(&L, hi ? nx : 0, j, k); }
                else if (ax == 1) { j = hi ? ny - 1 : 0; i = u; k = v; kf = VKY(&L, i, hi ? ny : 0, k); }
                else              { k = hi ? nz - 1 : 0; i = u; j = v; kf = VKZ(&L, i, j, hi ? nz : 0); }
                const double t = kinds[fc] == OR_DIRICHLET ? 2.0 * kf * g / (h * h)
                                 : kinds[fc] == OR_NEUMANN ? kf * g / h : 0.0;
                b[((size_t)k * ny + j) * nx + i] += t;
            }
    }
}

/* V(nu1,nu2)-cycles for the variable-permittivity operator (same cycle as
 * or_solve: smoothing, residual, averaging restriction, zero coarse guess,
 * CG on the coarsest level, nearest-neighbour prolongation times omega),
 * every level's face coefficients by Galerkin coarsening of the finest. */
int or_vc_solve(int nx, int ny, int nz, double h, const int* kinds, int levels, int nu1, int nu2, double omega,
                double cg_rtol, int cg_maxit, const double* eps, const double* b, double* phi, double rtol,
                int max_cycles, double* hist, int* cycles_out)
{
    if (levels < 1 || levels > OR_MAXLEVELS) return OR_E_ARG;
    const int div = 1 << (levels - 1);
    if (nx % div || ny % div || nz % div) return OR_E_ARG;
    vc_level L[OR_MAXLEVELS];
    double *ph[OR_MAXLEVELS], *bb[OR_MAXLEVELS], *rr[OR_MAXLEVELS];
    for (int l = 0; l < levels; ++l) {
        const int a = nx >> l, bq = ny >> l, c = nz >> l;
        L[l] = vc_make(a, bq, c, h, l, kinds, (double*)malloc(vc_nkx(a, bq, c) * sizeof(double)),
                       (double*)malloc(vc_nky(a, bq, c) * sizeof(double)),
                       (double*)malloc(vc_nkz(a, bq, c) * sizeof(double)));
        const size_t n = vc_cells(&L[l]);
        ph[l] = l == 0 ? phi : (double*)calloc(n, sizeof(double));
        bb[l] = l == 0 ? (double*)b : (double*)calloc(n, sizeof(double));
        rr[l] = (double*)calloc(n, sizeof(double));
        if (l == 0) vc_faces_from_eps(&L[0], eps);
        else vc_coarsen(&L[l - 1], &L[l]);
    }
    const size_t n0 = vc_cells(&L[0]);
    const double bnorm = norm2_d(n0, b);
    int k = 0, status = OR_OK;
    if (bnorm == 0.0) {
        memset(phi, 0, n0 * sizeof(double));
        if (hist) hist[0] = 0.0;
    } else {
        vc_residual(&L[0], phi, b, rr[0]);
        double rho = norm2_d(n0, rr[0]) / bnorm;
        if (hist) hist[0] = rho;
        while (isfinite(rho) && rho >= rtol && k < max_cycles) {
            for (int l = 0; l < levels - 1; ++l) {
                for (int s = 0; s < nu1; ++s) vc_rbgs_sweep(&L[l], ph[l], bb[l]);
                vc_residual(&L[l], ph[l], bb[l], rr[l]);
                const or_level dims = make_level(L[l].nx, L[l].ny, L[l].nz, h, l, kinds);
                restrict_avg_d(&dims, rr[l], bb[l + 1]);
                memset(ph[l + 1], 0, vc_cells(&L[l + 1]) * sizeof(double));
            }
            vc_cg(&L[levels - 1], bb[levels - 1], ph[levels - 1], cg_rtol, cg_maxit);
            for (int l = levels - 2; l >= 0; --l) {
                const or_level dims = make_level(L[l].nx, L[l].ny, L[l].nz, h, l, kinds);
                prolong_add_d(&dims, ph[l + 1], omega, ph[l]);
                for (int s = 0; s < nu2; ++s) vc_rbgs_sweep(&L[l], ph[l], bb[l]);
            }
            ++k;
            vc_residual(&L[0], phi, b, rr[0]);
            rho = norm2_d(n0, rr[0]) / bnorm;
            if (hist) hist[k] = rho;
        }
        if (!isfinite(rho)) status = OR_E_NONFINITE;
        else if (rho >= rtol) status = OR_E_NOCONV;
    }
    if (cycles_out) *cycles_out = k;
    for (int l = 0; l < levels; ++l) {
        free(L[l].kx); free(L[l].ky); free(L[l].kz);
        if (l > 0) { free(ph[l]); free(bb[l]); }
        free(rr[l]);
    }
    return status;
}

/* ====================== Poisson-Boltzmann (extension) =========================
 * The paper's outlook names the Poisson-Boltzmann equation (charged particles in
 * an electrolyte, with double layers) as a further equation for this solver and
 * its boundary treatment (Sec. 9), without writing it out.  Reading taken: a
 * symmetric electrolyte in dimensionless potential psi (e psi / k_B T for a
 * monovalent salt) and inverse Debye length kappa,
 *     -Lap(psi) + kappa^2 sinh(psi) = f,
 * with the reaction term taken at the cell centre (midpoint rule of the finite
 * volume), the same stencil and boundary folding as Poisson's equation, and the
 * linearised (Debye-Hueckel) operator -Lap + kappa^2 as its small-potential
 * limit.  Coarse operators: 2^l times the operator rediscretised at spacing
 * 2^l h, A_l + 2^l kappa^2 I.  For the Laplacian part this is the Galerkin
 * product of Sec. 3 (the reason for the correction factor about 2); with
 * omega = 2 the cycle is then the rediscretised cycle with omega = 1 for the
 * whole operator.  (The Galerkin product of the reaction term alone would be
 * kappa^2 I on every level, R P = I; with omega = 2 it over-corrects the smooth
 * modes that the reaction term dominates.)  The nonlinear equation is solved
 * by a shifted chord iteration with the linear multigrid as inner solver:
 *     r_k = b - A psi_k - kappa^2 sinh(psi_k),   c_k = cosh(max |psi_k|),
 *     (A + c_k kappa^2 I) delta = r_k  by `inner` V-cycles from delta = 0,
 *     psi_{k+1} = psi_k + delta,
 * while ||r_k|| / ||b|| >= rtol.  With c_k >= cosh(psi) everywhere on the
 * segment between iterate and solution the error map is a contraction, so the
 * iteration converges for any potential; for |psi| <~ 1 it is Newton's method
 * up to the variation of cosh. */

static void hier_set_k2(or_hier* H, double k2)
{
    for (int l = 0; l < H->nlev; ++l) H->lev[l].k2 = ldexp(k2, l);
}

void or_pb_apply(int nx, int ny, int nz, double h, int level, const int* kinds, double k2,
                 const double* phi, double* out)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    L.k2 = k2;
    apply_d(&L, phi, out);
}

void or_pb_rbgs_sweep(int nx, int ny, int nz, double h, int level, const int* kinds, double k2,
                      double* phi, const double* b)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    L.k2 = k2;
    rbgs_sweep_d(&L, phi, b);
}

int or_pb_cg(int nx, int ny, int nz, double h, int level, const int* kinds, double k2,
             const double* b, double* x, double rtol, int maxit)
{
    or_level L = make_level(nx, ny, nz, h, level, kinds);
    L.k2 = k2;
    return cg_d(&L, b, x, rtol, maxit);
}

/* Linear Poisson-Boltzmann (Debye-Hueckel) solve: or_solve with A_l + 2^l k2 I
 * on level l. */
int or_pb_solve(int nx, int ny, int nz, double h, const int* kinds, int levels, int nu1, int nu2,
                double omega, double cg_rtol, int cg_maxit, double k2, const double* b, double* phi,
                double rtol, int max_cycles, double* hist, int* cycles_out)
{
    or_hier H;
    if (hier_init(&H, nx, ny, nz, h, kinds, levels, nu1, nu2, omega, cg_rtol, cg_maxit, 0))
        return OR_E_ARG;
    hier_set_k2(&H, k2);
    const or_level* L0 = &H.lev[0];
    const size_t n = or_cells(L0);
    H.phi[0] = phi;
    H.b[0] = (double*)b;
    const double bnorm = norm2_d(n, b);
    int k = 0, status = OR_OK;
    if (bnorm == 0.0) {
        memset(phi, 0, n * sizeof(double));
        if (hist) hist[0] = 0.0;
    } else {
        residual_d(L0, phi, b, H.r[0]);
        double rho = norm2_d(n, H.r[0]) / bnorm;
        if (hist) hist[0] = rho;
        while (isfinite(rho) && rho >= rtol && k < max_cycles) {
            vcycle_d(&H, 0);
            ++k;
            residual_d(L0, phi, b, H.r[0]);
            rho = norm2_d(n, H.r[0]) / bnorm;
            if (hist) hist[k] = rho;
        }
        if (!isfinite(rho)) status = OR_E_NONFINITE;
        else if (rho >= rtol) status = OR_E_NOCONV;
    }
    if (cycles_out) *cycles_out = k;
    H.phi[0] = NULL; H.b[0] = NULL;
    hier_free(&H);
    return status;
}

/* r = b - A psi - k2 sinh(psi) on level 0 (the nonlinear residual). */
void or_pb_nl_residual(int nx, int ny, int nz, double h, const int* kinds, double k2, const double* psi,
                       const double* b, double* r)
{
    or_level L = make_level(nx, ny, nz, h, 0, kinds);
    residual_d(&L, psi, b, r);
    const size_t n = or_cells(&L);
    for (size_t c = 0; c < n; ++c) r[c] -= k2 * sinh(psi[c]);
}

/* Nonlinear Poisson-Boltzmann solve by the shifted chord iteration above.
 * psi: initial guess in, last iterate out; hist[0..outer] receives the
 * relative nonlinear residuals.  ||b|| = 0 gives psi = 0 (sinh(0) = 0). */
int or_pb_nl_solve(int nx, int ny, int nz, double h, const int* kinds, int levels, int nu1, int nu2,
                   double omega, double cg_rtol, int cg_maxit, double k2, int inner, const double* b,
                   double* psi, double rtol, int max_outer, double* hist, int* outer_out)
{
    or_hier H;
    if (hier_init(&H, nx, ny, nz, h, kinds, levels, nu1, nu2, omega, cg_rtol, cg_maxit, 0))
        return OR_E_ARG;
    const or_level* L0 = &H.lev[0];
    const size_t n = or_cells(L0);
    double* r = (double*)malloc(n * sizeof(double));
    double* delta = (double*)malloc(n * sizeof(double));
    const double bnorm = norm2_d(n, b);
    int k = 0, status = OR_OK;
    if (bnorm == 0.0) {
        memset(psi, 0, n * sizeof(double));
        if (hist) hist[0] = 0.0;
    } else {
        or_pb_nl_residual(nx, ny, nz, h, kinds, k2, psi, b, r);
        double rho = norm2_d(n, r) / bnorm;
        if (hist) hist[0] = rho;
        while (isfinite(rho) && rho >= rtol && k < max_outer) {
            double m = 0.0;
            for (size_t c = 0; c < n; ++c) m = fmax(m, fabs(psi[c]));
            hier_set_k2(&H, k2 * cosh(m));
            memset(delta, 0, n * sizeof(double));
            H.phi[0] = delta;
            H.b[0] = r;
            for (int i = 0; i < inner; ++i) vcycle_d(&H, 0);
            for (size_t c = 0; c < n; ++c) psi[c] += delta[c];
            ++k;
            or_pb_nl_residual(nx, ny, nz, h, kinds, k2, psi, b, r);
            rho = norm2_d(n, r) / bnorm;
            if (hist) hist[k] = rho;
        }
        if (!isfinite(rho)) status = OR_E_NONFINITE;
        else if (rho >= rtol) status = OR_E_NOCONV;
    }
    if (outer_out) *outer_out = k;
    H.phi[0] = NULL; H.b[0] = NULL;
    hier_free(&H);
    free(r); free(delta);
    return status;
}
