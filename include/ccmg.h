/*
 * ccmg.h -- C ABI of the cell-centered geometric multigrid Poisson solver for
 * AMD Instinct MI355X (gfx950).
 *
 * The solver computes the electric potential phi of
 *     -Lap(phi) = rho / eps                 (Sec. 2.4, Eq. Poisson)
 * on a uniform cell grid with the finite-volume 7-point stencil and
 * per-face Dirichlet or Neumann conditions folded into stencil and right-hand
 * side (Sec. 2.4, "Boundary conditions"; Sec. 5.3), by the cell-centered
 * multigrid of Sec. 3 / Sec. 5.3 (2x2x2 coarsening, averaging restriction,
 * nearest-neighbour prolongation with the correction magnified by omega,
 * Galerkin coarse operators, red-black Gauss-Seidel smoothing, CG on the
 * coarsest grid, V-cycles until the residual L2 norm drops below a tolerance,
 * Alg. 1), of D. Bartuschat and U. Ruede, "Parallel Multiphysics Simulations
 * of Charged Particles in Microfluidic Flows", arXiv:1410.6609.
 * Two extensions: FP32 V-cycles inside FP64 iterative refinement, and the
 * adjoint solve giving gradients with respect to the charges.
 *
 * Conventions for every entry point:
 *  - Arrays are contiguous [nz][ny][nx] (x fastest).  Cell (i,j,k) has its
 *    centre at ((i+1/2)h, (j+1/2)h, (k+1/2)h).
 *  - Pointers named d_* must be device memory of the current HIP device; the
 *    caller owns them.  The library never allocates device memory: its
 *    scratch space is a caller-owned workspace (ccmg_set_workspace).
 *  - Work is enqueued on the HIP stream given to ccmg_create (0 = the null
 *    stream).  Calls that return norms or statistics synchronise that stream;
 *    all others return without waiting.
 *  - Return value: CCMG_OK (0) or a negative CCMG_E_* code; then
 *    ccmg_last_error() holds a message.  No C++ exception crosses the ABI.
 *  - One solver object must not be used by two threads at once.
 */
#ifndef CCMG_H
#define CCMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccmg_solver ccmg_solver;

/* face kinds; faces are numbered 0..5 = x-, x+, y-, y+, z-, z+.
 * CCMG_PERIODIC (Sec. 2.4: the domain is cyclically extended; the cells at
 * opposite sides are neighbours) must be set on both faces of an axis; its
 * value is ignored.  A solver with a periodic axis runs on the stored-stencil
 * operator of ccmg_set_permittivity (unit permittivity until one is set; its
 * workspace includes the face coefficients) and in FP64 only.  Spheres of the
 * deposition and force calls are clipped at every face, periodic ones
 * included: keep them clear of periodic boundaries. */
enum { CCMG_DIRICHLET = 0, CCMG_NEUMANN = 1, CCMG_PERIODIC = 2 };

/* precision modes */
enum { CCMG_FP64 = 0, CCMG_FP32_IR = 1 };

/* status codes */
enum {
    CCMG_OK = 0,
    CCMG_E_ARG = -1,       /* bad argument (null, host pointer, out of range) */
    CCMG_E_DIMS = -2,      /* dims not divisible by 2^(levels-1), or coarsest grid too large */
    CCMG_E_SINGULAR = -3,  /* no Dirichlet face: the operator is singular */
    CCMG_E_HIP = -4,       /* a HIP runtime call failed */
    CCMG_E_NONFINITE = -5, /* the residual became NaN or Inf */
    CCMG_E_NOCONV = -6,    /* max_cycles reached before the tolerance (phi holds the last iterate) */
    CCMG_E_STATE = -7      /* no (or too small) workspace attached */
};

#define CCMG_MAX_LEVELS 16
#define CCMG_MAX_CYCLES 1000
#define CCMG_MAX_COARSE_CELLS 4096

/* One boundary face.  Dirichlet: value = phi on the face (half a cell outside
 * the last cell centre).  Neumann: value = outward normal derivative dphi/dn. */
typedef struct {
    int kind;
    double value;
} ccmg_face;

typedef struct {
    int nu1, nu2;         /* pre- and post-smoothing RB-GS sweeps (default 2, 2; Sec. 3: V(1,1) is unreliable) */
    int levels;           /* hierarchy depth; 0 = coarsen while the dims stay even and the grid exceeds 512 cells */
    double omega;         /* coarse-correction factor (default 2.0; Sec. 3 "about 2") */
    int precision;        /* CCMG_FP64 or CCMG_FP32_IR */
    int ir_inner_cycles;  /* FP32 V-cycles per refinement step (default 4) */
    double cg_rtol;       /* coarsest-grid CG: stop at ||r|| <= cg_rtol ||b|| (default 1e-13) */
    int cg_maxit;         /* coarsest-grid CG iteration cap (0 = 2 x coarsest cells) */
    int fuse_sweeps;      /* RB-GS sweeps fused per smoother kernel pass: 1 or 2 (default 2); iterates are identical */
    int bottom_cells;     /* the coarse levels from the first one with at most this many cells down to the
                             coarsest run in one workgroup, in LDS (default 4096, the maximum; 0 = off) */
    int variable_eps;     /* 1: reserve stored face coefficients for a cell-wise permittivity
                             (ccmg_set_permittivity; FP64 only); default 0 */
    double ir_cg_rtol;    /* FP32-IR: coarsest-grid CG tolerance inside the FP32 cycles (default 1e-6:
                             an FP32 correction carries about seven digits; the FP64 cycles use cg_rtol) */
    double kappa2;        /* Poisson-Boltzmann (the outlook of Sec. 9): kappa^2 >= 0, the squared inverse
                             Debye length in 1/length^2.  Every linear call (solve, cycles, residual,
                             smoothing, adjoint, FP32-IR) then uses the linearised (Debye-Hueckel) operator
                             -Lap + kappa^2 on the finest level, with 2^l-scaled coarse reaction terms (the
                             operator rediscretised at spacing 2^l h, times 2^l, as the Galerkin product is for
                             the Laplacian); ccmg_solve_pb solves the nonlinear equation.  Default 0 (Poisson).
                             Constant coefficients only: not with variable_eps or periodic faces. */
} ccmg_options;

typedef struct {
    int cycles;           /* V-cycles (FP64) or refinement steps (FP32-IR) performed */
    int inner_cycles;     /* FP32 V-cycles performed (FP32-IR), else equal to cycles */
    double rel_res0;      /* ||b - A phi_0|| / ||b|| of the initial guess */
    double rel_res;       /* ||b - A phi|| / ||b|| on return */
    double seconds;       /* host wall time of the call, including the final synchronisation */
} ccmg_stats;

/* Fill *opt with the defaults listed above. */
void ccmg_default_options(ccmg_options* opt);

/* Create a solver for an nx x ny x nz cell grid of spacing h > 0 with the six
 * face conditions bc[0..5] (x-, x+, y-, y+, z-, z+).  opt may be NULL for the
 * defaults.  hip_stream is a hipStream_t (NULL = null stream).  Builds the
 * level hierarchy on the host (Sec. 3: a level is coarsened by 2x2x2 while the
 * cell counts per dimension stay even); touches no device memory.
 * Errors: E_ARG (null out/bc, h <= 0, bad kinds or options, an unpaired
 * periodic face, FP32-IR with variable permittivity or a periodic axis),
 * E_DIMS (a dim not divisible by 2^(levels-1), coarsest grid over
 * CCMG_MAX_COARSE_CELLS cells, an x-y plane of 2 GiB or more in FP64),
 * E_SINGULAR (no Dirichlet face: every face Neumann or periodic). */
int ccmg_create(ccmg_solver** out, int nx, int ny, int nz, double h, const ccmg_face bc[6],
                const ccmg_options* opt, void* hip_stream);

/* Bytes of device workspace the solver needs (hierarchy arrays, ping-pong
 * buffers, norm partials, the control block, per-cell boundary values and,
 * with variable permittivity or a periodic axis, the face coefficients of
 * every level). */
size_t ccmg_workspace_bytes(const ccmg_solver* s);

/* Attach caller-owned device memory of at least ccmg_workspace_bytes() bytes,
 * 256-byte aligned.  It must stay valid while the solver is used.
 * Errors: E_ARG (null, host memory, misaligned), E_STATE (too small). */
int ccmg_set_workspace(ccmg_solver* s, void* d_ptr, size_t bytes);

/* Enqueue later calls on another stream. */
int ccmg_set_stream(ccmg_solver* s, void* hip_stream);

/* Number of levels and the cell counts of level l (l = 0 finest). */
int ccmg_num_levels(const ccmg_solver* s);
int ccmg_level_dims(const ccmg_solver* s, int l, int dims_out[3]);

/* Charge deposition (Sec. 2.4, naive volume mapping): for each sphere s with
 * centre d_centers[3s..3s+2], radius d_radii[s] (physical units) and charge
 * d_q[s], the cells whose centre lies in the closed ball are its n_s cells,
 * and every one of them receives q_s / (eps n_s h^3) in d_f = rho / eps, which
 * is overwritten.  Overlapping spheres add (in unspecified order).  A sphere
 * covering no cell centre deposits nothing.  d_counts (nullable, int[n])
 * receives n_s.  n = 0 just zeroes d_f. */
int ccmg_deposit_charges(ccmg_solver* s, int n, const double* d_centers, const double* d_radii,
                         const double* d_q, double eps, double* d_f, int* d_counts);

/* Normalisations of the sub-sampled deposition */
enum {
    CCMG_CHARGE_SPREAD = 0, /* rho = q w / (W h^3): the sphere's charge is conserved exactly */
    CCMG_CHARGE_VOLUME = 1  /* rho = q w / (4/3 pi R^3): the paper's charge density q / V per
                               overlapped volume fraction (total charge q W h^3 / V) */
};
#define CCMG_MAX_SUBSAMPLE 8

/* Sub-sampled charge deposition (Sec. 2.4, "Subsampling"; accuracy of the
 * factors in Sec. 6.3): every cell is split equidistantly into subsample^3
 * sub-cells, and its overlap ratio w with sphere s is the fraction of the
 * sub-cell centres ((i + (a + 1/2)/subsample) h, ...), a = 0..subsample-1,
 * that lie in the closed ball (distance test (dx*dx + dy*dy) + dz*dz <= R*R
 * without contraction).  W_s = sum over cells of w.  Each overlapped cell
 * receives q_s w / (eps norm_s) in d_f (overwritten; overlapping spheres add
 * in unspecified order), with norm_s = W_s h^3 (CCMG_CHARGE_SPREAD) or
 * 4/3 pi R_s^3 (CCMG_CHARGE_VOLUME).  A sphere with W_s = 0 deposits nothing.
 * subsample = 1 with CCMG_CHARGE_SPREAD equals ccmg_deposit_charges, with
 * CCMG_CHARGE_VOLUME the paper's naive q / V density.  d_weights (nullable,
 * double[n]) receives W_s.  subsample in 1..CCMG_MAX_SUBSAMPLE, else E_ARG. */
int ccmg_deposit_charges_sub(ccmg_solver* s, int n, const double* d_centers, const double* d_radii,
                             const double* d_q, double eps, int subsample, int mode, double* d_f,
                             double* d_weights);

/* Charge gradient of a loss for the sub-sampled deposition: given the adjoint
 * field d_lambda = dL/df (from ccmg_adjoint_solve), d_dq[s] = dL/dq_s =
 * sum over cells of lambda_c w_{s,c} / (eps norm_s), with w, norm_s and the
 * arguments as in ccmg_deposit_charges_sub (0 for a sphere with W_s = 0 in
 * CCMG_CHARGE_SPREAD mode).  Enqueued without waiting. */
int ccmg_charge_gradient(ccmg_solver* s, int n, const double* d_centers, const double* d_radii, double eps,
                         int subsample, int mode, const double* d_lambda, double* d_dq);

/* Gradient of the potential (Sec. 2.4, "Coulomb force": second-order finite
 * differences, the isotropic D3Q19 lattice stencil where possible): on cells
 * whose 18 D3Q19 neighbours all lie in the domain,
 *     grad phi = (1/w_1) sum_q w_q phi(x + h c_q) c_q / h,
 * w_1 = 1/3, w = 1/18 along the axes and 1/36 along the face diagonals;
 * on the boundary layer the D3Q7 central differences, with the value beyond
 * a face taken from the solver's boundary treatment (Sec. 2.4: Dirichlet
 * 2 g - phi, Neumann phi + h g_n, per-cell face values when set).
 * d_grad: 3 fields [3][nz][ny][nx] (x, y, z components), overwritten. */
int ccmg_gradient(ccmg_solver* s, const double* d_phi, double* d_grad);

/* Electrostatic force on each sphere (Sec. 2.4, Eq. ElectrostatForce):
 *     F_s = -h^3 sum_b grad phi(x_b) rho_s(x_b),
 * with the gradient of ccmg_gradient and rho_s the sphere's own charge
 * density of the sub-sampled deposition with the given subsample and mode
 * (ccmg_deposit_charges_sub; rho, not rho / eps).  d_force (double[3n],
 * device): F_s in d_force[3s..3s+2], 0 for a sphere covering no sub-cell
 * centre.  Enqueued without waiting. */
int ccmg_coulomb_force(ccmg_solver* s, const double* d_phi, int n, const double* d_centers,
                       const double* d_radii, const double* d_q, int subsample, int mode, double* d_force);

/* Adjoint of the electrostatic force, for a loss L(F) with d_gF[3s..3s+2] =
 * dL/dF_s (device, double[3n]).  The force of ccmg_coulomb_force is affine in
 * phi; this call writes
 *   d_mu     = dL/dphi (a field, overwritten): the transposed gradient
 *              stencil applied to -h^3 (q_s / norm_s) w_{s,b} dL/dF_s,
 *              summed over spheres (boundary ghosts contribute their linear
 *              part: -phi_b Dirichlet, +phi_b Neumann);
 *   d_direct = the derivative of L through each force's charge factor at
 *              fixed phi, dL/dF_s . F_s / q_s (double[n]).
 * With lambda from ccmg_adjoint_solve(d_mu), dL/dq_s = d_direct[s] + the
 * deposition's charge gradient of lambda (ccmg_charge_gradient, with the
 * deposition's own subsample and mode).  Arguments as ccmg_coulomb_force.
 * Enqueued without waiting. */
int ccmg_coulomb_adjoint(ccmg_solver* s, const double* d_phi, int n, const double* d_centers,
                         const double* d_radii, const double* d_q, int subsample, int mode, const double* d_gF,
                         double* d_mu, double* d_direct);

/* Charge gradient of a loss on the forces, through the whole chain
 * q -> deposition -> phi = A^-1 b -> F (Sec. 2.4, Eq. ElectrostatForce; the
 * force is affine in phi and phi is linear in q):
 *     dL/dq_s = d_direct[s] + sum_c lambda_c w_{s,c} / (eps norm_s),
 * with d_direct and mu = dL/dphi from ccmg_coulomb_adjoint (force_subsample,
 * force_mode) and lambda = A^-1 mu from the adjoint solve (homogeneous
 * boundary values, stopping rule rtol / max_cycles as ccmg_solve), the last
 * term the deposition's charge gradient (ccmg_charge_gradient with
 * deposit_subsample, deposit_mode) added on the device.  d_phi: the potential
 * the forces were computed from; d_gF: dL/dF_s (double[3n]).  Outputs
 * (device, caller-owned, overwritten): d_mu = dL/dphi and d_lambda = dL/df
 * (fields [nz][ny][nx]), d_dq = dL/dq (double[n]).  st (nullable): the
 * adjoint solve's statistics (synchronises).  Returns the adjoint solve's
 * status: E_NOCONV still fills d_dq from the last iterate of lambda. */
int ccmg_force_charge_gradient(ccmg_solver* s, const double* d_phi, int n, const double* d_centers,
                               const double* d_radii, const double* d_q, double eps, int force_subsample,
                               int force_mode, int deposit_subsample, int deposit_mode, const double* d_gF,
                               double* d_mu, double* d_lambda, double* d_dq, double rtol, int max_cycles,
                               ccmg_stats* st);

/* Cell-wise permittivity (extension for discontinuous dielectricity, which
 * the paper's solver is designed for by Galerkin coarsening, Sec. 3, with
 * per-unknown stencils, Sec. 5.3).  Needs a solver created with
 * opt.variable_eps = 1 (else E_STATE) and its workspace.  d_eps: one positive
 * value per cell, [nz][ny][nx] (device; read during the call's kernels only).
 * From then on every solve, cycle, residual and smoothing call of this solver
 * uses -div(eps grad phi) = f with d_f = rho (not rho / eps):
 *   - the flux across an interior face is eps_f (phi_b - phi_a) / h with the
 *     harmonic mean eps_f = 2 eps_a eps_b / (eps_a + eps_b); a boundary face
 *     takes its cell's eps (Dirichlet 2 eps_f (phi_c - g) / h, Neumann flux
 *     eps_f g_n);
 *   - coarse levels by Galerkin coarsening R A P with the cell-centred
 *     transfers, which keeps a 7-point stencil whose face coefficients are
 *     the means of the 4 fine face coefficients (times the level scale);
 *   - the same V(nu1,nu2)-cycle, stopping rule, adjoint and statistics.
 * d_eps = NULL returns to the constant-coefficient operator (-Lap phi = f).
 * Enqueued without waiting. */
int ccmg_set_permittivity(ccmg_solver* s, const double* d_eps);

/* Per-cell boundary values on one face (Sec. 2.4, "Boundary conditions"; the
 * validation of Sec. 6.3 sets them to the analytic potential): d_values holds
 * one value per boundary cell of the face, x faces [nz][ny], y faces [nz][nx],
 * z faces [ny][nx] (first index slowest); each is the Dirichlet value at the
 * face centre or the outward normal derivative there, by the face's kind.
 * The values are copied (stream-ordered) into the workspace, so d_values may
 * be freed once the copy has run; they replace the face's constant value in
 * every later forward fold (the adjoint solve keeps homogeneous values).
 * d_values = NULL restores the constant value.  Needs the workspace
 * (E_STATE otherwise). */
int ccmg_set_face_values(ccmg_solver* s, int face, const double* d_values);

/* One V(nu1,nu2)-cycle on d_phi (in/out) for the right-hand side d_f (= rho/eps,
 * boundary values taken from the faces).  rel_res_out (nullable): the relative
 * residual ||b - A phi|| / ||b|| after the cycle (synchronises). */
int ccmg_vcycle(ccmg_solver* s, double* d_phi, const double* d_f, double* rel_res_out);

/* Warm-started cycles for a time-step loop (Sec. 8.1 runs five V(3,3)-cycles
 * at the first time step and one per later step from the previous
 * solution): `ncycles` cycles (FP64) or refinement steps (FP32-IR) on d_phi
 * (in/out) for the right-hand side d_f, all enqueued without waiting.
 * d_rel_out (nullable, one double of device memory) receives the relative
 * residual ||b - A phi|| / ||b|| after the last cycle (NaN if it is not
 * finite), written on the stream; nothing is synchronised.  ncycles in
 * 0..CCMG_MAX_CYCLES (0: nothing is enqueued). */
int ccmg_vcycles(ccmg_solver* s, double* d_phi, const double* d_f, int ncycles, double* d_rel_out);

/* Multigrid solve (Alg. 1): d_phi holds the initial guess on entry (it is not
 * zeroed) and the solution on return.  Cycles (FP64) or refinement steps
 * (FP32-IR) are performed while ||b - A phi|| / ||b|| >= rtol, at most
 * max_cycles (<= CCMG_MAX_CYCLES).  If ||b|| = 0, phi is set to 0.
 * st (nullable) receives the statistics.  Returns E_NOCONV if the tolerance
 * was not reached (phi holds the last iterate), E_NONFINITE on NaN/Inf. */
int ccmg_solve(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles,
               ccmg_stats* st);

/* The same solve from the initial guess phi = 0 (Alg. 1 started from zero):
 * d_phi is output only, its contents on entry are never read.  phi is not
 * loaded before it is first written: the initial residual is b-tilde itself
 * (its norm passes read no phi), the first cycle's finest pre-smoothing pass
 * starts from zero and the first refinement step reads no phi; only variable
 * permittivity on a periodic axis zeroes phi on the device first.  The iterates are those of ccmg_solve on a
 * zeroed d_phi.  If no cycle runs (||b|| = 0, rtol >= 1, non-finite input,
 * max_cycles = 0) phi is set to 0.  Arguments, statistics and errors as
 * ccmg_solve. */
int ccmg_solve_zero(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles,
                    ccmg_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc), and so
 * cannot provide the workspace of ccmg_set_workspace: the solve of
 * ccmg_solve_zero with the solver's workspace carved for the duration of the
 * call from a static device array of CCMG_STATIC_SCRATCH_BYTES bytes that the
 * library holds on every device it runs on until the process ends.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * the caller still passes d_phi (output only) and d_f.  No workspace needs to
 * be attached; an attached one is left untouched and in use for every other
 * call.  Same kernels, iterates, statistics and errors as ccmg_solve_zero.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents; the call synchronises the solver's stream before it
 * returns, and calls that overlap on one device (from several threads or
 * streams) race.  Errors: E_ARG if ccmg_workspace_bytes(s) exceeds
 * CCMG_STATIC_SCRATCH_BYTES (checked before any device work: attach a
 * workspace and call ccmg_solve_zero instead); E_STATE for solvers whose
 * solve needs data kept in an attached workspace (per-cell boundary values,
 * variable permittivity, periodic faces); otherwise as ccmg_solve_zero. */
#define CCMG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int ccmg_solve_zero_static(ccmg_solver* s, double* d_phi, const double* d_f, double rtol, int max_cycles,
                           ccmg_stats* st);

/* Adjoint solve for a loss L(phi): given d_g = dL/dphi, solves A lambda = g
 * with the same operator and homogeneous boundary values (A is symmetric), from
 * lambda = 0 (as ccmg_solve_zero: d_lambda is output only, never read), into
 * d_lambda = dL/df.  With n > 0 spheres (same arrays as the
 * deposition) d_dq (nullable, double[n]) receives dL/dq_s = sum over the
 * sphere's cells of lambda_c / (eps n_s h^3); d_drho (nullable) receives
 * dL/drho = lambda / eps.  Stopping rule, statistics and errors as ccmg_solve. */
int ccmg_adjoint_solve(ccmg_solver* s, const double* d_g, double* d_lambda, int n,
                       const double* d_centers, const double* d_radii, double eps, double* d_dq,
                       double* d_drho, double rtol, int max_cycles, ccmg_stats* st);

/* Nonlinear Poisson-Boltzmann equation (the outlook of Sec. 9: charged
 * particles in an electrolyte, with double layers), read as
 *     -Lap(psi) + kappa^2 sinh(psi) = f
 * for a symmetric electrolyte in dimensionless potential, kappa^2 the solver's
 * option (> 0), f and the face conditions as for ccmg_solve (the reaction term
 * is taken at cell centres).  d_psi holds the initial guess on entry (it is not
 * zeroed) and the last iterate on return.  Shifted chord iteration: with the
 * nonlinear residual r = b - A psi - kappa^2 sinh(psi) and c = cosh(max|psi|),
 * `inner` (1..16) V-cycles from zero on (A + c kappa^2) delta = r, then
 * psi += delta; the step contracts for any potential (c bounds cosh(psi)),
 * and for |psi| up to about 1 it is close to Newton's method.  Repeated while
 * ||r|| / ||b|| >= rtol, at most max_outer steps; the host synchronises once per
 * step (max|psi| sets c).  FP64 only.  Statistics: cycles = outer steps,
 * inner_cycles = their V-cycles, rel_res0 / rel_res the relative nonlinear
 * residuals.  Errors as ccmg_solve; E_STATE if kappa2 = 0. */
int ccmg_solve_pb(ccmg_solver* s, double* d_psi, const double* d_f, double rtol, int max_outer, int inner,
                  ccmg_stats* st);

/* Residual of the finest level: d_r (nullable) = b - A phi with b the folded
 * right-hand side of d_f; rel_res_out (nullable) = ||b - A phi|| / ||b||. */
int ccmg_residual(ccmg_solver* s, const double* d_phi, const double* d_f, double* d_r,
                  double* rel_res_out);

/* The smoother alone: `sweeps` red-black Gauss-Seidel sweeps on the finest
 * level for the folded right-hand side of d_f, in place on d_phi (the same
 * smoother kernels the cycle runs; for tests and bandwidth measurement). */
int ccmg_smooth(ccmg_solver* s, double* d_phi, const double* d_f, int sweeps);

/* Relative residuals rho_0..rho_k of the last solve (k = cycles); copies at
 * most `max` values into host memory and returns how many it copied. */
int ccmg_history(const ccmg_solver* s, double* out, int max);

/* Kernel timing for measurement: with profiling on, every finest-level
 * smoother pass of a cycle is bracketed by HIP events on the solver's stream.
 * `which` selects the pass by its position in the finest level's pass list of
 * a cycle (0 = first pre-smoothing pass; with the default V(2,2) and two
 * sweeps fused per pass: 0 = pre-smoothing + residual + restriction,
 * 1 = prolongation + post-smoothing + residual norm).  Only cycles that ran
 * (not those skipped after convergence) are counted.  ccmg_profile_read
 * returns the summed milliseconds and the launch count, then clears them if
 * reset != 0.  Timing adds two event records per pass. */
int ccmg_profile_enable(ccmg_solver* s, int on);
int ccmg_profile_read(ccmg_solver* s, int which, double* total_ms, int* launches, int reset);

/* Message of the last error on this solver ("" if none); s may be NULL for
 * errors of ccmg_create. */
const char* ccmg_last_error(const ccmg_solver* s);

void ccmg_destroy(ccmg_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* CCMG_H */
