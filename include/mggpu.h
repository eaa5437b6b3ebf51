/*
 * mggpu.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of MG-GLAM (Ruan et al., "Fast full N-body simulations of generic
 * modified gravity: conformal coupling models", arXiv:2110.00328):
 *
 *   cloud-in-cell density  ->  nonlinear FAS multigrid solve of the
 *   scalar-field equation  ->  fifth-force gradient  (+ adjoints)
 *
 * Conventions shared by every entry point
 *   - Grids are periodic cubes of n^3 cells (n even), C-contiguous
 *     [k][j][i] with i (x) fastest, code units of Sec. 3.1.1: cell size 1,
 *     c~ = n (c/H0) / L with c/H0 = 2997.92458 Mpc/h.
 *   - Every array pointer is a DEVICE pointer owned by the caller; nothing
 *     is retained after a call returns.  Host pointers (params, options,
 *     stats, boxes) are read during the call only.
 *   - Calls are ordered on the context's HIP stream.  mg_solve,
 *     mg_solve_adjoint and mg_solve_batched synchronise that stream once per
 *     outer iteration to read the residual norm; the others are asynchronous.
 *   - Return value: MG_OK (0) or a negative MG_E* code; on MG_EINVAL no
 *     output has been written.  mg_last_error() gives a message.
 *   - A context is not thread-safe; use one context per stream.
 *
 * The solved field ("field") follows the paper's test quantities
 * (eq:field_uniform_dens_test): f(R) -> f_R (negative); symmetron ->
 * u = phi/phi_*; coupled quintessence -> phi~ = c~^2 delta-phi.
 */
#ifndef MGGPU_H
#define MGGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MG_OK = 0, MG_EINVAL = -1, MG_ENOCONV = -2, MG_ENAN = -3, MG_EHIP = -4 };

/* Models: Hu-Sawicki f(R) (Sec. 2.3, 3.2.5), symmetron (Sec. 2.2, 3.2.4),
 * coupled quintessence (Sec. 2.1, 3.2.3). */
enum { MG_FR = 0, MG_SYMMETRON = 1, MG_CQ = 2 };

/* MG_FP64: the paper's direct nonlinear Gauss-Seidel in FP64 throughout.
 * MG_FP32_REFINED: FP64 master field and FP64 residuals; each outer step
 * solves the correction equation F(w + e) - F(w) = -F(w) for e with FP32
 * multigrid, then w += e. */
enum { MG_FP64 = 0, MG_FP32_REFINED = 1 };

/* Cycle shapes (Sec. 3.2.1, fig:multigrid_cycles). */
enum { MG_CYCLE_V = 0, MG_CYCLE_F = 1, MG_CYCLE_W = 2 };

typedef struct {
  double a;          /* scale factor */
  double omega_m;    /* Omega_m today; Omega_Lambda = 1 - Omega_m */
  double box_mpch;   /* box size L in Mpc/h (sets c~) */
  int fr_n;          /* f(R): Hu-Sawicki n (eq:fR_HS): 0, 1 or 2 */
  double fr_fr0_abs; /* f(R): |f_R0| > 0 */
  double sym_a_star; /* symmetron: a_* (< a) */
  double sym_xi;     /* symmetron: xi = H0/m_* (xi c/H0 = Compton length) */
  double sym_beta_star; /* symmetron: beta_* (force prefactor only) */
  double cq_alpha;   /* CQ: alpha > 0 (eq:csf_potential) */
  double cq_beta;    /* CQ: beta (eq:csf_coupling_function) */
  double cq_phibar;  /* CQ: background field phi-bar(a) > 0 */
  double cq_lambda;  /* CQ: lambda of eq:csf_param_lambda */
  int cq_keep_exp;   /* CQ: 1 keeps exp(beta phi~/c~^2) before (1+delta) as in
                        eq:csf_eom_code; 0 drops it as the paper's runs did */
} mg_model_params;

typedef struct {
  int cycle;        /* MG_CYCLE_V / _F / _W */
  int nu_pre;       /* Gauss-Seidel sweeps (each = both colours) before coarsening, >= 0 */
  int nu_post;      /* sweeps after the correction, >= 1 */
  int inner_cycles; /* cycles between FP64 residual checks (refined mode: FP32
                       cycles per outer step); 0 = automatic: 2 before the
                       first check, then enough to reach tol at the measured
                       contraction per cycle (taken no better than 0.18 from
                       256^3 cells up) (1..8) */
  int max_cycles;   /* cap on cycles (FP64) or outer steps (refined), 1..64 */
  int precision;    /* MG_FP64 / MG_FP32_REFINED */
  int coarse_sweeps;/* cap on sweeps of the coarsest level (they stop once its
                       residual has dropped by 1e-8); 0 = default: for a
                       coarsest level of n <= 8, 24 in hierarchies of at most
                       4 levels and 8 from 5 levels up; else 2 n^2 */
  int fixed_cycles; /* 0: iterate to tol.  k > 0: run exactly k cycles from
                       field_in (or the background) with no convergence test,
                       as the paper's production runs do with two V-cycles per
                       time step warm-started from the previous step's field
                       (Sec. 4.3); returns MG_OK unless the residual is
                       non-finite.  Refined mode: one outer step of k FP32
                       cycles.  stats->rel_resid is the residual after them
                       (computed only when stats is given in FP64 mode). */
} mg_solver_opts;

typedef struct {
  int cycles;            /* FP64 residual checks (= outer steps in refined mode) */
  int status;            /* return code of the call */
  double rel_resid;      /* final RMS(d)/RMS(d at background) */
  double resid_hist[64]; /* rel_resid at each check */
  double ms_total;       /* wall time of the call (stream-synchronised) */
  int vcycles;           /* multigrid cycles run on the finest level */
  int fallback;          /* 1: the FP32-refined solve diverged and the result
                            is that of the plain FP64 solve rerun from the
                            same start */
} mg_stats;

typedef struct mg_ctx mg_ctx;

/* Create a context for n^3 grids on a HIP stream (NULL = default stream).
 * n must be even, 4 <= n <= 1600; the level pyramid is n, n/2, ... while the half
 * is even and >= 4 (4^3 coarsest for n = 2^l, 6^3 for n = 96).  Device
 * workspace is allocated on first use of each mode and kept until destroy.
 * The environment variable MGGPU_MARCH_MIN_BLOCKS, read here, sets from how
 * many workgroups up the smoother and residual/restriction kernels march in
 * z (default 4096; the results are identical either way), MGGPU_SMOOTH_MARCH_KT sets
 * the planes per thread of the z-marching FP32 smoother used on large levels
 * (default 4; 0 selects the per-row form; identical results),
 * MGGPU_PROLONG_SMOOTH_KT sets the coarse planes per workgroup (default 8;
 * 0 runs prolongation and half-sweep as separate kernels; identical
 * results) of the kernel that forms the prolonged correction inside the
 * first post-smoothing half-sweep of the f(R), symmetron and linear
 * (adjoint) FP32 cycles, used on the levels where its grid reaches
 * MGGPU_PROLONG_SMOOTH_MIN_BLOCKS workgroups (default 512; the depth is
 * halved to reach it), and
 * MGGPU_FP16_STORAGE=0 keeps the finest level's X and rho of the
 * FP32-refined solve in FP32 instead of 16-bit floats (default 1; n % 8 == 0
 * grids; changes rounding inside the FP32 correction cycles only, the FP64
 * residual and the solution's tolerance are unaffected).  MGGPU_CIC_DIRECT=1
 * makes cic_assign always take its direct atomic path (identical results).
 * Returns MG_EINVAL for a bad n or NULL out. */
int mg_ctx_create(mg_ctx **out, int n, void *hip_stream);
void mg_ctx_destroy(mg_ctx *ctx);
const char *mg_last_error(const mg_ctx *ctx);
int mg_ctx_levels(const mg_ctx *ctx);

/* Cloud-in-cell density contrast (Sec. 3.1).  pos: n_part x 3 floats (x,y,z)
 * in code units [0, n); cell c covers [c, c+1) with centre c + 1/2.  Out:
 * delta[n^3] = rho/mean - 1.  Deposits are 32.32 fixed-point integer
 * sums, so the result does not depend on the order of the particles and
 * the total mass is exact.  For n % 16 == 0 (and n_part < 2^32 - 8192) runs
 * of consecutive particles in one (16^3 tile, boundary class) bin are sorted
 * by bin and each tile is summed in LDS; otherwise each corner is a global
 * 64-bit atomic.  Particles in a spatially coherent order (a Lagrangian grid
 * order) form runs of several particles and are assigned fastest; any order
 * gives the same result.  Workspace: 16 bytes per particle (run records and
 * placed runs, at most one run per particle) plus 96 bytes per tile.
 * MG_EINVAL if n_part <= 0. */
int cic_assign(mg_ctx *ctx, const float *pos_xyz, int64_t n_part, float *delta_out);

/* Solve the model's scalar-field equation for delta (n^3 floats):
 *   f(R)      eq:fR_eom_codeunit2 (n = 1), per-cell cubic eq:fR_eom_codeunit
 *   symmetron eq:sym_eom_code_unit, per-cell cubic eq:sym_cubic_eqn
 *   CQ        eq:csf_eom_code, Newton-Gauss-Seidel eq:relaxation_iteration
 * with red-black Gauss-Seidel, FAS coarse equations
 * (eq:general_pde_numerical_coarse), 8-cell mean restriction and 27/9/3/1
 * prolongation (eq:solution_correction).  Stops when
 * RMS(d)/RMS(d at background) <= tol (Sec. 3.2.1 global residual).
 * field_in: initial guess (NULL = background value); field_out: solution
 * (n^3 doubles; may equal field_in).  Returns MG_ENOCONV with the last
 * iterate in field_out if max_cycles is reached, MG_ENAN on a non-finite
 * residual.  Divergence: when the FP64 residual has grown at two
 * consecutive checks and exceeds twice the best one, the FP64 mode stops
 * with MG_ENOCONV and the FP32-refined mode (also on a non-finite residual
 * after a finite start) reruns the plain FP64 solve once from the same
 * start and returns its result (stats->fallback = 1).  stats may be NULL.
 * Environment, read at context creation: MGGPU_TEST_CORRECTION_SCALE = s
 * scales each FP32 correction by s before it is added to the FP64 field
 * (a test hook that forces the divergence path from the host; default 1). */
int mg_solve(mg_ctx *ctx, int model, const mg_model_params *params,
             const mg_solver_opts *opts, const float *delta, const double *field_in,
             double *field_out, double tol, mg_stats *stats);

/* mg_solve without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, arithmetic and results as mg_solve (bit for
 * bit), but the call's whole workspace (the FP32-refined and the FP64 level
 * pyramids and the reduction partials) lives in one static 16 MiB device
 * array per GPU instead of the context's allocations: it calls no hipMalloc,
 * hipFree or other allocating routine, and the context must only have been
 * created (mg_ctx_create, which allocates its few scalars, at set-up).
 * Limit: the workspace of an n^3 solve must fit the array, which holds
 * n <= 64 (about 15 MB at n = 64); larger n returns MG_EINVAL.  Every call
 * on one GPU shares that GPU's array, whatever the context or stream, and
 * leaves its contents behind (the solve reads nothing it has not written):
 * calls that overlap on one GPU race. */
int mg_solve_noalloc(mg_ctx *ctx, int model, const mg_model_params *params,
                     const mg_solver_opts *opts, const float *delta, const double *field_in,
                     double *field_out, double tol, mg_stats *stats);

/* Residual of a field: d = F(field) in FP64 (n^3 doubles out, may be NULL)
 * and its RMS relative to the background residual in *rel. */
int mg_residual(mg_ctx *ctx, int model, const mg_model_params *params,
                const float *delta, const double *field, double *d_out, double *rel);

/* Fifth force g5 = -grad Phi5 by 3-point central differences (Sec. 3.1)
 * with Phi5 = -c~^2 f_R/2 (eq:F5_fR_codeunit), 3 xi^2 Om beta*^2 c~^2
 * a*^-3 u^2 (eq:F_5_codeunit) or beta phi~ (eq:csf_particle_geodesic_code2);
 * the time factor H0/a-dot is left to the caller.  Out: [3][n^3] floats. */
int mg_force(mg_ctx *ctx, int model, const mg_model_params *params, const double *field,
             float *force_out);

/* Transpose of mg_force at the given field: grad_force [3][n^3] floats ->
 * grad_field[n^3] doubles (dLoss/dfield). */
int mg_force_adjoint(mg_ctx *ctx, int model, const mg_model_params *params,
                     const double *field, const float *grad_force, double *grad_field_out);

/* Adjoint of mg_solve at a converged field: given dLoss/dfield, return
 * dLoss/ddelta = -(dF/ddelta) J^{-1} dLoss/dfield, with J = dF/dfield the
 * symmetric "Laplacian plus diagonal" Jacobian of the same equation, solved
 * by linear multigrid (FP64, or FP32 inner cycles with FP64 residuals as
 * selected by opts->precision) to ||r||/||b|| <= tol (opts->fixed_cycles is
 * ignored: the adjoint always iterates to tol).  All arrays n^3; delta
 * float, the rest double. */
int mg_solve_adjoint(mg_ctx *ctx, int model, const mg_model_params *params,
                     const mg_solver_opts *opts, const float *delta, const double *field,
                     const double *grad_field, double *grad_delta_out, double tol,
                     mg_stats *stats);

/* Loss = sum over the listed cells of |g5|^2 and its gradient with respect
 * to the force (zero elsewhere).  cells: n_cells int64 linear cell indices.
 * loss_out: one double on the device. */
int mg_loss_force_sq(mg_ctx *ctx, const float *force, const int64_t *cells, int64_t n_cells,
                     float *grad_force_out, double *loss_out);

/* One red-black half-sweep of the finest level in FP64 on a natural-layout
 * field (the smoother on its own, for parity checks): cells with
 * (i+j+k)%2 == colour are replaced by their exact per-cell solution. */
int mg_relax_halfsweep(mg_ctx *ctx, int model, const mg_model_params *params,
                       const float *delta, double *field, int colour);

/* Restriction (mean of 8 children) and prolongation-add (27/9/3/1) of
 * natural-layout double grids; coarse grids are (n/2)^3. */
int mg_restrict(mg_ctx *ctx, const double *fine, double *coarse);
int mg_prolong_add(mg_ctx *ctx, const double *coarse, double *fine);

/* ---- The particle side after the fifth force (a particle-mesh step) ---- */

/* CIC interpolation of a mesh field to particles: the same cells and weights
 * as cic_assign (Sec. 3.1), so it is that assignment's transpose.
 * grid: ncomp (1..3) components of n^3 device floats, [ncomp][k][j][i];
 * pos: [n_part][3] device floats in [0, n); out: [n_part][ncomp] device
 * floats.  Weights and sums in FP64.  n_part = 0 does nothing (pointers
 * unused); MG_EINVAL on a negative n_part, ncomp outside 1..3 or NULL. */
int mg_interp_to_particles(mg_ctx *ctx, const float *grid, int ncomp, const float *pos,
                           int64_t n_part, float *out);
/* The same for one FP64 field (n^3 doubles), out: n_part doubles. */
int mg_interp_field_to_particles(mg_ctx *ctx, const double *field, const float *pos,
                                 int64_t n_part, double *out);
/* Newtonian potential of eq:GR_poisson_codeunit on the grid: the zero-mean
 * solution of (7-point discrete Laplacian) Phi = (3/2) Omega_m a^-1 delta,
 * exact by FFT in FP64 (rocFFT, opened at first use; MG_EHIP if absent).
 * delta: n^3 device floats; phi_out: n^3 device doubles, natural layout.
 * Uses params->a and params->omega_m only. */
int mg_poisson_newton(mg_ctx *ctx, const mg_model_params *params, const float *delta,
                      double *phi_out);
/* -grad phi by central differences, (phi(c+e) - phi(c-e))/2 per axis, the
 * Newtonian force of eq:F_N_codeunit without H0/a-dot.  phi: n^3 device
 * doubles; force_out: [3][n^3] device floats (x, y, z). */
int mg_gradient(mg_ctx *ctx, const double *phi, float *force_out);
/* Total force without H0/a-dot: -grad of (s_N phi_n + Phi5(field)) by the
 * same central differences, the two potentials summed before differencing
 * as the paper does for coupled quintessence after
 * eq:csf_particle_geodesic_code2.  phi_n: the potential of the standard
 * Poisson equation (mg_poisson_newton); s_N = exp(beta phibar) for MG_CQ
 * (the background factor of eq:csf_poisson_code applied to the force) and 1
 * otherwise; Phi5 as in mg_force.  phi_n, field: n^3 device doubles;
 * force_out: [3][n^3] device floats.  MG_EINVAL for NULL arrays or bad
 * parameters. */
int mg_total_force(mg_ctx *ctx, int model, const mg_model_params *params, const double *phi_n,
                   const double *field, float *force_out);
/* Symmetron friction term dp~/da of eq:csf_particle_geodesic_qsa in code
 * units, -(dA/dphi)(d phi-bar/da) p~ with A of eq:sym_coupling_function,
 * phi_* of eq:varphi_ast and phi-bar(a) of eq:varphi_min_symm:
 * -9 Omega_m beta_*^2 xi^2 a^-4 (u(x_p) / u-bar) p_p, u-bar =
 * sqrt(1 - (a_* / a)^3) (eq:F_x_codeunit prints u-bar in place of 1/u-bar),
 * with u the solved symmetron field (n^3 device doubles) CIC-interpolated to
 * each particle.  pos, mom, out: [n_part][3] device floats.  MG_EINVAL unless
 * 0 < a_* < a; n_part = 0 does nothing. */
int mg_symmetron_friction(mg_ctx *ctx, const mg_model_params *params, const double *u_field,
                          const float *pos, const float *mom, int64_t n_part, float *out);

/* Coupled-quintessence background (Sec. 4.3, background cosmology solver;
 * eq:csf_background_eom, eq:csf_background_Friedmann,
 * eq:csf_background_Raychaudhuri and their forms in N = ln a).  Host code in
 * FP64; no context and no GPU needed.  The potential coefficient of the
 * printed forms in N is taken as lambda^2/3, lambda being that of
 * eq:csf_param_lambda (the lambda that mg_model_params.cq_lambda takes). */
typedef struct mg_cq_background_params {
  double omega_m;   /* Omega_m today, in (0, 1) */
  double h;         /* H0 / (100 km/s/Mpc), > 0 (sets Omega_r) */
  double t_cmb;     /* CMB temperature today in K (the paper: 2.7255) */
  double n_eff;     /* massless neutrino species (the paper: 3.046) */
  double alpha;     /* potential exponent, >= 0 (eq:csf_potential) */
  double beta;      /* coupling (eq:csf_coupling_function) */
  double z_init;    /* start of the integration (the paper: 1e5) */
  double phi_init;  /* phi-bar at z_init, > 0 and small */
  double dphi_init; /* d phi-bar / d ln a at z_init, small */
  double tol;       /* target |H(a=1)/H0 - 1| of the lambda shooting, > 0 */
} mg_cq_background_params;

typedef struct mg_cq_background_info {
  double lambda;  /* lambda of eq:csf_param_lambda giving H(a=1) = H0 */
  double omega_r; /* Omega_r from h, t_cmb, n_eff */
  double h_today; /* H(a=1)/H0 reached */
  int shots;      /* integrations spent on the shooting */
  long steps;     /* accepted integrator steps, all shots */
} mg_cq_background_info;

/* Solves for lambda by shooting from z_init to a = 1 (H(1) grows with
 * lambda: the bracket starts at lambda = 1 and doubles, then false position
 * until |H(1)/H0 - 1| <= tol), then integrates once more and fills
 * table[n_table][6] (host doubles, row-major) at n_table nodes uniform in
 * ln a from 1/(1+z_init) to 1, columns: a, H/H0, (dH/dt)/H0^2, phi-bar,
 * d phi-bar/da, (d phi-bar/dt)/H0.  MG_EINVAL for bad parameters,
 * n_table < 2 or NULL table; MG_ENAN if the field leaves phi-bar > 0 (or
 * the kinetic term reaches the Friedmann bound); MG_ENOCONV if no lambda
 * reaches H0 (matter and radiation alone exceed it).  info may be NULL. */
int mg_cq_background(const mg_cq_background_params *p, int n_table, double *table,
                     mg_cq_background_info *info);
/* Linear interpolation in a of every column of a table made by
 * mg_cq_background (the paper's lookup); row: 6 host doubles.  MG_EINVAL if a
 * lies outside the table. */
int mg_cq_background_at(const double *table, int n_table, double a, double *row);

/* Many independent boxes of different n and model in one call (the paper
 * runs independent realisations side by side over MPI, Sec. 3.1), each solved
 * with the scheme of mg_solve with MG_FP32_REFINED, then its force if
 * requested.  Two designs, chosen by the autotuner:
 *  - grouped level launches (teams = 2): boxes of the same (n, model) form a
 *    class; each level operation of the cycle is one launch per class with
 *    the box index in the grid, per-box constants and pointers from a table,
 *    and a per-box control word that switches a box off once it has
 *    converged or run its planned cycles; one synchronisation per outer
 *    step serves all boxes;
 *  - one persistent cooperative launch (teams = 0/1) that never has more
 *    workgroups than can be resident: each box is run by a team of
 *    workgroups, either one team per box sized by its cell count (levels of
 *    n <= 16 on one workgroup of the team) or single-workgroup teams each
 *    running a longest-first list of boxes.  Team barriers wait for a
 *    bounded time; if one times out every workgroup leaves and the call
 *    returns MG_EHIP.
 * Workspace for all boxes lives in ctx (its n is not used).  The shape
 * (design; for the persistent launch the workgroup size, 1 or 4 cells per
 * thread and the team split) comes from mg_batched_set_config if pinned,
 * else from the last tuning of this context for the same multiset of
 * (n, model), else from the cache file $MGGPU_TUNE_CACHE (default
 * $HOME/.mggpu_tune.json), else mg_batched_tune runs first.  opts->precision must be MG_FP32_REFINED and
 * opts->fixed_cycles 0.
 * Returns MG_OK when every box converged, else MG_ENAN / MG_ENOCONV
 * (per-box status in per_box, which may be NULL). */
typedef struct {
  int n;                   /* grid size of this box (even, 8 <= n <= 1024) */
  int model;               /* MG_FR / MG_SYMMETRON / MG_CQ */
  mg_model_params params;
  const float *delta;      /* n^3 device floats */
  double *field;           /* n^3 device doubles: solution out (and guess in) */
  float *force;            /* [3][n^3] device floats, or NULL */
  int field_in;            /* 1: field holds the initial guess; 0: background */
} mg_box_desc;

/* Kernel timing with HIP events recorded on the context's stream around
 * every launch of the finest-level smoothers (off by default; enabling
 * clears the totals).  Classes: MG_PROF_SMOOTH32 (FP32 correction-form
 * half-sweep), MG_PROF_SMOOTH64 (FP64 direct half-sweep), MG_PROF_LIN32 /
 * MG_PROF_LIN64 (adjoint half-sweeps).  mg_prof_read waits for the stream
 * and returns the summed duration and the launch count of one class. */
enum { MG_PROF_SMOOTH32 = 0, MG_PROF_SMOOTH64 = 1, MG_PROF_LIN32 = 2, MG_PROF_LIN64 = 3 };
int mg_prof_enable(mg_ctx *ctx, int on);
int mg_prof_read(mg_ctx *ctx, int kernel_class, double *total_ms, int64_t *launches);

int mg_solve_batched(mg_ctx *ctx, int n_box, const mg_box_desc *boxes,
                     const mg_solver_opts *opts, double tol, mg_stats *per_box);

/* Autotuner of the batched solve: times one outer step (2 FP32 cycles) of
 * the given batch with the grouped level launches and, for batches below
 * 8M cells in all, with the persistent launch for each workgroup size in
 * {256, 512, 1024}, 1 or 4 cells per thread, and both team splits; keeps
 * the fastest for this context and writes it to the cache file.
 * Overwrites nothing the caller owns.  The persistent launch is cooperative;
 * after any cooperative launch the grouped launches of the process run
 * slower (their class streams no longer overlap as well: 16.6 instead of
 * 11.8 ms for 64 boxes of 64^3..128^3), which is why larger batches do not
 * try it. */
int mg_batched_tune(mg_ctx *ctx, int n_box, const mg_box_desc *boxes,
                    const mg_solver_opts *opts, int *block_out, int *vec_out);
/* Shape the last batched call used: workgroup size, vec (1: 4 cells per
 * thread), teams (2: grouped level launches, block and vec then unused; 1:
 * persistent launch, one sized team per box; 0: persistent launch,
 * single-workgroup teams).  (0, -1, -1) before any. */
int mg_batched_config(const mg_ctx *ctx, int *block, int *vec, int *teams);
/* Pins the shape for later batched calls (block 256/512/1024, vec 0/1,
 * teams 0/1/2); block = 0 unpins.  MG_EINVAL on other values. */
int mg_batched_set_config(mg_ctx *ctx, int block, int vec, int teams);

#ifdef __cplusplus
}
#endif
#endif
