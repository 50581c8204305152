/*
 * lowmach.h - C ABI of liblowmach.so, an MI355X (gfx950) implementation of one
 * predictor-corrector time step of the low-Mach fractional-step method of
 * Severino et al., "Numerical method for strongly variable-density flows at
 * low Mach number" (section 3).
 *
 * Conventions
 *  - Every entry point returns an lm_status; lm_last_error() gives the text of
 *    the last failure on a context. Entry points never abort the process.
 *  - All arrays crossing the ABI are float64, C order with x fastest: a cell
 *    field has shape (nz, ny, nx) (2D: (ny, nx)); a face-flux array F_d has
 *    n_d + 1 entries along direction d (entry f is the face between cells f-1
 *    and f), the interior count along the others. Pointers are host or device
 *    memory as the `mem` argument says (LM_HOST / LM_DEVICE); nothing is
 *    retained after a call returns. Device copies are ordered on the
 *    context's stream; host copies complete before the call returns.
 *  - The caller owns the device workspace (lm_workspace_size bytes, 256-byte
 *    aligned) and the HIP stream. The context carves every device array from
 *    the workspace and never calls hipMalloc; it allocates only a small host
 *    struct and a few bytes of pinned host memory for solver flags.
 *  - A context is not thread safe; use one context per stream.
 */
#ifndef LOWMACH_H
#define LOWMACH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lm_ctx lm_ctx;

typedef enum {
  LM_OK = 0,
  LM_EINVAL = -1,        /* invalid argument (sizes, parameters, non-positive T) */
  LM_ENOMEM = -2,        /* workspace smaller than lm_workspace_size */
  LM_EHIP = -3,          /* a HIP runtime call failed */
  LM_ENOCONV = -4,       /* Poisson solver hit poisson_maxit before poisson_rtol */
  LM_ENONFINITE = -5,    /* a NaN/Inf appeared in the step */
  LM_ESTATE = -6,        /* call out of order (e.g. lm_step before lm_set_fields) */
  LM_EUNSUPPORTED = -7   /* valid request that is not implemented    */
} lm_status;

/* Side kinds (section 3.6 ghost rules, section 3.3 flux boundary conditions). */
enum {
  LM_SIDE_PERIODIC = 0, /* Eq 3.45 for all fields                              */
  LM_SIDE_SLIP = 1,     /* zero normal flux; normal v Dirichlet 0 (Eq 3.43),   */
                        /* tangential v, Z, H Neumann 0 (Eq 3.44)              */
  LM_SIDE_NOSLIP = 2,   /* zero normal flux; v Dirichlet 0; Z, H Neumann 0     */
  LM_SIDE_INFLOW = 3,   /* given normal mass flux; v, Z, H Dirichlet (given)   */
  LM_SIDE_OUTFLOW = 4   /* v, Z, H extrapolated (Eq 3.46); flux extrapolated   */
                        /* and shifted uniformly to close global mass          */
};

enum { LM_FP64 = 0, LM_MIXED = 1, LM_MIXED_FLEXIBLE = 2 };   /* Poisson preconditioner precision */
enum { LM_BETA_ONE = 0, LM_BETA_INV_RHO = 1 };  /* Poisson face coefficient forms (lm_params)   */
enum { LM_HOST = 0, LM_DEVICE = 1 };  /* where caller arrays live           */

/* Grid: ndim in {2,3}; n[d] interior cells and L[d] length per direction
 * (n[2] = 1, L[2] ignored in 2D); bc[d][0] / bc[d][1] the low / high side.
 * faces[d] (host, may be NULL): the n[d] + 1 face coordinates of a
 * stretched direction, strictly increasing from 0 to L[d] (section 3.2.1:
 * the operators of Eq 3.20-3.21 take the local spacings; each cell centre
 * is the midpoint of its faces, ghost cells mirror the first interior cell
 * at a wall). Copied at init, not kept. Stretched grids: 2D, no outflow
 * side, no adjoint, the step's constant-coefficient Poisson operator only
 * (poisson_beta LM_BETA_ONE), p0_closed 0 or 1; otherwise LM_EUNSUPPORTED. */
typedef struct {
  int ndim;
  int n[3];
  double L[3];
  int bc[3][2];
  const double *faces[3];
} lm_grid;

/* Dimensionless parameters (section 2.6, Eq 2.42-2.50; section 4.1):
 *  Re, Pr        Pe = Re Pr; viscous factor Pr/Pe (Eq 2.43)
 *  sigma         kappa = T^sigma (Eq 2.50) unless sutherland_C > 0
 *  inv_Fr2       buoyancy 1/Fr^2 (Eq 2.43, 3.8b)
 *  reacting      0: Z not transported, T = qs (H - 1); 1: flame sheet
 *  S, qs         generalised stoichiometric coefficient; qs = Q/(S+1)
 *  eps, tol      regularisation width and tolerance (section 3.5, Eq 3.34)
 *  Le_F, Le_O    fuel / oxidiser Lewis numbers (Eq 3.35)
 *  Da_ib         immersed-boundary Darcy number (Eq 3.30-3.32)
 *  p0            constant thermodynamic pressure (Eq 2.41)
 *  dt            time step; 0 = fixed once from cfl and the initial state
 *  cfl           CFL number used when dt == 0
 *  precision     LM_FP64: FP64 V-cycle in FP64 single-reduction CG;
 *                LM_MIXED: FP32 V-cycle in the same FP64 single-reduction
 *                CG (residual, operator, dot products and updates FP64);
 *                LM_MIXED_FLEXIBLE: FP32 V-cycle in FP64 flexible
 *                (Polak-Ribiere) CG
 *  poisson_rtol  stop when ||b - A P||_2 <= rtol ||b||_2 (b mean-free)
 *  poisson_maxit iteration cap (LM_ENOCONV beyond it)
 *  mg_nu         smoothing sweeps per level and direction (0 = default 2)
 *  with_ib       1 = reserve immersed-boundary arrays (needed by lm_set_fields
 *                with a non-NULL lm_ib)
 *  with_adjoint  1 = reserve the adjoint arrays (lm_step_adjoint and its
 *                helpers; FP64, constant p0, fixed dt; the grids and sides
 *                listed at lm_adjoint)
 *  poisson_beta  LM_BETA_ONE (0): the step's operator only; LM_BETA_INV_RHO:
 *                also reserve the arrays of the variable-coefficient form
 *                beta = 1/rho_f for lm_project with a density (needs a grid
 *                that coarsens to <= 128 cells). The step itself always
 *                uses beta = 1: its constraint is on the mass flux
 *                (Eq 3.9, 3.24), for which the density never enters A.
 *  p0_closed     0: p0 constant (open or periodic systems, Eq 2.41);
 *                1: enclosed system: p0 = m / integral(1/T) dV with the mass
 *                m of the initial state (Eq 2.40), the predicted and new
 *                levels' p0 from their temperatures before rho = p0/T
 *                (Eq 3.6, 3.15), and the source zeta d_t p0 inside the
 *                (1/rho)[...] of the excess-enthalpy residual (Eq 3.4b),
 *                zeta = (S+1)(gamma-1)/(gamma Q) = (gamma-1)/(gamma qs),
 *                d_t p0 by BDF2 over the levels before (Eq 3.5, 3.14; BDF1
 *                with one earlier level; on the first step from the time
 *                derivative of Eq 2.40 with the step's residuals). Needs
 *                non-reacting flow, periodic or wall sides and no mass
 *                source S_m (LM_EUNSUPPORTED / LM_EINVAL otherwise); p0 is
 *                then the initial thermodynamic pressure;
 *                2: semi-enclosed system: p0 from the ordinary differential
 *                equation of Eq 2.38, d_t p0 = (gamma/V) [qs/Pe
 *                int (div(kappa grad H) + N'(Z) div(kappa grad Z)) dV
 *                - p0 int div v dV], the first integral the sum over cells
 *                of the H residual's diffusion term (the boundary faces'
 *                conductive fluxes) plus, with reaction, N' of Eq 2.39
 *                (Heaviside regularised as in Eq 3.35) times the Z
 *                diffusion term; the second the volume flux out through
 *                the inflow sides (their given normal velocities); p0
 *                advanced by the step's AB2 predictor (Euler on the first
 *                step) and trapezoid corrector, each level's rate entering
 *                its residual as d_t p0 (Eq 3.4b). Inflow sides and
 *                reacting flow are allowed; outflow sides, S_m and
 *                immersed bodies (Eq 2.38 has no term for the heat of the
 *                penalisation) are not
 *  gamma         ratio of specific heats (p0_closed only; > 1)
 *  sutherland_C  0: kappa = T^sigma; C > 0: Sutherland's law
 *                kappa = T^{3/2} (1 + C) / (T + C) (Eq 4.12), C the
 *                Sutherland temperature over the reference temperature
 *  dt_tol        0: fixed time step. > 0: adaptive step driven by the
 *                predictor-corrector difference (the local-error estimate
 *                of the step, O(dt^3)): err = the largest of the RMS of
 *                |v* - v^{n+1}|, of H* - H^{n+1} and (reacting) of
 *                (Z* - Z^{n+1})/(S+1). After the fourth or a later step of
 *                exactly one size, the factor 0.9 (dt_tol/err)^{1/3}
 *                (in [0.5, 1.5]) is applied when it lies outside
 *                [0.9, 1.1]; growth stops at the CFL step of the new state
 *                (cfl > 0 required) and the step drops to 0.9 of it when
 *                that falls below the current step. Unequal steps use
 *                Adams-Bashforth 2 and BDF2 for unequal spacing (also for
 *                the d_t p0 of p0_closed systems). Steps are never
 *                rejected. Not with with_adjoint.                         */
typedef struct {
  double Re, Pr, sigma, inv_Fr2;
  int reacting;
  double S, qs, eps, tol, Le_F, Le_O;
  double Da_ib, p0, dt, cfl;
  int precision;
  double poisson_rtol;
  int poisson_maxit;
  int mg_nu;
  int with_ib;
  int with_adjoint;
  int poisson_beta;
  int p0_closed;
  double gamma;
  double sutherland_C;
  double dt_tol;
} lm_params;

/* Field set for lm_set_fields / lm_get_fields; NULL entries are skipped.
 * rho is output only (always p0/T). P holds P = p dt (Eq 3.8c).           */
typedef struct {
  double *rho, *v[3], *Z, *H, *T, *P, *F[3];
} lm_fields;

/* Immersed-boundary data (section 3.4): chi mask (0/1 bytes), targets of
 * Eq 3.30-3.32 and the mass source S_m of Eq 3.33; NULL = zero.           */
typedef struct {
  const unsigned char *chi;
  const double *v_ib[3], *Z_ib, *H_ib, *S_m;
} lm_ib;

/* Boundary data of one side: per-cell arrays over the side (C order, the
 * side's own direction removed).
 * Inflow side: NULL = zero. `wall` (bytes, NULL = none) flags cells of the
 * side covered by a solid footprint: there Z and H take zero-gradient
 * ghosts (Eq 3.44) instead of Dirichlet ones (Eq 3.43); give F = 0 and
 * v = 0 on those cells.
 * Slip or no-slip wall: only H may be given (the other entries must be
 * NULL): the wall is then isothermal, H Dirichlet with the given wall
 * values (Eq 3.43, Eq 4.16a-b) instead of zero-gradient (adiabatic,
 * Eq 4.16c); H = NULL makes it adiabatic again. Non-reacting flow only.
 * The conductivity of an isothermal wall's faces is that of the wall
 * temperature T_w = qs (H_w - 1): the mirrored ghost temperature
 * 2 T_w - T can leave the range where kappa(T) is defined.               */
typedef struct {
  const double *v[3], *Z, *H, *F;
  const unsigned char *wall;
} lm_side_data;

typedef struct {
  int steps;                 /* steps taken by the call                      */
  double dt;                 /* size of the last step taken (lm_get_dt: next) */
  double time;               /* simulated time since lm_set_fields           */
  int poisson_iters[2];      /* last step: predictor, corrector iterations   */
  double poisson_relres[2];  /* last step: final recursive relative residual */
  double compat[2];          /* last step: mean(b) removed before each solve */
  long long total_poisson_iters;
  double p0;                 /* thermodynamic pressure at the end of the call */
  double pc_err;             /* adaptive steps: last step's error estimate    */
  int pc_err_used;           /* adaptive steps: 1 if it decided the next step */
} lm_step_stats;

/* RHS-mode projection: solve A P = b for the zero-mean P, with
 * A P = sum_d delta_1 (beta delta_1 P) (Eq 3.24 composed with Eq 3.23).
 * rho NULL: beta = 1 (the step's operator). rho given (a cell field, same
 * layout and `mem` as b; needs params.poisson_beta = LM_BETA_INV_RHO, else
 * LM_EUNSUPPORTED): beta = 1/rho_f on every face, rho_f = (rho_a + rho_b)/2
 * the two-point face average of the adjacent cells (Eq 3.20, n = 1), i.e.
 * the variable-coefficient form div(grad P / rho) = b; zero flux through
 * non-periodic sides either way; LM_EINVAL if rho is not positive and
 * finite everywhere. b is a cell field (mem says where); the solve starts
 * from zero in solver scratch and P (NULL: not returned) receives the
 * zero-mean solution; the context's state, its pressure included, is left
 * as it was. rho is copied; no pointer is kept.                           */
typedef struct {
  const double *b;
  const double *rho;
  double *P;
  int mem;
  double rtol;               /* 0 = params.poisson_rtol                     */
  int iters;                 /* out */
  double relres;             /* out */
  double mean_b;             /* out: compatibility residue removed          */
} lm_project_args;

/* Bytes of device workspace needed for (grid, params). */
lm_status lm_workspace_size(const lm_grid *grid, const lm_params *params, size_t *bytes);

/* Create a context on the current HIP device over a caller workspace of
 * `bytes` bytes (>= lm_workspace_size) and a caller stream (hipStream_t,
 * NULL = default stream). Errors: LM_EINVAL (bad grid: ndim, n < 4, a
 * periodic pair broken, non-positive L; bad params), LM_ENOMEM.
 * The environment variable LM_STAGE_KERNEL, read here, picks the form of
 * the explicit stage kernel: unset, the LDS halo-tile kernel in 2D and the
 * one-thread-per-cell kernel in 3D; "lds" or "direct", that form in both
 * (grids whose planes do not tile by 64 x 4, and 3D grids with an
 * immersed body, always take the one-thread-per-cell kernel). The forms
 * compute the same arithmetic. LM_BLOCK_PCG=0, also read here, keeps
 * grids of at most 4096 cells on the multi-kernel pressure solve (by
 * default their whole solve runs in one workgroup and lm_step checks its
 * outcome after the step); the equations and the tolerance are the same.   */
lm_status lm_init_grid(const lm_grid *grid, const lm_params *params, void *dev_workspace,
                       size_t bytes, void *hip_stream, lm_ctx **out);

/* level 0: set the state at time n from T (or H) and v, optionally Z, P
 * and F (section 3.1 start-up). H is obtained by inverting Eq 3.42 when T is
 * given; T is re-evaluated from (Z, H) and rho = p0/T (Eq 2.49). Unless F is
 * given, F_d is the face average of rho v (Eq 3.20, n = 1). Setting level 0
 * clears the level n-1 history, so the next step is a Heun start (Euler
 * predictor, BDF1 density derivative). `ib` may be NULL.
 * level 1 (after level 0): the fields at time n-1 (T or H, v, optionally Z
 * and F as for level 0; P is not used; `ib` must be NULL, the body is that
 * of level 0). The library forms from them the history the next step reads:
 * rho^{n-1} = p0/T^{n-1} and the residuals R_Z, R_H, R_v at level n-1
 * (Eq 3.2, 3.4, 3.8), so the next step takes the AB2 predictor (Eq 3.1, 3.3,
 * 3.10) and the BDF2 density derivative (Eq 3.11, 3.19) instead of the Heun
 * start; the step from n-1 to n is taken to have the current step size.
 * Needs a constant p0 (p0_closed = 0, else LM_EUNSUPPORTED); LM_ESTATE
 * before level 0. LM_EINVAL if T <= 0 anywhere; other levels
 * LM_EUNSUPPORTED.                                                        */
lm_status lm_set_fields(lm_ctx *ctx, int level, const lm_fields *f, const lm_ib *ib, int mem);

/* Boundary data of side (d, side), side 0 = low, 1 = high: an inflow side,
 * or the wall temperature of a slip / no-slip wall (see lm_side_data).
 * LM_EINVAL for periodic or outflow sides, entries a wall cannot take;
 * LM_EUNSUPPORTED for an isothermal wall in reacting flow.                */
lm_status lm_set_side(lm_ctx *ctx, int d, int side, const lm_side_data *data, int mem);

/* Advance nsteps predictor-corrector steps (section 3.1, Eq 3.1-3.19).
 * On LM_ENOCONV / LM_ENONFINITE from a stage the state stays at the last
 * completed step. With an adaptive step (dt_tol > 0), a non-finite error
 * estimate or CFL step after a step returns LM_ENONFINITE with that step
 * committed. Either way stats (if not NULL) gives the steps completed,
 * the step size and the time reached.                                     */
lm_status lm_step(lm_ctx *ctx, int nsteps, lm_step_stats *stats);

/* Poisson solve in RHS mode (see lm_project_args). */
lm_status lm_project(lm_ctx *ctx, lm_project_args *args);

/* Copy a level into caller arrays: level 0, the current state (time n);
 * LM_LEVEL_PREDICTED, the predicted level of the last step taken (the
 * starred fields of Eq 3.1-3.11 and P*; the difference to level 0 is the
 * step's predictor-corrector difference, Tab 2). LM_ESTATE if no step was
 * taken since lm_set_fields / lm_load_state; LM_EUNSUPPORTED for other
 * levels.                                                                */
enum { LM_LEVEL_PREDICTED = 2 };
lm_status lm_get_fields(lm_ctx *ctx, int level, lm_fields *f, int mem);

/* The time step of the next lm_step (fixed once after lm_set_fields when
 * params.dt == 0; updated after every step when params.dt_tol > 0). */
lm_status lm_get_dt(const lm_ctx *ctx, double *dt);

/* ---- checkpoint / restart ------------------------------------------------
 * The complete state of a context (level n, its pressure, the level n-1
 * density and residuals used by the next AB2/BDF2 step, the step counter,
 * the time and, for an enclosed system, the p0 history and mass) copied to or from a caller device buffer of
 * lm_state_size bytes; restoring it and stepping reproduces the original
 * run bit for bit.                                                          */
lm_status lm_state_size(const lm_ctx *ctx, size_t *bytes);
lm_status lm_save_state(lm_ctx *ctx, void *dev_buf);
lm_status lm_load_state(lm_ctx *ctx, const void *dev_buf);

/* ---- adjoint of the step (reverse mode, hand-written) ---------------------
 * The adjoint state is the cotangent of the context's state: fields H, v,
 * F (faces) and the history rho^{n-1}, R_H^{n-1}, R_v^{n-1}, with ndim
 * entries in each per-direction array (the rest are ignored), and in
 * reacting flow also Z and R_Z^{n-1}. Supported for 2D and 3D grids on
 * uniform spacing whose sides are periodic, slip or no-slip walls
 * (isothermal or adiabatic) or inflow, with an outflow side on the high
 * end of at most one direction, in FP64, reacting or not, with or without
 * an immersed body (the body arrays, wall and inflow values are constants
 * of the step: they carry no cotangent) (params with_adjoint = 1;
 * otherwise LM_EUNSUPPORTED). Face cotangents: a wall or inflow face
 * carries a constant flux and its cotangent is 0; an outflow face flux is
 * a state variable; face 0 of a periodic direction duplicates face n,
 * whose cotangent holds the pair's.                                        */
typedef struct {
  double *H, *v[3], *F[3], *rho_prev, *R_H, *R_v[3];
  double *T;   /* lm_adjoint_set only: a cotangent of the temperature,
                  folded into those of H and Z by the transpose of
                  T = qs (F~(Z) + H) (Eq 3.42; qs (H - 1) without reaction):
                  H_bar += qs T_bar, Z_bar += qs F~'(Z) T_bar at the
                  current state, on the device; ignored by lm_adjoint_get */
  double *Z, *R_Z; /* reacting flow only (else NULL): the cotangents of Z
                      and of R_Z^{n-1}                                    */
} lm_adjoint;

/* Kinetic energy sum_cells 1/2 rho |v|^2 dV of the current state (uniform
 * grids; LM_EUNSUPPORTED on stretched ones). */
lm_status lm_kinetic_energy(lm_ctx *ctx, double *ke);
/* Adjoint state := d(kinetic energy)/d(state) at the current state. */
lm_status lm_adjoint_seed_ke(lm_ctx *ctx);
/* Adjoint state := the given cotangents (NULL entries = 0). */
lm_status lm_adjoint_set(lm_ctx *ctx, const lm_adjoint *a, int mem);
lm_status lm_adjoint_get(lm_ctx *ctx, lm_adjoint *a, int mem);
/* One step back: with the forward state at level n and the adjoint state
 * holding the cotangent of the state at n+1, replace it by the cotangent of
 * the state at n (the step is recomputed internally; the forward state is
 * left at n). Each stage needs one adjoint Poisson solve with the same
 * symmetric operator, started from that stage's solution of the previous
 * lm_step_adjoint call since the last lm_adjoint_set / lm_adjoint_seed_ke,
 * or the linear extrapolation of its last two (a reverse sweep steps back
 * in time; the tolerance is poisson_rtol as ever); errors as lm_step.      */
lm_status lm_step_adjoint(lm_ctx *ctx);
/* The reverse step without the recompute, for callers that replay steps
 * anyway (a checkpointed reverse sweep): right after lm_step took one step
 * from a state, lm_save_step_levels copies that step's predicted level (rho,
 * H, Z in reacting flow, v, F) and its new level (rho, H, Z, v) into a
 * caller device buffer of lm_step_levels_size bytes (LM_ESTATE when no step
 * was taken since the state was set or loaded); with the state restored to
 * the one the step was taken from, lm_step_adjoint_levels does what
 * lm_step_adjoint does, reading those levels instead of recomputing them
 * (the same results bit for bit). The buffer is read, not kept.            */
lm_status lm_step_levels_size(const lm_ctx *ctx, size_t *bytes);
lm_status lm_save_step_levels(lm_ctx *ctx, void *dev_buf);
lm_status lm_step_adjoint_levels(lm_ctx *ctx, const void *dev_buf);
/* With the forward state freshly set from (T0, v0) (and Z0 in reacting
 * flow) by lm_set_fields and the adjoint state holding its cotangent:
 * cotangents of T0, v0 and Z0 (through H0 = T0/qs - F~(Z0), or T0/qs + 1
 * without reaction, rho0 = p0/T0, F0 = face average of rho0 v0). v0_bar
 * entries and Z0_bar may be NULL; Z0_bar must be NULL without reaction
 * (LM_EINVAL).                                                             */
lm_status lm_adjoint_initial(lm_ctx *ctx, double *T0_bar, double *v0_bar[3], double *Z0_bar, int mem);

/* Kernel timing hook: launches one kernel class `reps` times back to back on
 * the context's stream between two HIP events and returns the mean duration
 * of one launch in *avg_ms. Needs a state (after lm_set_fields); the kernels
 * write solver scratch arrays and the predicted level only, and the next
 * lm_step recomputes those. which:
 *   0 finest multigrid down kernel (fused) or one half-sweep
 *   1 predictor stage kernel                   2 CG direction update + operator
 *   3 finest multigrid up kernel (fused) or the restriction
 *   4 CG solution/residual update              5 coarse-grid V-cycle block
 *   6 Poisson right-hand side                  7 projection                    */
lm_status lm_bench_kernel(lm_ctx *ctx, int which, int reps, double *avg_ms);

/* In-step timing of one solver kernel class, which = 0: the finest
 * multigrid down kernel (the fused 2D or 3D level kernel); 1: the finest
 * fused 3D up kernel; 2: the separate single-reduction CG update (grids
 * whose finest level is not a fused 2D one). With capacity > 0, the next
 * launches of that kernel made by lm_step (up to capacity of them) each
 * carry a start and a stop HIP event bound to the dispatch on the context's
 * stream (recorded when the kernel starts and ends, so the queueing gap
 * before it is not counted); capacity = 0 stops and releases the events.
 * lm_kernel_timing_read waits for the stream, then returns the mean
 * event-measured duration (ms) and the number of the recorded launches
 * that did the full work of a CG iteration with a previous direction
 * (iterations 2 .. the solve's iteration count: launches queued after
 * convergence return at once);
 * 0 when the grid has no such kernel. LM_EINVAL for another which.       */
lm_status lm_kernel_timing(lm_ctx *ctx, int which, int capacity);
lm_status lm_kernel_timing_read(lm_ctx *ctx, double *avg_ms, int *count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * RHS-mode solve of lm_project (beta = 1, zero-mean P with A P = b, the
 * same multigrid-preconditioned CG and stopping rule) in one call, with no
 * context, no workspace and no allocation. Every solver array lives in a
 * static device buffer of 64 MiB that the library holds on each GPU it runs
 * on until the process ends (enough for about 512^2 or 64^3 cells in FP64).
 * grid, params: as for lm_init_grid (params gives precision, mg_nu,
 * poisson_rtol and poisson_maxit); stream: a hipStream_t (NULL = default
 * stream), the call returns after it has drained. args: b (required) and P
 * (NULL: not returned) are cell fields in C order, host or device as
 * args->mem says; rho must be NULL; rtol 0 = params->poisson_rtol; iters,
 * relres and mean_b are written as for lm_project. The solve starts from
 * zero. Errors (text by lm_last_error(NULL)): LM_EINVAL for bad arguments,
 * LM_EUNSUPPORTED for a density or a grid whose coarsest multigrid level
 * has more than 128 cells, LM_ENOMEM when the grid needs more than the
 * 64 MiB (checked before any device work), LM_ENOCONV, LM_EHIP. All calls on
 * one GPU share its buffer: calls that overlap on one GPU (from several
 * threads or streams) race and must be serialised by the caller.          */
lm_status lm_project_static(const lm_grid *grid, const lm_params *params, void *hip_stream,
                            lm_project_args *args);

/* Text of the last error of ctx; with ctx == NULL, of the last failed
 * lm_workspace_size, lm_init_grid or lm_project_static of the calling
 * thread. */
const char *lm_last_error(const lm_ctx *ctx);

/* Release the context (the caller still owns workspace and stream). */
void lm_destroy(lm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LOWMACH_H */
