// Internal declarations of liblowmach: data layout, kernel parameter blocks,
// device reduction helpers and the host-side launch functions shared by the
// translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/lowmach.h"

namespace lm {

constexpr int kBlock = 256;          // threads per block of the cell kernels
constexpr int kBX = 64, kBY = 4;     // 2D block shape (one wavefront per row)

// Padded cell layout of one grid level. Every cell array carries one ghost
// layer per direction (2D arrays have no z ghosts). Rows are padded so that
// the first interior cell of every row starts on a 128-byte boundary.
struct Lay {
  int ndim;
  int n[3];      // interior cells per direction (n[2] = 1 in 2D)
  long s[3];     // element strides: 1, row pitch, plane pitch
  long base;     // element index of interior cell (0,0,0)
  long total;    // elements to allocate per array
  __host__ __device__ long at(int i, int j, int k) const { return base + i + j * s[1] + k * s[2]; }
  __host__ __device__ long ncells() const { return (long)n[0] * n[1] * n[2]; }
};

Lay make_layout(int ndim, const int n[3], int elem_bytes);

// Boundary description handed to kernels.
struct Bnd {
  int kind[3][2];     // LM_SIDE_* per direction and side
  int periodic[3];    // 1 if direction is periodic
  int all_periodic;
};

// Physical and discretisation constants handed to the explicit kernels.
struct Phys {
  double h[3], ih[3];
  double Pe, Pr, sigma, inv_Fr2, Da, p0, dt;
  int reacting;
  double qs, S, k, Le_F, Le_O, N_F, N_O, fshift;  // fshift = -1 - F_eps(0)
  int has_ib;
  double nu_coef;   // max(Pr, 1, 1/Le_F, 1/Le_O)
  int closed;       // 1: p0 from the conserved mass (Eq 2.40); 2: from the ODE of Eq 2.38
  double vol_out;   // Eq 2.38: volume flux out through the inflow sides (given normal velocities)
  double volume;    // domain volume
  double gamma;     // ratio of specific heats (p0_closed)
  double zeta;      // (gamma - 1)/(gamma qs): factor of the d_t p0 source (Eq 3.4b)
  double suth_C;    // > 0: Sutherland's law for kappa (Eq 4.12); 0: kappa = T^sigma
  int stage_form;   // stage kernel form (host side): 0 LDS tiles in 2D, one thread per cell in 3D; 1 LDS; 2 direct
  // stretched grid (2D): packed spacing arrays per direction (device, see
  // met_view), cell volumes on the cell layout, and the Eq 3.28 weights of
  // the mirrored pressure ghost per side; met NULL on a uniform grid
  const double *met = nullptr;
  const double *vol = nullptr;
  double gx[3][2][3] = {};
  // unequal steps (adaptive time step): AB2 weights of R^n, R^{n-1}; BDF2
  // d_t rho = (bd0 (rho^{new} - rho^n) - bd2 (rho^n - rho^{n-1})) / dt
  int var_step;
  double ab0, ab1, bd0, bd2;
};

// Thermodynamic pressure of an enclosed system, on the device (the step
// never reads it back): committed p0 at levels n, n-1, n-2, the pending
// predicted and new levels and the d_t p0 each stage's residual uses.
struct P0Dev {
  double p0[3];        // levels n, n-1, n-2
  double mass;         // conserved mass m = sum(rho dV)
  double p0_star, p0_new;
  double dtp0_n;       // d_t p0 at level n (predictor residual); 0 on the first step
  double dtp0_star;    // d_t p0 at the predicted level (corrector residual)
  double dtp0_start;   // first step: d_t p0 at level n from the balance of Eq 2.40
  double rate_prev;    // Eq 2.38 systems: d_t p0 at level n-1 (AB2 of the predictor)
  double dt_hist[2];   // sizes of the last two committed steps (newest first; adaptive steps)
  int nhist;           // committed levels before n (0, 1, 2)
};

// One time level of the state (device pointers into the workspace).
struct Level {
  double *rho, *v[3], *Z, *H, *T, *kap, *F[3];
};

// Residual set of one time level.
struct Resid {
  double *H, *Z, *v[3];
};

// Immersed-boundary arrays (padded layout; NULL when absent).
struct IB {
  const unsigned char *chi;
  const double *v_ib[3], *Z_ib, *H_ib, *S_m;
};

// Side data (compact, per side cell), device pointers or NULL: the values
// of an inflow side, or the wall H of an isothermal slip / no-slip wall.
struct SideData {
  const double *v[3], *Z, *H, *F;
  const unsigned char *wall;  // solid footprint cells of an inflow side
};

struct Sides {
  SideData s[3][2];
};

// Device scalars of the Poisson solver, one block per solve.
struct SolverScalars {
  double rzh[2];     // r.z of the last two iterations (slot = iteration & 1)
  double alh[2];     // alpha of the last two iterations (single-reduction CG)
  double rr, cc;     // last ||r||^2 and ||c||^2 (c: mean-free right-hand side)
  double mean_b, sum_b, outflow_c, mean_x;
  int done, iters, zero, nonconv;  // kept contiguous (cleared together)
  int rho_bad;                     // a density given for beta = 1/rho_f is not positive and finite
};

// Outcome of one pressure solve, written on the device when the host
// checks it later (after the step) instead of waiting for it.
struct SolveLog {
  double rr, cc, mean_b;
  int iters, done, nonconv, pad;
};

// Multigrid level storage (precision chosen at run time, hence void*).
struct MGLevel {
  Lay lay;
  void *x, *xpost, *b;  // pre- and post-smoothed correction, right-hand side
  double ih2[3];        // 1/h^2 per direction
};

// ---- helpers -------------------------------------------------------------

inline unsigned ceil_div(long a, long b) { return (unsigned)((a + b - 1) / b); }

inline dim3 grid_for(const Lay &L) {
  return dim3(ceil_div(L.n[0], kBX), ceil_div(L.n[1], kBY), L.n[2]);
}
inline long nblocks_for(const Lay &L) {
  dim3 g = grid_for(L);
  return (long)g.x * g.y * g.z;
}

// ---- launchers (explicit part, lm_explicit.hip) --------------------------
hipError_t launch_ghosts(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                         double *v[3], double *Z, double *H, double *T, double *kap);
hipError_t launch_stage(hipStream_t st, int corrector, int first, const Lay &L, const Phys &P,
                        const Level &cur, const Level &n0, const Resid &rprev, const Resid &rn,
                        const IB &ib, Level &out, double *M[3], const double *dtp0);
// Enclosed-system thermodynamic pressure (lm_explicit.hip). what:
//   0 set-up: mass of the level, p0 = params.p0, no history
//   1 predicted level: p0* = m / sum(dV/T*), rho* = p0*/T*, d_t p0 at it
//   2 new level: p0^{n+1} = m / sum(dV/T^{n+1}), rho^{n+1} = p0^{n+1}/T^{n+1}
//   3 first step, after the predictor stage kernel: d_t p0 at level n from
//     the balance of Eq 2.40, added to the stored level-n residual R_H and
//     to the Euler-predicted H* (then T*, kappa*)
//   4 commit of a completed step (history shift, d_t p0 for the next step)
// Semi-enclosed systems (Eq 2.38), on ghost-filled levels:
//   5 before the predictor stage kernel: d_t p0 at level n (lv)
//   6 after it: p0* by AB2 (Euler on the first step), rho* = p0*/T*
//   7 before the corrector stage kernel: d_t p0 at the predicted level (lv)
//   8 after it: p0^{n+1} by the trapezoid rule, rho^{n+1} = p0^{n+1}/T^{n+1}
hipError_t launch_p0(hipStream_t st, int what, const Lay &L, const Phys &P, P0Dev *p0, Level *lv, const Level *n0,
                     double *RH, double *partials);
hipError_t launch_rhs(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                      double *const M[3], const double *rho_new, const double *rho_n,
                      const double *rho_prev, int bdf2, const double *S_m, double *b,
                      double *partials, SolverScalars *sc);
hipError_t launch_project(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                          double *const M[3], const double *x, const double *rho_new,
                          const SolverScalars *sc, double *F[3], double *v[3], double *P_out,
                          int *nonfinite);
hipError_t launch_pack(hipStream_t st, const Lay &L, const double *src_compact, double *dst_padded,
                       int face_dir);
hipError_t launch_unpack(hipStream_t st, const Lay &L, const double *src_padded, double *dst_compact,
                         int face_dir);
hipError_t launch_pack_u8(hipStream_t st, const Lay &L, const unsigned char *src, unsigned char *dst);
hipError_t launch_init_state(hipStream_t st, const Lay &L, const Phys &P, const Bnd &B,
                             const Sides &sd, int from_T, Level &lv, int *bad_flag);
hipError_t launch_face_flux(hipStream_t st, const Lay &L, const Bnd &B, const Sides &sd,
                            const Level &lv, double *M[3], const double *met);
hipError_t launch_cfl(hipStream_t st, const Lay &L, const Phys &P, const Level &lv,
                      const unsigned char *chi, double *partials, double *out_max);
hipError_t launch_mean(hipStream_t st, const Lay &L, const double *a, double *partials, SolverScalars *sc,
                       const double *vol, double volume);
// Sums over cells of |v* - v^{n+1}|^2, (H* - H^{n+1})^2, (Z* - Z^{n+1})^2
// into out[0..2] (partials: at least 3 * kErrBlocks doubles).
constexpr int kErrBlocks = 256;
// y[0..n) = a x[0..n)
hipError_t launch_scale_copy(hipStream_t st, long n, double a, const double *x, double *y);
hipError_t launch_pc_err(hipStream_t st, const Lay &L, int reacting, const Level &star, const Level &nw,
                         double *partials, double *out);

// ---- adjoint (lm_adjoint.hip): 2D/3D, periodic or wall sides ----------------
struct AdjPhys {
  double h[3];
  double Pe, Pr, sigma, inv_Fr2, p0, qs, dt;
  double suth_C;  // > 0: Sutherland's law for kappa (Eq 4.12)
  double Da;      // Darcy number of the body penalisation (Eq 3.30)
  int reacting;   // flame map and Z transport (section 3.5)
  double S, k, Le_F, Le_O, N_F, N_O, fshift;
};
// Per-direction arrays hold ndim entries; Z entries are used in reacting
// flow only.
struct AdjResidArgs {
  Lay L;
  AdjPhys P;
  Bnd B;                                // periodic or slip / no-slip wall sides
  Sides sd;                             // wall values (H of isothermal walls, v)
  const double *H, *Z, *v[3], *F[3];    // level at which the residuals are taken
  const double *RbH, *RbZ, *Rbv[3];     // residual cotangents
  double *Hb, *Zb, *vb[3], *Fb[3];      // accumulated adjoints
  const unsigned char *chi;             // body mask (null: no body)
  const double *H_ib, *Z_ib, *v_ib[3];  // body targets (null: 0)
  const double *kap, *dkap;             // the level's kappa and d kappa/dT (launch_adj_kappa)
  int box_mode;                         // 0 every cell; 1 only cells in the box; 2 only cells outside it
  int box_lo[3], box_hi[3];             // inclusive cell ranges per direction
};
struct AdjProjArgs {
  Lay L;
  AdjPhys P;
  Bnd B;
  const double *Fb[3], *vb[3], *v[3], *rho;
  double *Mb[3], *rhob, *Pb;
};
// Cell-wise transposes (EOS, temperature, kinetic-energy seed, initial
// state) and the kinetic-energy sum.
struct AdjCellArgs {
  Lay L;
  AdjPhys P;
  Bnd B;
  double dV;
  const double *H, *Z, *rho, *v[3], *Fb[3], *Hb_in, *Zb_in, *rhob, *Tb;
  double *Hb, *Zb, *vb[3], *Zb0, *part;
  double *Tb_out;
};
struct AdjTailArgs {
  Lay L;
  AdjPhys P;
  Bnd B;
  int first, corrector;
  const double *bb;
  double *Mb[3];
  double *rhob_new;
  const double *H_new, *Z_new, *rho_new;
  const double *v_n[3], *rho_n;
  const double *Hb_out, *Zb_out, *RbH_out, *RbZ_out, *Rbv_out[3], *rhoprevb_out;
  double *Hb_star, *Zb_star;
  double *Hb_n, *Zb_n, *vb_n[3], *rhob_n;
  double *RbH_star, *RbZ_star, *Rbv_star[3];
  double *RbH_n, *RbZ_n, *Rbv_n[3];
  double *rhoprevb_in, *RbH_prev_in, *RbZ_prev_in, *Rbv_prev_in[3];
};
hipError_t launch_adj_resid(hipStream_t st, const AdjResidArgs &a);
hipError_t launch_adj_proj(hipStream_t st, const AdjProjArgs &a);
hipError_t launch_adj_tail(hipStream_t st, const AdjTailArgs &a);
// (Hb, Zb) += d rho/d(H, Z) rhob (H, Z, rho, rhob -> Hb, Zb)
hipError_t launch_adj_eos(hipStream_t st, const AdjCellArgs &a);
// (Hb, Zb) += transpose of T(Z, H) applied to Tb (H, Z, Tb -> Hb, Zb)
hipError_t launch_adj_add_T(hipStream_t st, const AdjCellArgs &a);
// kinetic-energy cotangent (dV, H, Z, rho, v -> Hb, Zb, vb)
hipError_t launch_adj_seed_ke(hipStream_t st, const AdjCellArgs &a);
// initial-state transpose (H, Z, rho, v, Fb, Hb_in, Zb_in -> Tb_out, Zb0, vb += )
hipError_t launch_adj_init(hipStream_t st, const AdjCellArgs &a);
// kappa(T(Z, H)) and d kappa/dT of a level's cells (H, Z -> Hb: kappa,
// Zb0: d kappa/dT)
hipError_t launch_adj_kappa(hipStream_t st, const AdjCellArgs &a);
hipError_t launch_ke(hipStream_t st, const Lay &L, const double *rho, double *const v[3], double dV, double *part,
                     double *out);
// out = 2 x1 - x2 on the cells (extrapolated initial guess).
hipError_t launch_adj_extrap(hipStream_t st, const Lay &L, const double *x1, const double *x2, double *out);
// Transpose of the outflow closure of a high outflow side in direction d:
// y += (-sum_side y/h - sum_side Fb) dV/area (scratch: one double).
hipError_t launch_adj_outflow(hipStream_t st, const Lay &L, const AdjPhys &P, int d, double *y, const double *Fb,
                              double *scratch);
hipError_t launch_shift(hipStream_t st, const Lay &L, const double *x, const SolverScalars *sc, double *out);

// ---- Poisson (lm_solver.hip) -----------------------------------------------
// Bump allocator over the caller workspace; with base == nullptr it only
// counts bytes (sizing pass).
struct Carver {
  char *base;
  size_t off;
  void *take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void *p = base ? (void *)(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

constexpr int kMaxLev = 24;
constexpr long kCoarseCells = 4096;   // levels at or below this size: one-block LDS kernel
constexpr long kMaxCoarsest = 1024;   // dense pseudo-inverse limit
constexpr int kVcCoarsest = 128;      // coarsest cells of a variable-coefficient solve (inverse built on the device)

struct PoissonWS {
  int met = 0;             // stretched 2D grid: volume-weighted operator (set before poisson_plan)
  double *vol = nullptr;   // its cell volumes (fine layout, FP64)
  double *met_w = nullptr; // its cell widths per level and direction (x then y, level after level)
  double volume = 0.0;     // its domain area (the weight of the solution mean)
  void *met_tab = nullptr; // its coarse-level spacing tables (MG precision)
  Lay lay;                 // fine layout (FP64 CG vectors)
  Bnd bnd;
  int nlev, lc;            // MG levels; first level handled by the coarse kernel
  int mixed, nu;
  MGLevel lev[kMaxLev];    // level 0 uses r, zpre and z below
  int tx[kMaxLev], ty[kMaxLev];  // 2D tile of the fused level kernels (0: level not tiled)
  double *x, *r[2], *p[2], *q;
  int cgcg;                // single-reduction (Chronopoulos-Gear) CG in FP64 mode
  int block_pcg;           // the whole solve in one workgroup (finest level <= kCoarseCells)
  double *blk;             // its scratch (face coefficients, p, s)
  double tol2;             // rtol^2 of the solve in progress
  double *w, *s[2];        // its A u and s = A p vectors
  void *z[2];              // preconditioned residuals in MG precision
  void *zpre;              // finest-level pre-smoothed correction
  void *pinv;              // dense pseudo-inverse of the coarsest operator
  double *part_cc, *part_pq, *part_rz;  // per-block partial sums
  long np_max;
  double *partials;        // scratch partials of once-per-solve reductions
  SolverScalars *sc;       // device scalars
  SolverScalars *host_sc;  // pinned host copy
  // variable-coefficient form A P = sum_d delta_1 (beta delta_1 P), beta = 1/rho_f
  int vc_cap;              // arrays below reserved
  int vc;                  // the solve in progress uses beta = 1/rho_f
  int vtx[kMaxLev], vty[kMaxLev];  // 2D tile of the variable-coefficient level kernels
  double *rho64;           // finest-level density (FP64, fine layout)
  void *rho[kMaxLev];      // density per level in MG precision (level 0 aliases rho64 in FP64)
  void *rho_c;             // densities of the coarse-kernel levels, packed as its LDS
  void *pinv_vc;           // pseudo-inverse of the coarsest variable-coefficient operator
  void *cf[kMaxLev][3];    // tiled 2D levels: west-face and south-face beta, 1/diagonal of L
  hipEvent_t *tev;         // in-step timing of the finest down kernel: event pairs
  int *tk;                 // CG iteration of each timed launch; -1: not a full-work launch
  int tcap, tcount, tsolve0;
  int twhich;              // timed kernel class (see lm_kernel_timing)
};

// Plans the hierarchy and carves (or sizes, base == nullptr) the solver
// arrays. Returns false if the grid does not coarsen to <= kMaxCoarsest cells.
bool poisson_plan(PoissonWS &ws, Carver &cv, const Lay &fine, const Bnd &B, const double h[3], int mixed, int flexible,
                  int nu, int vc_cap, std::string *err);
// Host-side set-up of the coarsest-level pseudo-inverse (after carving).
hipError_t poisson_setup(hipStream_t st, PoissonWS &ws, const double h[3]);
// The same pseudo-inverse built on the device (one block, Gauss-Jordan in
// LDS); needs a coarsest level of <= kVcCoarsest cells
// (hipErrorInvalidValue otherwise).
hipError_t poisson_setup_device(hipStream_t st, PoissonWS &ws);
// Solve A x = b for the zero-mean x (A P = sum_d delta_1 delta_1 P with
// zero-flux non-periodic sides), warm-started from x0 (NULL = 0). b is read
// with sc->mean_b and the outflow shift sc->outflow_c removed on the fly.
// The solution stays in ws.x with its mean in sc->mean_x. With log (only
// when ws.block_pcg) the call returns once the solve is queued and its
// outcome lands in *log on the device; iters, relres and converged are then
// not written.
hipError_t poisson_solve(hipStream_t st, PoissonWS &ws, const double *b, const double *x0, double rtol,
                         int maxit, int expect_iters, int *iters, double *relres, int *converged,
                         SolveLog *log = nullptr);
// Prepares a variable-coefficient solve from the density in ws.rho64 (fine
// layout): the density on every level (2^d-cell averages), the packed
// coarse-level densities and the coarsest pseudo-inverse. Sets
// sc->rho_bad when a density is not positive and finite. The caller then
// sets ws.vc for the solve.
hipError_t poisson_set_beta(hipStream_t st, PoissonWS &ws);
// Stretched 2D grid (ws.met, planned with vc_cap): from the finest cell
// widths wx (n[0]) and wy (n[1]) (host arrays), every level's cell ratios
// dx/dy, the finest cell volumes, the packed coarse-level ratios and the
// coarsest pseudo-inverse; leaves ws.vc set for every later solve.
hipError_t poisson_set_metric(hipStream_t st, PoissonWS &ws, const double *wx, const double *wy);
// One launch of a solver kernel class for timing (see lm_bench_kernel);
// the caller has cleared sc->done. Returns hipErrorInvalidValue for an
// unknown class.
hipError_t poisson_bench_launch(hipStream_t st, PoissonWS &ws, int which);

}  // namespace lm
