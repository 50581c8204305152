// C ABI of liblowmach: context, workspace carving, field transfer and the
// predictor-corrector step driver (section 3.1 of Severino et al.).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lm_internal.h"

using namespace lm;

// Cotangent of the context's state (per-direction entries beyond ndim are
// unused and null).
struct AdjState {
  double *H, *Z, *v[3], *F[3], *rho_prev, *R_H, *R_Z, *R_v[3];
};
// Work arrays of one reverse step.
struct AdjWork {
  double *Mb[3], *rhob_new, *Pb, *bb;
  double *Hb_star, *Zb_star, *vb_star[3], *Fb_star[3];
  double *RbH_star, *RbZ_star, *Rbv_star[3], *RbH_n, *RbZ_n, *Rbv_n[3], *rhob_n;
  double *Tb_set, *Tb_init, *Zb_init;
  // the last adjoint Poisson solution of each stage (0 corrector, 1
  // predictor): the initial guess of the same stage's solve one step back
  double *xa[2], *xa_old[2], *xa_guess;
  int xa_valid[2], xa_iters[2];
  double *kap, *dkap;  // kappa and d kappa/dT of the level a residual gather reads
};

struct lm_ctx {
  lm_grid grid;
  lm_params prm;
  hipStream_t st;
  Lay lay;
  Bnd bnd;
  Phys phys;
  Level lev[3];          // roles rotate: cur (n), nxt (n+1), star
  double *P[3];          // pressure of each level slot
  int icur, inxt, istar;
  double *rho_prev;
  Resid R[2];
  int rprev;             // index of R^{n-1}; R^n is rprev ^ 1
  double *M[3], *b;
  IB ib;
  double *ib_store[6];
  unsigned char *chi_store;
  Sides sides;
  double *side_store[3][2][7];  // v[3], Z, H, F, wall flags (bytes)
  double *staging;
  size_t staging_bytes;
  int *dflags;           // [0] bad T, [1] non-finite
  double *dscalar;       // [0] CFL max rate
  PoissonWS pws;
  int *hflags;           // pinned
  double *hscalar;       // pinned
  SolveLog *dlog;        // outcome of the step's two solves (one-block solver), checked after the step
  SolveLog *hlog;        // pinned copy
  int have_state, have_prev;
  double time;
  long long total_iters;
  int last_iters[2];
  std::string err;
  // adjoint: two sets of the adjoint state (input and output of a reverse
  // step) and work arrays
  AdjState ad[2];
  int ad_cur;
  AdjWork aw;
  P0Dev *p0d;            // enclosed-system thermodynamic pressure (device)
  // adaptive time step
  double dt_prev;        // size of the step that made level n (0 before the first)
  int nsame;             // steps of that size in a row
  double dt_last;        // size of the last step taken
  double pc_err;         // its predictor-corrector estimate
  int pc_used;           // 1 if that estimate decided the next step
  int have_star;         // the predicted level of the last step is readable
  // stretched grid (section 3.2.1): host cell widths per direction, the
  // packed device spacing arrays of the explicit kernels
  int stretched;
  std::vector<double> wid[3];
  double *met_dev;
};

namespace {

// Text of the last failed call of this thread made without a context
// (lm_workspace_size, lm_init_grid, lm_project_static).
thread_local char g_init_err[512];

lm_status init_fail(lm_status s, const char *msg) {
  snprintf(g_init_err, sizeof(g_init_err), "%s", msg);
  return s;
}
lm_status init_fail(lm_status s, const std::string &msg) { return init_fail(s, msg.c_str()); }

lm_status fail(lm_ctx *c, lm_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(ctx, LM_EHIP, std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
  } while (0)

// Argument checks; *err receives a static message on failure.
bool valid_grid(const lm_grid *g, const char **err) {
  if (!g || (g->ndim != 2 && g->ndim != 3)) {
    *err = "ndim must be 2 or 3";
    return false;
  }
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < 4) {
      *err = "each direction needs at least 4 cells";
      return false;
    }
    if (!(g->L[d] > 0.0)) {
      *err = "lengths must be positive";
      return false;
    }
    for (int s = 0; s < 2; ++s)
      if (g->bc[d][s] < LM_SIDE_PERIODIC || g->bc[d][s] > LM_SIDE_OUTFLOW) {
        *err = "unknown side kind";
        return false;
      }
    if ((g->bc[d][0] == LM_SIDE_PERIODIC) != (g->bc[d][1] == LM_SIDE_PERIODIC)) {
      *err = "periodic sides come in pairs";
      return false;
    }
  }
  if (g->ndim == 2 && g->n[2] != 1) {
    *err = "2D grids need n[2] == 1";
    return false;
  }
  for (int d = 0; d < g->ndim; ++d) {
    const double *f = g->faces[d];
    if (!f) continue;
    bool ok = std::fabs(f[0]) <= 1e-14 * g->L[d] && std::fabs(f[g->n[d]] - g->L[d]) <= 1e-12 * g->L[d];
    for (int q = 0; q < g->n[d] && ok; ++q) ok = f[q + 1] > f[q];
    if (!ok) {
      *err = "faces[d] must hold n[d] + 1 strictly increasing values from 0 to L[d]";
      return false;
    }
  }
  return true;
}

// Cell widths of every direction (stretched grids; uniform directions get
// L/n) from the caller's face coordinates, copied.
void setup_metric(lm_ctx *c) {
  const lm_grid &g = c->grid;
  c->stretched = 0;
  for (int d = 0; d < g.ndim; ++d) c->stretched = c->stretched || g.faces[d] != nullptr;
  for (int d = 0; d < 3; ++d) {
    c->wid[d].clear();
    if (!c->stretched || d >= g.ndim) continue;
    c->wid[d].resize(g.n[d]);
    for (int q = 0; q < g.n[d]; ++q)
      c->wid[d][q] = g.faces[d] ? g.faces[d][q + 1] - g.faces[d][q] : g.L[d] / g.n[d];
  }
  for (int d = 0; d < 3; ++d) c->grid.faces[d] = nullptr;  // not kept
  c->pws.met = c->stretched;
}

// Packed spacing arrays of the explicit kernels (the layout of met_view)
// and the Eq 3.28 weights of the mirrored pressure ghost per side.
std::vector<double> metric_arrays(lm_ctx *c) {
  std::vector<double> out;
  for (int d = 0; d < c->grid.ndim; ++d) {
    const std::vector<double> &w = c->wid[d];
    const int n = (int)w.size();
    const bool per = c->bnd.periodic[d] != 0;
    std::vector<double> wp(n + 2);
    for (int q = 0; q < n; ++q) wp[q + 1] = w[q];
    wp[0] = per ? w[n - 1] : w[0];        // ghosts: the wrapped cell, or the mirrored first cell
    wp[n + 1] = per ? w[0] : w[n - 1];
    for (int p = 0; p < n + 2; ++p) out.push_back(1.0 / wp[p]);
    for (int f = 0; f <= n; ++f) out.push_back(1.0 / (0.5 * (wp[f] + wp[f + 1])));
    for (int f = 0; f <= n; ++f) out.push_back(wp[f + 1] / (wp[f] + wp[f + 1]));
    for (int f = 0; f <= n; ++f) out.push_back(wp[f] / (wp[f] + wp[f + 1]));
    for (int i = 0; i < n; ++i) out.push_back(1.0 / (0.5 * wp[i] + wp[i + 1] + 0.5 * wp[i + 2]));
    for (int s = 0; s < 2; ++s) {
      const double a = s == 0 ? w[0] : w[n - 1], b = s == 0 ? w[1] : w[n - 2], e = s == 0 ? w[2] : w[n - 3];
      const double x0 = -0.5 * a, x1 = 0.5 * a, x2 = a + 0.5 * b, x3 = a + b + 0.5 * e;
      c->phys.gx[d][s][0] = (x2 - x0) * (x3 - x0) / ((x2 - x1) * (x3 - x1));
      c->phys.gx[d][s][1] = (x1 - x0) * (x3 - x0) / ((x1 - x2) * (x3 - x2));
      c->phys.gx[d][s][2] = (x1 - x0) * (x2 - x0) / ((x1 - x3) * (x2 - x3));
    }
  }
  return out;
}

bool valid_params(const lm_params *p, const char **err) {
  if (!p) {
    *err = "params is NULL";
    return false;
  }
  if (!(p->Re > 0 && p->Pr > 0 && p->sigma >= 0 && p->p0 > 0)) {
    *err = "Re, Pr, p0 must be positive and sigma >= 0";
    return false;
  }
  if (!(p->dt > 0) && !(p->cfl > 0)) {
    *err = "need dt > 0 or cfl > 0";
    return false;
  }
  if (p->reacting && !(p->S > 0 && p->eps > 0 && p->tol > 0 && p->tol < 0.5)) {
    *err = "reacting needs S > 0, eps > 0, 0 < tol < 0.5";
    return false;
  }
  if (!(p->qs > 0) || !(p->Le_F > 0) || !(p->Le_O > 0)) {
    *err = "qs, Le_F, Le_O must be positive";
    return false;
  }
  if (p->with_ib && !(p->Da_ib > 0)) {
    *err = "Da_ib must be positive with immersed boundaries";
    return false;
  }
  if (!(p->poisson_rtol > 0) || p->poisson_maxit <= 0) {
    *err = "poisson_rtol > 0 and poisson_maxit > 0 required";
    return false;
  }
  if (p->precision != LM_FP64 && p->precision != LM_MIXED && p->precision != LM_MIXED_FLEXIBLE) {
    *err = "precision must be LM_FP64, LM_MIXED or LM_MIXED_FLEXIBLE";
    return false;
  }
  if (p->poisson_beta != LM_BETA_ONE && p->poisson_beta != LM_BETA_INV_RHO) {
    *err = "poisson_beta must be LM_BETA_ONE or LM_BETA_INV_RHO";
    return false;
  }
  if (p->p0_closed < 0 || p->p0_closed > 2) {
    *err = "p0_closed must be 0, 1 or 2";
    return false;
  }
  if (p->p0_closed && !(p->gamma > 1.0)) {
    *err = "gamma must exceed 1 for an enclosed system";
    return false;
  }
  if (!(p->sutherland_C >= 0.0 && p->sutherland_C < 1e300)) {
    *err = "sutherland_C must be >= 0 and finite";
    return false;
  }
  if (!(p->dt_tol >= 0.0 && p->dt_tol < 1e300)) {
    *err = "dt_tol must be >= 0 and finite";
    return false;
  }
  if (p->dt_tol > 0.0 && !(p->cfl > 0.0)) {
    *err = "an adaptive step (dt_tol > 0) needs cfl > 0";
    return false;
  }
  if (p->with_adjoint && p->dt_tol > 0.0) {
    *err = "the adjoint needs a fixed time step";
    return false;
  }
  if (p->with_adjoint && p->p0_closed) {
    *err = "the adjoint needs a constant thermodynamic pressure";
    return false;
  }
  if (p->with_adjoint && p->precision != LM_FP64) {
    *err = "the adjoint supports FP64 runs";
    return false;
  }
  return true;
}

void setup_phys(lm_ctx *c) {
  const lm_grid &g = c->grid;
  const lm_params &p = c->prm;
  Phys &P = c->phys;
  for (int d = 0; d < 3; ++d) {
    P.h[d] = d < g.ndim ? g.L[d] / g.n[d] : 1.0;
    P.ih[d] = 1.0 / P.h[d];
  }
  P.Pe = p.Re * p.Pr;
  P.Pr = p.Pr;
  P.sigma = p.sigma;
  P.inv_Fr2 = p.inv_Fr2;
  P.Da = p.Da_ib > 0 ? p.Da_ib : 1.0;
  P.p0 = p.p0;
  P.dt = p.dt;
  P.reacting = p.reacting;
  P.qs = p.qs;
  P.S = p.reacting ? p.S : 1.0;
  P.k = p.reacting ? std::log((1.0 - p.tol) / p.tol) / (2.0 * p.eps) : 1.0;
  P.Le_F = p.Le_F;
  P.Le_O = p.Le_O;
  P.N_F = (1.0 - p.Le_F) / (P.S * p.Le_F);
  P.N_O = (p.Le_O - 1.0) / p.Le_O;
  // F_eps(0) of Eq 3.41: ln cosh(-k) = k + log1p(exp(-2k)) - ln 2
  const double k = P.k, S = P.S;
  const double lc = k + std::log1p(std::exp(-2.0 * k)) - std::log(2.0);
  const double f0 = (-(S + 1.0) * lc / k + (S - 1.0) * (-1.0)) / (2.0 * S);
  P.fshift = -1.0 - f0;
  P.has_ib = 0;
  double nc = p.Pr;
  if (1.0 > nc) nc = 1.0;
  if (1.0 / p.Le_F > nc) nc = 1.0 / p.Le_F;
  if (1.0 / p.Le_O > nc) nc = 1.0 / p.Le_O;
  P.nu_coef = nc;
  P.closed = p.p0_closed;
  P.zeta = p.p0_closed ? (p.gamma - 1.0) / (p.gamma * p.qs) : 0.0;
  P.gamma = p.gamma;
  P.volume = 1.0;
  for (int d = 0; d < g.ndim; ++d) P.volume *= g.L[d];
  P.vol_out = 0.0;
  P.suth_C = p.sutherland_C;
  // stage kernel form: by default the LDS halo tiles in 2D and one thread
  // per cell in 3D (the faster of the two forms measured at 1024^2 and
  // 256^3); LM_STAGE_KERNEL=lds or =direct forces one form everywhere the
  // grid allows it (tuning and comparison)
  const char *sk = std::getenv("LM_STAGE_KERNEL");
  P.stage_form = !sk ? 0 : std::strcmp(sk, "lds") == 0 ? 1 : std::strcmp(sk, "direct") == 0 ? 2 : 0;
}

// Carves every device array (or only sizes them when cv.base == nullptr).
bool carve(lm_ctx *c, Carver &cv, std::string *err) {
  const int nd = c->grid.ndim;
  c->met_dev = nullptr;
  if (c->stretched) {
    bool outflow = false;
    for (int d = 0; d < nd; ++d)
      for (int s = 0; s < 2; ++s) outflow = outflow || c->grid.bc[d][s] == LM_SIDE_OUTFLOW;
    if (nd != 2 || outflow || c->prm.with_adjoint || c->prm.poisson_beta != LM_BETA_ONE || c->prm.p0_closed == 2) {
      if (err)
        *err = "stretched grids: 2D, no outflow side, no adjoint, poisson_beta LM_BETA_ONE, p0_closed 0 or 1";
      return false;
    }
    long m = 0;
    for (int d = 0; d < nd; ++d) m += 5L * c->grid.n[d] + 5;
    c->met_dev = (double *)cv.take((size_t)m * 8);
  }
  if (c->prm.p0_closed) {
    // enclosed (1): periodic or wall sides; semi-enclosed (2, Eq 2.38):
    // inflow sides too; never an outflow side (its flux closes the mass)
    bool open = false;
    for (int d = 0; d < nd; ++d)
      for (int s = 0; s < 2; ++s)
        open = open || (c->grid.bc[d][s] == LM_SIDE_INFLOW && c->prm.p0_closed == 1) ||
               c->grid.bc[d][s] == LM_SIDE_OUTFLOW;
    // the mass form of Eq 2.40 maps T with the non-reacting T(H) only;
    // Eq 2.38 carries the flame's heat through its N' term
    if (open || (c->prm.reacting && c->prm.p0_closed == 1)) {
      if (err)
        *err = "p0_closed needs periodic or wall sides (inflow sides too with 2); 1 needs non-reacting flow";
      return false;
    }
    // Eq 2.38 has no term for the heat and species the penalisation of
    // Eq 3.31-3.32 puts in or takes out (the mass form needs none)
    if (c->prm.p0_closed == 2 && c->prm.with_ib) {
      if (err) *err = "p0_closed = 2 (Eq 2.38) takes no immersed body";
      return false;
    }
  }
  c->p0d = (P0Dev *)cv.take(sizeof(P0Dev));
  const Lay &L = c->lay;
  const size_t ab = (size_t)L.total * 8;
  const bool reacting = c->prm.reacting != 0;
  for (int s = 0; s < 3; ++s) {
    Level &lv = c->lev[s];
    memset(&lv, 0, sizeof(lv));
    lv.rho = (double *)cv.take(ab);
    for (int d = 0; d < nd; ++d) lv.v[d] = (double *)cv.take(ab);
    lv.Z = reacting ? (double *)cv.take(ab) : nullptr;
    lv.H = (double *)cv.take(ab);
    lv.T = (double *)cv.take(ab);
    lv.kap = (double *)cv.take(ab);
    for (int d = 0; d < nd; ++d) lv.F[d] = (double *)cv.take(ab);
    c->P[s] = (double *)cv.take(ab);
  }
  c->rho_prev = (double *)cv.take(ab);
  for (int r = 0; r < 2; ++r) {
    memset(&c->R[r], 0, sizeof(Resid));
    c->R[r].H = (double *)cv.take(ab);
    c->R[r].Z = reacting ? (double *)cv.take(ab) : nullptr;
    for (int d = 0; d < nd; ++d) c->R[r].v[d] = (double *)cv.take(ab);
  }
  for (int d = 0; d < 3; ++d) c->M[d] = d < nd ? (double *)cv.take(ab) : nullptr;
  c->b = (double *)cv.take(ab);
  memset(&c->ib, 0, sizeof(c->ib));
  for (int q = 0; q < 6; ++q) c->ib_store[q] = nullptr;
  c->chi_store = nullptr;
  if (c->prm.with_ib) {
    c->chi_store = (unsigned char *)cv.take((size_t)L.total);
    for (int q = 0; q < nd + 3; ++q) c->ib_store[q] = (double *)cv.take(ab);
  }
  memset(&c->sides, 0, sizeof(c->sides));
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < 7; ++q) c->side_store[d][s][q] = nullptr;
  for (int d = 0; d < nd; ++d)
    for (int s = 0; s < 2; ++s)
      if (c->grid.bc[d][s] == LM_SIDE_INFLOW || c->grid.bc[d][s] == LM_SIDE_SLIP ||
          c->grid.bc[d][s] == LM_SIDE_NOSLIP) {
        const size_t nside = (size_t)(L.ncells() / L.n[d]);
        for (int q = 0; q < 7; ++q) c->side_store[d][s][q] = (double *)cv.take(nside * 8);
      }
  long mx = 1;
  for (int d = 0; d < 3; ++d) mx *= (L.n[d] + 1);
  c->staging_bytes = (size_t)mx * 8;
  c->staging = (double *)cv.take(c->staging_bytes);
  c->dflags = (int *)cv.take(64);
  c->dscalar = (double *)cv.take(64);
  c->dlog = (SolveLog *)cv.take(2 * sizeof(SolveLog));
  {
    const bool adj = c->prm.with_adjoint;
    auto take = [&](bool on) { return adj && on ? (double *)cv.take(ab) : nullptr; };
    for (int s = 0; s < 2; ++s) {
      AdjState &a = c->ad[s];
      a.H = take(true);
      a.Z = take(c->prm.reacting);
      a.rho_prev = take(true);
      a.R_H = take(true);
      a.R_Z = take(c->prm.reacting);
      for (int d = 0; d < 3; ++d) {
        a.v[d] = take(d < nd);
        a.F[d] = take(d < nd);
        a.R_v[d] = take(d < nd);
      }
    }
    AdjWork &w = c->aw;
    for (double **q : {&w.rhob_new, &w.Pb, &w.bb, &w.Hb_star, &w.RbH_star, &w.RbH_n, &w.rhob_n, &w.Tb_set,
                       &w.Tb_init})
      *q = take(true);
    for (double **q : {&w.Zb_star, &w.RbZ_star, &w.RbZ_n, &w.Zb_init}) *q = take(c->prm.reacting);
    for (int q = 0; q < 2; ++q) {
      w.xa[q] = take(true);
      w.xa_old[q] = take(true);
      w.xa_valid[q] = w.xa_iters[q] = 0;
    }
    w.xa_guess = take(true);
    w.kap = take(true);
    w.dkap = take(true);
    for (int d = 0; d < 3; ++d)
      for (double **q : {&w.Mb[d], &w.vb_star[d], &w.Fb_star[d], &w.Rbv_star[d], &w.Rbv_n[d]}) *q = take(d < nd);
    c->ad_cur = 0;
  }
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = c->phys.h[d];
  if (!poisson_plan(c->pws, cv, L, c->bnd, h, c->prm.precision != LM_FP64, c->prm.precision == LM_MIXED_FLEXIBLE,
                    c->prm.mg_nu > 0 ? c->prm.mg_nu : 2, c->prm.poisson_beta == LM_BETA_INV_RHO || c->stretched,
                    err))
    return false;
  c->phys.met = c->met_dev;
  c->phys.vol = c->pws.vol;
  return true;
}

void setup_layout(lm_ctx *c) {
  c->lay = make_layout(c->grid.ndim, c->grid.n, 8);
  Bnd &B = c->bnd;
  B.all_periodic = 1;
  for (int d = 0; d < 3; ++d) {
    for (int s = 0; s < 2; ++s) B.kind[d][s] = d < c->grid.ndim ? c->grid.bc[d][s] : LM_SIDE_PERIODIC;
    B.periodic[d] = B.kind[d][0] == LM_SIDE_PERIODIC;
    if (d < c->grid.ndim && !B.periodic[d]) B.all_periodic = 0;
  }
}

Level &cur(lm_ctx *c) { return c->lev[c->icur]; }

lm_status copy_in(lm_ctx *c, const double *src, double *dst, int face_dir, int mem) {
  const Lay &L = c->lay;
  long m = L.ncells();
  if (face_dir >= 0) m = m / L.n[face_dir] * (L.n[face_dir] + 1);
  const double *dsrc = src;
  if (mem == LM_HOST) {
    HIPCHK(c, hipMemcpyAsync(c->staging, src, (size_t)m * 8, hipMemcpyHostToDevice, c->st));
    dsrc = c->staging;
  }
  HIPCHK(c, launch_pack(c->st, L, dsrc, dst, face_dir));
  if (mem == LM_HOST) HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

lm_status copy_out(lm_ctx *c, const double *src, double *dst, int face_dir, int mem) {
  const Lay &L = c->lay;
  long m = L.ncells();
  if (face_dir >= 0) m = m / L.n[face_dir] * (L.n[face_dir] + 1);
  if (mem == LM_HOST) {
    HIPCHK(c, launch_unpack(c->st, L, src, c->staging, face_dir));
    HIPCHK(c, hipMemcpyAsync(dst, c->staging, (size_t)m * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  } else {
    HIPCHK(c, launch_unpack(c->st, L, src, dst, face_dir));
  }
  return LM_OK;
}

lm_status copy_side(lm_ctx *c, const double *src, double *dst, size_t n, int mem) {
  if (!src) {
    HIPCHK(c, hipMemsetAsync(dst, 0, n * 8, c->st));
    return LM_OK;
  }
  HIPCHK(c, hipMemcpyAsync(dst, src, n * 8, mem == LM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           c->st));
  if (mem == LM_HOST) HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

}  // namespace

extern "C" {

lm_status lm_workspace_size(const lm_grid *grid, const lm_params *params, size_t *bytes) {
  const char *bad = "bytes is NULL";
  if (!bytes || !valid_grid(grid, &bad) || !valid_params(params, &bad)) return init_fail(LM_EINVAL, bad);
  std::string err;
  lm_ctx *c = new (std::nothrow) lm_ctx();
  if (!c) return init_fail(LM_ENOMEM, "out of host memory");
  c->grid = *grid;
  c->prm = *params;
  setup_phys(c);
  setup_layout(c);
  setup_metric(c);
  Carver cv{nullptr, 0};
  bool ok = carve(c, cv, &err);
  delete c;
  if (!ok) return init_fail(LM_EUNSUPPORTED, err);
  *bytes = cv.off + 256;
  return LM_OK;
}

lm_status lm_init_grid(const lm_grid *grid, const lm_params *params, void *ws, size_t bytes, void *stream,
                       lm_ctx **out) {
  if (!out) return init_fail(LM_EINVAL, "out is NULL");
  *out = nullptr;
  const char *bad = nullptr;
  if (!valid_grid(grid, &bad) || !valid_params(params, &bad)) return init_fail(LM_EINVAL, bad);
  if (!ws) return init_fail(LM_EINVAL, "workspace is NULL");
  std::string err;
  size_t need = 0;
  lm_status s = lm_workspace_size(grid, params, &need);
  if (s != LM_OK) return s;
  if (bytes < need) return init_fail(LM_ENOMEM, "workspace smaller than lm_workspace_size");
  lm_ctx *c = new (std::nothrow) lm_ctx();
  if (!c) return init_fail(LM_ENOMEM, "out of host memory");
  c->grid = *grid;
  c->prm = *params;
  c->st = (hipStream_t)stream;
  setup_phys(c);
  setup_layout(c);
  setup_metric(c);
  char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  Carver cv{base, 0};
  if (!carve(c, cv, &err)) {
    delete c;
    return init_fail(LM_EUNSUPPORTED, err);
  }
  c->icur = 0;
  c->inxt = 1;
  c->istar = 2;
  c->rprev = 0;
  c->have_state = 0;
  c->have_prev = 0;
  c->time = 0;
  c->total_iters = 0;
  c->last_iters[0] = c->last_iters[1] = 0;
  hipError_t e = hipHostMalloc((void **)&c->hflags, 64);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hscalar, 64);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hlog, 2 * sizeof(SolveLog));
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->pws.host_sc, sizeof(SolverScalars));
  if (e != hipSuccess) {
    lm_destroy(c);
    return init_fail(LM_EHIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  // zero the whole carved region once (ghost layers, padding, scalars)
  e = hipMemsetAsync(base, 0, cv.off, c->st);
  if (e != hipSuccess) {
    lm_destroy(c);
    return init_fail(LM_EHIP, std::string("hipMemsetAsync of the workspace: ") + hipGetErrorString(e));
  }
  double h[3] = {c->phys.h[0], c->phys.h[1], c->phys.h[2]};
  e = poisson_setup(c->st, c->pws, h);
  if (e != hipSuccess) {
    lm_destroy(c);
    return init_fail(LM_EHIP, std::string("coarse-grid set-up: ") + hipGetErrorString(e));
  }
  if (c->stretched) {
    const std::vector<double> m = metric_arrays(c);
    e = hipMemcpyAsync(c->met_dev, m.data(), m.size() * 8, hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e == hipSuccess) e = poisson_set_metric(c->st, c->pws, c->wid[0].data(), c->wid[1].data());
    if (e != hipSuccess) {
      lm_destroy(c);
      return init_fail(LM_EHIP, std::string("stretched-grid set-up: ") + hipGetErrorString(e));
    }
  }
  *out = c;
  return LM_OK;
}

// Eq 2.38 systems: the volume flux out through the inflow sides, the given
// normal velocities times the face areas (outward: minus on low sides).
static lm_status update_vol_out(lm_ctx *c) {
  c->phys.vol_out = 0.0;
  if (c->prm.p0_closed != 2) return LM_OK;
  const Lay &L = c->lay;
  std::vector<double> buf;
  for (int d = 0; d < c->grid.ndim; ++d)
    for (int s = 0; s < 2; ++s) {
      if (c->grid.bc[d][s] != LM_SIDE_INFLOW || !c->sides.s[d][s].v[d]) continue;
      const size_t n = (size_t)(L.ncells() / L.n[d]);
      buf.resize(n);
      HIPCHK(c, hipMemcpyAsync(buf.data(), c->sides.s[d][s].v[d], n * 8, hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      double sum = 0.0;
      for (size_t q = 0; q < n; ++q) sum += buf[q];
      double area = 1.0;
      for (int e = 0; e < c->grid.ndim; ++e)
        if (e != d) area *= c->phys.h[e];
      c->phys.vol_out += (s == 1 ? 1.0 : -1.0) * sum * area;
    }
  return LM_OK;
}

lm_status lm_set_side(lm_ctx *c, int d, int side, const lm_side_data *data, int mem) {
  if (!c || !data || d < 0 || d >= c->grid.ndim || side < 0 || side > 1)
    return fail(c, LM_EINVAL, "bad side arguments");
  const int kind = c->grid.bc[d][side];
  const size_t n = (size_t)(c->lay.ncells() / c->lay.n[d]);
  double **st = c->side_store[d][side];
  lm_status s;
  if (kind == LM_SIDE_SLIP || kind == LM_SIDE_NOSLIP) {
    // isothermal (H given) or adiabatic (H NULL) wall
    if (data->v[0] || data->v[1] || data->v[2] || data->Z || data->F || data->wall)
      return fail(c, LM_EINVAL, "a wall side takes only H (its wall temperature)");
    if (data->H && c->prm.reacting)
      return fail(c, LM_EUNSUPPORTED, "isothermal walls need non-reacting flow");
    SideData &sd = c->sides.s[d][side];
    sd.H = nullptr;
    if (data->H) {
      if ((s = copy_side(c, data->H, st[4], n, mem)) != LM_OK) return s;
      sd.H = st[4];
    }
    return LM_OK;
  }
  if (kind != LM_SIDE_INFLOW) return fail(c, LM_EINVAL, "side is not an inflow or wall side");
  for (int q = 0; q < 3; ++q) {
    if (q >= c->grid.ndim) break;
    if ((s = copy_side(c, data->v[q], st[q], n, mem)) != LM_OK) return s;
  }
  if ((s = copy_side(c, data->Z, st[3], n, mem)) != LM_OK) return s;
  if ((s = copy_side(c, data->H, st[4], n, mem)) != LM_OK) return s;
  if ((s = copy_side(c, data->F, st[5], n, mem)) != LM_OK) return s;
  SideData &sd = c->sides.s[d][side];
  sd.wall = nullptr;
  if (data->wall) {
    HIPCHK(c, hipMemcpyAsync(st[6], data->wall, n, mem == LM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                             c->st));
    if (mem == LM_HOST) HIPCHK(c, hipStreamSynchronize(c->st));
    sd.wall = (const unsigned char *)st[6];
  }
  for (int q = 0; q < 3; ++q) sd.v[q] = q < c->grid.ndim ? st[q] : nullptr;
  sd.Z = st[3];
  sd.H = st[4];
  sd.F = st[5];
  return update_vol_out(c);
}

// Velocity, Z and T (or H) of a level from caller arrays; the EOS, rho and
// the face fluxes follow in finish_level.
static lm_status load_level(lm_ctx *c, Level &lv, const lm_fields *f, int mem) {
  if (!f->T && !f->H) return fail(c, LM_EINVAL, "need T or H");
  const int nd = c->grid.ndim;
  for (int d = 0; d < nd; ++d)
    if (!f->v[d]) return fail(c, LM_EINVAL, "need every velocity component");
  lm_status s;
  for (int d = 0; d < nd; ++d)
    if ((s = copy_in(c, f->v[d], lv.v[d], -1, mem)) != LM_OK) return s;
  if (c->prm.reacting) {
    if (f->Z) {
      if ((s = copy_in(c, f->Z, lv.Z, -1, mem)) != LM_OK) return s;
    } else {
      HIPCHK(c, hipMemsetAsync(lv.Z, 0, (size_t)c->lay.total * 8, c->st));
    }
  }
  if (f->T) {
    if ((s = copy_in(c, f->T, lv.T, -1, mem)) != LM_OK) return s;
  } else {
    if ((s = copy_in(c, f->H, lv.H, -1, mem)) != LM_OK) return s;
  }
  return LM_OK;
}

// T, H, rho = p0/T and kappa of a loaded level (flags a non-positive T in
// dflags[0]), then its face fluxes: the given ones, or the face average of
// rho v.
static lm_status finish_level(lm_ctx *c, Level &lv, const lm_fields *f, int mem) {
  const int nd = c->grid.ndim;
  lm_status s;
  HIPCHK(c, launch_init_state(c->st, c->lay, c->phys, c->bnd, c->sides, f->T != nullptr, lv, c->dflags));
  if (f->F[0]) {
    for (int d = 0; d < nd; ++d) {
      if (!f->F[d]) return fail(c, LM_EINVAL, "give every face-flux component or none");
      if ((s = copy_in(c, f->F[d], lv.F[d], d, mem)) != LM_OK) return s;
    }
  } else {
    HIPCHK(c, launch_face_flux(c->st, c->lay, c->bnd, c->sides, lv, c->M, c->phys.met));
  }
  return LM_OK;
}

// Level n-1: the fields of the previous time level, from which the level
// n-1 density and residuals of the next step's AB2 predictor and BDF2
// density derivative are formed (section 3.1, Eq 3.1, 3.3, 3.10, 3.11).
static lm_status set_previous_level(lm_ctx *c, const lm_fields *f, const lm_ib *ib, int mem) {
  if (!c->have_state) return fail(c, LM_ESTATE, "set level 0 before level 1");
  if (ib) return fail(c, LM_EINVAL, "the immersed body is set with level 0");
  if (c->prm.p0_closed) return fail(c, LM_EUNSUPPORTED, "level 1 needs a constant thermodynamic pressure");
  // the level's fields go to the predicted slot; the stage kernel writes
  // the (discarded) Euler update into the next-level slot
  Level &pv = c->lev[c->istar];
  lm_status s = load_level(c, pv, f, mem);
  if (s != LM_OK) return s;
  HIPCHK(c, hipMemsetAsync(c->dflags, 0, 64, c->st));
  if ((s = finish_level(c, pv, f, mem)) != LM_OK) return s;
  HIPCHK(c, hipMemcpyAsync(c->hflags, c->dflags, 16, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (c->hflags[0]) return fail(c, LM_EINVAL, "temperature must be positive everywhere");
  HIPCHK(c, launch_ghosts(c->st, c->lay, c->bnd, c->phys, c->sides, pv.v, pv.Z, pv.H, pv.T, pv.kap));
  // residuals of level n-1 into the history slot R^{n-1}
  HIPCHK(c, launch_stage(c->st, 0, 1, c->lay, c->phys, pv, pv, c->R[c->rprev ^ 1], c->R[c->rprev], c->ib,
                         c->lev[c->inxt], c->M, &c->p0d->dtp0_n));
  std::swap(c->rho_prev, pv.rho);
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->have_prev = 1;
  c->have_star = 0;
  c->dt_prev = c->phys.dt;  // the step from n-1 to n: the current step
  c->nsame = 1;
  return LM_OK;
}

lm_status lm_set_fields(lm_ctx *c, int level, const lm_fields *f, const lm_ib *ib, int mem) {
  if (!c || !f) return fail(c, LM_EINVAL, "NULL argument");
  if (level == 1) return set_previous_level(c, f, ib, mem);
  if (level != 0) return fail(c, LM_EUNSUPPORTED, "level must be 0 or 1");
  const int nd = c->grid.ndim;
  Level &lv = cur(c);
  lm_status s = load_level(c, lv, f, mem);
  if (s != LM_OK) return s;
  if (f->P) {
    if ((s = copy_in(c, f->P, c->P[c->icur], -1, mem)) != LM_OK) return s;
  } else {
    HIPCHK(c, hipMemsetAsync(c->P[c->icur], 0, (size_t)c->lay.total * 8, c->st));
  }
  // immersed boundary
  c->phys.has_ib = 0;
  memset(&c->ib, 0, sizeof(c->ib));
  if (ib) {
    if (!c->prm.with_ib) return fail(c, LM_EINVAL, "context created without with_ib");
    if (ib->chi) {
      const unsigned char *src = ib->chi;
      if (mem == LM_HOST) {
        HIPCHK(c, hipMemcpyAsync(c->staging, ib->chi, (size_t)c->lay.ncells(), hipMemcpyHostToDevice, c->st));
        src = (const unsigned char *)c->staging;
      }
      HIPCHK(c, launch_pack_u8(c->st, c->lay, src, c->chi_store));
      if (mem == LM_HOST) HIPCHK(c, hipStreamSynchronize(c->st));
      c->ib.chi = c->chi_store;
      c->phys.has_ib = 1;
    }
    const double *srcs[6] = {ib->v_ib[0], ib->v_ib[1], nd == 3 ? ib->v_ib[2] : nullptr, ib->Z_ib, ib->H_ib,
                             ib->S_m};
    const int slot[6] = {0, 1, 2, nd, nd + 1, nd + 2};
    for (int q = 0; q < 6; ++q) {
      if (!srcs[q]) continue;
      double *dst = c->ib_store[slot[q]];
      if ((s = copy_in(c, srcs[q], dst, -1, mem)) != LM_OK) return s;
      if (q < 3) c->ib.v_ib[q] = dst;
      if (q == 3) c->ib.Z_ib = dst;
      if (q == 4) c->ib.H_ib = dst;
      if (q == 5) c->ib.S_m = dst;
    }
  }
  if (c->prm.p0_closed && c->ib.S_m) return fail(c, LM_EINVAL, "an enclosed system takes no mass source S_m");
  HIPCHK(c, hipMemsetAsync(c->dflags, 0, 64, c->st));
  if ((s = finish_level(c, lv, f, mem)) != LM_OK) return s;
  if (c->prm.p0_closed) {  // conserved mass of this state, p0 history cleared
    HIPCHK(c, launch_p0(c->st, 0, c->lay, c->phys, c->p0d, &lv, nullptr, nullptr, c->pws.partials));
    if ((s = update_vol_out(c)) != LM_OK) return s;
  }
  if (!(c->prm.dt > 0)) {
    HIPCHK(c, launch_cfl(c->st, c->lay, c->phys, lv, c->ib.chi, c->pws.partials, c->dscalar));
  }
  HIPCHK(c, hipMemcpyAsync(c->hflags, c->dflags, 16, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(c->hscalar, c->dscalar, 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (c->hflags[0]) return fail(c, LM_EINVAL, "temperature must be positive everywhere");
  if (!(c->prm.dt > 0)) {
    const double m = c->hscalar[0];
    if (!(m > 0) || !std::isfinite(m)) return fail(c, LM_EINVAL, "cannot fix dt from the CFL condition");
    c->phys.dt = c->prm.cfl / m;
  } else {
    c->phys.dt = c->prm.dt;
  }
  c->have_state = 1;
  c->have_prev = 0;
  c->have_star = 0;
  c->time = 0.0;
  c->dt_prev = 0.0;
  c->nsame = 0;
  c->dt_last = c->phys.dt;
  c->pc_err = 0.0;
  c->pc_used = 0;
  c->phys.var_step = 0;
  return LM_OK;
}

// Weights of the predictor's AB2 and of the BDF2 density derivative for a
// step after one of another size (adaptive steps), w = dt / dt_prev:
// AB2 integrates the line through R^{n-1}, R^n over the step,
// R^n (1 + w/2) - R^{n-1} w/2; BDF2 differentiates the parabola through
// rho^{n-1}, rho^n, rho^{n+1} at t_{n+1}, taken in the differences of the
// levels (weights (1+2w)/(1+w) and w^2/(1+w)) so that rounding scales with
// the change of rho, not with rho / dt.
static void set_step_weights(lm_ctx *c) {
  Phys &P = c->phys;
  P.var_step = 0;
  if (!(c->prm.dt_tol > 0.0) || !c->have_prev) return;
  const double dt = P.dt, w = dt / c->dt_prev;
  P.var_step = 1;
  P.ab0 = 1.0 + 0.5 * w;
  P.ab1 = -0.5 * w;
  P.bd0 = (1.0 + 2.0 * w) / (1.0 + w);
  P.bd2 = w * w / (1.0 + w);
}

// After a committed step (adaptive steps): the step's error estimate from
// the predicted and new levels, then the next step. Only the fourth or a
// later step of exactly one size decides: levels made by steps of different
// sizes differ by O(h^2 |dt - dt_prev|) in the cell velocity (the
// projection subtracts delta_2 P with P = p dt), which the AB2
// extrapolation of the next two steps carries into the estimate; the
// Euler-predicted first step behaves alike.
static lm_status adapt_dt(lm_ctx *c, int first) {
  const Lay &L = c->lay;
  Level &nw = c->lev[c->icur];
  HIPCHK(c, launch_pc_err(c->st, L, c->prm.reacting, c->lev[c->istar], nw, c->pws.partials, c->dscalar + 1));
  HIPCHK(c, launch_cfl(c->st, L, c->phys, nw, c->ib.chi, c->pws.partials + 3 * kErrBlocks, c->dscalar));
  HIPCHK(c, hipMemcpyAsync(c->hscalar, c->dscalar, 32, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double N = (double)L.ncells();
  double err = std::max(std::sqrt(c->hscalar[1] / N), std::sqrt(c->hscalar[2] / N));
  if (c->prm.reacting) err = std::max(err, std::sqrt(c->hscalar[3] / N) / (c->prm.S + 1.0));
  const double dt = c->phys.dt;
  const double cap = c->prm.cfl / c->hscalar[0];
  if (!(cap > 0) || !std::isfinite(cap) || !std::isfinite(err))
    return fail(c, LM_ENONFINITE, "adaptive step: non-finite error estimate or CFL step");
  c->nsame = (!first && dt == c->dt_prev) ? c->nsame + 1 : 1;
  c->pc_err = err;
  c->pc_used = c->nsame >= 4;
  double nd = dt;
  if (c->pc_used) {
    const double fac =
        err <= 0.0 ? 1.5 : std::min(1.5, std::max(0.5, 0.9 * std::cbrt(c->prm.dt_tol / err)));
    if (fac <= 0.9 || fac >= 1.1) nd = std::min(dt * fac, cap);
  }
  if (nd > cap) nd = 0.9 * cap;
  c->dt_last = dt;
  c->dt_prev = dt;
  c->phys.dt = nd;
  return LM_OK;
}

static lm_status do_stage(lm_ctx *c, int corrector, int &iters, double &relres, double &compat) {
  const Lay &L = c->lay;
  Level &A = c->lev[c->icur];
  Level &out = corrector ? c->lev[c->inxt] : c->lev[c->istar];
  Level &src = corrector ? c->lev[c->istar] : A;
  Resid &rprev = c->R[c->rprev];
  Resid &rn = c->R[c->rprev ^ 1];
  HIPCHK(c, launch_ghosts(c->st, L, c->bnd, c->phys, c->sides, src.v, src.Z, src.H, src.T, src.kap));
  const int first = !c->have_prev;
  const double *dtp0 = corrector ? &c->p0d->dtp0_star : &c->p0d->dtp0_n;
  const bool ode = c->prm.p0_closed == 2;
  // Eq 2.38: d_t p0 of the residual's level from its heat integral
  if (ode) HIPCHK(c, launch_p0(c->st, corrector ? 7 : 5, L, c->phys, c->p0d, &src, nullptr, nullptr, c->pws.partials));
  HIPCHK(c, launch_stage(c->st, corrector, first, L, c->phys, src, A, rprev, rn, c->ib, out, c->M, dtp0));
  if (ode) {
    // p0 of the predicted (AB2) / new (trapezoid) level, then rho = p0 / T
    HIPCHK(c, launch_p0(c->st, corrector ? 8 : 6, L, c->phys, c->p0d, &out, nullptr, nullptr, c->pws.partials));
  } else if (c->prm.p0_closed) {
    // first step: d_t p0 at level n from the balance, into R_H^n and H*
    if (!corrector && first) HIPCHK(c, launch_p0(c->st, 3, L, c->phys, c->p0d, &out, &A, rn.H, c->pws.partials));
    // p0 of the predicted / new level from the mass, then rho = p0 / T
    HIPCHK(c, launch_p0(c->st, corrector ? 2 : 1, L, c->phys, c->p0d, &out, &A, nullptr, c->pws.partials));
  }
  HIPCHK(c, launch_rhs(c->st, L, c->bnd, c->phys, c->sides, c->M, out.rho, A.rho, c->rho_prev, !first, c->ib.S_m,
                       c->b, c->pws.partials, c->pws.sc));
  const double *x0 = corrector ? c->P[c->istar] : c->P[c->icur];
  if (!corrector && c->phys.var_step && c->phys.dt != c->dt_prev) {
    // P = p dt: after a change of step the previous pressure, scaled by
    // dt / dt_prev, is the warm start (in the predicted level's slot,
    // which the predictor overwrites anyway)
    HIPCHK(c, launch_scale_copy(c->st, L.total, c->phys.dt / c->dt_prev, c->P[c->icur], c->P[c->istar]));
    x0 = c->P[c->istar];
  }
  int conv = 0;
  const int expect = c->last_iters[corrector];
  // the one-block solver leaves its outcome on the device; lm_step reads
  // both stages' after the step (one wait per step instead of three)
  SolveLog *log = c->pws.block_pcg ? c->dlog + corrector : nullptr;
  HIPCHK(c, poisson_solve(c->st, c->pws, c->b, x0, c->prm.poisson_rtol, c->prm.poisson_maxit, expect, &iters,
                          &relres, &conv, log));
  if (!log) {
    compat = c->pws.host_sc->mean_b;
    c->last_iters[corrector] = iters > 0 ? iters : 1;
    c->total_iters += iters;
    if (!conv) return fail(c, LM_ENOCONV, "Poisson solver did not reach poisson_rtol");
  }
  double *P_out = corrector ? c->P[c->inxt] : c->P[c->istar];
  HIPCHK(c, launch_project(c->st, L, c->bnd, c->phys, c->sides, c->M, c->pws.x, out.rho, c->pws.sc, out.F, out.v,
                           P_out, c->dflags + 1));
  return LM_OK;
}

// Reads back the outcome of both stage solves when the one-workgroup solver
// deferred it to the device log (stage solves then skip their own host
// check), synchronising the stream; otherwise only synchronises.
static lm_status read_solve_logs(lm_ctx *c, int it[2], double rr[2], double cm[2]) {
  if (c->pws.block_pcg)
    HIPCHK(c, hipMemcpyAsync(c->hlog, c->dlog, 2 * sizeof(SolveLog), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (!c->pws.block_pcg) return LM_OK;
  for (int q = 0; q < 2; ++q) {
    const SolveLog &g = c->hlog[q];
    it[q] = g.iters;
    rr[q] = g.cc > 0 ? std::sqrt(g.rr / g.cc) : 0.0;
    cm[q] = g.mean_b;
    c->last_iters[q] = g.iters > 0 ? g.iters : 1;
    c->total_iters += g.iters;
    if (!(g.done && !g.nonconv)) return fail(c, LM_ENOCONV, "Poisson solver did not reach poisson_rtol");
  }
  return LM_OK;
}

lm_status lm_step(lm_ctx *c, int nsteps, lm_step_stats *stats) {
  if (!c) return LM_EINVAL;
  if (!c->have_state) return fail(c, LM_ESTATE, "lm_set_fields must come first");
  if (nsteps < 0) return fail(c, LM_EINVAL, "nsteps < 0");
  int done = 0;
  int it[2] = {0, 0};
  double rr[2] = {0, 0}, cm[2] = {0, 0};
  for (int n = 0; n < nsteps; ++n) {
    set_step_weights(c);
    HIPCHK(c, hipMemsetAsync(c->dflags + 1, 0, 4, c->st));
    lm_status s = do_stage(c, 0, it[0], rr[0], cm[0]);
    if (s == LM_OK) s = do_stage(c, 1, it[1], rr[1], cm[1]);
    if (s == LM_OK) {
      HIPCHK(c, hipMemcpyAsync(c->hflags + 1, c->dflags + 1, 4, hipMemcpyDeviceToHost, c->st));
      s = read_solve_logs(c, it, rr, cm);
      if (s == LM_OK && c->hflags[1]) s = fail(c, LM_ENONFINITE, "non-finite velocity after the step");
    }
    if (s != LM_OK) {
      if (stats) {
        stats->steps = done;
        stats->dt = c->dt_last;
        stats->time = c->time;
      }
      return s;
    }
    // commit: level n+1 becomes current; rho^n becomes rho^{n-1}
    if (c->prm.p0_closed)
      HIPCHK(c, launch_p0(c->st, 4, c->lay, c->phys, c->p0d, nullptr, nullptr, nullptr, nullptr));
    double *old_prev = c->rho_prev;
    c->rho_prev = c->lev[c->icur].rho;
    c->lev[c->icur].rho = old_prev;
    std::swap(c->icur, c->inxt);
    c->rprev ^= 1;
    const int first = !c->have_prev;
    c->have_prev = 1;
    c->have_star = 1;
    c->time += c->phys.dt;
    ++done;
    if (c->prm.dt_tol > 0.0) {
      if ((s = adapt_dt(c, first)) != LM_OK) {
        // the step that produced the estimate is committed
        if (stats) {
          stats->steps = done;
          stats->dt = c->phys.dt;
          stats->time = c->time;
        }
        return s;
      }
    } else {
      c->dt_last = c->phys.dt;
    }
  }
  if (stats) {
    stats->steps = done;
    stats->dt = c->dt_last;
    stats->time = c->time;
    stats->pc_err = c->pc_err;
    stats->pc_err_used = c->pc_used;
    for (int q = 0; q < 2; ++q) {
      stats->poisson_iters[q] = it[q];
      stats->poisson_relres[q] = rr[q];
      stats->compat[q] = cm[q];
    }
    stats->total_poisson_iters = c->total_iters;
    stats->p0 = c->prm.p0;
    if (c->prm.p0_closed) {
      HIPCHK(c, hipMemcpyAsync(c->hscalar + 1, &c->p0d->p0[0], 8, hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      stats->p0 = c->hscalar[1];
    }
  }
  return LM_OK;
}

lm_status lm_project(lm_ctx *c, lm_project_args *a) {
  if (!c || !a || !a->b) return fail(c, LM_EINVAL, "NULL argument");
  if (a->rho && (!c->pws.vc_cap || c->stretched))
    return fail(c, LM_EUNSUPPORTED, "a density needs params.poisson_beta = LM_BETA_INV_RHO (uniform grids)");
  lm_status s = copy_in(c, a->b, c->b, -1, a->mem);
  if (s != LM_OK) return s;
  const Lay &L = c->lay;
  if (a->rho) {
    if ((s = copy_in(c, a->rho, c->pws.rho64, -1, a->mem)) != LM_OK) return s;
    HIPCHK(c, poisson_set_beta(c->st, c->pws));  // an invalid density ends the solve at once
  }
  HIPCHK(c, launch_mean(c->st, L, c->b, c->pws.partials, c->pws.sc, c->phys.vol, c->phys.volume));
  int iters = 0, conv = 0;
  double relres = 0;
  const double rtol = a->rtol > 0 ? a->rtol : c->prm.poisson_rtol;
  c->pws.vc = c->pws.met || a->rho != nullptr;
  // a standalone solve: zero start in solver scratch, the state untouched
  const hipError_t e = poisson_solve(c->st, c->pws, c->b, nullptr, rtol, c->prm.poisson_maxit, 0, &iters,
                                     &relres, &conv);
  c->pws.vc = c->pws.met;
  HIPCHK(c, e);
  if (a->rho && c->pws.host_sc->rho_bad) return fail(c, LM_EINVAL, "rho must be positive and finite");
  a->iters = iters;
  a->relres = relres;
  a->mean_b = c->pws.host_sc->mean_b;
  if (!conv) return fail(c, LM_ENOCONV, "Poisson solver did not reach rtol");
  HIPCHK(c, launch_shift(c->st, L, c->pws.x, c->pws.sc, c->pws.x));  // zero mean, in place
  if (a->P) return copy_out(c, c->pws.x, a->P, -1, a->mem);
  return LM_OK;
}

lm_status lm_get_fields(lm_ctx *c, int level, lm_fields *f, int mem) {
  if (!c || !f) return fail(c, LM_EINVAL, "NULL argument");
  if (level != 0 && level != LM_LEVEL_PREDICTED)
    return fail(c, LM_EUNSUPPORTED, "level must be 0 or LM_LEVEL_PREDICTED");
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  if (level == LM_LEVEL_PREDICTED && !c->have_star)
    return fail(c, LM_ESTATE, "no step taken since the state was set or loaded");
  Level &lv = level == 0 ? cur(c) : c->lev[c->istar];
  double *Pl = level == 0 ? c->P[c->icur] : c->P[c->istar];
  lm_status s;
  const int nd = c->grid.ndim;
  if (f->rho && (s = copy_out(c, lv.rho, f->rho, -1, mem)) != LM_OK) return s;
  for (int d = 0; d < nd; ++d)
    if (f->v[d] && (s = copy_out(c, lv.v[d], f->v[d], -1, mem)) != LM_OK) return s;
  if (f->Z) {
    if (!lv.Z) return fail(c, LM_EINVAL, "Z is not transported (reacting = 0)");
    if ((s = copy_out(c, lv.Z, f->Z, -1, mem)) != LM_OK) return s;
  }
  if (f->H && (s = copy_out(c, lv.H, f->H, -1, mem)) != LM_OK) return s;
  if (f->T && (s = copy_out(c, lv.T, f->T, -1, mem)) != LM_OK) return s;
  if (f->P && (s = copy_out(c, Pl, f->P, -1, mem)) != LM_OK) return s;
  for (int d = 0; d < nd; ++d)
    if (f->F[d] && (s = copy_out(c, lv.F[d], f->F[d], d, mem)) != LM_OK) return s;
  if (mem == LM_DEVICE) HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

lm_status lm_get_dt(const lm_ctx *c, double *dt) {
  if (!c || !dt) return LM_EINVAL;
  if (!c->have_state && !(c->prm.dt > 0)) return LM_ESTATE;
  *dt = c->phys.dt;
  return LM_OK;
}

const char *lm_last_error(const lm_ctx *c) { return c ? c->err.c_str() : g_init_err; }

void lm_destroy(lm_ctx *c) {
  if (!c) return;
  (void)lm_kernel_timing(c, 0, 0);
  if (c->hflags) (void)hipHostFree(c->hflags);
  if (c->hscalar) (void)hipHostFree(c->hscalar);
  if (c->hlog) (void)hipHostFree(c->hlog);
  if (c->pws.host_sc) (void)hipHostFree(c->pws.host_sc);
  delete c;
}

}  // extern "C"

extern "C" lm_status lm_bench_kernel(lm_ctx *c, int which, int reps, double *avg_ms) {
  if (!c || !avg_ms || reps <= 0) return fail(c, LM_EINVAL, "bad arguments");
  if (!c->have_state) return fail(c, LM_ESTATE, "lm_set_fields must come first");
  if (which < 0 || which > 7) return fail(c, LM_EINVAL, "unknown kernel class");
  if (which == 3 && c->pws.lc == 0) return fail(c, LM_EUNSUPPORTED, "grid has no multi-block MG level");
  // solver kernels run only while the device flag `done` is clear
  SolverScalars sc{};
  sc.done = 0;
  sc.rzh[0] = sc.rzh[1] = 1.0;
  sc.cc = 1.0;
  HIPCHK(c, hipMemcpyAsync(c->pws.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  Level &A = c->lev[c->icur];
  Level &S = c->lev[c->istar];
  auto one = [&]() -> hipError_t {
    switch (which) {
      case 1:
        return launch_stage(c->st, 0, 1, c->lay, c->phys, A, A, c->R[c->rprev], c->R[c->rprev ^ 1], c->ib, S,
                            c->M, &c->p0d->dtp0_n);
      case 6:
        return launch_rhs(c->st, c->lay, c->bnd, c->phys, c->sides, c->M, S.rho, A.rho, c->rho_prev, 0, c->ib.S_m,
                          c->b, c->pws.partials, c->pws.sc);
      case 7:
        return launch_project(c->st, c->lay, c->bnd, c->phys, c->sides, c->M, c->pws.x, S.rho, c->pws.sc, S.F,
                              S.v, c->P[c->istar], c->dflags + 1);
      default: return poisson_bench_launch(c->st, c->pws, which);
    }
  };
  hipError_t e = one();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = one();
  if (e == hipSuccess) e = hipEventRecord(e1, c->st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the solver flag so later predicated launches stay idle
  sc.done = 1;
  if (e == hipSuccess) e = hipMemcpyAsync(c->pws.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) return fail(c, LM_EHIP, std::string("HIP error in lm_bench_kernel: ") + hipGetErrorString(e));
  *avg_ms = (double)ms / reps;
  return LM_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint / restart
// ---------------------------------------------------------------------------
namespace {

struct StateHeader {
  int have_prev, have_state;
  double time;
  int last_iters[2];
  double dt, dt_prev, dt_last, pc_err;  // time step and the adaptive-step history
  int nsame, pc_used;
};
// Header bytes [0, 128): StateHeader; [128, 256): the device p0 state.
static_assert(sizeof(StateHeader) <= 128 && sizeof(P0Dev) <= 128, "state header layout");

// Arrays making up the state, in a fixed order.
int state_arrays(lm_ctx *c, double **out) {
  int k = 0;
  const int nd = c->grid.ndim;
  Level &lv = c->lev[c->icur];
  out[k++] = lv.rho;
  for (int d = 0; d < nd; ++d) out[k++] = lv.v[d];
  if (lv.Z) out[k++] = lv.Z;
  out[k++] = lv.H;
  out[k++] = lv.T;
  out[k++] = lv.kap;
  for (int d = 0; d < nd; ++d) out[k++] = lv.F[d];
  out[k++] = c->P[c->icur];
  out[k++] = c->rho_prev;
  Resid &r = c->R[c->rprev];
  out[k++] = r.H;
  if (r.Z) out[k++] = r.Z;
  for (int d = 0; d < nd; ++d) out[k++] = r.v[d];
  return k;
}

// Direction of the outflow side (-1: none).
int outflow_dir(const lm_ctx *c) {
  for (int d = 0; d < c->grid.ndim; ++d)
    for (int s = 0; s < 2; ++s)
      if (c->grid.bc[d][s] == LM_SIDE_OUTFLOW) return d;
  return -1;
}

// The adjoint covers periodic, slip / no-slip wall and inflow sides, and an
// outflow side on the high end of at most one direction, on uniform spacing
// with at least 3 cells per direction.
bool adjoint_ok(lm_ctx *c) {
  if (!c->prm.with_adjoint || c->stretched) return false;
  // the residual gather tells a periodic stencil position from the cell it
  // wraps to by its unwrapped offset: 3 cells per direction at least (the
  // set-up already asks for 4)
  for (int d = 0; d < c->grid.ndim; ++d)
    if (c->grid.n[d] < 3) return false;
  int nout = 0;
  for (int d = 0; d < c->grid.ndim; ++d)
    for (int s = 0; s < 2; ++s)
      if (c->grid.bc[d][s] == LM_SIDE_OUTFLOW) {
        if (s == 0 || c->grid.n[d] < 3) return false;
        ++nout;
      }
  return nout <= 1;
}

// The arrays of an adjoint state with the face direction of each (-1 for
// cell arrays), in the order H, Z, v, F, rho_prev, R_H, R_Z, R_v (Z and R_Z
// in reacting flow only); returns the count.
int adj_arrays(const AdjState &a, int nd, bool react, double *arr[14], int fd[14]) {
  int k = 0;
  auto put = [&](double *x, int f) {
    arr[k] = x;
    fd[k++] = f;
  };
  put(a.H, -1);
  if (react) put(a.Z, -1);
  for (int d = 0; d < nd; ++d) put(a.v[d], -1);
  for (int d = 0; d < nd; ++d) put(a.F[d], d);
  put(a.rho_prev, -1);
  put(a.R_H, -1);
  if (react) put(a.R_Z, -1);
  for (int d = 0; d < nd; ++d) put(a.R_v[d], -1);
  return k;
}

// The caller's lm_adjoint as an adjoint state view.
AdjState adj_view(const lm_adjoint *in, int nd) {
  AdjState v{};
  v.H = in->H;
  v.Z = in->Z;
  v.rho_prev = in->rho_prev;
  v.R_H = in->R_H;
  v.R_Z = in->R_Z;
  for (int d = 0; d < nd; ++d) {
    v.v[d] = in->v[d];
    v.F[d] = in->F[d];
    v.R_v[d] = in->R_v[d];
  }
  return v;
}

AdjPhys adj_phys(const lm_ctx *c) {
  AdjPhys P;
  for (int d = 0; d < 3; ++d) P.h[d] = c->phys.h[d];
  P.Pe = c->phys.Pe;
  P.Pr = c->phys.Pr;
  P.sigma = c->phys.sigma;
  P.inv_Fr2 = c->phys.inv_Fr2;
  P.p0 = c->phys.p0;
  P.qs = c->phys.qs;
  P.dt = c->phys.dt;
  P.suth_C = c->phys.suth_C;
  P.Da = c->phys.Da;
  P.reacting = c->phys.reacting;
  P.S = c->phys.S;
  P.k = c->phys.k;
  P.Le_F = c->phys.Le_F;
  P.Le_O = c->phys.Le_O;
  P.N_F = c->phys.N_F;
  P.N_O = c->phys.N_O;
  P.fshift = c->phys.fshift;
  return P;
}

}  // namespace

extern "C" lm_status lm_state_size(const lm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return LM_EINVAL;
  double *arr[32];
  const int k = state_arrays(const_cast<lm_ctx *>(c), arr);
  *bytes = 256 + (size_t)k * c->lay.total * 8;
  return LM_OK;
}

extern "C" lm_status lm_save_state(lm_ctx *c, void *buf) {
  if (!c || !buf) return fail(c, LM_EINVAL, "NULL argument");
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  double *arr[32];
  const int k = state_arrays(c, arr);
  StateHeader h{c->have_prev, c->have_state, c->time, {c->last_iters[0], c->last_iters[1]},
                c->phys.dt,  c->dt_prev,     c->dt_last, c->pc_err,
                c->nsame,    c->pc_used};
  HIPCHK(c, hipMemcpyAsync(buf, &h, sizeof(h), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync((char *)buf + 128, c->p0d, sizeof(P0Dev), hipMemcpyDeviceToDevice, c->st));
  char *p = (char *)buf + 256;
  const size_t ab = (size_t)c->lay.total * 8;
  for (int q = 0; q < k; ++q) HIPCHK(c, hipMemcpyAsync(p + q * ab, arr[q], ab, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

extern "C" lm_status lm_load_state(lm_ctx *c, const void *buf) {
  if (!c || !buf) return fail(c, LM_EINVAL, "NULL argument");
  double *arr[32];
  const int k = state_arrays(c, arr);
  StateHeader h;
  HIPCHK(c, hipMemcpyAsync(&h, buf, sizeof(h), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(c->p0d, (const char *)buf + 128, sizeof(P0Dev), hipMemcpyDeviceToDevice, c->st));
  const char *p = (const char *)buf + 256;
  const size_t ab = (size_t)c->lay.total * 8;
  for (int q = 0; q < k; ++q) HIPCHK(c, hipMemcpyAsync(arr[q], p + q * ab, ab, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->have_prev = h.have_prev;
  c->have_state = h.have_state;
  c->have_star = 0;
  c->time = h.time;
  c->last_iters[0] = h.last_iters[0];
  c->last_iters[1] = h.last_iters[1];
  c->phys.dt = h.dt;
  c->dt_prev = h.dt_prev;
  c->dt_last = h.dt_last;
  c->pc_err = h.pc_err;
  c->nsame = h.nsame;
  c->pc_used = h.pc_used;
  return LM_OK;
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------
extern "C" lm_status lm_kinetic_energy(lm_ctx *c, double *ke) {
  if (!c || !ke) return LM_EINVAL;
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  Level &lv = c->lev[c->icur];
  double dV = 1.0;
  for (int d = 0; d < c->grid.ndim; ++d) dV *= c->phys.h[d];
  if (c->stretched) return fail(c, LM_EUNSUPPORTED, "kinetic energy implemented for uniform grids");
  HIPCHK(c, launch_ke(c->st, c->lay, lv.rho, lv.v, dV, c->pws.partials, c->dscalar));
  HIPCHK(c, hipMemcpyAsync(c->hscalar, c->dscalar, 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  *ke = c->hscalar[0];
  return LM_OK;
}

static const char *kAdjUnsupported =
    "adjoint needs with_adjoint, uniform spacing and at most one outflow side, on a high end";

extern "C" lm_status lm_adjoint_seed_ke(lm_ctx *c) {
  if (!c) return LM_EINVAL;
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  const int nd = c->grid.ndim;
  AdjState &a = c->ad[c->ad_cur];
  double *arr[14];
  int fd[14];
  const int k = adj_arrays(a, nd, c->prm.reacting, arr, fd);
  const size_t ab = (size_t)c->lay.total * 8;
  for (int q = 0; q < k; ++q) HIPCHK(c, hipMemsetAsync(arr[q], 0, ab, c->st));
  c->aw.xa_valid[0] = c->aw.xa_valid[1] = 0;  // a new reverse sweep: no warm start
  Level &lv = c->lev[c->icur];
  AdjCellArgs g{};
  g.L = c->lay;
  g.P = adj_phys(c);
  g.dV = 1.0;
  for (int d = 0; d < nd; ++d) g.dV *= c->phys.h[d];
  g.H = lv.H;
  g.Z = lv.Z;
  g.rho = lv.rho;
  g.Hb = a.H;
  g.Zb = a.Z;
  for (int d = 0; d < nd; ++d) {
    g.v[d] = lv.v[d];
    g.vb[d] = a.v[d];
  }
  HIPCHK(c, launch_adj_seed_ke(c->st, g));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

extern "C" lm_status lm_adjoint_set(lm_ctx *c, const lm_adjoint *in, int mem) {
  if (!c || !in) return LM_EINVAL;
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  const int nd = c->grid.ndim;
  const bool react = c->prm.reacting;
  if (!react && (in->Z || in->R_Z)) return fail(c, LM_EINVAL, "Z cotangents need reacting flow");
  AdjState &a = c->ad[c->ad_cur];
  c->aw.xa_valid[0] = c->aw.xa_valid[1] = 0;  // a new reverse sweep: no warm start
  double *arr[14], *src[14];
  int fd[14], fd2[14];
  const int k = adj_arrays(a, nd, react, arr, fd);
  adj_arrays(adj_view(in, nd), nd, react, src, fd2);
  for (int q = 0; q < k; ++q) {
    HIPCHK(c, hipMemsetAsync(arr[q], 0, (size_t)c->lay.total * 8, c->st));
    if (src[q]) {
      lm_status s = copy_in(c, src[q], arr[q], fd[q], mem);
      if (s != LM_OK) return s;
    }
  }
  if (in->T) {
    // T = qs (F~(Z) + H) (qs (H - 1) without reaction) at the current level:
    // the cotangent of T adds qs T_bar to H_bar and qs F~'(Z) T_bar to Z_bar
    if (react && !c->have_state) return fail(c, LM_ESTATE, "a T cotangent in reacting flow needs the state");
    double *Tb = c->aw.Tb_set;
    lm_status s = copy_in(c, in->T, Tb, -1, mem);
    if (s != LM_OK) return s;
    AdjCellArgs g{};
    g.L = c->lay;
    g.P = adj_phys(c);
    g.Z = c->lev[c->icur].Z;
    g.Tb = Tb;
    g.Hb = a.H;
    g.Zb = a.Z;
    HIPCHK(c, launch_adj_add_T(c->st, g));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

extern "C" lm_status lm_adjoint_get(lm_ctx *c, lm_adjoint *out, int mem) {
  if (!c || !out) return LM_EINVAL;
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  const int nd = c->grid.ndim;
  const bool react = c->prm.reacting;
  double *arr[14], *dst[14];
  int fd[14], fd2[14];
  const int k = adj_arrays(c->ad[c->ad_cur], nd, react, arr, fd);
  adj_arrays(adj_view(out, nd), nd, react, dst, fd2);
  for (int q = 0; q < k; ++q) {
    if (!dst[q]) continue;
    lm_status s = copy_out(c, arr[q], dst[q], fd[q], mem);
    if (s != LM_OK) return s;
  }
  if (mem == LM_DEVICE) HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

// The arrays of a step's levels that its reverse step reads: the predicted
// level (rho, H, Z in reacting flow, v, F) and the new level (rho, H, Z, v).
static int step_level_arrays(const lm_ctx *c, const Level &S, const Level &X, double **out) {
  const int nd = c->grid.ndim;
  const bool react = c->prm.reacting;
  int k = 0;
  out[k++] = S.rho;
  out[k++] = S.H;
  if (react) out[k++] = S.Z;
  for (int d = 0; d < nd; ++d) out[k++] = S.v[d];
  for (int d = 0; d < nd; ++d) out[k++] = S.F[d];
  out[k++] = X.rho;
  out[k++] = X.H;
  if (react) out[k++] = X.Z;
  for (int d = 0; d < nd; ++d) out[k++] = X.v[d];
  return k;
}

extern "C" lm_status lm_step_levels_size(const lm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return LM_EINVAL;
  double *arr[16];
  const Level &l = c->lev[0];
  *bytes = (size_t)step_level_arrays(c, l, l, arr) * c->lay.total * 8;
  return LM_OK;
}

extern "C" lm_status lm_save_step_levels(lm_ctx *c, void *buf) {
  if (!c || !buf) return fail(c, LM_EINVAL, "NULL argument");
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  if (!c->have_star) return fail(c, LM_ESTATE, "no step taken since the state was set or loaded");
  double *arr[16];
  // after a committed step the new level is the current one
  const int k = step_level_arrays(c, c->lev[c->istar], c->lev[c->icur], arr);
  const size_t ab = (size_t)c->lay.total * 8;
  for (int q = 0; q < k; ++q)
    HIPCHK(c, hipMemcpyAsync((char *)buf + q * ab, arr[q], ab, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

static lm_status step_adjoint(lm_ctx *c, const void *levels);

extern "C" lm_status lm_step_adjoint(lm_ctx *c) { return step_adjoint(c, nullptr); }

extern "C" lm_status lm_step_adjoint_levels(lm_ctx *c, const void *levels) {
  if (!levels) return fail(c, LM_EINVAL, "NULL argument");
  return step_adjoint(c, levels);
}

static lm_status step_adjoint(lm_ctx *c, const void *levels) {
  if (!c) return LM_EINVAL;
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  const Lay &L = c->lay;
  const int nd = c->grid.ndim;
  const bool react = c->prm.reacting;
  const size_t ab = (size_t)L.total * 8;
  lm_status s = LM_OK;
  if (levels) {
    // the step's predicted and new levels as saved right after it was
    // taken from this state
    double *arr[16];
    const int k = step_level_arrays(c, c->lev[c->istar], c->lev[c->inxt], arr);
    for (int q = 0; q < k; ++q)
      HIPCHK(c, hipMemcpyAsync(arr[q], (const char *)levels + q * ab, ab, hipMemcpyDeviceToDevice, c->st));
  } else {
    // forward recompute of the step (state at n untouched: outputs go to the
    // predicted and next levels)
    int it[2];
    double rr[2], cm[2];
    s = do_stage(c, 0, it[0], rr[0], cm[0]);
    if (s == LM_OK) s = do_stage(c, 1, it[1], rr[1], cm[1]);
    if (s == LM_OK) s = read_solve_logs(c, it, rr, cm);
    if (s != LM_OK) return s;
  }
  const int first = !c->have_prev;
  const AdjPhys P = adj_phys(c);
  Level &N = c->lev[c->icur], &S = c->lev[c->istar], &X = c->lev[c->inxt];
  AdjState &ain = c->ad[c->ad_cur];        // cotangent of the step's outputs
  AdjState &aout = c->ad[c->ad_cur ^ 1];   // cotangent of the step's inputs
  AdjWork &w = c->aw;
  // zero what is accumulated into
  HIPCHK(c, hipMemsetAsync(w.Hb_star, 0, ab, c->st));
  if (react) HIPCHK(c, hipMemsetAsync(w.Zb_star, 0, ab, c->st));
  for (int d = 0; d < nd; ++d)
    for (double *z : {w.vb_star[d], w.Fb_star[d], aout.F[d]}) HIPCHK(c, hipMemsetAsync(z, 0, ab, c->st));
  // the stage's adjoint solve starts from its solution one step later in
  // time (the previous call's), which the pressure cotangents of
  // consecutive steps leave close; the tolerance is the same
  auto adjoint_solve = [&](double *rhs, double *out, int stage) -> lm_status {
    HIPCHK(c, launch_mean(c->st, L, rhs, c->pws.partials, c->pws.sc, c->phys.vol, c->phys.volume));
    int iters = 0, conv = 0;
    double relres = 0.0;
    const double *x0 = w.xa_valid[stage] ? w.xa[stage] : nullptr;
    if (w.xa_valid[stage] >= 2) {
      HIPCHK(c, launch_adj_extrap(c->st, L, w.xa[stage], w.xa_old[stage], w.xa_guess));
      x0 = w.xa_guess;
    }
    HIPCHK(c, poisson_solve(c->st, c->pws, rhs, x0, c->prm.poisson_rtol, c->prm.poisson_maxit, w.xa_iters[stage],
                            &iters, &relres, &conv));
    if (!conv) return fail(c, LM_ENOCONV, "adjoint Poisson solve did not converge");
    HIPCHK(c, launch_shift(c->st, L, c->pws.x, c->pws.sc, out));
    std::swap(w.xa[stage], w.xa_old[stage]);
    HIPCHK(c, hipMemcpyAsync(w.xa[stage], out, ab, hipMemcpyDeviceToDevice, c->st));
    w.xa_valid[stage] = w.xa_valid[stage] + 1 > 2 ? 2 : w.xa_valid[stage] + 1;
    w.xa_iters[stage] = iters;
    return LM_OK;
  };
  auto proj = [&](double *const Fb[3], double *const vb[3], const Level &lv) -> hipError_t {
    AdjProjArgs a{};
    a.L = L;
    a.P = P;
    a.B = c->bnd;
    for (int d = 0; d < nd; ++d) {
      a.Fb[d] = Fb[d];
      a.vb[d] = vb[d];
      a.v[d] = lv.v[d];
      a.Mb[d] = w.Mb[d];
    }
    a.rho = lv.rho;
    a.rhob = w.rhob_new;
    a.Pb = w.Pb;
    return launch_adj_proj(c->st, a);
  };
  const IB *ib = c->phys.has_ib ? &c->ib : nullptr;
  auto resid = [&](const Level &lv, const double *RbH, const double *RbZ, double *const Rbv[3], double *Hb,
                   double *Zb, double *const vb[3], double *const Fb[3]) -> hipError_t {
    AdjResidArgs a{};
    a.L = L;
    a.P = P;
    a.B = c->bnd;
    a.sd = c->sides;
    a.H = lv.H;
    a.Z = lv.Z;
    a.RbH = RbH;
    a.RbZ = RbZ;
    a.Hb = Hb;
    a.Zb = Zb;
    for (int d = 0; d < nd; ++d) {
      a.v[d] = lv.v[d];
      a.F[d] = lv.F[d];
      a.Rbv[d] = Rbv[d];
      a.vb[d] = vb[d];
      a.Fb[d] = Fb[d];
    }
    if (ib && ib->chi) {
      a.chi = ib->chi;
      a.H_ib = ib->H_ib;
      a.Z_ib = ib->Z_ib;
      for (int d = 0; d < nd; ++d) a.v_ib[d] = ib->v_ib[d];
    }
    AdjCellArgs kk{};
    kk.L = L;
    kk.P = P;
    kk.H = lv.H;
    kk.Z = lv.Z;
    kk.Hb = w.kap;
    kk.Zb0 = w.dkap;
    hipError_t e = launch_adj_kappa(c->st, kk);
    if (e != hipSuccess) return e;
    a.kap = w.kap;
    a.dkap = w.dkap;
    return launch_adj_resid(c->st, a);
  };
  // outflow closure: the cotangent of the stage's right-hand side b from
  // that of the shifted one (y, the adjoint solve's output) and of the
  // outflow face fluxes
  const int dout = outflow_dir(c);
  auto closure = [&](double *const Fb[3]) -> hipError_t {
    if (dout < 0) return hipSuccess;
    return launch_adj_outflow(c->st, L, P, dout, w.bb, Fb[dout], c->dscalar + 1);
  };
  // corrector: projection, Poisson, right-hand side, EOS and AM2 transposes
  HIPCHK(c, proj(ain.F, ain.v, X));
  if ((s = adjoint_solve(w.Pb, w.bb, 0)) != LM_OK) return s;
  HIPCHK(c, closure(ain.F));
  AdjTailArgs t{};
  t.L = L;
  t.P = P;
  t.B = c->bnd;
  t.first = first;
  t.corrector = 1;
  t.bb = w.bb;
  t.rhob_new = w.rhob_new;
  t.H_new = X.H;
  t.Z_new = X.Z;
  t.rho_new = X.rho;
  t.rho_n = N.rho;
  t.Hb_out = ain.H;
  t.Zb_out = ain.Z;
  t.RbH_out = ain.R_H;
  t.RbZ_out = ain.R_Z;
  t.rhoprevb_out = ain.rho_prev;
  t.Hb_star = w.Hb_star;
  t.Zb_star = w.Zb_star;
  t.Hb_n = aout.H;
  t.Zb_n = aout.Z;
  t.rhob_n = w.rhob_n;
  t.RbH_star = w.RbH_star;
  t.RbZ_star = w.RbZ_star;
  t.RbH_n = w.RbH_n;
  t.RbZ_n = w.RbZ_n;
  t.rhoprevb_in = aout.rho_prev;
  t.RbH_prev_in = aout.R_H;
  t.RbZ_prev_in = aout.R_Z;
  for (int d = 0; d < nd; ++d) {
    t.Mb[d] = w.Mb[d];
    t.v_n[d] = N.v[d];
    t.Rbv_out[d] = ain.R_v[d];
    t.vb_n[d] = aout.v[d];
    t.Rbv_star[d] = w.Rbv_star[d];
    t.Rbv_n[d] = w.Rbv_n[d];
    t.Rbv_prev_in[d] = aout.R_v[d];
  }
  HIPCHK(c, launch_adj_tail(c->st, t));
  // residuals at the predicted level
  HIPCHK(c, resid(S, w.RbH_star, w.RbZ_star, w.Rbv_star, w.Hb_star, w.Zb_star, w.vb_star, w.Fb_star));
  // predictor: projection, Poisson, right-hand side, EOS and AB2 transposes
  HIPCHK(c, proj(w.Fb_star, w.vb_star, S));
  if ((s = adjoint_solve(w.Pb, w.bb, 1)) != LM_OK) return s;
  HIPCHK(c, closure(w.Fb_star));
  t.corrector = 0;
  t.H_new = S.H;
  t.Z_new = S.Z;
  t.rho_new = S.rho;
  HIPCHK(c, launch_adj_tail(c->st, t));
  // residuals at level n, then the EOS of level n
  HIPCHK(c, resid(N, w.RbH_n, w.RbZ_n, w.Rbv_n, aout.H, aout.Z, aout.v, aout.F));
  AdjCellArgs e{};
  e.L = L;
  e.P = P;
  e.H = N.H;
  e.Z = N.Z;
  e.rho = N.rho;
  e.rhob = w.rhob_n;
  e.Hb = aout.H;
  e.Zb = aout.Z;
  HIPCHK(c, launch_adj_eos(c->st, e));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->ad_cur ^= 1;
  return LM_OK;
}

extern "C" lm_status lm_adjoint_initial(lm_ctx *c, double *T0_bar, double *v0_bar[3], double *Z0_bar, int mem) {
  if (!c || !T0_bar) return LM_EINVAL;
  if (!adjoint_ok(c)) return fail(c, LM_EUNSUPPORTED, kAdjUnsupported);
  if (!c->have_state) return fail(c, LM_ESTATE, "no state set");
  if (Z0_bar && !c->prm.reacting) return fail(c, LM_EINVAL, "Z0_bar needs reacting flow");
  const int nd = c->grid.ndim;
  Level &N = c->lev[c->icur];
  AdjState &a = c->ad[c->ad_cur];
  AdjCellArgs g{};
  g.L = c->lay;
  g.P = adj_phys(c);
  g.B = c->bnd;
  g.H = N.H;
  g.Z = N.Z;
  g.rho = N.rho;
  g.Hb_in = a.H;
  g.Zb_in = a.Z;
  g.Tb_out = c->aw.Tb_init;
  g.Zb0 = c->aw.Zb_init;
  for (int d = 0; d < nd; ++d) {
    g.v[d] = N.v[d];
    g.Fb[d] = a.F[d];
    g.vb[d] = a.v[d];
  }
  HIPCHK(c, launch_adj_init(c->st, g));
  lm_status s = copy_out(c, g.Tb_out, T0_bar, -1, mem);
  if (s != LM_OK) return s;
  if (Z0_bar && (s = copy_out(c, g.Zb0, Z0_bar, -1, mem)) != LM_OK) return s;
  if (v0_bar) {
    for (int d = 0; d < nd; ++d)
      if (v0_bar[d] && (s = copy_out(c, a.v[d], v0_bar[d], -1, mem)) != LM_OK) return s;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  return LM_OK;
}

// ---------------------------------------------------------------------------
// In-step kernel timing
// ---------------------------------------------------------------------------
extern "C" lm_status lm_kernel_timing(lm_ctx *c, int which, int capacity) {
  if (!c || capacity < 0 || which < 0 || which > 2) return fail(c, LM_EINVAL, "bad arguments");
  PoissonWS &ws = c->pws;
  if (ws.tev) {
    (void)hipStreamSynchronize(c->st);
    for (int q = 0; q < 2 * ws.tcap; ++q) (void)hipEventDestroy(ws.tev[q]);
    delete[] ws.tev;
    delete[] ws.tk;
    ws.tev = nullptr;
    ws.tk = nullptr;
  }
  ws.tcap = ws.tcount = ws.tsolve0 = 0;
  ws.twhich = which;
  if (capacity == 0) return LM_OK;
  ws.tev = new (std::nothrow) hipEvent_t[2 * (size_t)capacity];
  ws.tk = new (std::nothrow) int[(size_t)capacity];
  if (!ws.tev || !ws.tk) {
    delete[] ws.tev;
    delete[] ws.tk;
    ws.tev = nullptr;
    ws.tk = nullptr;
    return fail(c, LM_ENOMEM, "out of host memory");
  }
  for (int q = 0; q < 2 * capacity; ++q) {
    const hipError_t e = hipEventCreate(&ws.tev[q]);
    if (e != hipSuccess) {
      for (int r = 0; r < q; ++r) (void)hipEventDestroy(ws.tev[r]);
      delete[] ws.tev;
      delete[] ws.tk;
      ws.tev = nullptr;
      ws.tk = nullptr;
      return fail(c, LM_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  ws.tcap = capacity;
  return LM_OK;
}

extern "C" lm_status lm_kernel_timing_read(lm_ctx *c, double *avg_ms, int *count) {
  if (!c || !avg_ms || !count) return fail(c, LM_EINVAL, "NULL argument");
  PoissonWS &ws = c->pws;
  HIPCHK(c, hipStreamSynchronize(c->st));
  double tot = 0.0;
  int n = 0;
  for (int q = 0; q < ws.tcount; ++q) {
    if (ws.tk[q] < 0) continue;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, ws.tev[2 * q], ws.tev[2 * q + 1]));
    tot += ms;
    ++n;
  }
  *count = n;
  *avg_ms = n ? tot / n : 0.0;
  return LM_OK;
}

// ---------------------------------------------------------------------------
// Pressure solve without allocation (lm_project_static)
// ---------------------------------------------------------------------------
namespace {

// Every device array of the solve lives here: 64 MiB per GPU, held from the
// first call on that GPU until the process ends. Calls on one GPU share it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kScratchDevices];     // device address of `scratch`, per device
SolverScalars g_scratch_sc[kScratchDevices];       // host copy of the solver scalars, per device

__global__ void __launch_bounds__(kBlock) k_zero_bytes(ulonglong2 *p, size_t n16) {
  const ulonglong2 z = make_ulonglong2(0ull, 0ull);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

// Carves the arrays of a pressure solve (right-hand side, host staging and
// the solver) from cv; cv.base == nullptr only sizes them.
bool carve_solve(PoissonWS &ws, Carver &cv, const Lay &L, const Bnd &B, const double h[3], const lm_params &p,
                 double **b, double **staging) {
  *b = (double *)cv.take((size_t)L.total * 8);
  *staging = (double *)cv.take((size_t)L.ncells() * 8);
  return poisson_plan(ws, cv, L, B, h, p.precision != LM_FP64, p.precision == LM_MIXED_FLEXIBLE,
                      p.mg_nu > 0 ? p.mg_nu : 2, 0, nullptr);
}

#define STATIC_HIPCHK(expr)                                                                        \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      snprintf(g_init_err, sizeof(g_init_err), "HIP error in %s: %s", #expr, hipGetErrorString(e_)); \
      return LM_EHIP;                                                                              \
    }                                                                                              \
  } while (0)

}  // namespace

extern "C" lm_status lm_project_static(const lm_grid *grid, const lm_params *params, void *stream,
                                       lm_project_args *a) {
  if (!grid || !params || !a || !a->b) return init_fail(LM_EINVAL, "NULL argument");
  if (a->rho) return init_fail(LM_EUNSUPPORTED, "lm_project_static solves the beta = 1 form only");
  if (grid->faces[0] || grid->faces[1] || grid->faces[2])
    return init_fail(LM_EUNSUPPORTED, "lm_project_static takes uniform grids only");
  if (a->mem != LM_HOST && a->mem != LM_DEVICE) return init_fail(LM_EINVAL, "mem must be LM_HOST or LM_DEVICE");
  const char *bad = nullptr;
  if (!valid_grid(grid, &bad) || !valid_params(params, &bad)) return init_fail(LM_EINVAL, bad);
  // layout, sides and spacings as lm_init_grid sets them up
  Lay L = make_layout(grid->ndim, grid->n, 8);
  Bnd B;
  B.all_periodic = 1;
  for (int d = 0; d < 3; ++d) {
    for (int q = 0; q < 2; ++q) B.kind[d][q] = d < grid->ndim ? grid->bc[d][q] : LM_SIDE_PERIODIC;
    B.periodic[d] = B.kind[d][0] == LM_SIDE_PERIODIC;
    if (d < grid->ndim && !B.periodic[d]) B.all_periodic = 0;
  }
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = d < grid->ndim ? grid->L[d] / grid->n[d] : 1.0;
  // sizing pass: rejected before any device work when it does not fit
  PoissonWS ws{};
  double *b = nullptr, *staging = nullptr;
  Carver sz{nullptr, 0};
  if (!carve_solve(ws, sz, L, B, h, *params, &b, &staging))
    return init_fail(LM_EUNSUPPORTED, "grid does not coarsen far enough for the multigrid solver");
  if (ws.lev[ws.nlev - 1].lay.ncells() > kVcCoarsest)
    return init_fail(LM_EUNSUPPORTED, "lm_project_static needs a grid that coarsens to <= 128 cells");
  const size_t need = (sz.off + 255) & ~(size_t)255;
  if (need > kScratchBytes) {
    snprintf(g_init_err, sizeof(g_init_err),
             "grid needs %zu bytes of solver scratch; lm_project_static holds %zu (64 MiB)", need, kScratchBytes);
    return LM_ENOMEM;
  }
  // the device address of this GPU's copy of `scratch`, taken once per device
  int dev = 0;
  STATIC_HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return init_fail(LM_EUNSUPPORTED, "device index beyond 64");
  unsigned char *base;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *ptr = nullptr;
      STATIC_HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    base = g_scratch_ptr[dev];
  }
  hipStream_t st = (hipStream_t)stream;
  ws = PoissonWS{};
  Carver cv{(char *)base, 0};
  carve_solve(ws, cv, L, B, h, *params, &b, &staging);
  ws.host_sc = &g_scratch_sc[dev];
  // the previous call's contents: ghost layers and padding start at zero
  hipLaunchKernelGGL(k_zero_bytes, dim3(1024), dim3(kBlock), 0, st, (ulonglong2 *)base, need / 16);
  STATIC_HIPCHK(hipGetLastError());
  STATIC_HIPCHK(poisson_setup_device(st, ws));
  const double *src = a->b;
  if (a->mem == LM_HOST) {
    STATIC_HIPCHK(hipMemcpyAsync(staging, a->b, (size_t)L.ncells() * 8, hipMemcpyHostToDevice, st));
    src = staging;
  }
  STATIC_HIPCHK(launch_pack(st, L, src, b, -1));
  STATIC_HIPCHK(launch_mean(st, L, b, ws.partials, ws.sc, nullptr, 0.0));
  int iters = 0, conv = 0;
  double relres = 0.0;
  const double rtol = a->rtol > 0 ? a->rtol : params->poisson_rtol;
  STATIC_HIPCHK(poisson_solve(st, ws, b, nullptr, rtol, params->poisson_maxit, 0, &iters, &relres, &conv));
  a->iters = iters;
  a->relres = relres;
  a->mean_b = ws.host_sc->mean_b;
  if (!conv) return init_fail(LM_ENOCONV, "Poisson solver did not reach rtol");
  STATIC_HIPCHK(launch_shift(st, L, ws.x, ws.sc, ws.x));  // zero mean, in place
  if (a->P) {
    if (a->mem == LM_HOST) {
      STATIC_HIPCHK(launch_unpack(st, L, ws.x, staging, -1));
      STATIC_HIPCHK(hipMemcpyAsync(a->P, staging, (size_t)L.ncells() * 8, hipMemcpyDeviceToHost, st));
    } else {
      STATIC_HIPCHK(launch_unpack(st, L, ws.x, a->P, -1));
    }
  }
  STATIC_HIPCHK(hipStreamSynchronize(st));
  return LM_OK;
}
