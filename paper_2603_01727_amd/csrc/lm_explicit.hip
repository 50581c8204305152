// Explicit part of the predictor-corrector step on the collocated grid:
// ghost cells (section 3.6), the fused residual + Adams update + equation of
// state kernel (sections 3.1, 3.2, 3.4, 3.5), the Poisson right-hand side
// with the outflow mass closure (section 3.1, 3.3) and the projection of
// face fluxes and cell velocities (Eq 3.23, 3.25).
#include "lm_device.h"
#include "lm_sides.h"

namespace lm {

// Value of field `a` (rule set f) at ghost position (i, j, k): the rules of
// the highest out-of-range direction are applied first, which reproduces
// filling directions in the order x, y, z with each pass covering the ghosts
// of the directions already filled.
template <int DIM>
__device__ double ghost_value(const Lay &L, const Bnd &B, const Sides &sd, const double *a, int f, int i,
                              int j, int k) {
  double w[27];
  int pos[27][3];
  int nt = 1;
  w[0] = 1.0;
  pos[0][0] = i;
  pos[0][1] = j;
  pos[0][2] = k;
  double cst = 0.0;
  for (int d = DIM - 1; d >= 0; --d) {
    const int n = L.n[d];
    const int cur = nt;
    for (int t = 0; t < cur; ++t) {
      const int q = pos[t][d];
      if (q >= 0 && q < n) continue;
      const int s = q < 0 ? 0 : 1;
      const int i1 = s == 0 ? 0 : n - 1, i2 = s == 0 ? 1 : n - 2, i3 = s == 0 ? 2 : n - 3;
      switch (ghost_rule(B, sd, L, d, s, f, pos[t][0], pos[t][1], pos[t][2])) {
        case R_PER: pos[t][d] = s == 0 ? n - 1 : 0; break;
        case R_DIR:
          cst += 2.0 * w[t] * side_value(sd, L, d, s, f, pos[t][0], pos[t][1], pos[t][2]);
          w[t] = -w[t];
          pos[t][d] = i1;
          break;
        case R_NEU: pos[t][d] = i1; break;
        default: {
          const double wt = w[t];
          w[t] = 3.0 * wt;
          pos[t][d] = i1;
          w[nt] = -3.0 * wt;
          pos[nt][0] = pos[t][0]; pos[nt][1] = pos[t][1]; pos[nt][2] = pos[t][2];
          pos[nt][d] = i2;
          ++nt;
          w[nt] = wt;
          pos[nt][0] = pos[t][0]; pos[nt][1] = pos[t][1]; pos[nt][2] = pos[t][2];
          pos[nt][d] = i3;
          ++nt;
        }
      }
    }
  }
  double v = cst;
  for (int t = 0; t < nt; ++t) v += w[t] * a[L.at(pos[t][0], pos[t][1], pos[t][2])];
  return v;
}

// Ghost position number t of the padded box (box minus interior).
template <int DIM>
__device__ inline bool ghost_pos(const Lay &L, long t, int &i, int &j, int &k) {
  const long nx2 = L.n[0] + 2, ny2 = L.n[1] + 2;
  if (DIM == 3) {
    const long a = 2 * nx2 * ny2;
    if (t < a) {
      k = (t / (nx2 * ny2)) ? L.n[2] : -1;
      long r = t % (nx2 * ny2);
      j = (int)(r / nx2) - 1;
      i = (int)(r % nx2) - 1;
      return true;
    }
    t -= a;
  }
  const int nz = L.n[2];
  const long b = 2 * nx2 * nz;
  if (t < b) {
    long plane = t / (2 * nx2);
    long r = t % (2 * nx2);
    k = DIM == 3 ? (int)plane : 0;
    j = (r / nx2) ? L.n[1] : -1;
    i = (int)(r % nx2) - 1;
    return true;
  }
  t -= b;
  const long c = 2L * L.n[1] * nz;
  if (t < c) {
    long plane = t / (2L * L.n[1]);
    long r = t % (2L * L.n[1]);
    k = DIM == 3 ? (int)plane : 0;
    j = (int)(r / 2);
    i = (r % 2) ? L.n[0] : -1;
    return true;
  }
  return false;
}

template <int DIM>
inline long ghost_count(const Lay &L) {
  long nx2 = L.n[0] + 2, ny2 = L.n[1] + 2;
  long cnt = 2 * nx2 * L.n[2] + 2L * L.n[1] * L.n[2];
  if (DIM == 3) cnt += 2 * nx2 * ny2;
  return cnt;
}

struct GhostArgs {
  double *v[3], *Z, *H, *T, *kap;
};

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_ghosts_periodic(Lay L, GhostArgs g, long count) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int i, j, k;
  if (!ghost_pos<DIM>(L, t, i, j, k)) return;
  const int si = i < 0 ? L.n[0] - 1 : (i >= L.n[0] ? 0 : i);
  const int sj = j < 0 ? L.n[1] - 1 : (j >= L.n[1] ? 0 : j);
  const int sk = DIM == 3 ? (k < 0 ? L.n[2] - 1 : (k >= L.n[2] ? 0 : k)) : k;
  const long dst = L.at(i, j, k), src = L.at(si, sj, sk);
  for (int c = 0; c < DIM; ++c) g.v[c][dst] = g.v[c][src];
  g.H[dst] = g.H[src];
  if (g.Z) g.Z[dst] = g.Z[src];
  g.T[dst] = g.T[src];
  g.kap[dst] = g.kap[src];
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_ghosts_general(Lay L, Bnd B, Phys P, Sides sd, GhostArgs g,
                                                           long count) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int i, j, k;
  if (!ghost_pos<DIM>(L, t, i, j, k)) return;
  const long dst = L.at(i, j, k);
  for (int c = 0; c < DIM; ++c) g.v[c][dst] = ghost_value<DIM>(L, B, sd, g.v[c], c, i, j, k);
  const double H = ghost_value<DIM>(L, B, sd, g.H, 4, i, j, k);
  double Z = 0.0;
  if (P.reacting) Z = ghost_value<DIM>(L, B, sd, g.Z, 3, i, j, k);
  g.H[dst] = H;
  if (g.Z) g.Z[dst] = Z;
  // ghost temperature (boundary-face conductivity only) with Z clamped to
  // its realizable range [0, S+1]
  const double Zc = P.reacting ? fmin(fmax(Z, 0.0), P.S + 1.0) : 0.0;
  const double T = temperature(P, Zc, H);
  g.T[dst] = T;
  int dw, sw;
  if (isothermal_ghost<DIM>(L, B, sd, i, j, k, dw, sw)) {
    // the wall face takes the conductivity of the wall temperature: the
    // ghost is its mirror through the face (the mirrored temperature
    // 2 T_w - T can be out of the range of kappa in a start-up transient)
    const double Tw = temperature(P, 0.0, side_value(sd, L, dw, sw, 4, i, j, k));
    const long src = L.at(min(max(i, 0), L.n[0] - 1), min(max(j, 0), L.n[1] - 1),
                          DIM == 3 ? min(max(k, 0), L.n[2] - 1) : k);
    g.kap[dst] = 2.0 * kappa_of(P, Tw) - kappa_of(P, g.T[src]);
  } else {
    g.kap[dst] = kappa_of(P, T);
  }
}

hipError_t launch_ghosts(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                         double *v[3], double *Z, double *H, double *T, double *kap) {
  GhostArgs g{{v[0], v[1], v[2]}, Z, H, T, kap};
  const long cnt = L.ndim == 3 ? ghost_count<3>(L) : ghost_count<2>(L);
  const unsigned nb = ceil_div(cnt, kBlock);
  if (B.all_periodic) {
    if (L.ndim == 3)
      hipLaunchKernelGGL(k_ghosts_periodic<3>, dim3(nb), dim3(kBlock), 0, st, L, g, cnt);
    else
      hipLaunchKernelGGL(k_ghosts_periodic<2>, dim3(nb), dim3(kBlock), 0, st, L, g, cnt);
  } else {
    if (L.ndim == 3)
      hipLaunchKernelGGL(k_ghosts_general<3>, dim3(nb), dim3(kBlock), 0, st, L, B, P, sd, g, cnt);
    else
      hipLaunchKernelGGL(k_ghosts_general<2>, dim3(nb), dim3(kBlock), 0, st, L, B, P, sd, g, cnt);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residuals at one time level and the Adams update
// ---------------------------------------------------------------------------

// ---- field access ---------------------------------------------------------
// The residual arithmetic reads every field through an accessor, at offsets
// (o0, o1, o2) in cells from the cell the residual is taken at, so one body
// of arithmetic serves both the direct kernel (padded arrays in HBM) and the
// z-marching 3D kernel (LDS planes and registers).
// Spacings of a uniform grid: the inverse distance across a face (lo = 0:
// the high face, -1: the low face), the inverse cell width, the inverse
// distance between the centres on either side along k (Eq 3.21, n = 2),
// and the interpolation from two centres to their face (Eq 3.20, n = 1).
#define LM_UNIFORM_SPACING                                                                   \
  __device__ static double ihf(const Phys &P, int d, int) { return P.ih[d]; }                \
  __device__ static double ihc(const Phys &P, int d) { return P.ih[d]; }                     \
  __device__ static double i2h(const Phys &P, int k) { return 0.5 * P.ih[k]; }               \
  __device__ static double interp(int, int, double a, double b) { return 0.5 * (a + b); }

struct DirectAcc {
  LM_UNIFORM_SPACING
  static constexpr bool kPhased = false;
  const Level &lv;
  const IB &ib;
  long c, s1, s2;
  int has_ib;
  __device__ long at(int o0, int o1, int o2) const { return c + o0 + o1 * s1 + o2 * s2; }
  __device__ double v(int i, int o0, int o1, int o2) const { return lv.v[i][at(o0, o1, o2)]; }
  __device__ double kap(int o0, int o1, int o2) const { return lv.kap[at(o0, o1, o2)]; }
  // scalar field f: 0 H, 1 Z
  __device__ double s(int f, int o0, int o1, int o2) const { return (f ? lv.Z : lv.H)[at(o0, o1, o2)]; }
  // face flux F_d on the face of the cell at offset o (0 or -1) along d
  __device__ double F(int d, int o) const { return lv.F[d][c + o * (d == 0 ? 1 : (d == 1 ? s1 : s2))]; }
  __device__ double rho() const { return lv.rho[c]; }
  __device__ double chi() const { return (has_ib && ib.chi) ? (double)ib.chi[c] : 0.0; }
  __device__ double v_ib(int i) const { return ib.v_ib[i] ? ib.v_ib[i][c] : 0.0; }
  __device__ double Z_ib() const { return ib.Z_ib ? ib.Z_ib[c] : 0.0; }
  __device__ double H_ib() const { return ib.H_ib ? ib.H_ib[c] : 0.0; }
};

// Stretched 2D grid: the direct accessor with the local spacings of the
// cell at interior coordinates q.
struct StretchedAcc {
  static constexpr bool kPhased = false;
  DirectAcc g;
  MetView m[2];
  int q[2];
  __device__ double v(int i, int o0, int o1, int o2) const { return g.v(i, o0, o1, o2); }
  __device__ double kap(int o0, int o1, int o2) const { return g.kap(o0, o1, o2); }
  __device__ double s(int f, int o0, int o1, int o2) const { return g.s(f, o0, o1, o2); }
  __device__ double F(int d, int o) const { return g.F(d, o); }
  __device__ double rho() const { return g.rho(); }
  __device__ double chi() const { return g.chi(); }
  __device__ double v_ib(int i) const { return g.v_ib(i); }
  __device__ double Z_ib() const { return g.Z_ib(); }
  __device__ double H_ib() const { return g.H_ib(); }
  __device__ double ihf(const Phys &, int d, int lo) const { return m[d].idfc[q[d] + 1 + lo]; }
  __device__ double ihc(const Phys &, int d) const { return m[d].iwid[q[d] + 1]; }
  __device__ double i2h(const Phys &, int k) const { return m[k].id2[q[k]]; }
  __device__ double interp(int d, int lo, double x, double y) const {
    const int f = q[d] + 1 + lo;
    return m[d].wlo[f] * x + m[d].whi[f] * y;
  }
};

// Scheduling fence between the phases of a residual, for accessors that
// ask for it (LDS-fed forms: their operands are cheap to fetch late, and
// holding them all at once would exhaust the register file).
template <class A>
__device__ inline void phase_fence() {
  if constexpr (A::kPhased) asm volatile("" ::: "memory");
}

// tau_id on the face between the cells at offsets lo e_d and (lo + 1) e_d
// (lo = 0 or -1; Eq 2.46 on d-faces), all components i at once: kappa_f
// [D_d v_i + D_i v_d - 2/3 delta_id div], D_d the difference across the
// face, D_k (k != d) the mean of the two cells' centred differences. Only
// the derivatives the face needs are formed: the normal ones of every
// component, and along each k != d those of v_d and v_k.
template <int DIM, class A>
__device__ inline void face_stress(const A &a, const Phys &P, int lo, int d, double tau[3]) {
  int o[3] = {0, 0, 0}, q[3] = {0, 0, 0};
  o[d] = lo;
  q[d] = lo + 1;
  const double kf = a.interp(d, lo, a.kap(o[0], o[1], o[2]), a.kap(q[0], q[1], q[2]));
  double Dn[3];       // D_d v_c
  double Dkd[3];      // D_k v_d (k != d)
  double Dkk[3];      // D_k v_k (k != d)
  const double ihd = a.ihf(P, d, lo);
#pragma unroll
  for (int c = 0; c < DIM; ++c) Dn[c] = (a.v(c, q[0], q[1], q[2]) - a.v(c, o[0], o[1], o[2])) * ihd;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (k == d) continue;
    const double i2h = a.i2h(P, k);  // 1/(2h): centred differences
    int op[3] = {o[0], o[1], o[2]}, om[3] = {o[0], o[1], o[2]};
    int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
    op[k] += 1;
    om[k] -= 1;
    qp[k] += 1;
    qm[k] -= 1;
    Dkd[k] = a.interp(d, lo, (a.v(d, op[0], op[1], op[2]) - a.v(d, om[0], om[1], om[2])) * i2h,
                      (a.v(d, qp[0], qp[1], qp[2]) - a.v(d, qm[0], qm[1], qm[2])) * i2h);
    Dkk[k] = a.interp(d, lo, (a.v(k, op[0], op[1], op[2]) - a.v(k, om[0], om[1], om[2])) * i2h,
                      (a.v(k, qp[0], qp[1], qp[2]) - a.v(k, qm[0], qm[1], qm[2])) * i2h);
  }
  double div = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) div += (k == d) ? Dn[d] : Dkk[k];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    const double t = (i == d) ? (Dn[d] + Dn[d]) - (2.0 / 3.0) * div : Dn[i] + Dkd[i];
    tau[i] = kf * t;
  }
}

// Scalar terms of Eq 3.26b and the centred diffusion of section 3.2 for the
// scalar field f (0 H, 1 Z).
template <int DIM, class A>
__device__ inline void scalar_terms(const A &a, const Phys &P, int f, double &adv, double &dif) {
  adv = 0.0;
  dif = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int p[3] = {0, 0, 0}, m[3] = {0, 0, 0};
    p[d] = 1;
    m[d] = -1;
    const double sc = a.s(f, 0, 0, 0);
    const double gp = (a.s(f, p[0], p[1], p[2]) - sc) * a.ihf(P, d, 0);
    const double gm = (sc - a.s(f, m[0], m[1], m[2])) * a.ihf(P, d, -1);
    const double kc = a.kap(0, 0, 0);
    const double kp = a.interp(d, 0, kc, a.kap(p[0], p[1], p[2]));
    const double km = a.interp(d, -1, a.kap(m[0], m[1], m[2]), kc);
    // face to centre: the centroid lies midway between its faces
    adv = adv + 0.5 * (a.F(d, 0) * gp + a.F(d, -1) * gm);
    dif = dif + (kp * gp - km * gm) * a.ihc(P, d);
  }
}

// Direct form for kernels that take the scalar terms alone.
template <int DIM>
__device__ inline void scalar_terms(const Lay &L, const Phys &P, const Level &lv, int f, long c, double &adv,
                                    double &dif) {
  const IB ib{};
  const DirectAcc a{lv, ib, c, L.s[1], L.s[2], 0};
  scalar_terms<DIM>(a, P, f, adv, dif);
}

template <int DIM, class A>
__device__ inline void residuals(const A &a, const Phys &P, double dtp0, double &RH, double &RZ, double Rv[3]) {
  const double rho = a.rho();
  const double kap = a.kap(0, 0, 0);
  const double chi = a.chi();
  double advH, difH;
  phase_fence<A>();
  scalar_terms<DIM>(a, P, 0, advH, difH);
  phase_fence<A>();
  double rH = -advH + difH / P.Pe;
  RZ = 0.0;
  if (P.reacting) {
    double advZ, difZ;
    scalar_terms<DIM>(a, P, 1, advZ, difZ);
    phase_fence<A>();
    const double Z = a.s(1, 0, 0, 0);
    const double th = theta_eps(P, Z);
    const double le = (P.Le_F - P.Le_O) * th + P.Le_O;
    const double nn = (P.N_F - P.N_O) * th + P.N_O;
    double rZ = -advZ + difZ / (le * P.Pe);
    rH = rH + nn * difZ / P.Pe;
    if (chi != 0.0) rZ = rZ - chi * kap * (Z - a.Z_ib()) / (le * P.Pe * P.Da);
    RZ = rZ / rho;
  }
  if (chi != 0.0) rH = rH - chi * kap * (a.s(0, 0, 0, 0) - a.H_ib()) / (P.Pe * P.Da);
  if (P.closed) rH = rH + P.zeta * dtp0;  // zeta d_t p0 (Eq 3.4b), enclosed systems
  RH = rH / rho;
  double visc_all[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double tp[3], tm[3];
    face_stress<DIM>(a, P, 0, d, tp);
    phase_fence<A>();
    face_stress<DIM>(a, P, -1, d, tm);
    phase_fence<A>();
#pragma unroll
    for (int i = 0; i < DIM; ++i) visc_all[i] = visc_all[i] + (tp[i] - tm[i]) * a.ihc(P, d);
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double conv = 0.0;
    const double visc = visc_all[i];
    const double vc = a.v(i, 0, 0, 0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int p[3] = {0, 0, 0}, m[3] = {0, 0, 0};
      p[d] = 1;
      m[d] = -1;
      const double flp = a.F(d, 0) * a.interp(d, 0, vc, a.v(i, p[0], p[1], p[2]));
      const double flm = a.F(d, -1) * a.interp(d, -1, a.v(i, m[0], m[1], m[2]), vc);
      conv = conv + (flp - flm) * a.ihc(P, d);
    }
    double r = -conv + (P.Pr / P.Pe) * visc;
    if (i == 1 && P.inv_Fr2 != 0.0) r = r + P.inv_Fr2 * (1.0 - rho);
    if (chi != 0.0) r = r - chi * (P.Pr / (P.Pe * P.Da)) * kap * (vc - a.v_ib(i));
    Rv[i] = r;
    phase_fence<A>();
  }
}

struct StageArgs {
  Level cur, n0, out;
  Resid rprev, rn;
  IB ib;
  double *M[3];
  const double *dtp0;  // d_t p0 of the level the residuals are taken at (enclosed systems)
};

// Values at the cell the Adams update reads besides the residuals: level n
// and the stored residuals (R^{n-1} in the predictor, R^n in the corrector).
struct Centre {
  double rho0, H0, Z0, v0[3];
  double rH, rZ, rv[3];
};

template <int DIM, int CORR>
__device__ inline void load_centre(const Phys &P, const StageArgs &a, long c, int first, Centre &q) {
  q.rho0 = a.n0.rho[c];
  q.H0 = a.n0.H[c];
  q.Z0 = P.reacting ? a.n0.Z[c] : 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) q.v0[i] = a.n0.v[i][c];
  const Resid &r = CORR ? a.rn : a.rprev;
  const bool need = CORR || !first;
  q.rH = need ? r.H[c] : 0.0;
  q.rZ = (need && P.reacting) ? r.Z[c] : 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) q.rv[i] = need ? r.v[i][c] : 0.0;
}

// Predictor (corrector = 0): residuals of level n stored for the corrector
// and the next step; AB2 (Euler on the first step) for H, Z and rho v
// (Eq 3.1, 3.3, 3.10); T*, rho*, kappa* from the equation of state (Eq 3.6).
// Corrector: AM2 with the stored level-n residuals (Eq 3.12, 3.13, 3.18);
// T, rho, kappa at n+1 (Eq 3.15).
template <int DIM, int CORR>
__device__ inline void stage_update(const Phys &P, const StageArgs &a, long c, int first, const Centre &q,
                                    double RH, double RZ, const double Rv[3]) {
  const double dt = P.dt;
  double H, Z = 0.0;
  if (!CORR) {
    a.rn.H[c] = RH;
    if (P.reacting) a.rn.Z[c] = RZ;
#pragma unroll
    for (int i = 0; i < DIM; ++i) a.rn.v[i][c] = Rv[i];
    if (first) {
      H = q.H0 + dt * RH;
      if (P.reacting) Z = q.Z0 + dt * RZ;
#pragma unroll
      for (int i = 0; i < DIM; ++i) a.M[i][c] = q.rho0 * q.v0[i] + dt * Rv[i];
    } else if (P.var_step) {
      // AB2 for unequal steps: weights 1 + w/2 and -w/2, w = dt / dt_prev
      H = q.H0 + dt * (P.ab0 * RH + P.ab1 * q.rH);
      if (P.reacting) Z = q.Z0 + dt * (P.ab0 * RZ + P.ab1 * q.rZ);
#pragma unroll
      for (int i = 0; i < DIM; ++i) a.M[i][c] = q.rho0 * q.v0[i] + dt * (P.ab0 * Rv[i] + P.ab1 * q.rv[i]);
    } else {
      H = q.H0 + dt * (1.5 * RH - 0.5 * q.rH);
      if (P.reacting) Z = q.Z0 + dt * (1.5 * RZ - 0.5 * q.rZ);
#pragma unroll
      for (int i = 0; i < DIM; ++i) a.M[i][c] = q.rho0 * q.v0[i] + dt * (1.5 * Rv[i] - 0.5 * q.rv[i]);
    }
  } else {
    H = q.H0 + 0.5 * dt * (RH + q.rH);
    if (P.reacting) Z = q.Z0 + 0.5 * dt * (RZ + q.rZ);
#pragma unroll
    for (int i = 0; i < DIM; ++i) a.M[i][c] = q.rho0 * q.v0[i] + 0.5 * dt * (Rv[i] + q.rv[i]);
  }
  const double T = temperature(P, Z, H);
  a.out.H[c] = H;
  if (P.reacting) a.out.Z[c] = Z;
  a.out.T[c] = T;
  a.out.rho[c] = P.p0 / T;
  a.out.kap[c] = kappa_of(P, T);
}

// One thread per cell, every field read straight from the padded arrays
// (MET: a stretched 2D grid, local spacings).
template <int DIM, int CORR, bool MET = false>
__global__ void __launch_bounds__(kBlock) k_stage(Lay L, Phys P, StageArgs a, int first) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  double RH, RZ, Rv[3];
  const double dtp0 = P.closed ? *a.dtp0 : 0.0;
  const DirectAcc acc{a.cur, a.ib, c, L.s[1], L.s[2], P.has_ib};
  if constexpr (MET) {
    const StretchedAcc sa{acc, {met_view(P.met, L, 0), met_view(P.met, L, 1)}, {p.i, p.j}};
    residuals<DIM>(sa, P, dtp0, RH, RZ, Rv);
  } else {
    residuals<DIM>(acc, P, dtp0, RH, RZ, Rv);
  }
  Centre q;
  load_centre<DIM, CORR>(P, a, c, first, q);
  stage_update<DIM, CORR>(P, a, c, first, q, RH, RZ, Rv);
}

// ---- z-marching 3D stage ------------------------------------------------
// A block owns a 64 x 4 column of cells and a run of planes; it marches up
// the planes. The velocity components are read at edge neighbours in all
// three planes z-1, z, z+1, so they sit in a ring of four LDS planes (three
// read, one being filled); kappa, H, Z and the x / y face fluxes are read
// off-centre only within the plane, so they sit in two LDS planes (read,
// filled); their z-1 / z+1 values and the z face flux come from registers
// of the thread's own column. The halo tiles go from HBM straight into LDS
// (16-byte global-to-LDS loads, no registers held), one plane ahead of use
// (two for the velocity ring), so one barrier per plane suffices and the
// next plane streams in while this one is computed. Every field is read
// from HBM once, plus the tile's halo.
constexpr int kMX = 64, kMY = 4;            // cells of a block's column
constexpr int kMW = kMX + 4;                // LDS row: x0-2 .. x0+65 (16-byte pairs from an even x)
constexpr int kMP = kMW * (kMY + 2);        // doubles per LDS plane
constexpr int kMPairs = kMP / 2;            // 16-byte pairs per plane (one per thread, first kMPairs threads)
constexpr int kMarchBlocks = 2048;          // target grid (chooses the run of planes)
static_assert(kMPairs <= kBlock, "one pair per thread");

struct MarchShared {
  double v[3][4][kMP];  // velocity components, ring of four planes (plane z in slot z & 3)
  double s[5][2][kMP];  // kappa, H, Z, F_0, F_1: plane z in slot z & 1
};

typedef __attribute__((address_space(3))) void lds_void_t;

// Global-to-LDS copy of one 16-byte pair per lane; lane l of the wavefront
// writes pairs 64 w + l of the plane (w = the wavefront of the block).
__device__ inline void pair_to_lds(const double *src, double *plane) {
  double *dst = plane + 2 * (threadIdx.x & ~63u);
  __builtin_amdgcn_global_load_lds((const void *)src, (lds_void_t *)dst, 16, 0, 0);
}

// Accessor of the z-marching kernel (all offsets are compile-time after
// unrolling: each picks one LDS plane or register).
struct MarchAcc {
  LM_UNIFORM_SPACING
  static constexpr bool kPhased = true;
  const MarchShared &sm;
  int me;                  // this cell in an LDS plane
  int vm, v0, vp;          // ring slots of planes z-1, z, z+1
  int sc;                  // slot of the scalar planes
  double kz[2], sz[2][2];  // own column: kappa and H, Z at z-1, z+1
  double F2m, F2c;         // z face fluxes below and at the cell
  double rho_c;
  __device__ double v(int i, int o0, int o1, int o2) const {
    const int slot = o2 < 0 ? vm : (o2 > 0 ? vp : v0);
    return sm.v[i][slot][me + o0 + o1 * kMW];
  }
  __device__ double kap(int o0, int o1, int o2) const {
    if (o2 != 0) return kz[o2 > 0];
    return sm.s[0][sc][me + o0 + o1 * kMW];
  }
  __device__ double s(int f, int o0, int o1, int o2) const {
    if (o2 != 0) return sz[f][o2 > 0];
    return sm.s[1 + f][sc][me + o0 + o1 * kMW];
  }
  __device__ double F(int d, int o) const {
    if (d == 0) return sm.s[3][sc][me + o];
    if (d == 1) return sm.s[4][sc][me + o * kMW];
    return o < 0 ? F2m : F2c;
  }
  __device__ double rho() const { return rho_c; }
  __device__ double chi() const { return 0.0; }
  __device__ double v_ib(int) const { return 0.0; }
  __device__ double Z_ib() const { return 0.0; }
  __device__ double H_ib() const { return 0.0; }
};

// Empty asm statements that claim to change their operands: applied at the
// top of each plane of a march, they keep the compiler from hoisting the
// work derived from the step constants and the column address out of the
// plane loop, where it would pin most of the register file for the whole
// march (recomputing it costs a few instructions per plane).
__device__ inline void refresh(Phys &P, long &cc, int &me) {
  asm volatile("" : "+s"(P.ih[0]), "+s"(P.ih[1]), "+s"(P.ih[2]), "+s"(P.Pe), "+s"(P.Pr), "+s"(P.Da), "+s"(P.dt),
               "+s"(P.p0));
  asm volatile("" : "+s"(P.sigma), "+s"(P.inv_Fr2), "+s"(P.qs), "+s"(P.S), "+s"(P.k), "+s"(P.Le_F), "+s"(P.Le_O),
               "+s"(P.N_F));
  asm volatile("" : "+s"(P.N_O), "+s"(P.fshift), "+s"(P.zeta), "+s"(P.suth_C), "+s"(P.ab0), "+s"(P.ab1));
  asm volatile("" : "+v"(cc), "+v"(me));
}

template <int CORR>
__global__ void __launch_bounds__(kBlock) k_stage_march(Lay L, Phys P, StageArgs a, int first, int ntx, int nty,
                                                        int tz) {
  __shared__ MarchShared sm;
  const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = (int)(b % ntx), rest = (int)(b / ntx);
  const int by = rest % nty, ch = rest / nty;
  const int x0 = bx * kMX, y0 = by * kMY;
  const int z0 = ch * tz, z1 = min(z0 + tz, L.n[2]);
  if (z0 >= z1) return;
  const int tid = threadIdx.x;
  const int lx = tid & (kMX - 1), ly = tid / kMX;
  const long s2 = L.s[2];
  // this thread's pair of the halo tile (offset from its plane)
  const bool hp = tid < kMPairs;
  const int pr = tid / (kMW / 2), pc = tid - pr * (kMW / 2);
  const long gp = L.at(x0 - 2 + 2 * pc, y0 - 1 + pr, 0);
  const int me = (ly + 1) * kMW + lx + 2;
  const long cc = L.at(x0 + lx, y0 + ly, 0);  // own column at plane 0
  const double *vs[3] = {a.cur.v[0], a.cur.v[1], a.cur.v[2]};
  const double *ss[5] = {a.cur.kap, a.cur.H, a.cur.Z, a.cur.F[0], a.cur.F[1]};
  const double dtp0 = P.closed ? *a.dtp0 : 0.0;

  // prologue: velocity planes z0-1, z0, z0+1; scalar plane z0; own column
  if (hp) {
    for (int z = z0 - 1; z <= z0 + 1; ++z)
#pragma unroll
      for (int i = 0; i < 3; ++i) pair_to_lds(vs[i] + gp + z * s2, sm.v[i][z & 3]);
#pragma unroll
    for (int f = 0; f < 5; ++f)
      if (f != 2 || P.reacting) pair_to_lds(ss[f] + gp + z0 * s2, sm.s[f][z0 & 1]);
  }
  double kz[3], Hz[3], Zz[3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const long c = cc + (z0 + dz) * s2;
    kz[dz + 1] = a.cur.kap[c];
    Hz[dz + 1] = a.cur.H[c];
    Zz[dz + 1] = P.reacting ? a.cur.Z[c] : 0.0;
  }
  double F2m = a.cur.F[2][cc + (z0 - 1) * s2], F2c = a.cur.F[2][cc + z0 * s2];
  double rho_c = a.cur.rho[cc + z0 * s2];
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int z = z0; z < z1; ++z) {
    Phys Pz = P;
    long ccz = cc;
    int mez = me;
    refresh(Pz, ccz, mez);
    const bool more = z + 1 < z1;
    // next planes: velocity tiles of z+2 and scalar tiles of z+1 into
    // their free LDS slots; the own column's kappa, H, Z of z+2, z face
    // flux and density of z+1
    double kN = 0.0, HN = 0.0, ZN = 0.0, F2N = 0.0, rhoN = 0.0;
    if (more) {
      if (hp) {
#pragma unroll
        for (int i = 0; i < 3; ++i) pair_to_lds(vs[i] + gp + (z + 2) * s2, sm.v[i][(z + 2) & 3]);
#pragma unroll
        for (int f = 0; f < 5; ++f)
          if (f != 2 || P.reacting) pair_to_lds(ss[f] + gp + (z + 1) * s2, sm.s[f][(z + 1) & 1]);
      }
      const long cn = ccz + (z + 2) * s2, c1 = ccz + (z + 1) * s2;
      kN = a.cur.kap[cn];
      HN = a.cur.H[cn];
      ZN = P.reacting ? a.cur.Z[cn] : 0.0;
      F2N = a.cur.F[2][c1];
      rhoN = a.cur.rho[c1];
    }
    const long c = ccz + z * s2;
    Centre q;
    load_centre<3, CORR>(Pz, a, c, first, q);
    {
      MarchAcc acc{sm, mez, (z - 1) & 3, z & 3, (z + 1) & 3, z & 1, {kz[0], kz[2]}, {{Hz[0], Hz[2]}, {Zz[0], Zz[2]}},
                   F2m, F2c, rho_c};
      double RH, RZ, Rv[3];
      residuals<3>(acc, Pz, dtp0, RH, RZ, Rv);
      stage_update<3, CORR>(Pz, a, c, first, q, RH, RZ, Rv);
    }
    kz[0] = kz[1];
    kz[1] = kz[2];
    kz[2] = kN;
    Hz[0] = Hz[1];
    Hz[1] = Hz[2];
    Hz[2] = HN;
    Zz[0] = Zz[1];
    Zz[1] = Zz[2];
    Zz[2] = ZN;
    F2m = F2c;
    F2c = F2N;
    rho_c = rhoN;
    // the global-to-LDS copies of this step have landed before any
    // wavefront reads them after the barrier
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// The z-marching form covers 3D grids without an immersed body whose
// planes tile by 64 x 4 (any sides: the ghosts are filled beforehand).
// ---- LDS-staged 2D stage ----------------------------------------------------
// One block per 64 x 4 tile: the seven stencil fields' tiles with their
// one-cell halo go from HBM (or the last-level cache) straight into LDS,
// the centre-only fields are loaded meanwhile, one barrier, then the same
// residual arithmetic reads the neighbours from LDS.
struct Tile2DShared {
  double t[7][kMP];  // v_0, v_1, kappa, H, Z, F_0, F_1
};

struct Tile2DAcc {
  LM_UNIFORM_SPACING
  static constexpr bool kPhased = false;
  const Tile2DShared &sm;
  int me;
  const Level &lv;
  const IB &ib;
  long c;
  int has_ib;
  __device__ double v(int i, int o0, int o1, int) const { return sm.t[i][me + o0 + o1 * kMW]; }
  __device__ double kap(int o0, int o1, int) const { return sm.t[2][me + o0 + o1 * kMW]; }
  __device__ double s(int f, int o0, int o1, int) const { return sm.t[3 + f][me + o0 + o1 * kMW]; }
  __device__ double F(int d, int o) const { return d == 0 ? sm.t[5][me + o] : sm.t[6][me + o * kMW]; }
  __device__ double rho() const { return lv.rho[c]; }
  __device__ double chi() const { return (has_ib && ib.chi) ? (double)ib.chi[c] : 0.0; }
  __device__ double v_ib(int i) const { return ib.v_ib[i] ? ib.v_ib[i][c] : 0.0; }
  __device__ double Z_ib() const { return ib.Z_ib ? ib.Z_ib[c] : 0.0; }
  __device__ double H_ib() const { return ib.H_ib ? ib.H_ib[c] : 0.0; }
};

template <int CORR>
__global__ void __launch_bounds__(kBlock) k_stage_tile2d(Lay L, Phys P, StageArgs a, int first, int ntx) {
  __shared__ Tile2DShared sm;
  const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % ntx) * kMX, y0 = (int)(b / ntx) * kMY;
  const int tid = threadIdx.x;
  if (tid < kMPairs) {
    const int pr = tid / (kMW / 2), pc = tid - pr * (kMW / 2);
    const long gp = L.at(x0 - 2 + 2 * pc, y0 - 1 + pr, 0);
    const double *src[7] = {a.cur.v[0], a.cur.v[1], a.cur.kap, a.cur.H, a.cur.Z, a.cur.F[0], a.cur.F[1]};
#pragma unroll
    for (int f = 0; f < 7; ++f)
      if (f != 4 || P.reacting) pair_to_lds(src[f] + gp, sm.t[f]);
  }
  const int lx = tid & (kMX - 1), ly = tid / kMX;
  const long c = L.at(x0 + lx, y0 + ly, 0);
  Centre q;
  load_centre<2, CORR>(P, a, c, first, q);
  const double dtp0 = P.closed ? *a.dtp0 : 0.0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const Tile2DAcc acc{sm, (ly + 1) * kMW + lx + 2, a.cur, a.ib, c, P.has_ib};
  double RH, RZ, Rv[3];
  residuals<2>(acc, P, dtp0, RH, RZ, Rv);
  stage_update<2, CORR>(P, a, c, first, q, RH, RZ, Rv);
}

// The LDS-staged forms need planes that tile by 64 x 4 (any sides: the
// ghosts are filled beforehand; 3D: no immersed body) and, for the 16-byte
// tile copies, stencil fields on 16-byte boundaries (workspace arrays
// start on 256-byte ones).
static bool lds_stage_ok(const Lay &L, const Phys &P, const Level &cur) {
  if (P.met || L.n[0] % kMX != 0 || L.n[1] % kMY != 0 || (L.base & 1)) return false;
  if (L.ndim == 3 && (P.has_ib || L.n[2] < 8)) return false;
  const double *f[7] = {cur.v[0], cur.v[1], L.ndim == 3 ? cur.v[2] : cur.v[0], cur.kap, cur.H, cur.F[0], cur.F[1]};
  for (const double *p : f)
    if ((uintptr_t)p & 15) return false;
  return !P.reacting || ((uintptr_t)cur.Z & 15) == 0;
}

hipError_t launch_stage(hipStream_t st, int corrector, int first, const Lay &L, const Phys &P,
                        const Level &cur, const Level &n0, const Resid &rprev, const Resid &rn,
                        const IB &ib, Level &out, double *M[3], const double *dtp0) {
  StageArgs a;
  a.dtp0 = dtp0;
  a.cur = cur;
  a.n0 = n0;
  a.out = out;
  a.rprev = rprev;
  a.rn = rn;
  a.ib = ib;
  for (int i = 0; i < 3; ++i) a.M[i] = M[i];
  if (P.stage_form != 2 && L.ndim == 2 && lds_stage_ok(L, P, cur)) {
    const int ntx = L.n[0] / kMX;
    const dim3 g(ntx * (L.n[1] / kMY));
    if (corrector)
      hipLaunchKernelGGL((k_stage_tile2d<1>), g, dim3(kBlock), 0, st, L, P, a, first, ntx);
    else
      hipLaunchKernelGGL((k_stage_tile2d<0>), g, dim3(kBlock), 0, st, L, P, a, first, ntx);
    return hipGetLastError();
  }
  if (P.stage_form == 1 && L.ndim == 3 && lds_stage_ok(L, P, cur)) {
    const int ntx = L.n[0] / kMX, nty = L.n[1] / kMY;
    const int tiles = ntx * nty;
    int nch = std::max(1, (kMarchBlocks + tiles - 1) / tiles);
    int tz = std::max(8, (L.n[2] + nch - 1) / nch);
    nch = (L.n[2] + tz - 1) / tz;
    const dim3 g(tiles * nch);
    if (corrector)
      hipLaunchKernelGGL((k_stage_march<1>), g, dim3(kBlock), 0, st, L, P, a, first, ntx, nty, tz);
    else
      hipLaunchKernelGGL((k_stage_march<0>), g, dim3(kBlock), 0, st, L, P, a, first, ntx, nty, tz);
    return hipGetLastError();
  }
  dim3 g = grid_for(L), b(kBX, kBY);
  if (P.met) {  // stretched 2D grid
    if (corrector)
      hipLaunchKernelGGL((k_stage<2, 1, true>), g, b, 0, st, L, P, a, first);
    else
      hipLaunchKernelGGL((k_stage<2, 0, true>), g, b, 0, st, L, P, a, first);
    return hipGetLastError();
  }
  if (L.ndim == 3) {
    if (corrector)
      hipLaunchKernelGGL((k_stage<3, 1>), g, b, 0, st, L, P, a, first);
    else
      hipLaunchKernelGGL((k_stage<3, 0>), g, b, 0, st, L, P, a, first);
  } else {
    if (corrector)
      hipLaunchKernelGGL((k_stage<2, 1>), g, b, 0, st, L, P, a, first);
    else
      hipLaunchKernelGGL((k_stage<2, 0>), g, b, 0, st, L, P, a, first);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Poisson right-hand side and projection
// ---------------------------------------------------------------------------

// Eq 3.20 (n = 1) from the centres of two neighbouring cells (lower,
// upper) along d to their face f (see met_view): the two-point mean on a
// uniform grid (met NULL).
__device__ inline double face_interp(const double *met, const Lay &L, int d, int f, double lo, double hi) {
  if (!met) return 0.5 * (lo + hi);
  const MetView m = met_view(met, L, d);
  return m.wlo[f] * lo + m.whi[f] * hi;
}

// Prescribed normal mass flux on the boundary face of side (d, s) next to
// cell p; outflow sides extrapolate the cell momentum quadratically to the
// face (cells at 1/2, 3/2, 5/2 spacings: weights 15/8, -10/8, 3/8).
__device__ inline double boundary_flux(const Lay &L, const Bnd &B, const Sides &sd, const double *Md,
                                       const CellPos &p, int d, int s) {
  const int kind = B.kind[d][s];
  if (kind == LM_SIDE_SLIP || kind == LM_SIDE_NOSLIP) return 0.0;
  if (kind == LM_SIDE_INFLOW) {
    const double *F = sd.s[d][s].F;
    return F ? F[side_index(L, d, p.i, p.j, p.k)] : 0.0;
  }
  const long sdd = L.s[d];
  const int q = coord(p, d);
  long c1 = p.c + (long)((s == 0 ? 0 : L.n[d] - 1) - q) * sdd;
  long c2 = c1 + (s == 0 ? sdd : -sdd);
  long c3 = c2 + (s == 0 ? sdd : -sdd);
  return (15.0 * Md[c1] - 10.0 * Md[c2] + 3.0 * Md[c3]) / 8.0;
}

struct RhsArgs {
  const double *M[3];
  const double *rho_new, *rho_n, *rho_prev, *S_m;
  double *b, *partials;
  SolverScalars *sc;
  int bdf2;
  int has_outflow;
  double outflow_area, dV;
};

// b = sum_d delta_1 G_d + d_t rho - S_m, G_d the face average of the
// predicted momentum on interior faces and the prescribed flux on boundary
// faces (Eq 3.9-3.11, 3.17-3.19, 3.24, 3.33). The last block forms mean(b)
// (periodic / closed) or the uniform outflow shift that makes sum(b) = 0.
template <int DIM, bool MET = false>
__global__ void __launch_bounds__(kBlock) k_rhs(Lay L, Bnd B, Phys P, Sides sd, RhsArgs a) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double part = 0.0;
  if (cell_of_thread(L, p)) {
    const long c = p.c;
    double div = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double *Md = a.M[d];
      const int q = coord(p, d);
      const long nh = nbr(L, B, c, q, d, +1), nl = nbr(L, B, c, q, d, -1);
      const double Gh = nh >= 0 ? face_interp(MET ? P.met : nullptr, L, d, q + 1, Md[c], Md[nh]) : boundary_flux(L, B, sd, Md, p, d, 1);
      const double Gl = nl >= 0 ? face_interp(MET ? P.met : nullptr, L, d, q, Md[nl], Md[c]) : boundary_flux(L, B, sd, Md, p, d, 0);
      div = div + (Gh - Gl) * (MET ? met_view(P.met, L, d).iwid[q + 1] : P.ih[d]);
    }
    double drho;
    if (a.bdf2)
      drho = P.var_step ? (P.bd0 * (a.rho_new[c] - a.rho_n[c]) - P.bd2 * (a.rho_n[c] - a.rho_prev[c])) / P.dt
                        : (3.0 * a.rho_new[c] - 4.0 * a.rho_n[c] + a.rho_prev[c]) / (2.0 * P.dt);
    else
      drho = (a.rho_new[c] - a.rho_n[c]) / P.dt;
    const double src = a.S_m ? drho - a.S_m[c] : drho;
    const double b = div + src;
    a.b[c] = b;
    part = MET ? b * P.vol[c] : b;   // stretched: the integral of b
  }
  const double s = block_sum(part, sh);
  if (linear_tid() == 0) a.partials[linear_block()] = s;
}

// One block: total of the right-hand side; mean(b) for periodic / closed
// domains, or the uniform outflow shift that makes sum(b) = 0.
__global__ void __launch_bounds__(kBlock) k_rhs_finish(const double *partials, int np, double ncells,
                                                       int has_outflow, double dV, double area, SolverScalars *sc) {
  __shared__ double sh[kBlock / 64];
  const double tot = sum_partials(partials, (unsigned)np, sh);
  if (threadIdx.x == 0) {
    sc->sum_b = tot;
    if (has_outflow) {
      sc->outflow_c = tot * dV / area;
      sc->mean_b = 0.0;
    } else {
      sc->outflow_c = 0.0;
      sc->mean_b = tot / ncells;
    }
  }
}

hipError_t launch_rhs(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                      double *const M[3], const double *rho_new, const double *rho_n,
                      const double *rho_prev, int bdf2, const double *S_m, double *b,
                      double *partials, SolverScalars *sc) {
  RhsArgs a;
  for (int i = 0; i < 3; ++i) a.M[i] = M[i];
  a.rho_new = rho_new;
  a.rho_n = rho_n;
  a.rho_prev = rho_prev;
  a.S_m = S_m;
  a.b = b;
  a.partials = partials;
  a.sc = sc;
  a.bdf2 = bdf2;
  a.has_outflow = 0;
  a.outflow_area = 0.0;
  a.dV = 1.0;
  for (int d = 0; d < L.ndim; ++d) a.dV *= P.h[d];
  for (int d = 0; d < L.ndim; ++d)
    for (int s = 0; s < 2; ++s)
      if (B.kind[d][s] == LM_SIDE_OUTFLOW) {
        a.has_outflow = 1;
        a.outflow_area += a.dV / P.h[d] * (double)L.ncells() / L.n[d];
      }
  dim3 g = grid_for(L), bl(kBX, kBY);
  if (L.ndim == 3)
    hipLaunchKernelGGL(k_rhs<3>, g, bl, 0, st, L, B, P, sd, a);
  else if (P.met)
    hipLaunchKernelGGL((k_rhs<2, true>), g, bl, 0, st, L, B, P, sd, a);
  else
    hipLaunchKernelGGL(k_rhs<2>, g, bl, 0, st, L, B, P, sd, a);
  hipLaunchKernelGGL(k_rhs_finish, dim3(1), dim3(kBlock), 0, st, (const double *)partials, (int)nblocks_for(L),
                     P.met ? P.volume : (double)L.ncells(), a.has_outflow, a.dV, a.outflow_area, sc);
  return hipGetLastError();
}

struct ProjArgs {
  const double *M[3];
  const double *x, *rho_new;
  const SolverScalars *sc;
  double *F[3], *v[3], *P_out;
  int *nonfinite;
};

// F_d = G_d - delta_1 P on interior faces and the prescribed flux on
// boundary faces (Eq 3.23; outflow faces carry the uniform shift);
// v = (M - delta_2 P)/rho_new (Eq 3.25) with P ghosts by quadratic
// extrapolation at non-periodic sides (Eq 3.27-3.28); P stored zero-mean.
template <int DIM, bool MET = false>
__global__ void __launch_bounds__(kBlock) k_project(Lay L, Bnd B, Phys P, Sides sd, ProjArgs a) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double *x = a.x;
  const double oc = a.sc->outflow_c;
  const double xc = x ? x[c] : 0.0;
  bool bad = false;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double *Md = a.M[d];
    const int q = coord(p, d);
    const long sdd = L.s[d];
    const long nh = nbr(L, B, c, q, d, +1), nl = nbr(L, B, c, q, d, -1);
    double xp, xm;
    if (nh >= 0) {
      xp = x ? x[nh] : 0.0;
      const double G = face_interp(MET ? P.met : nullptr, L, d, q + 1, Md[c], Md[nh]);
      a.F[d][c] = G - (xp - xc) * (MET ? met_view(P.met, L, d).idfc[q + 1] : P.ih[d]);
    } else {
      double G = boundary_flux(L, B, sd, Md, p, d, 1);
      if (B.kind[d][1] == LM_SIDE_OUTFLOW) G -= oc;
      a.F[d][c] = G;
      if (!MET)
        xp = x ? 3.0 * xc - 3.0 * x[c - sdd] + x[c - 2 * sdd] : 0.0;
      else  // Eq 3.28 with the stretched positions
        xp = x ? P.gx[d][1][0] * xc + P.gx[d][1][1] * x[c - sdd] + P.gx[d][1][2] * x[c - 2 * sdd] : 0.0;
    }
    if (nl >= 0) {
      xm = x ? x[nl] : 0.0;
      if (q == 0) {  // periodic: duplicate of the wrapped face, same arithmetic
        const double G = face_interp(MET ? P.met : nullptr, L, d, 0, Md[nl], Md[c]);
        a.F[d][c - sdd] = G - (xc - xm) * (MET ? met_view(P.met, L, d).idfc[0] : P.ih[d]);
      }
    } else {
      double G = boundary_flux(L, B, sd, Md, p, d, 0);
      if (B.kind[d][0] == LM_SIDE_OUTFLOW) G += oc;
      a.F[d][c - sdd] = G;
      if (!MET)
        xm = x ? 3.0 * xc - 3.0 * x[c + sdd] + x[c + 2 * sdd] : 0.0;
      else
        xm = x ? P.gx[d][0][0] * xc + P.gx[d][0][1] * x[c + sdd] + P.gx[d][0][2] * x[c + 2 * sdd] : 0.0;
    }
    const double v = MET ? (Md[c] - (xp - xm) * met_view(P.met, L, d).id2[q]) / a.rho_new[c]
                           : (Md[c] - (xp - xm) / (2.0 * P.h[d])) / a.rho_new[c];
    a.v[d][c] = v;
    bad |= !isfinite(v);
  }
  if (a.P_out) a.P_out[c] = (x == nullptr || a.sc->zero) ? 0.0 : xc - a.sc->mean_x;
  if (bad) atomicOr(a.nonfinite, 1);
}

hipError_t launch_project(hipStream_t st, const Lay &L, const Bnd &B, const Phys &P, const Sides &sd,
                          double *const M[3], const double *x, const double *rho_new,
                          const SolverScalars *sc, double *F[3], double *v[3], double *P_out,
                          int *nonfinite) {
  ProjArgs a;
  for (int i = 0; i < 3; ++i) {
    a.M[i] = M[i];
    a.F[i] = F[i];
    a.v[i] = v[i];
  }
  a.x = x;
  a.rho_new = rho_new;
  a.sc = sc;
  a.P_out = P_out;
  a.nonfinite = nonfinite;
  dim3 g = grid_for(L), bl(kBX, kBY);
  if (L.ndim == 3)
    hipLaunchKernelGGL(k_project<3>, g, bl, 0, st, L, B, P, sd, a);
  else if (P.met)
    hipLaunchKernelGGL((k_project<2, true>), g, bl, 0, st, L, B, P, sd, a);
  else
    hipLaunchKernelGGL(k_project<2>, g, bl, 0, st, L, B, P, sd, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------

// H from T by inverting Eq 3.42 (or T from H), then T re-evaluated from
// (Z, H), rho = p0/T (Eq 2.49), kappa = T^sigma (Eq 2.50).
__global__ void __launch_bounds__(kBlock) k_init_state(Lay L, Phys P, Level lv, int from_T, int *bad) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double Z = P.reacting ? lv.Z[c] : 0.0;
  double H;
  if (from_T) {
    const double T0 = lv.T[c];
    H = P.reacting ? T0 / P.qs - f_tilde(P, Z) : T0 / P.qs + 1.0;
    lv.H[c] = H;
  } else {
    H = lv.H[c];
  }
  const double T = temperature(P, Z, H);
  if (!(T > 0.0)) atomicOr(bad, 1);
  lv.T[c] = T;
  lv.rho[c] = P.p0 / T;
  lv.kap[c] = kappa_of(P, T);
}

hipError_t launch_init_state(hipStream_t st, const Lay &L, const Phys &P, const Bnd &B,
                             const Sides &sd, int from_T, Level &lv, int *bad_flag) {
  (void)B;
  (void)sd;
  dim3 g = grid_for(L), bl(kBX, kBY);
  hipLaunchKernelGGL(k_init_state, g, bl, 0, st, L, P, lv, from_T, bad_flag);
  return hipGetLastError();
}

// M = rho v at cells (scratch for the initial face flux).
__global__ void __launch_bounds__(kBlock) k_momentum(Lay L, Level lv, double *M0, double *M1, double *M2) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double r = lv.rho[c];
  M0[c] = r * lv.v[0][c];
  M1[c] = r * lv.v[1][c];
  if (L.ndim == 3) M2[c] = r * lv.v[2][c];
}

// Initial face flux: face average of rho v (Eq 3.20, n = 1), prescribed
// flux on boundary faces, extrapolated flux on outflow faces.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_face_flux(Lay L, Bnd B, Sides sd, ProjArgs a, const double *met) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double *Md = a.M[d];
    const int q = coord(p, d);
    const long nh = nbr(L, B, c, q, d, +1), nl = nbr(L, B, c, q, d, -1);
    a.F[d][c] = nh >= 0 ? face_interp(met, L, d, q + 1, Md[c], Md[nh]) : boundary_flux(L, B, sd, Md, p, d, 1);
    if (q == 0)
      a.F[d][c - L.s[d]] = nl >= 0 ? face_interp(met, L, d, 0, Md[nl], Md[c]) : boundary_flux(L, B, sd, Md, p, d, 0);
  }
}

hipError_t launch_face_flux(hipStream_t st, const Lay &L, const Bnd &B, const Sides &sd,
                            const Level &lv, double *M[3], const double *met) {
  dim3 g = grid_for(L), bl(kBX, kBY);
  hipLaunchKernelGGL(k_momentum, g, bl, 0, st, L, lv, M[0], M[1], M[2]);
  ProjArgs a{};
  for (int i = 0; i < 3; ++i) {
    a.M[i] = M[i];
    a.F[i] = lv.F[i];
  }
  if (L.ndim == 3)
    hipLaunchKernelGGL(k_face_flux<3>, g, bl, 0, st, L, B, sd, a, met);
  else
    hipLaunchKernelGGL(k_face_flux<2>, g, bl, 0, st, L, B, sd, a, met);
  return hipGetLastError();
}

// dt = CFL / max over cells of sum_d |v_d|/h_d + 2 nu sum_d 1/h_d^2 + chi nu/Da,
// nu = max(Pr, 1, 1/Le_F, 1/Le_O) kappa/(Pe rho).
__global__ void __launch_bounds__(kBlock) k_cfl(Lay L, Phys P, Level lv, const unsigned char *chi,
                                                double *partials) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double rate = 0.0;
  if (cell_of_thread(L, p)) {
    const long c = p.c;
    const double nu = P.nu_coef * lv.kap[c] / (P.Pe * lv.rho[c]);
    double a = 0.0, q = 0.0;
    for (int d = 0; d < L.ndim; ++d) {
      if (P.met) {  // stretched: the cell's own width
        const double iw = met_view(P.met, L, d).iwid[coord(p, d) + 1];
        a = a + fabs(lv.v[d][c]) * iw;
        q = q + iw * iw;
      } else {
        a = a + fabs(lv.v[d][c]) / P.h[d];
        q = q + 1.0 / (P.h[d] * P.h[d]);
      }
    }
    rate = a + 2.0 * nu * q;
    if (chi) rate = rate + (double)chi[c] * nu / P.Da;
  }
  const double m = block_max(rate, sh);
  if (linear_tid() == 0) partials[linear_block()] = m;
}

__global__ void __launch_bounds__(kBlock) k_cfl_finish(const double *partials, int np, double *out) {
  __shared__ double sh[kBlock / 64];
  double v = -1.0;
  for (int q = threadIdx.x; q < np; q += kBlock) v = fmax(v, partials[q]);
  v = block_max(v, sh);
  if (threadIdx.x == 0) *out = v;
}

hipError_t launch_cfl(hipStream_t st, const Lay &L, const Phys &P, const Level &lv,
                      const unsigned char *chi, double *partials, double *out_max) {
  dim3 g = grid_for(L), bl(kBX, kBY);
  hipLaunchKernelGGL(k_cfl, g, bl, 0, st, L, P, lv, chi, partials);
  hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(kBlock), 0, st, (const double *)partials, (int)nblocks_for(L),
                     out_max);
  return hipGetLastError();
}

// Predictor-corrector differences of a step (the local-error estimate of an
// adaptive step): per block sums of |v* - v^{n+1}|^2, (H* - H^{n+1})^2 and
// (Z* - Z^{n+1})^2 over the cells of a grid-stride loop (fixed grid, so
// the summation order does not depend on the launch).
__global__ void __launch_bounds__(kBlock) k_pc_err(Lay L, int reacting, Level s, Level q, double *partials) {
  __shared__ double sh[kBlock / 64];
  const long N = L.ncells();
  const int nx = L.n[0], ny = L.n[1];
  double ev = 0.0, eh = 0.0, ez = 0.0;
  for (long t = (long)blockIdx.x * kBlock + threadIdx.x; t < N; t += (long)kErrBlocks * kBlock) {
    const int i = (int)(t % nx);
    const int j = (int)((t / nx) % ny);
    const int k = (int)(t / ((long)nx * ny));
    const long c = L.at(i, j, k);
    for (int d = 0; d < L.ndim; ++d) {
      const double dv = s.v[d][c] - q.v[d][c];
      ev = ev + dv * dv;
    }
    const double dh = s.H[c] - q.H[c];
    eh = eh + dh * dh;
    if (reacting) {
      const double dz = s.Z[c] - q.Z[c];
      ez = ez + dz * dz;
    }
  }
  ev = block_sum(ev, sh);
  eh = block_sum(eh, sh);
  ez = block_sum(ez, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = ev;
    partials[kErrBlocks + blockIdx.x] = eh;
    partials[2 * kErrBlocks + blockIdx.x] = ez;
  }
}

__global__ void __launch_bounds__(kBlock) k_pc_err_finish(const double *partials, double *out) {
  __shared__ double sh[kBlock / 64];
  for (int q = 0; q < 3; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < kErrBlocks; b += kBlock) v = v + partials[q * kErrBlocks + b];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[q] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_scale_copy(long n, double a, const double *x, double *y) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] = a * x[t];
}

hipError_t launch_scale_copy(hipStream_t st, long n, double a, const double *x, double *y) {
  hipLaunchKernelGGL(k_scale_copy, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, st, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_pc_err(hipStream_t st, const Lay &L, int reacting, const Level &star, const Level &nw,
                         double *partials, double *out) {
  hipLaunchKernelGGL(k_pc_err, dim3(kErrBlocks), dim3(kBlock), 0, st, L, reacting, star, nw, partials);
  hipLaunchKernelGGL(k_pc_err_finish, dim3(1), dim3(kBlock), 0, st, (const double *)partials, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversion between compact caller arrays and padded device arrays
// ---------------------------------------------------------------------------

// face_dir < 0: cell field (nz, ny, nx). face_dir = d: face array with
// n_d + 1 entries along d, entry f stored at padded cell f - 1 (its high face).
__global__ void __launch_bounds__(kBlock) k_pack(Lay L, const double *src, double *dst, int fd, int unpack) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long m[3] = {L.n[0], L.n[1], L.n[2]};
  if (fd >= 0) m[fd] += 1;
  const long tot = m[0] * m[1] * m[2];
  if (t >= tot) return;
  const int i = (int)(t % m[0]);
  const int j = (int)((t / m[0]) % m[1]);
  const int k = (int)(t / (m[0] * m[1]));
  const int o0 = fd == 0 ? -1 : 0, o1 = fd == 1 ? -1 : 0, o2 = fd == 2 ? -1 : 0;
  const long pidx = L.at(i + o0, j + o1, k + o2);
  if (unpack)
    dst[t] = src[pidx];
  else
    dst[pidx] = src[t];
}

hipError_t launch_pack(hipStream_t st, const Lay &L, const double *src, double *dst, int face_dir) {
  long m = L.ncells();
  if (face_dir >= 0) m = m / L.n[face_dir] * (L.n[face_dir] + 1);
  hipLaunchKernelGGL(k_pack, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, st, L, src, dst, face_dir, 0);
  return hipGetLastError();
}

hipError_t launch_unpack(hipStream_t st, const Lay &L, const double *src, double *dst, int face_dir) {
  long m = L.ncells();
  if (face_dir >= 0) m = m / L.n[face_dir] * (L.n[face_dir] + 1);
  hipLaunchKernelGGL(k_pack, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, st, L, src, dst, face_dir, 1);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) k_pack_u8(Lay L, const unsigned char *src, unsigned char *dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.ncells()) return;
  const int i = (int)(t % L.n[0]);
  const int j = (int)((t / L.n[0]) % L.n[1]);
  const int k = (int)(t / ((long)L.n[0] * L.n[1]));
  dst[L.at(i, j, k)] = src[t];
}

hipError_t launch_pack_u8(hipStream_t st, const Lay &L, const unsigned char *src, unsigned char *dst) {
  hipLaunchKernelGGL(k_pack_u8, dim3(ceil_div(L.ncells(), kBlock)), dim3(kBlock), 0, st, L, src, dst);
  return hipGetLastError();
}

}  // namespace lm

namespace lm {

// mean(a) over the interior into sc->mean_b (outflow shift cleared).
__global__ void __launch_bounds__(kBlock) k_mean(Lay L, const double *a, double *partials, SolverScalars *sc,
                                                 const double *vol) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double v = 0.0;
  if (cell_of_thread(L, p)) v = vol ? a[p.c] * vol[p.c] : a[p.c];
  const double s = block_sum(v, sh);
  if (linear_tid() == 0) partials[linear_block()] = s;
}

hipError_t launch_mean(hipStream_t st, const Lay &L, const double *a, double *partials, SolverScalars *sc,
                       const double *vol, double volume) {
  dim3 g = grid_for(L), bl(kBX, kBY);
  hipLaunchKernelGGL(k_mean, g, bl, 0, st, L, a, partials, sc, vol);
  hipLaunchKernelGGL(k_rhs_finish, dim3(1), dim3(kBlock), 0, st, (const double *)partials, (int)nblocks_for(L),
                     vol ? volume : (double)L.ncells(), 0, 1.0, 1.0, sc);
  return hipGetLastError();
}

// out = x - mean(x) (zero-mean pressure), or 0 when the right-hand side vanished.
__global__ void __launch_bounds__(kBlock) k_shift(Lay L, const double *x, const SolverScalars *sc, double *out) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  out[p.c] = sc->zero ? 0.0 : x[p.c] - sc->mean_x;
}

hipError_t launch_shift(hipStream_t st, const Lay &L, const double *x, const SolverScalars *sc, double *out) {
  dim3 g = grid_for(L), bl(kBX, kBY);
  hipLaunchKernelGGL(k_shift, g, bl, 0, st, L, x, sc, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Thermodynamic pressure of an enclosed system (Eq 2.40)
// ---------------------------------------------------------------------------

// Per-block partial sums over the cells: 0 rho, 1 1/T, 2 R_H/T^2, 3 1/(rho T^2).
template <int WHAT>
__global__ void __launch_bounds__(kBlock) k_p0_sum(Lay L, const double *T, const double *rho, const double *RH,
                                                   double *part, const double *vol) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double v = 0.0;
  if (cell_of_thread(L, p)) {
    const long c = p.c;
    if (WHAT == 0) v = rho[c];
    if (WHAT == 1) v = 1.0 / T[c];
    if (WHAT == 2) v = RH[c] / (T[c] * T[c]);
    if (WHAT == 3) v = 1.0 / (rho[c] * (T[c] * T[c]));
    if (vol) v = v * vol[c];  // stretched: cell volumes enter each sum (dV = 1 below)
  }
  const double s = block_sum(v, sh);
  if (linear_tid() == 0) part[linear_block()] = s;
}

// Derivative at the newest of three levels spaced dt_new (newest pair) and
// dt_old: BDF2 for unequal steps in level differences, w = dt_new / dt_old.
__device__ inline double bdf2_unequal(double p_new, double p_mid, double p_old, double dt_new, double dt_old) {
  const double w = dt_new / dt_old;
  return ((1.0 + 2.0 * w) / (1.0 + w) * (p_new - p_mid) - w * w / (1.0 + w) * (p_mid - p_old)) / dt_new;
}

// Per-block partial sums over the cells of the H residual's diffusion term
// sum_d delta_1(kappa_f delta_1 H) (ghost-filled level): times dV it is the
// integral of div(kappa grad H) of Eq 2.38, the boundary faces' fluxes. With
// reaction each cell adds N'(Z) sum_d delta_1(kappa_f delta_1 Z), N' of
// Eq 2.39 (-1/S on the fuel side, 1 on the oxidiser side) with the Heaviside
// regularised as in Eq 3.35: the heat the flame releases.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_p0_heat(Lay L, Phys P, Level lv, double *part) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double v = 0.0;
  if (cell_of_thread(L, p)) {
    double adv;
    scalar_terms<DIM>(L, P, lv, 0, p.c, adv, v);
    if (P.reacting) {
      double difZ;
      scalar_terms<DIM>(L, P, lv, 1, p.c, adv, difZ);
      v += ((-1.0 / P.S - 1.0) * theta_eps(P, lv.Z[p.c]) + 1.0) * difZ;
    }
  }
  const double s = block_sum(v, sh);
  if (linear_tid() == 0) part[linear_block()] = s;
}

// One block: the sum of the partials (fixed order) and the update of the
// device p0 state. what: 0 mass and set-up, 1 predicted level, 2 new level,
// 3 first half of the start-up balance (stores the sum), 4 second half;
// Eq 2.38: 5 / 7 d_t p0 at level n / the predicted level from the heat
// integral, 6 / 8 p0 of the predicted / new level (no sum).
__global__ void __launch_bounds__(kBlock) k_p0_finish(int what, const double *part, int np, P0Dev *q, double dV,
                                                      Phys P) {
  __shared__ double sh[kBlock / 64];
  const double p_init = P.p0, qs = P.qs, zeta = P.zeta, dt = P.dt;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  const double s = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  if (what == 0) {
    q->mass = s * dV;
    q->p0[0] = q->p0[1] = q->p0[2] = p_init;
    q->p0_star = q->p0_new = p_init;
    q->dtp0_n = q->dtp0_star = q->dtp0_start = q->rate_prev = 0.0;
    q->dt_hist[0] = q->dt_hist[1] = 0.0;
    q->nhist = 0;
  } else if (what == 5 || what == 7) {
    // Eq 2.38: (gamma/V) [qs/Pe int div(kappa grad H) - p0 int div v]
    const double p0 = what == 5 ? q->p0[0] : q->p0_star;
    const double r = P.gamma / P.volume * (qs / P.Pe * (s * dV) - p0 * P.vol_out);
    if (what == 5)
      q->dtp0_n = r;
    else
      q->dtp0_star = r;
  } else if (what == 6) {
    if (q->nhist == 0)
      q->p0_star = q->p0[0] + dt * q->dtp0_n;
    else if (P.var_step)
      q->p0_star = q->p0[0] + dt * (P.ab0 * q->dtp0_n + P.ab1 * q->rate_prev);
    else
      q->p0_star = q->p0[0] + dt * (1.5 * q->dtp0_n - 0.5 * q->rate_prev);
  } else if (what == 8) {
    q->p0_new = q->p0[0] + 0.5 * dt * (q->dtp0_star + q->dtp0_n);
  } else if (what == 1) {
    const double ps = q->mass / (s * dV);
    q->p0_star = ps;
    // d_t p0 at the predicted level: BDF2 over levels n, n-1 (Eq 3.14), BDF1 with level n only;
    // after a step of another size BDF2 for unequal steps (level differences)
    if (q->nhist >= 1 && P.var_step)
      q->dtp0_star = bdf2_unequal(ps, q->p0[0], q->p0[1], dt, q->dt_hist[0]);
    else
      q->dtp0_star = q->nhist >= 1 ? (3.0 * ps - 4.0 * q->p0[0] + q->p0[1]) / (2.0 * dt) : (ps - q->p0[0]) / dt;
  } else if (what == 2) {
    q->p0_new = q->mass / (s * dV);
  } else if (what == 3) {
    q->dtp0_start = s;  // sum of R_H / T^2, finished below
  } else {
    // d_t p0 = (p0^2/m) sum(dV qs R_H / T^2) with R_H = R_H|0 + zeta d_t p0 / rho: solved for d_t p0
    const double w = q->p0[0] * q->p0[0] / q->mass * dV * qs;
    const double A = w * q->dtp0_start, B = w * zeta * s;
    q->dtp0_start = A / (1.0 - B);
  }
}

// rho = p0 / T with p0 of the predicted (which = 0) or new (1) level.
__global__ void __launch_bounds__(kBlock) k_p0_eos(Lay L, const double *T, double *rho, const P0Dev *q, int which) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  rho[p.c] = (which ? q->p0_new : q->p0_star) / T[p.c];
}

// First step: the balance's d_t p0 at level n enters the stored level-n
// residual R_H and the Euler-predicted H*, whose T* and kappa* follow.
__global__ void __launch_bounds__(kBlock) k_p0_startup(Lay L, Phys P, const P0Dev *q, const double *rho_n,
                                                       double *RH, Level out) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double add = P.zeta * q->dtp0_start / rho_n[c];
  RH[c] += add;
  const double H = out.H[c] + P.dt * add;
  const double T = temperature(P, 0.0, H);
  out.H[c] = H;
  out.T[c] = T;
  out.kap[c] = kappa_of(P, T);
}

// Commit of a completed step: history shift and d_t p0 at the new level n
// for the next predictor (BDF2, Eq 3.5; BDF1 with one earlier level).
__global__ void k_p0_commit(P0Dev *q, double dt, int unequal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  q->rate_prev = q->dtp0_n;  // Eq 2.38 systems: the level-n rate for the next AB2
  q->p0[2] = q->p0[1];
  q->p0[1] = q->p0[0];
  q->p0[0] = q->p0_new;
  q->dt_hist[1] = q->dt_hist[0];
  q->dt_hist[0] = dt;
  q->nhist = q->nhist < 2 ? q->nhist + 1 : 2;
  if (q->nhist >= 2 && unequal)
    q->dtp0_n = bdf2_unequal(q->p0[0], q->p0[1], q->p0[2], q->dt_hist[0], q->dt_hist[1]);
  else
    q->dtp0_n = q->nhist >= 2 ? (3.0 * q->p0[0] - 4.0 * q->p0[1] + q->p0[2]) / (2.0 * dt) : (q->p0[0] - q->p0[1]) / dt;
}

hipError_t launch_p0(hipStream_t st, int what, const Lay &L, const Phys &P, P0Dev *p0, Level *lv, const Level *n0,
                     double *RH, double *partials) {
  const dim3 g = grid_for(L), bl(kBX, kBY);
  const int np = (int)nblocks_for(L);
  const double dV = P.met ? 1.0 : P.h[0] * P.h[1] * (L.ndim == 3 ? P.h[2] : 1.0);
  const double *vol = P.met ? P.vol : nullptr;
  auto finish = [&](int w) {
    hipLaunchKernelGGL(k_p0_finish, dim3(1), dim3(kBlock), 0, st, w, (const double *)partials, np, p0, dV, P);
  };
  switch (what) {
    case 0:
      hipLaunchKernelGGL(k_p0_sum<0>, g, bl, 0, st, L, (const double *)lv->T, (const double *)lv->rho,
                         (const double *)nullptr, partials, vol);
      finish(0);
      break;
    case 1:
    case 2:
      hipLaunchKernelGGL(k_p0_sum<1>, g, bl, 0, st, L, (const double *)lv->T, (const double *)nullptr,
                         (const double *)nullptr, partials, vol);
      finish(what);
      hipLaunchKernelGGL(k_p0_eos, g, bl, 0, st, L, (const double *)lv->T, lv->rho, (const P0Dev *)p0, what - 1);
      break;
    case 3:
      hipLaunchKernelGGL(k_p0_sum<2>, g, bl, 0, st, L, (const double *)n0->T, (const double *)nullptr,
                         (const double *)RH, partials, vol);
      finish(3);
      hipLaunchKernelGGL(k_p0_sum<3>, g, bl, 0, st, L, (const double *)n0->T, (const double *)n0->rho,
                         (const double *)nullptr, partials, vol);
      finish(4);
      hipLaunchKernelGGL(k_p0_startup, g, bl, 0, st, L, P, (const P0Dev *)p0, (const double *)n0->rho, RH, *lv);
      break;
    case 4:
      hipLaunchKernelGGL(k_p0_commit, dim3(1), dim3(64), 0, st, p0, P.dt, P.var_step);
      break;
    case 5:
    case 7:
      if (L.ndim == 3)
        hipLaunchKernelGGL(k_p0_heat<3>, g, bl, 0, st, L, P, *lv, partials);
      else
        hipLaunchKernelGGL(k_p0_heat<2>, g, bl, 0, st, L, P, *lv, partials);
      finish(what);
      break;
    case 6:
    case 8:
      hipLaunchKernelGGL(k_p0_finish, dim3(1), dim3(kBlock), 0, st, what, (const double *)partials, 0, p0, dV, P);
      hipLaunchKernelGGL(k_p0_eos, g, bl, 0, st, L, (const double *)lv->T, lv->rho, (const P0Dev *)p0,
                         what == 6 ? 0 : 1);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lm
