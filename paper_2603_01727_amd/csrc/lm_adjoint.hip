// Adjoint (reverse mode) of one predictor-corrector step for the 2D
// periodic, non-reacting configuration without immersed boundary. The step
// is recomputed forward from the stored state (not committed); the sweep
// back applies, in reverse order, the transposes of
//   projection   F = avg(M) - delta_1 P,  v = (M - delta_2 P)/rho   (Eq 3.23, 3.25)
//   Poisson      P = Pi A^+ Pi b  (A symmetric, Pi the mean projector)   (Eq 3.24)
//   right side   b = delta_2 . M + BDF(rho)                            (Eq 3.9-3.11)
//   EOS          rho = p0 / (Q/(S+1) (H - 1))                           (Eq 2.49, 3.42)
//   Adams steps  AB2 predictor / AM2 corrector                          (Eq 3.1-3.18)
//   residuals    R_H, R_v of Eq 3.4, 3.8, 3.26 with tau of Eq 2.46.
// The residual transpose is a gather: for every input cell m the residuals
// of the 3 x 3 cells whose stencils reach m are re-evaluated with dual
// numbers seeded at m (derivatives with respect to H, v1, v2, F1, F2 at m)
// and contracted with the residual cotangents. No atomics; deterministic.
#include "lm_device.h"

namespace lm {

// ---------------------------------------------------------------------------
// Dual numbers with N derivative components
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  __device__ Dual() {}
  __device__ explicit Dual(double x) : v(x) {
#pragma unroll
    for (int q = 0; q < N; ++q) d[q] = 0.0;
  }
};

template <int N>
__device__ inline Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = a.d[q] + b.d[q];
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = a.d[q] - b.d[q];
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = -a.d[q];
  return r;
}
template <int N>
__device__ inline Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
  return r;
}
template <int N>
__device__ inline Dual<N> operator*(double s, const Dual<N> &a) {
  Dual<N> r;
  r.v = s * a.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = s * a.d[q];
  return r;
}
template <int N>
__device__ inline Dual<N> operator*(const Dual<N> &a, double s) {
  return s * a;
}
template <int N>
__device__ inline Dual<N> operator/(const Dual<N> &a, double s) {
  Dual<N> r;
  r.v = a.v / s;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = a.d[q] / s;
  return r;
}
template <int N>
__device__ inline Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = (a.d[q] - r.v * b.d[q]) * ib;
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(const Dual<N> &a, double s) {
  Dual<N> r = a;
  r.v = a.v - s;
  return r;
}
template <int N>
__device__ inline Dual<N> operator-(double s, const Dual<N> &a) {
  Dual<N> r = -a;
  r.v = s - a.v;
  return r;
}
template <int N>
__device__ inline Dual<N> operator+(const Dual<N> &a, double s) {
  Dual<N> r = a;
  r.v = a.v + s;
  return r;
}
// x^p for x > 0
template <int N>
__device__ inline Dual<N> dpow(const Dual<N> &x, double p) {
  Dual<N> r;
  r.v = pow(x.v, p);
  const double dv = p * r.v / x.v;
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = dv * x.d[q];
  return r;
}

// ---------------------------------------------------------------------------
// Residuals of one cell, written over a loader of dual-valued fields
// ---------------------------------------------------------------------------
using D5 = Dual<5>;

// Periodic 2D loader of the level fields; values at cell (mi, mj) carry unit
// seeds: H -> 0, v1 -> 1, v2 -> 2, F1 -> 3, F2 -> 4.
struct Loader {
  Lay L;
  const double *H, *v[2], *F[2];
  int mi, mj;
  __device__ int wx(int i) const { return i < 0 ? i + L.n[0] : (i >= L.n[0] ? i - L.n[0] : i); }
  __device__ int wy(int j) const { return j < 0 ? j + L.n[1] : (j >= L.n[1] ? j - L.n[1] : j); }
  __device__ D5 load(const double *a, int i, int j, int seed) const {
    i = wx(i);
    j = wy(j);
    D5 r(a[L.at(i, j, 0)]);
    if (i == mi && j == mj) r.d[seed] = 1.0;
    return r;
  }
  __device__ D5 hh(int i, int j) const { return load(H, i, j, 0); }
  __device__ D5 vv(int c, int i, int j) const { return load(v[c], i, j, 1 + c); }
  __device__ D5 ff(int d, int i, int j) const { return load(F[d], i, j, 3 + d); }
};

__device__ inline D5 temp_of(const AdjPhys &P, const D5 &H) { return P.qs * (H - 1.0); }

// kappa(T) with its derivative: T^sigma (Eq 2.50), or Sutherland's law
// T^{3/2} (1 + C)/(T + C) (Eq 4.12), d kappa/dT = kappa (3/(2T) - 1/(T + C)).
__device__ inline D5 kappa_dual(const AdjPhys &P, const D5 &T) {
  if (P.suth_C > 0.0) {
    const double C = P.suth_C, t = T.v;
    D5 r;
    r.v = t * sqrt(t) * (1.0 + C) / (t + C);
    const double dv = r.v * (1.5 / t - 1.0 / (t + C));
#pragma unroll
    for (int q = 0; q < 5; ++q) r.d[q] = dv * T.d[q];
    return r;
  }
  return dpow(T, P.sigma);
}

__device__ inline D5 kap_at(const AdjPhys &P, const Loader &ld, int i, int j) {
  return kappa_dual(P, temp_of(P, ld.hh(i, j)));
}

// tau_id on the face between (i, j) and its +d neighbour (Eq 2.46 on d-faces).
__device__ inline D5 tau_face_d(const AdjPhys &P, const Loader &ld, int i, int j, int d, int comp) {
  const int di = d == 0 ? 1 : 0, dj = d == 1 ? 1 : 0;
  const D5 kf = 0.5 * (kap_at(P, ld, i, j) + kap_at(P, ld, i + di, j + dj));
  D5 D[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k == d) {
        D[k][c] = (ld.vv(c, i + di, j + dj) - ld.vv(c, i, j)) * (1.0 / P.h[d]);
      } else {
        const int ki = k == 0 ? 1 : 0, kj = k == 1 ? 1 : 0;
        const double h2 = 2.0 * P.h[k];
        const D5 a = (ld.vv(c, i + ki, j + kj) - ld.vv(c, i - ki, j - kj)) / h2;
        const D5 b = (ld.vv(c, i + di + ki, j + dj + kj) - ld.vv(c, i + di - ki, j + dj - kj)) / h2;
        D[k][c] = 0.5 * (a + b);
      }
    }
  }
  D5 t = D[d][comp] + D[comp][d];
  if (comp == d) t = t - (2.0 / 3.0) * (D[0][0] + D[1][1]);
  return kf * t;
}

// R_H, R_v1, R_v2 at cell (i, j): the arithmetic of the forward residual
// (Eq 3.4a, 3.8a with the flux forms of Eq 3.26), non-reacting, no body.
__device__ inline void resid_cell(const AdjPhys &P, const Loader &ld, int i, int j, D5 &RH, D5 Rv[2]) {
  const D5 Hc = ld.hh(i, j);
  const D5 Tc = temp_of(P, Hc);
  const D5 rho = D5(P.p0) / Tc;
  const D5 kc = kappa_dual(P, Tc);
  D5 adv(0.0), dif(0.0);
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int di = d == 0 ? 1 : 0, dj = d == 1 ? 1 : 0;
    const D5 Hp = ld.hh(i + di, j + dj), Hm = ld.hh(i - di, j - dj);
    const D5 gp = (Hp - Hc) / P.h[d];
    const D5 gm = (Hc - Hm) / P.h[d];
    const D5 kp = 0.5 * (kc + kap_at(P, ld, i + di, j + dj));
    const D5 km = 0.5 * (kap_at(P, ld, i - di, j - dj) + kc);
    adv = adv + 0.5 * (ld.ff(d, i, j) * gp + ld.ff(d, i - di, j - dj) * gm);
    dif = dif + (kp * gp - km * gm) / P.h[d];
  }
  RH = (-adv + dif / P.Pe) / rho;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    D5 conv(0.0), visc(0.0);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int di = d == 0 ? 1 : 0, dj = d == 1 ? 1 : 0;
      const D5 vc = ld.vv(c, i, j);
      const D5 flp = ld.ff(d, i, j) * (0.5 * (vc + ld.vv(c, i + di, j + dj)));
      const D5 flm = ld.ff(d, i - di, j - dj) * (0.5 * (ld.vv(c, i - di, j - dj) + vc));
      conv = conv + (flp - flm) / P.h[d];
      const D5 tp = tau_face_d(P, ld, i, j, d, c);
      const D5 tm = tau_face_d(P, ld, i - di, j - dj, d, c);
      visc = visc + (tp - tm) / P.h[d];
    }
    D5 r = -conv + (P.Pr / P.Pe) * visc;
    if (c == 1 && P.inv_Fr2 != 0.0) r = r + P.inv_Fr2 * (1.0 - rho);
    Rv[c] = r;
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
struct AdjResidArgs {
  Lay L;
  AdjPhys P;
  const double *H, *v[2], *F[2];        // level at which the residuals are taken
  const double *RbH, *Rbv[2];           // residual cotangents
  double *Hb, *vb[2], *Fb[2];           // accumulated adjoints
};

// (Hb, vb, Fb) += (dR/d(H, v, F))^T (RbH, Rbv) by gather over the 3 x 3
// cells whose residual stencils reach the cell.
__global__ void __launch_bounds__(kBlock) k_adj_resid(AdjResidArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  Loader ld;
  ld.L = a.L;
  ld.H = a.H;
  ld.v[0] = a.v[0];
  ld.v[1] = a.v[1];
  ld.F[0] = a.F[0];
  ld.F[1] = a.F[1];
  ld.mi = p.i;
  ld.mj = p.j;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      const int ci = ld.wx(p.i + di), cj = ld.wy(p.j + dj);
      D5 RH, Rv[2];
      resid_cell(a.P, ld, ci, cj, RH, Rv);
      const long c = a.L.at(ci, cj, 0);
      const double rh = a.RbH[c], r0 = a.Rbv[0][c], r1 = a.Rbv[1][c];
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] += rh * RH.d[q] + r0 * Rv[0].d[q] + r1 * Rv[1].d[q];
    }
  const long m = p.c;
  a.Hb[m] += acc[0];
  a.vb[0][m] += acc[1];
  a.vb[1][m] += acc[2];
  a.Fb[0][m] += acc[3];
  a.Fb[1][m] += acc[4];
}

hipError_t launch_adj_resid(hipStream_t st, const Lay &L, const AdjPhys &P, const double *H, double *const v[2],
                            double *const F[2], const double *RbH, double *const Rbv[2], double *Hb, double *vb[2],
                            double *Fb[2]) {
  AdjResidArgs a;
  a.L = L;
  a.P = P;
  a.H = H;
  for (int d = 0; d < 2; ++d) {
    a.v[d] = v[d];
    a.F[d] = F[d];
    a.Rbv[d] = Rbv[d];
    a.vb[d] = vb[d];
    a.Fb[d] = Fb[d];
  }
  a.RbH = RbH;
  a.Hb = Hb;
  hipLaunchKernelGGL(k_adj_resid, grid_for(L), dim3(kBX, kBY), 0, st, a);
  return hipGetLastError();
}

__device__ inline long pw(const Lay &L, int i, int j) {
  i = i < 0 ? i + L.n[0] : (i >= L.n[0] ? i - L.n[0] : i);
  j = j < 0 ? j + L.n[1] : (j >= L.n[1] ? j - L.n[1] : j);
  return L.at(i, j, 0);
}

// Transpose of the projection: from (Fb, vb) at the projected level to the
// momentum cotangent Mb, the density cotangent rhob and the pressure
// cotangent Pb (= -delta_1^T Fb + delta_2 (vb/rho)).
__global__ void __launch_bounds__(kBlock) k_adj_proj(Lay L, AdjPhys P, const double *Fb0, const double *Fb1,
                                                     const double *vb0, const double *vb1, const double *v0,
                                                     const double *v1, const double *rho, double *Mb0, double *Mb1,
                                                     double *rhob, double *Pb) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const int i = p.i, j = p.j;
  const long c = p.c;
  const double *Fb[2] = {Fb0, Fb1};
  const double *vb[2] = {vb0, vb1};
  const double *vv[2] = {v0, v1};
  double *Mb[2] = {Mb0, Mb1};
  const double r = rho[c];
  double rb = 0.0, pb = 0.0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const long cm = d == 0 ? pw(L, i - 1, j) : pw(L, i, j - 1);
    const long cp = d == 0 ? pw(L, i + 1, j) : pw(L, i, j + 1);
    const double w = vb[d][c] / r;
    rb -= vb[d][c] * vv[d][c] / r;
    Mb[d][c] = 0.5 * (Fb[d][c] + Fb[d][cm]) + w;
    const double wp = vb[d][cp] / rho[cp], wm = vb[d][cm] / rho[cm];
    pb += (Fb[d][c] - Fb[d][cm]) / P.h[d] + (wp - wm) / (2.0 * P.h[d]);
  }
  rhob[c] = rb;
  Pb[c] = pb;
}

// Transposes of the right-hand side, the EOS and the Adams update of one
// stage (corrector or predictor). AdjTailArgs: bb the zero-mean Poisson
// right-hand-side cotangent; Mb the momentum cotangent from the projection
// transpose; rhob_new the cotangent of the stage's new density; for the
// corrector the cotangents of the step's outputs (Hb_out, RbH_out, Rbv_out,
// rhoprevb_out); for the predictor Hb_star from the corrector residual
// transpose; outputs the level-n accumulators, the residual cotangents and
// the cotangents of the level n-1 history.
__global__ void __launch_bounds__(kBlock) k_adj_tail(AdjTailArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const int i = p.i, j = p.j;
  const long c = p.c;
  const double dt = a.P.dt;
  double c1, c2, c3;
  if (a.first) {
    c1 = 1.0 / dt;
    c2 = -1.0 / dt;
    c3 = 0.0;
  } else {
    c1 = 3.0 / (2.0 * dt);
    c2 = -4.0 / (2.0 * dt);
    c3 = 1.0 / (2.0 * dt);
  }
  const double bb = a.bb[c];
  double Mb[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const long cm = d == 0 ? pw(a.L, i - 1, j) : pw(a.L, i, j - 1);
    const long cp = d == 0 ? pw(a.L, i + 1, j) : pw(a.L, i, j + 1);
    Mb[d] = a.Mb[d][c] - (a.bb[cp] - a.bb[cm]) / (2.0 * a.P.h[d]);
  }
  const double rnew = a.rho_new[c];
  const double Tnew = a.P.qs * (a.H_new[c] - 1.0);
  const double drho = -rnew * a.P.qs / Tnew;      // d rho / d H
  const double rhob_new = a.rhob_new[c] + c1 * bb;
  const double rho_n = a.rho_n[c];
  double rhob_n = c2 * bb;
  double prevb = c3 * bb;
  if (a.corrector) {
    const double Hb = a.Hb_out[c] + drho * rhob_new;   // cotangent of H^{n+1}
    a.Hb_n[c] = Hb;
    a.RbH_star[c] = 0.5 * dt * Hb;
    a.RbH_n[c] = 0.5 * dt * Hb + a.RbH_out[c];
    rhob_n += a.rhoprevb_out[c];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      a.Rbv_star[d][c] = 0.5 * dt * Mb[d];
      a.Rbv_n[d][c] = 0.5 * dt * Mb[d] + a.Rbv_out[d][c];
      rhob_n += Mb[d] * a.v_n[d][c];
      a.vb_n[d][c] = rho_n * Mb[d];
    }
    a.rhob_n[c] = rhob_n;
    a.rhoprevb_in[c] = prevb;
  } else {
    const double ca = a.first ? 1.0 : 1.5, cb = a.first ? 0.0 : 0.5;
    const double Hb = a.Hb_star[c] + drho * rhob_new;  // cotangent of H*
    a.Hb_n[c] += Hb;
    a.RbH_n[c] += dt * ca * Hb;
    a.RbH_prev_in[c] = -dt * cb * Hb;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      rhob_n += Mb[d] * a.v_n[d][c];
      a.vb_n[d][c] += rho_n * Mb[d];
      a.Rbv_n[d][c] += dt * ca * Mb[d];
      a.Rbv_prev_in[d][c] = -dt * cb * Mb[d];
    }
    a.rhob_n[c] += rhob_n;
    a.rhoprevb_in[c] += prevb;
  }
}

hipError_t launch_adj_proj(hipStream_t st, const Lay &L, const AdjPhys &P, double *const Fb[2],
                           double *const vb[2], double *const v[2], const double *rho, double *Mb[2], double *rhob,
                           double *Pb) {
  hipLaunchKernelGGL(k_adj_proj, grid_for(L), dim3(kBX, kBY), 0, st, L, P, (const double *)Fb[0],
                     (const double *)Fb[1], (const double *)vb[0], (const double *)vb[1], (const double *)v[0],
                     (const double *)v[1], rho, Mb[0], Mb[1], rhob, Pb);
  return hipGetLastError();
}

hipError_t launch_adj_tail(hipStream_t st, const AdjTailArgs &a) {
  hipLaunchKernelGGL(k_adj_tail, grid_for(a.L), dim3(kBX, kBY), 0, st, a);
  return hipGetLastError();
}

// Hb += (d rho/d H) rhob at level n; the step's input cotangent is complete.
__global__ void __launch_bounds__(kBlock) k_adj_eos(Lay L, AdjPhys P, const double *H, const double *rho,
                                                    const double *rhob, double *Hb) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double T = P.qs * (H[c] - 1.0);
  Hb[c] += -rho[c] * P.qs / T * rhob[c];
}

hipError_t launch_adj_eos(hipStream_t st, const Lay &L, const AdjPhys &P, const double *H, const double *rho,
                          const double *rhob, double *Hb) {
  hipLaunchKernelGGL(k_adj_eos, grid_for(L), dim3(kBX, kBY), 0, st, L, P, H, rho, rhob, Hb);
  return hipGetLastError();
}

// A cotangent of the temperature folded into that of H: T = qs (H - 1) in
// non-reacting flow, so H_bar += qs T_bar.
__global__ void __launch_bounds__(kBlock) k_adj_add_T(Lay L, AdjPhys P, const double *Tb, double *Hb) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  Hb[p.c] += P.qs * Tb[p.c];
}

hipError_t launch_adj_add_T(hipStream_t st, const Lay &L, const AdjPhys &P, const double *Tb, double *Hb) {
  hipLaunchKernelGGL(k_adj_add_T, grid_for(L), dim3(kBX, kBY), 0, st, L, P, Tb, Hb);
  return hipGetLastError();
}

// Cotangent of J = sum 1/2 rho |v|^2 dV at the current level: vb = rho v dV,
// Hb = (d rho/d H) |v|^2/2 dV, all other cotangents zero.
__global__ void __launch_bounds__(kBlock) k_adj_seed_ke(Lay L, AdjPhys P, double dV, const double *H,
                                                        const double *rho, const double *v0, const double *v1,
                                                        double *Hb, double *vb0, double *vb1) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const long c = p.c;
  const double r = rho[c];
  const double T = P.qs * (H[c] - 1.0);
  const double e = 0.5 * (v0[c] * v0[c] + v1[c] * v1[c]);
  vb0[c] = r * v0[c] * dV;
  vb1[c] = r * v1[c] * dV;
  Hb[c] = -r * P.qs / T * e * dV;
}

hipError_t launch_adj_seed_ke(hipStream_t st, const Lay &L, const AdjPhys &P, double dV, const double *H,
                              const double *rho, double *const v[2], double *Hb, double *vb[2]) {
  hipLaunchKernelGGL(k_adj_seed_ke, grid_for(L), dim3(kBX, kBY), 0, st, L, P, dV, H, rho, (const double *)v[0],
                     (const double *)v[1], Hb, vb[0], vb[1]);
  return hipGetLastError();
}

// Adjoint of the initial state built from (T0, v0): F0 = avg(rho0 v0),
// rho0 = p0/T(H0), H0 = T0/qs + 1. Outputs Tb (cotangent of T0) and adds
// rho0 avg^T(Fb) to vb.
__global__ void __launch_bounds__(kBlock) k_adj_init(Lay L, AdjPhys P, const double *H, const double *rho,
                                                     const double *v0, const double *v1, const double *Fb0,
                                                     const double *Fb1, const double *Hb, double *vb0, double *vb1,
                                                     double *Tb) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const int i = p.i, j = p.j;
  const long c = p.c;
  const double r = rho[c];
  const double mb0 = 0.5 * (Fb0[c] + Fb0[pw(L, i - 1, j)]);
  const double mb1 = 0.5 * (Fb1[c] + Fb1[pw(L, i, j - 1)]);
  const double rhob = mb0 * v0[c] + mb1 * v1[c];
  vb0[c] += r * mb0;
  vb1[c] += r * mb1;
  const double T = P.qs * (H[c] - 1.0);
  const double hb = Hb[c] - r * P.qs / T * rhob;
  Tb[c] = hb / P.qs;
}

hipError_t launch_adj_init(hipStream_t st, const Lay &L, const AdjPhys &P, const double *H, const double *rho,
                           double *const v[2], double *const Fb[2], const double *Hb, double *vb[2], double *Tb) {
  hipLaunchKernelGGL(k_adj_init, grid_for(L), dim3(kBX, kBY), 0, st, L, P, H, rho, (const double *)v[0],
                     (const double *)v[1], (const double *)Fb[0], (const double *)Fb[1], Hb, vb[0], vb[1], Tb);
  return hipGetLastError();
}

// sum over cells of 1/2 rho |v|^2 into per-block partials.
__global__ void __launch_bounds__(kBlock) k_ke(Lay L, const double *rho, const double *v0, const double *v1,
                                               double *part) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double e = 0.0;
  if (cell_of_thread(L, p)) e = 0.5 * rho[p.c] * (v0[p.c] * v0[p.c] + v1[p.c] * v1[p.c]);
  const double s = block_sum(e, sh);
  if (linear_tid() == 0) part[linear_block()] = s;
}

__global__ void __launch_bounds__(kBlock) k_ke_finish(const double *part, int np, double dV, double *out) {
  __shared__ double sh[kBlock / 64];
  const double s = sum_partials(part, (unsigned)np, sh);
  if (threadIdx.x == 0) *out = s * dV;
}

hipError_t launch_ke(hipStream_t st, const Lay &L, const double *rho, double *const v[2], double dV, double *part,
                     double *out) {
  hipLaunchKernelGGL(k_ke, grid_for(L), dim3(kBX, kBY), 0, st, L, rho, (const double *)v[0], (const double *)v[1],
                     part);
  hipLaunchKernelGGL(k_ke_finish, dim3(1), dim3(kBlock), 0, st, (const double *)part, (int)nblocks_for(L), dV, out);
  return hipGetLastError();
}

}  // namespace lm
