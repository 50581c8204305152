// Adjoint (reverse mode) of one predictor-corrector step for the periodic,
// non-reacting configuration, in 2D and 3D, with or without an immersed body
// (volume penalisation, Eq 3.30-3.32; the mass source S_m does not depend on
// the state and has no cotangent). The step
// is recomputed forward from the stored state (not committed); the sweep
// back applies, in reverse order, the transposes of
//   projection   F = avg(M) - delta_1 P,  v = (M - delta_2 P)/rho   (Eq 3.23, 3.25)
//   Poisson      P = Pi A^+ Pi b  (A symmetric, Pi the mean projector)   (Eq 3.24)
//   right side   b = delta_2 . M + BDF(rho)                            (Eq 3.9-3.11)
//   EOS          rho = p0 / (Q/(S+1) (H - 1))                           (Eq 2.49, 3.42)
//   Adams steps  AB2 predictor / AM2 corrector                          (Eq 3.1-3.18)
//   residuals    R_H, R_v of Eq 3.4, 3.8, 3.26 with tau of Eq 2.46 and the
//                penalisation terms of Eq 3.30-3.32.
// The residual transpose is a gather: for every input cell m the residuals
// of the 3^DIM cells whose stencils reach m are re-evaluated with dual
// numbers seeded at m (derivatives with respect to H, the DIM velocity
// components and the DIM face fluxes at m) and contracted with the residual
// cotangents. No atomics; deterministic.
#include <type_traits>

#include "lm_device.h"
#include "lm_sides.h"

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
// Dual numbers carrying derivatives with respect to H, Z (reacting flow
// only, R = 1), v (DIM) and F (DIM).
template <int DIM, int R>
using DD = Dual<1 + R + 2 * DIM>;

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void adj_static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    adj_static_for<B + 1, E>(f);
  }
}

struct Ix {
  int i, j, k;
};
// x shifted by s cells along direction d
__device__ inline Ix off(Ix x, int d, int s) {
  if (d == 0)
    x.i += s;
  else if (d == 1)
    x.j += s;
  else
    x.k += s;
  return x;
}
__device__ inline int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ inline Ix wrap(const Lay &L, Ix x) { return Ix{wrap(x.i, L.n[0]), wrap(x.j, L.n[1]), wrap(x.k, L.n[2])}; }
__device__ inline long pw(const Lay &L, Ix x) {
  x = wrap(L, x);
  return L.at(x.i, x.j, x.k);
}

// Loader of the level fields at cell positions, interior or ghost; values
// at cell m carry unit seeds: H -> 0, Z -> 1 (R = 1), v_c -> 1 + R + c,
// F_d -> 1 + R + DIM + d. W = 0: every direction periodic (positions wrap);
// W = 1: slip / no-slip wall sides as well, whose ghost values follow the
// forward ghost rules (mirror, or 2 x side value - mirror; corner ghosts by
// the rules of the highest out-of-range direction first), so that a ghost
// carries the seed of the interior cell it mirrors with weight -1 or +1.
// The body mask and targets are constants (null: no body, or a zero
// target).
template <int DIM, int R, int W>
struct Loader {
  Lay L;
  Bnd B;
  Sides sd;
  const double *H, *Z, *v[3], *F[3];
  const double *kap, *dkap;  // the level's kappa(T) and d kappa/dT at the cells
  const unsigned char *chi;
  const double *H_ib, *Z_ib, *v_ib[3];
  Ix m;
  // cell constants at x (x wrapped into a periodic grid first)
  __device__ long cidx(Ix x) const {
    if (!W) x = wrap(L, x);
    return L.at(x.i, x.j, x.k);
  }
  __device__ double chi_at(Ix x) const { return chi ? (double)chi[cidx(x)] : 0.0; }
  __device__ double hib(Ix x) const { return H_ib ? H_ib[cidx(x)] : 0.0; }
  __device__ double zib(Ix x) const { return Z_ib ? Z_ib[cidx(x)] : 0.0; }
  __device__ double vib(int c, Ix x) const { return v_ib[c] ? v_ib[c][cidx(x)] : 0.0; }
  // field a with rule set f (0..2 velocity components, 3 Z, 4 H). An
  // outflow side's ghost is the quadratic extrapolation 3 u_0 - 3 u_1 + u_2
  // of the three cells inside; with at most one outflow direction (checked
  // at set-up) a ghost spans at most three cells.
  __device__ DD<DIM, R> load(const double *a, int f, Ix x, int seed) const {
    if (!W) {
      // periodic: the seed test on unwrapped coordinates (exact when every
      // direction has at least 3 cells, as readers lie within 2 of m), which
      // an unrolled gather resolves at compile time
      const bool seeded = x.i == m.i && x.j == m.j && x.k == m.k;
      x = wrap(L, x);
      DD<DIM, R> r(a[L.at(x.i, x.j, x.k)]);
      if (seeded) r.d[seed] = 1.0;
      return r;
    }
    int pos[3][3] = {{x.i, x.j, x.k}, {0, 0, 0}, {0, 0, 0}};
    double w[3] = {1.0, 0.0, 0.0};
    int nt = 1;
    double cst = 0.0;
#pragma unroll
    for (int d = DIM - 1; d >= 0; --d) {
      const int n = L.n[d];
      const int cur = nt;
      for (int t = 0; t < cur; ++t) {
        const int q = pos[t][d];
        if (q >= 0 && q < n) continue;
        const int s = q < 0 ? 0 : 1;
        if (B.periodic[d]) {
          pos[t][d] = s == 0 ? n - 1 : 0;
          continue;
        }
        const int i1 = s == 0 ? 0 : n - 1, step = s == 0 ? 1 : -1;
        const int rule = ghost_rule(B, sd, L, d, s, f, pos[t][0], pos[t][1], pos[t][2]);
        if (rule == R_DIR) {
          cst += 2.0 * w[t] * side_value(sd, L, d, s, f, pos[t][0], pos[t][1], pos[t][2]);
          w[t] = -w[t];
          pos[t][d] = i1;
        } else if (rule == R_NEU || nt != 1) {
          pos[t][d] = i1;
        } else {  // extrapolated (outflow)
          const double wt = w[t];
          for (int e = 0; e < 3; ++e) {
            pos[e][0] = pos[t][0];
            pos[e][1] = pos[t][1];
            pos[e][2] = pos[t][2];
            pos[e][d] = i1 + e * step;
          }
          w[0] = 3.0 * wt;
          w[1] = -3.0 * wt;
          w[2] = wt;
          nt = 3;
        }
      }
    }
    double val = cst, der = 0.0;
    for (int t = 0; t < nt; ++t) {
      val += w[t] * a[L.at(pos[t][0], pos[t][1], pos[t][2])];
      if (pos[t][0] == m.i && pos[t][1] == m.j && pos[t][2] == m.k) der += w[t];
    }
    DD<DIM, R> r(val);
    r.d[seed] = der;
    return r;
  }
  __device__ DD<DIM, R> hh(Ix x) const { return load(H, 4, x, 0); }
  __device__ DD<DIM, R> zz(Ix x) const { return load(Z, 3, x, 1); }  // R = 1 only
  __device__ DD<DIM, R> vv(int c, Ix x) const { return load(v[c], c, x, 1 + R + c); }
  // flux on the +d face of x (x interior, or one cell below the low side
  // along d: that side's face, a constant on a wall)
  __device__ DD<DIM, R> ff(int d, Ix x) const {
    if (!W) return load(F[d], 0, x, 1 + R + DIM + d);
    int pos[3] = {x.i, x.j, x.k};
    if (pos[d] < 0 && B.periodic[d]) pos[d] += L.n[d];
    DD<DIM, R> r(F[d][L.at(pos[0], pos[1], pos[2])]);
    if (pos[0] == m.i && pos[1] == m.j && pos[2] == m.k) r.d[1 + R + DIM + d] = 1.0;
    return r;
  }
  __device__ bool inside(Ix x) const {
    return x.i >= 0 && x.i < L.n[0] && x.j >= 0 && x.j < L.n[1] && (DIM == 2 || (x.k >= 0 && x.k < L.n[2]));
  }
};

// Flame map (section 3.5): F~(Z) = F_eps(Z) + fshift with
// F_eps = [-(S+1) ln cosh(k (Z-1))/k + (S-1)(Z-1)]/(2S) (Eq 3.41), so
// dF~/dZ = [-(S+1) tanh(k (Z-1)) + S - 1]/(2S).
__device__ inline double ftilde_of(const AdjPhys &P, double Z) {
  const double S = P.S, k = P.k;
  return (-(S + 1.0) * lncosh(k * (Z - 1.0)) / k + (S - 1.0) * (Z - 1.0)) / (2.0 * S) + P.fshift;
}
__device__ inline double dftilde_of(const AdjPhys &P, double Z) {
  return (-(P.S + 1.0) * tanh(P.k * (Z - 1.0)) + (P.S - 1.0)) / (2.0 * P.S);
}
template <int N>
__device__ inline Dual<N> ftilde_dual(const AdjPhys &P, const Dual<N> &Z) {
  Dual<N> r;
  r.v = ftilde_of(P, Z.v);
  const double dv = dftilde_of(P, Z.v);
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = dv * Z.d[q];
  return r;
}
// theta_eps(Z) = (1 + tanh(k (Z - 1)))/2 (Eq 3.34)
template <int N>
__device__ inline Dual<N> theta_dual(const AdjPhys &P, const Dual<N> &Z) {
  const double t = tanh(P.k * (Z.v - 1.0));
  Dual<N> r;
  r.v = 0.5 * (1.0 + t);
  const double dv = 0.5 * P.k * (1.0 - t * t);
#pragma unroll
  for (int q = 0; q < N; ++q) r.d[q] = dv * Z.d[q];
  return r;
}

// T(Z, H) of Eq 3.42; without reaction T = qs (H - 1).
template <int DIM, int R, int W>
__device__ inline DD<DIM, R> temp_at(const AdjPhys &P, const Loader<DIM, R, W> &ld, Ix x) {
  if (R) return P.qs * (ftilde_dual(P, ld.zz(x)) + ld.hh(x));
  return P.qs * (ld.hh(x) - 1.0);
}

// kappa(T) with its derivative: T^sigma (Eq 2.50), or Sutherland's law
// T^{3/2} (1 + C)/(T + C) (Eq 4.12), d kappa/dT = kappa (3/(2T) - 1/(T + C)).
template <int N>
__device__ inline Dual<N> kappa_dual(const AdjPhys &P, const Dual<N> &T) {
  if (P.suth_C > 0.0) {
    const double C = P.suth_C, t = T.v;
    Dual<N> r;
    r.v = t * sqrt(t) * (1.0 + C) / (t + C);
    const double dv = r.v * (1.5 / t - 1.0 / (t + C));
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = dv * T.d[q];
    return r;
  }
  return dpow(T, P.sigma);
}

// Conductivity at a cell position. Ghosts (W = 1) follow the forward ghost
// fill: at an isothermal wall 2 kappa(T_w) - kappa(T) of the interior cell
// the ghost position clamps to; elsewhere kappa of the ghost temperature,
// with the ghost Z clamped to [0, S+1].
template <int DIM, int R, int W>
__device__ inline DD<DIM, R> kap_at(const AdjPhys &P, const Loader<DIM, R, W> &ld, Ix x) {
  if (!W || ld.inside(x)) {
    // kappa of a cell from the level's precomputed kappa and d kappa/dT:
    // T = qs (F~(Z) + H) carries the seeds (dT/dH = qs, dT/dZ = qs F~'(Z))
    const bool seeded = x.i == ld.m.i && x.j == ld.m.j && x.k == ld.m.k;
    if (!W) x = wrap(ld.L, x);
    const long c = ld.L.at(x.i, x.j, x.k);
    DD<DIM, R> r(ld.kap[c]);
    if (seeded) {
      const double g = ld.dkap[c] * P.qs;
      r.d[0] = g;
      if (R) r.d[1] = g * dftilde_of(P, ld.Z[c]);
    }
    return r;
  }
  int dw, sw;
  if (isothermal_ghost<DIM>(ld.L, ld.B, ld.sd, x.i, x.j, x.k, dw, sw)) {
    const double Hw = side_value(ld.sd, ld.L, dw, sw, 4, x.i, x.j, x.k);
    const double Tw = P.reacting ? P.qs * (ftilde_of(P, 0.0) + Hw) : P.qs * (Hw - 1.0);
    const Ix src{min(max(x.i, 0), ld.L.n[0] - 1), min(max(x.j, 0), ld.L.n[1] - 1),
                 DIM == 3 ? min(max(x.k, 0), ld.L.n[2] - 1) : x.k};
    return 2.0 * kappa_dual(P, DD<DIM, R>(Tw)).v - kappa_dual(P, temp_at(P, ld, src));
  }
  const DD<DIM, R> H = ld.hh(x);
  if (!R) return kappa_dual(P, P.qs * (H - 1.0));
  DD<DIM, R> Z = ld.zz(x);
  if (Z.v < 0.0 || Z.v > P.S + 1.0) Z = DD<DIM, R>(fmin(fmax(Z.v, 0.0), P.S + 1.0));
  return kappa_dual(P, P.qs * (ftilde_dual(P, Z) + H));
}

// tau_{d c} for every component c on the face between cell x and its +d
// neighbour (Eq 2.46 on d-faces): normal derivatives across the face,
// tangential ones as the mean of the centred differences of the two cells.
template <int DIM, int R, int W>
__device__ inline void tau_face(const AdjPhys &P, const Loader<DIM, R, W> &ld, Ix x, int d, DD<DIM, R> tau[DIM]) {
  const Ix y = off(x, d, 1);
  const DD<DIM, R> kf = 0.5 * (kap_at(P, ld, x) + kap_at(P, ld, y));
  DD<DIM, R> D[DIM][DIM];  // D[k][c] = d v_c / d x_k on the face
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if (k == d) {
        D[k][c] = (ld.vv(c, y) - ld.vv(c, x)) * (1.0 / P.h[d]);
      } else {
        const double h2 = 2.0 * P.h[k];
        const DD<DIM, R> a = (ld.vv(c, off(x, k, 1)) - ld.vv(c, off(x, k, -1))) / h2;
        const DD<DIM, R> b = (ld.vv(c, off(y, k, 1)) - ld.vv(c, off(y, k, -1))) / h2;
        D[k][c] = 0.5 * (a + b);
      }
    }
  }
  DD<DIM, R> div = D[0][0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) div = div + D[k][k];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    DD<DIM, R> t = D[d][c] + D[c][d];
    if (c == d) t = t - (2.0 / 3.0) * div;
    tau[c] = kf * t;
  }
}

// Advection (face fluxes times the one-sided differences, averaged to the
// centre) and centred diffusion of a scalar at cell x (Eq 3.26b, section
// 3.2): field 0 H, 1 Z.
template <int DIM, int R, int W>
__device__ inline void scalar_dual(const AdjPhys &P, const Loader<DIM, R, W> &ld, Ix x, int f, const DD<DIM, R> &kc,
                                   DD<DIM, R> &adv, DD<DIM, R> &dif) {
  auto val = [&](Ix y) { return f == 0 ? ld.hh(y) : ld.zz(y); };
  const DD<DIM, R> sc = val(x);
  adv = DD<DIM, R>(0.0);
  dif = DD<DIM, R>(0.0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const Ix xp = off(x, d, 1), xm = off(x, d, -1);
    const DD<DIM, R> gp = (val(xp) - sc) / P.h[d];
    const DD<DIM, R> gm = (sc - val(xm)) / P.h[d];
    const DD<DIM, R> kp = 0.5 * (kc + kap_at(P, ld, xp));
    const DD<DIM, R> km = 0.5 * (kap_at(P, ld, xm) + kc);
    adv = adv + 0.5 * (ld.ff(d, x) * gp + ld.ff(d, xm) * gm);
    dif = dif + (kp * gp - km * gm) / P.h[d];
  }
}

// R_H, R_Z (R = 1) and R_v at cell x (wrapped into the grid): the
// arithmetic of the forward residual (Eq 3.2a, 3.4a, 3.8a with the flux
// forms of Eq 3.26, the Lewis-number factors of Eq 3.35), with the
// penalisation of the body mask chi (Eq 3.30-3.32).
template <int DIM, int R, int W>
__device__ inline void resid_cell(const AdjPhys &P, const Loader<DIM, R, W> &ld, Ix x, DD<DIM, R> &RH,
                                  DD<DIM, R> &RZ, DD<DIM, R> Rv[DIM]) {
  const DD<DIM, R> Hc = ld.hh(x);
  const DD<DIM, R> Tc = temp_at(P, ld, x);
  const DD<DIM, R> rho = DD<DIM, R>(P.p0) / Tc;
  const DD<DIM, R> kc = kappa_dual(P, Tc);
  const double chi = ld.chi_at(x);
  DD<DIM, R> adv, dif;
  scalar_dual(P, ld, x, 0, kc, adv, dif);
  DD<DIM, R> rH = -adv + dif / P.Pe;
  if (R) {
    DD<DIM, R> advZ, difZ;
    scalar_dual(P, ld, x, 1, kc, advZ, difZ);
    const DD<DIM, R> Zc = ld.zz(x);
    const DD<DIM, R> th = theta_dual(P, Zc);
    const DD<DIM, R> le = (P.Le_F - P.Le_O) * th + P.Le_O;
    const DD<DIM, R> nn = (P.N_F - P.N_O) * th + P.N_O;
    DD<DIM, R> rZ = -advZ + difZ / (le * P.Pe);
    rH = rH + nn * difZ / P.Pe;
    if (chi != 0.0) rZ = rZ - chi * (kc * (Zc - ld.zib(x))) / (le * (P.Pe * P.Da));
    RZ = rZ / rho;
  }
  if (chi != 0.0) rH = rH - chi * (kc * (Hc - ld.hib(x))) / (P.Pe * P.Da);
  RH = rH / rho;
  DD<DIM, R> visc[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) visc[c] = DD<DIM, R>(0.0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    DD<DIM, R> tp[DIM], tm[DIM];
    tau_face<DIM, R, W>(P, ld, x, d, tp);
    tau_face<DIM, R, W>(P, ld, off(x, d, -1), d, tm);
#pragma unroll
    for (int c = 0; c < DIM; ++c) visc[c] = visc[c] + (tp[c] - tm[c]) / P.h[d];
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const DD<DIM, R> vc = ld.vv(c, x);
    DD<DIM, R> conv(0.0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const Ix xp = off(x, d, 1), xm = off(x, d, -1);
      const DD<DIM, R> flp = ld.ff(d, x) * (0.5 * (vc + ld.vv(c, xp)));
      const DD<DIM, R> flm = ld.ff(d, xm) * (0.5 * (ld.vv(c, xm) + vc));
      conv = conv + (flp - flm) / P.h[d];
    }
    DD<DIM, R> r = -conv + (P.Pr / P.Pe) * visc[c];
    if (c == 1 && P.inv_Fr2 != 0.0) r = r + P.inv_Fr2 * (1.0 - rho);
    if (chi != 0.0) r = r - chi * (P.Pr / (P.Pe * P.Da)) * (kc * (vc - ld.vib(c, x)));
    Rv[c] = r;
  }
}

// Density of the equation of state rho = p0/T(Z, H) and its derivatives
// d rho/dH = -rho qs/T and d rho/dZ = -rho qs F~'(Z)/T.
struct EosD {
  double dH, dZ;
};
__device__ inline EosD eos_d(const AdjPhys &P, double rho, double H, double Z) {
  const double T = P.reacting ? P.qs * (ftilde_of(P, Z) + H) : P.qs * (H - 1.0);
  const double g = -rho * P.qs / T;
  return EosD{g, P.reacting ? g * dftilde_of(P, Z) : 0.0};
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Launch one of the <DIM, R> instances of a kernel.
#define LM_ADJ_LAUNCH(K, L, R, ...)                                                          \
  do {                                                                                       \
    if ((L).ndim == 3) {                                                                     \
      if (R)                                                                                 \
        hipLaunchKernelGGL((K<3, 1>), grid_for(L), dim3(kBX, kBY), 0, st, __VA_ARGS__);     \
      else                                                                                   \
        hipLaunchKernelGGL((K<3, 0>), grid_for(L), dim3(kBX, kBY), 0, st, __VA_ARGS__);     \
    } else {                                                                                 \
      if (R)                                                                                 \
        hipLaunchKernelGGL((K<2, 1>), grid_for(L), dim3(kBX, kBY), 0, st, __VA_ARGS__);     \
      else                                                                                   \
        hipLaunchKernelGGL((K<2, 0>), grid_for(L), dim3(kBX, kBY), 0, st, __VA_ARGS__);     \
    }                                                                                        \
  } while (0)

// kappa(T) and d kappa/dT of every cell of a level, T = T(Z, H): one
// evaluation per cell, which the residual gather reads (it meets each cell
// in up to 13 stencil positions of each of its 3^DIM residuals).
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_kappa(AdjCellArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const long c = p.c;
  const double T = R ? a.P.qs * (ftilde_of(a.P, a.Z[c]) + a.H[c]) : a.P.qs * (a.H[c] - 1.0);
  Dual<1> t(T);
  t.d[0] = 1.0;
  const Dual<1> k = kappa_dual(a.P, t);
  a.Hb[c] = k.v;     // kappa
  a.Zb0[c] = k.d[0]; // d kappa/dT
}

hipError_t launch_adj_kappa(hipStream_t st, const AdjCellArgs &a) {
  LM_ADJ_LAUNCH(k_adj_kappa, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// (Hb, Zb, vb, Fb) += (dR/d(H, Z, v, F))^T (RbH, RbZ, Rbv) by gather over
// the 3^DIM cells whose residual stencils reach the cell (with wall or
// inflow sides, the interior ones: a ghost mirrors a cell within one cell
// of the reader; towards a high outflow side two cells further, as its
// extrapolated ghost reads three cells in). The flux of a wall or inflow
// face is a constant of the step: its cotangent stays 0.
template <int DIM, int R, int W>
__global__ void __launch_bounds__(kBlock) k_adj_resid(AdjResidArgs a) {
  constexpr int N = 1 + R + 2 * DIM;
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  if (a.box_mode) {
    const bool in = p.i >= a.box_lo[0] && p.i <= a.box_hi[0] && p.j >= a.box_lo[1] && p.j <= a.box_hi[1] &&
                    p.k >= a.box_lo[2] && p.k <= a.box_hi[2];
    if (in != (a.box_mode == 1)) return;
  }
  Loader<DIM, R, W> ld;
  ld.L = a.L;
  ld.B = a.B;
  ld.sd = a.sd;
  ld.H = a.H;
  ld.Z = a.Z;
  ld.kap = a.kap;
  ld.dkap = a.dkap;
  ld.chi = a.chi;
  ld.H_ib = a.H_ib;
  ld.Z_ib = a.Z_ib;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ld.v[d] = a.v[d];
    ld.F[d] = a.F[d];
    ld.v_ib[d] = a.v_ib[d];
  }
  ld.m = Ix{p.i, p.j, p.k};
  double acc[N];
#pragma unroll
  for (int q = 0; q < N; ++q) acc[q] = 0.0;
  const int kr = DIM == 3 ? 1 : 0;
  // an outflow ghost reads the third cell inside: readers of cell m reach
  // two cells towards a high outflow side
  const int pm[3] = {p.i, p.j, p.k};
  int hi[3] = {1, 1, kr};
  if (W)
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (a.B.kind[d][1] == LM_SIDE_OUTFLOW && pm[d] == a.L.n[d] - 3) hi[d] = 2;
  // the residual of cell x (unwrapped in a periodic grid) contracted with
  // its cotangents into acc
  auto gather = [&](Ix x) __attribute__((always_inline)) {
    DD<DIM, R> RH, RZ, Rv[DIM];
    resid_cell<DIM, R, W>(a.P, ld, x, RH, RZ, Rv);
    const long c = ld.cidx(x);
    const double rh = a.RbH[c], rz = R ? a.RbZ[c] : 0.0;
    double r[DIM];
#pragma unroll
    for (int e = 0; e < DIM; ++e) r[e] = a.Rbv[e][c];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = rh * RH.d[q];
      if (R) s += rz * RZ.d[q];
#pragma unroll
      for (int e = 0; e < DIM; ++e) s += r[e] * Rv[e].d[q];
      acc[q] += s;
    }
  };
  if constexpr (!W) {
    // periodic: the 3^DIM offsets unrolled, so that every seed test (which
    // stencil position is cell m) is a constant and the derivative
    // arithmetic of the positions that are not m folds away
    adj_static_for<0, (DIM == 3 ? 27 : 9)>([&](auto T) __attribute__((always_inline)) {
      constexpr int t = decltype(T)::value;
      constexpr int di = t % 3 - 1, dj = (t / 3) % 3 - 1, dk = DIM == 3 ? t / 9 - 1 : 0;
      gather(Ix{p.i + di, p.j + dj, p.k + dk});
    });
  } else {
    for (int dk = -kr; dk <= hi[2]; ++dk)
      for (int dj = -1; dj <= hi[1]; ++dj)
        for (int di = -1; di <= hi[0]; ++di) {
          Ix x{p.i + di, p.j + dj, p.k + dk};
          if (!ld.inside(x)) {
            const int q[3] = {x.i, x.j, x.k};
            bool wall = false;
            for (int d = 0; d < DIM; ++d)
              if ((q[d] < 0 || q[d] >= a.L.n[d]) && !a.B.periodic[d]) wall = true;
            if (wall) continue;  // a ghost has no residual
          }
          gather(wrap(a.L, x));
        }
  }
  const long m = p.c;
  a.Hb[m] += acc[0];
  if (R) a.Zb[m] += acc[1];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    a.vb[d][m] += acc[1 + R + d];
    // the high face of the last cell: a state flux on an outflow side, a
    // constant on a wall or inflow side
    if (!W || a.B.periodic[d] || pm[d] + 1 < a.L.n[d] || a.B.kind[d][1] == LM_SIDE_OUTFLOW)
      a.Fb[d][m] += acc[1 + R + DIM + d];
  }
}

static void launch_resid_sel(hipStream_t st, const AdjResidArgs &a, int W) {
  const dim3 g = grid_for(a.L), bl(kBX, kBY);
  const int sel = (a.L.ndim == 3 ? 4 : 0) + (a.P.reacting ? 2 : 0) + W;
  switch (sel) {
    case 0: hipLaunchKernelGGL((k_adj_resid<2, 0, 0>), g, bl, 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_adj_resid<2, 0, 1>), g, bl, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_adj_resid<2, 1, 0>), g, bl, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_adj_resid<2, 1, 1>), g, bl, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_adj_resid<3, 0, 0>), g, bl, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_adj_resid<3, 0, 1>), g, bl, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_adj_resid<3, 1, 0>), g, bl, 0, st, a); break;
    default: hipLaunchKernelGGL((k_adj_resid<3, 1, 1>), g, bl, 0, st, a); break;
  }
}

// With wall, inflow or outflow sides: the cells whose readers' stencils
// stay inside the grid (at least 2 cells from every non-periodic side, 3
// from a high outflow side, whose gather reaches further) take the
// periodic kernel, exact there (no ghost is read and no position wraps
// across such a side); the band along those sides the kernel with the
// ghost rules.
hipError_t launch_adj_resid(hipStream_t st, const AdjResidArgs &a0) {
  AdjResidArgs a = a0;
  a.box_mode = 0;
  if (a.B.all_periodic) {
    launch_resid_sel(st, a, 0);
    return hipGetLastError();
  }
  bool empty = false;
  for (int d = 0; d < 3; ++d) {
    a.box_lo[d] = 0;
    a.box_hi[d] = a.L.n[d] - 1;
    if (d < a.L.ndim && !a.B.periodic[d]) {
      a.box_lo[d] = 2;
      a.box_hi[d] = a.L.n[d] - (a.B.kind[d][1] == LM_SIDE_OUTFLOW ? 4 : 3);
      empty = empty || a.box_hi[d] < a.box_lo[d];
    }
  }
  if (!empty) {
    a.box_mode = 1;
    launch_resid_sel(st, a, 0);
    a.box_mode = 2;
  }
  launch_resid_sel(st, a, 1);
  return hipGetLastError();
}

// Coefficient of x_q in (xm - xp) at cell qq of a direction with two wall
// sides (n >= 3): xp, xm are the neighbours of qq, or at the sides the
// ghost 3 x_0 - 3 x_1 + x_2 (mirrored at the high side) of the quadratic
// extrapolation the projection uses (Eq 3.27-3.28).
__device__ inline double xcoef(int qq, int q, int n) {
  const double cm = qq > 0 ? (double)(q == qq - 1)
                           : 3.0 * (q == qq) - 3.0 * (q == qq + 1) + (double)(q == qq + 2);
  const double cp = qq + 1 < n ? (double)(q == qq + 1)
                               : 3.0 * (q == qq) - 3.0 * (q == qq - 1) + (double)(q == qq - 2);
  return cm - cp;
}

// Outflow face flux on the high side of direction d: the quadratic
// extrapolation (15 M_{n-1} - 10 M_{n-2} + 3 M_{n-3})/8 of the cell
// momentum (less the uniform closure shift); the cotangent it passes to
// the momentum of cell q (zero away from the side) from the face
// cotangent Fb of its column.
__constant__ double kOutW[3] = {15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0};
__device__ inline double outflow_face_mb(const Lay &L, const Bnd &B, const double *Fb, long c, int d, int q) {
  const int n = L.n[d], j = n - 1 - q;
  if (B.kind[d][1] != LM_SIDE_OUTFLOW || j > 2) return 0.0;
  return kOutW[j] * Fb[c + (long)j * L.s[d]];
}

// Transpose of the projection: from (Fb, vb) at the projected level to the
// momentum cotangent Mb, the density cotangent rhob and the pressure
// cotangent Pb (= -delta_1^T Fb + delta_2^T (vb/rho)). Wall faces carry a
// constant flux (no cotangent); near a wall delta_2 reads the extrapolated
// ghost of P.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_proj(AdjProjArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const Ix x{p.i, p.j, p.k};
  const long c = p.c;
  const double r = a.rho[c];
  double rb = 0.0, pb = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double ih = 1.0 / a.P.h[d];
    const double w = a.vb[d][c] / r;
    rb -= a.vb[d][c] * a.v[d][c] / r;
    if (a.B.periodic[d]) {
      const long cm = pw(a.L, off(x, d, -1)), cp = pw(a.L, off(x, d, 1));
      a.Mb[d][c] = 0.5 * (a.Fb[d][c] + a.Fb[d][cm]) + w;
      const double wp = a.vb[d][cp] / a.rho[cp], wm = a.vb[d][cm] / a.rho[cm];
      pb += (a.Fb[d][c] - a.Fb[d][cm]) / a.P.h[d] + (wp - wm) / (2.0 * a.P.h[d]);
    } else {
      const int n = a.L.n[d], q = coord(p, d);
      const long sdd = a.L.s[d];
      const double fh = q + 1 < n ? a.Fb[d][c] : 0.0, fl = q > 0 ? a.Fb[d][c - sdd] : 0.0;
      a.Mb[d][c] = 0.5 * (fh + fl) + w + outflow_face_mb(a.L, a.B, a.Fb[d], c, d, q);
      double s2 = 0.0;
      for (int qq = max(q - 2, 0); qq <= min(q + 2, n - 1); ++qq) {
        const long cq = c + (long)(qq - q) * sdd;
        s2 += a.vb[d][cq] / a.rho[cq] * xcoef(qq, q, n);
      }
      pb += (fh - fl) * ih + s2 * (0.5 * ih);
    }
  }
  a.rhob[c] = rb;
  a.Pb[c] = pb;
}

hipError_t launch_adj_proj(hipStream_t st, const AdjProjArgs &a) {
  LM_ADJ_LAUNCH(k_adj_proj, a.L, 0, a);
  return hipGetLastError();
}

// Transposes of the right-hand side, the EOS and the Adams update of one
// stage (corrector or predictor). AdjTailArgs: bb the zero-mean Poisson
// right-hand-side cotangent; Mb the momentum cotangent from the projection
// transpose; rhob_new the cotangent of the stage's new density; for the
// corrector the cotangents of the step's outputs (Hb_out, Zb_out, RbH_out,
// RbZ_out, Rbv_out, rhoprevb_out); for the predictor Hb_star, Zb_star from
// the corrector residual transpose; outputs the level-n accumulators, the
// residual cotangents and the cotangents of the level n-1 history. H and Z
// follow the same Adams updates (Eq 3.1, 3.3, 3.12, 3.14).
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_tail(AdjTailArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const Ix x{p.i, p.j, p.k};
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
  double Mb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (a.B.periodic[d]) {
      const long cm = pw(a.L, off(x, d, -1)), cp = pw(a.L, off(x, d, 1));
      Mb[d] = a.Mb[d][c] - (a.bb[cp] - a.bb[cm]) / (2.0 * a.P.h[d]);
    } else {
      // a wall face carries no momentum: b's face averages exist on interior
      // faces only, so d b_c/d M_c = (hi - lo)/(2h) with hi, lo = 1 for an
      // interior face
      const int n = a.L.n[d], q = coord(p, d);
      const long sdd = a.L.s[d];
      const double hi = q + 1 < n ? 1.0 : 0.0, lo = q > 0 ? 1.0 : 0.0;
      const double bp = q + 1 < n ? a.bb[c + sdd] : 0.0, bm = q > 0 ? a.bb[c - sdd] : 0.0;
      Mb[d] = a.Mb[d][c] - (bp - bm) / (2.0 * a.P.h[d]) + bb * (hi - lo) / (2.0 * a.P.h[d]);
      // the last cell's high face on an outflow side is the extrapolated
      // momentum (unshifted in b)
      Mb[d] += outflow_face_mb(a.L, a.B, a.bb, c, d, q) / a.P.h[d];
    }
  }
  const EosD e = eos_d(a.P, a.rho_new[c], a.H_new[c], R ? a.Z_new[c] : 0.0);
  const double rhob_new = a.rhob_new[c] + c1 * bb;
  const double rho_n = a.rho_n[c];
  double rhob_n = c2 * bb;
  double prevb = c3 * bb;
  if (a.corrector) {
    const double Hb = a.Hb_out[c] + e.dH * rhob_new;   // cotangent of H^{n+1}
    a.Hb_n[c] = Hb;
    a.RbH_star[c] = 0.5 * dt * Hb;
    a.RbH_n[c] = 0.5 * dt * Hb + a.RbH_out[c];
    if (R) {
      const double Zb = a.Zb_out[c] + e.dZ * rhob_new;  // cotangent of Z^{n+1}
      a.Zb_n[c] = Zb;
      a.RbZ_star[c] = 0.5 * dt * Zb;
      a.RbZ_n[c] = 0.5 * dt * Zb + a.RbZ_out[c];
    }
    rhob_n += a.rhoprevb_out[c];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      a.Rbv_star[d][c] = 0.5 * dt * Mb[d];
      a.Rbv_n[d][c] = 0.5 * dt * Mb[d] + a.Rbv_out[d][c];
      rhob_n += Mb[d] * a.v_n[d][c];
      a.vb_n[d][c] = rho_n * Mb[d];
    }
    a.rhob_n[c] = rhob_n;
    a.rhoprevb_in[c] = prevb;
  } else {
    const double ca = a.first ? 1.0 : 1.5, cb = a.first ? 0.0 : 0.5;
    const double Hb = a.Hb_star[c] + e.dH * rhob_new;  // cotangent of H*
    a.Hb_n[c] += Hb;
    a.RbH_n[c] += dt * ca * Hb;
    a.RbH_prev_in[c] = -dt * cb * Hb;
    if (R) {
      const double Zb = a.Zb_star[c] + e.dZ * rhob_new;  // cotangent of Z*
      a.Zb_n[c] += Zb;
      a.RbZ_n[c] += dt * ca * Zb;
      a.RbZ_prev_in[c] = -dt * cb * Zb;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      rhob_n += Mb[d] * a.v_n[d][c];
      a.vb_n[d][c] += rho_n * Mb[d];
      a.Rbv_n[d][c] += dt * ca * Mb[d];
      a.Rbv_prev_in[d][c] = -dt * cb * Mb[d];
    }
    a.rhob_n[c] += rhob_n;
    a.rhoprevb_in[c] += prevb;
  }
}

hipError_t launch_adj_tail(hipStream_t st, const AdjTailArgs &a) {
  LM_ADJ_LAUNCH(k_adj_tail, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// (Hb, Zb) += (d rho/d(H, Z)) rhob at level n; the step's input cotangent
// is complete.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_eos(AdjCellArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const long c = p.c;
  const EosD e = eos_d(a.P, a.rho[c], a.H[c], R ? a.Z[c] : 0.0);
  a.Hb[c] += e.dH * a.rhob[c];
  if (R) a.Zb[c] += e.dZ * a.rhob[c];
}

hipError_t launch_adj_eos(hipStream_t st, const AdjCellArgs &a) {
  LM_ADJ_LAUNCH(k_adj_eos, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// A cotangent of the temperature folded into those of H and Z:
// T = qs (F~(Z) + H) (T = qs (H - 1) without reaction), so H_bar += qs T_bar
// and Z_bar += qs F~'(Z) T_bar.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_add_T(AdjCellArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const long c = p.c;
  a.Hb[c] += a.P.qs * a.Tb[c];
  if (R) a.Zb[c] += a.P.qs * dftilde_of(a.P, a.Z[c]) * a.Tb[c];
}

hipError_t launch_adj_add_T(hipStream_t st, const AdjCellArgs &a) {
  LM_ADJ_LAUNCH(k_adj_add_T, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// Cotangent of J = sum 1/2 rho |v|^2 dV at the current level: vb = rho v dV,
// (Hb, Zb) = (d rho/d(H, Z)) |v|^2/2 dV, all other cotangents zero.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_seed_ke(AdjCellArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const long c = p.c;
  const double r = a.rho[c];
  double e = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double u = a.v[d][c];
    e += u * u;
    a.vb[d][c] = r * u * a.dV;
  }
  const EosD g = eos_d(a.P, r, a.H[c], R ? a.Z[c] : 0.0);
  a.Hb[c] = g.dH * (0.5 * e) * a.dV;
  if (R) a.Zb[c] = g.dZ * (0.5 * e) * a.dV;
}

hipError_t launch_adj_seed_ke(hipStream_t st, const AdjCellArgs &a) {
  LM_ADJ_LAUNCH(k_adj_seed_ke, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// Adjoint of the initial state built from (T0, Z0, v0): H0 = T0/qs - F~(Z0)
// (T0/qs + 1 without reaction), rho0 = p0/T0, F0 = avg(rho0 v0) on interior
// faces (wall faces carry the constant wall flux). Outputs
// Tb (cotangent of T0), Zb0 (of Z0, reacting flow) and adds
// rho0 avg^T(Fb) to vb. rho0 depends on T0 alone, so the density cotangent
// from F0 enters T0 only; the state cotangents of H and Z map through the
// enthalpy map.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_adj_init(AdjCellArgs a) {
  CellPos p;
  if (!cell_of_thread(a.L, p)) return;
  const Ix x{p.i, p.j, p.k};
  const long c = p.c;
  const double r = a.rho[c];
  double rhob = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int q = coord(p, d);
    const bool per = a.B.periodic[d];
    const double fh = (per || q + 1 < a.L.n[d]) ? a.Fb[d][c] : 0.0;  // wall faces: constant flux
    const double fl = (per || q > 0) ? a.Fb[d][pw(a.L, off(x, d, -1))] : 0.0;
    const double mb = 0.5 * (fh + fl) + (per ? 0.0 : outflow_face_mb(a.L, a.B, a.Fb[d], c, d, q));
    rhob += mb * a.v[d][c];
    a.vb[d][c] += r * mb;
  }
  const double hb = a.Hb_in[c];
  a.Tb_out[c] = hb / a.P.qs - r * r / a.P.p0 * rhob;  // d rho0/d T0 = -rho0/T0 = -rho0^2/p0
  if (R) a.Zb0[c] = a.Zb_in[c] - dftilde_of(a.P, a.Z[c]) * hb;
}

hipError_t launch_adj_init(hipStream_t st, const AdjCellArgs &a) {
  LM_ADJ_LAUNCH(k_adj_init, a.L, a.P.reacting, a);
  return hipGetLastError();
}

// Outflow closure (one high outflow side, direction d): the forward shifts
// the Poisson right-hand side of the cells next to the side by oc/h and the
// outflow face fluxes by -oc, oc = sum(b) dV / area. Given the adjoint
// solve's output y (the cotangent of the shifted right-hand side) and the
// outflow face cotangents Fb, one block forms
//   s = (-sum_side y/h - sum_side Fb) dV / area
// and the second kernel adds it to every cell: b_bar = y + s.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_adj_outflow_sum(Lay L, AdjPhys P, int d, const double *y,
                                                            const double *Fb, double *out) {
  __shared__ double sh[kBlock / 64];
  const int n = L.n[d];
  const int a0 = d == 0 ? 1 : 0, a1 = d == 2 ? 1 : 2;  // the two other directions
  const long m0 = L.n[a0], m1 = DIM == 3 ? L.n[a1] : 1;
  double acc = 0.0;
  for (long t = threadIdx.x; t < m0 * m1; t += blockDim.x) {
    int q[3] = {0, 0, 0};
    q[d] = n - 1;
    q[a0] = (int)(t % m0);
    if (DIM == 3) q[a1] = (int)(t / m0);
    const long c = L.at(q[0], q[1], q[2]);
    acc += y[c] / P.h[d] + Fb[c];
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = -tot * P.h[d] / (double)(m0 * m1);  // dV/area = h_d / (faces on the side)
}

__global__ void __launch_bounds__(kBlock) k_adj_add_scalar(Lay L, double *y, const double *s) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  y[p.c] += *s;
}

hipError_t launch_adj_outflow(hipStream_t st, const Lay &L, const AdjPhys &P, int d, double *y, const double *Fb,
                              double *scratch) {
  if (L.ndim == 3)
    hipLaunchKernelGGL(k_adj_outflow_sum<3>, dim3(1), dim3(kBlock), 0, st, L, P, d, (const double *)y, Fb, scratch);
  else
    hipLaunchKernelGGL(k_adj_outflow_sum<2>, dim3(1), dim3(kBlock), 0, st, L, P, d, (const double *)y, Fb, scratch);
  hipLaunchKernelGGL(k_adj_add_scalar, grid_for(L), dim3(kBX, kBY), 0, st, L, y, (const double *)scratch);
  return hipGetLastError();
}

// out = 2 x1 - x2 on the cells: the linear extrapolation of a stage's last
// two adjoint Poisson solutions, the next solve's initial guess.
__global__ void __launch_bounds__(kBlock) k_adj_extrap(Lay L, const double *x1, const double *x2, double *out) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  out[p.c] = 2.0 * x1[p.c] - x2[p.c];
}

hipError_t launch_adj_extrap(hipStream_t st, const Lay &L, const double *x1, const double *x2, double *out) {
  hipLaunchKernelGGL(k_adj_extrap, grid_for(L), dim3(kBX, kBY), 0, st, L, x1, x2, out);
  return hipGetLastError();
}

// sum over cells of 1/2 rho |v|^2 into per-block partials.
template <int DIM, int R>
__global__ void __launch_bounds__(kBlock) k_ke(AdjCellArgs a) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double e = 0.0;
  if (cell_of_thread(a.L, p)) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) s += a.v[d][p.c] * a.v[d][p.c];
    e = 0.5 * a.rho[p.c] * s;
  }
  const double s = block_sum(e, sh);
  if (linear_tid() == 0) a.part[linear_block()] = s;
}

__global__ void __launch_bounds__(kBlock) k_ke_finish(const double *part, int np, double dV, double *out) {
  __shared__ double sh[kBlock / 64];
  const double s = sum_partials(part, (unsigned)np, sh);
  if (threadIdx.x == 0) *out = s * dV;
}

hipError_t launch_ke(hipStream_t st, const Lay &L, const double *rho, double *const v[3], double dV, double *part,
                     double *out) {
  AdjCellArgs a{};
  a.L = L;
  a.rho = rho;
  a.part = part;
  for (int d = 0; d < L.ndim; ++d) a.v[d] = v[d];
  LM_ADJ_LAUNCH(k_ke, L, 0, a);
  hipLaunchKernelGGL(k_ke_finish, dim3(1), dim3(kBlock), 0, st, (const double *)part, (int)nblocks_for(L), dV, out);
  return hipGetLastError();
}

}  // namespace lm
