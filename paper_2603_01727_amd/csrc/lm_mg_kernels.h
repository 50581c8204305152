// Multigrid kernels of the Poisson preconditioner that work out of LDS:
//  - fused 2D tile kernels with temporal blocking (one launch per level and
//    direction of the V-cycle), and
//  - the one-block coarse V-cycle over all levels of at most kCoarseCells
//    cells, with the dense pseudo-inverse on the coarsest grid.
// Each comes in the constant-coefficient form (beta = 1) and, with VC, in
// the variable-coefficient form beta = 1/rho_f (face_beta), whose level
// operators are rediscretised from the level's density (2^d-cell averages).
// Included by lm_solver.hip only.
#pragma once

namespace lm {

// ---------------------------------------------------------------------------
// Fused 2D tile kernels
// ---------------------------------------------------------------------------
template <typename T>
struct Down2DArgs {
  Lay Lf, Lc;
  Bnd B;
  T ihx, ihy, idg;          // 1/h^2 per direction; 1/diag for interior cells
  const void *b;            // right-hand side (FP64 r_{k-1} on the finest level)
  T *xpre, *bc;             // outputs: pre-smoothed x, coarse right-hand side
  // finest-level CG update (k >= 1)
  double *x;
  const double *p, *q;
  double *rnew;
  const double *part_pq;
  int np_pq;
  SolverScalars *sc;
  int k;                    // CG iteration (0: plain V-cycle on r_0)
  int finest;
  int tiles_x;
  // single-reduction CG (Chronopoulos-Gear): p, s, x, r updated here
  int cgcg;
  const T *u;               // z_{k-1} = M r_{k-1}
  const double *w;          // A u
  const double *s_old;      // s_{k-2}
  double *s_new, *p_io;     // s_{k-1}; p updated in place
  const double *part_g, *part_cc;  // [gamma | delta | rr] x np_g; ||c||^2 x np_cc
  int np_g, np_cc;
  double tol2;
  const T *cfx, *cfy, *cig;  // variable-coefficient kernels: west/south face beta, 1/diagonal
};

template <typename T>
struct Up2DArgs {
  Lay Lf, Lc;
  Bnd B;
  T ihx, ihy, idg;
  double dihx, dihy;  // FP64 1/h^2: w = A u is formed in FP64 whatever T is
  const T *xpre, *xc;
  const void *b;      // FP64 r_k on the finest level
  T *xout;
  const T *zold;      // flexible CG: z_{k-1}
  double *part_rz;    // finest level: [rz | rr | rzo] x np, or [r.u | w.u | rr] x np
  int np;
  const SolverScalars *sc;
  int finest;
  int tiles_x;
  double *w;          // single-reduction CG: w = A u written on the finest level
  const T *cfx, *cfy, *cig;  // variable-coefficient kernels: west/south face beta, 1/diagonal
  const double *rho64;  // the finest level's FP64 density (FP32 kernels: w = A u in FP64)
};

__device__ inline int wrap_or_out(int g, int n, int periodic) {
  if (g >= 0 && g < n) return g;
  if (!periodic) return -1;
  return g < 0 ? g + n : g - n;
}

// True when every frame position is a cell with all four neighbours, so
// the sweeps need no boundary tests (periodic directions always qualify).
__device__ inline bool frame_interior(const Bnd &B, int gx0, int gy0, int W, int HH, int nx, int ny) {
  const bool okx = B.periodic[0] || (gx0 > 0 && gx0 + W < nx);
  const bool oky = B.periodic[1] || (gy0 > 0 && gy0 + HH < ny);
  return okx && oky;
}

// Gauss-Seidel value of an interior cell. A cell is updated by its owner and
// by the halos of its neighbours' tiles, and all must get the same bits (the
// single-reduction CG needs w = A u consistent with the stored u): in FP32
// the expression is evaluated exactly as written, without contraction into
// fused multiply-adds.
template <typename T>
__device__ inline T gs5(T b, T xw, T xe, T xs_, T xn, T ihx, T ihy, T idg) {
  return (b + (ihx * (xw + xe) + ihy * (xs_ + xn))) * idg;
}
template <>
__device__ inline float gs5<float>(float b, float xw, float xe, float xs_, float xn, float ihx, float ihy, float idg) {
#pragma clang fp contract(off)
  return (b + (ihx * (xw + xe) + ihy * (xs_ + xn))) * idg;
}

// Gauss-Seidel value at frame offset o, general case: raw global position
// (gx, gy) possibly outside a non-periodic side, in which case the cell does
// not exist (returns false). A cell with all four neighbours takes exactly
// the arithmetic of the interior path (gs5), so that a tile computing it in
// its halo gets the owner's bits whichever path either tile runs.
template <typename T, int W>
__device__ inline bool gs_general(const T *xs, const T *bs, int o, int gx, int gy, int nx, int ny, const Bnd &B,
                                  T ihx, T ihy, T idg, bool zero_nb, T &out) {
  if (!B.periodic[0] && (gx < 0 || gx >= nx)) return false;
  if (!B.periodic[1] && (gy < 0 || gy >= ny)) return false;
  const bool inx = B.periodic[0] || (gx > 0 && gx + 1 < nx);
  const bool iny = B.periodic[1] || (gy > 0 && gy + 1 < ny);
  if (inx && iny) {
    out = zero_nb ? bs[o] * idg : gs5<T>(bs[o], xs[o - 1], xs[o + 1], xs[o - W], xs[o + W], ihx, ihy, idg);
    return true;
  }
  T sx = T(0), sy = T(0);
  int cx = 0, cy = 0;
  if (B.periodic[0] || gx > 0) {
    if (!zero_nb) sx += xs[o - 1];
    ++cx;
  }
  if (B.periodic[0] || gx + 1 < nx) {
    if (!zero_nb) sx += xs[o + 1];
    ++cx;
  }
  if (B.periodic[1] || gy > 0) {
    if (!zero_nb) sy += xs[o - W];
    ++cy;
  }
  if (B.periodic[1] || gy + 1 < ny) {
    if (!zero_nb) sy += xs[o + W];
    ++cy;
  }
  out = (bs[o] + (ihx * sx + ihy * sy)) / (ihx * (T)cx + ihy * (T)cy);
  return true;
}

// (L x) at frame offset o (cell known to exist).
template <typename T, int W, typename A = T>
__device__ inline A lx_general(const T *xs, int o, int gx, int gy, int nx, int ny, const Bnd &B, A ihx, A ihy) {
  A sx = A(0), sy = A(0);
  int cx = 0, cy = 0;
  if (B.periodic[0] || gx > 0) {
    sx += (A)xs[o - 1];
    ++cx;
  }
  if (B.periodic[0] || gx + 1 < nx) {
    sx += (A)xs[o + 1];
    ++cx;
  }
  if (B.periodic[1] || gy > 0) {
    sy += (A)xs[o - W];
    ++cy;
  }
  if (B.periodic[1] || gy + 1 < ny) {
    sy += (A)xs[o + W];
    ++cy;
  }
  return (ihx * (A)cx + ihy * (A)cy) * (A)xs[o] - (ihx * sx + ihy * sy);
}

// Half-sweeps s = S0 .. S1 on shrinking regions [s, W-s) x [s, HH-s) of a
// W x HH frame; colour of half-sweep s is (s + cshift) & 1 (0 = red).
// Cells of one colour are enumerated directly (two per row pair), so the
// loop has compile-time bounds and no parity test.
template <typename T, int W, int HH, int S0, int S1, int CSHIFT>
__device__ inline void sweeps(T *xs, const T *bs, int p0, int gx0, int gy0, int nx, int ny, const Bnd &B, T ihx,
                              T ihy, T idg, bool fast, bool zero_first) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = S0; s <= S1; ++s) {
    const int color = (s + CSHIFT) & 1;
    const int w = W - 2 * s, rows = HH - 2 * s;
    const int half = w / 2;
    const int cnt = half * rows;
    const bool zn = zero_first && s == S0;
    for (int o = tid; o < cnt; o += kBlock) {
      const int ly = s + o / half;
      const int lx = s + 2 * (o % half) + ((color + p0 + ly + s) & 1);
      const int off = ly * W + lx;
      if (fast) {
        if (zn)
          xs[off] = bs[off] * idg;
        else
          xs[off] = gs5<T>(bs[off], xs[off - 1], xs[off + 1], xs[off - W], xs[off + W], ihx, ihy, idg);
      } else {
        T v;
        if (gs_general<T, W>(xs, bs, off, gx0 + lx, gy0 + ly, nx, ny, B, ihx, ihy, idg, zn, v)) xs[off] = v;
      }
    }
    __syncthreads();
  }
}

// ---- variable-coefficient frames (beta = 1/rho_f) --------------------------
// The frame holds, per position, beta of the cell's west face (fx) and
// south face (fy) and 1/diagonal of L (ig), precomputed once per solve for
// the level (k_vc_coef2d), 0 for faces through non-periodic sides and for
// positions outside the grid: one branch-free update then serves interior
// and boundary cells, and leaves missing cells at 0.

// Gauss-Seidel value with face coefficients (evaluated as written, no
// contraction: halo copies of a cell get the owner's bits).
template <typename T>
__device__ inline T gs_vc(T b, T xw, T xe, T xs_, T xn, T bw, T be, T bs_, T bn, T ihx, T ihy, T ig) {
#pragma clang fp contract(off)
  return (b + (ihx * (bw * xw + be * xe) + ihy * (bs_ * xs_ + bn * xn))) * ig;
}

// (L x) at frame offset o with the frame's face coefficients.
template <typename T, int W, typename A = T>
__device__ inline A lx_vc(const T *xs, const T *fx, const T *fy, int o, A ihx, A ihy) {
#pragma clang fp contract(off)
  const A bw = fx[o], be = fx[o + 1], bs_ = fy[o], bn = fy[o + W];
  const A dg = ihx * (bw + be) + ihy * (bs_ + bn);
  return dg * (A)xs[o] -
         (ihx * (bw * (A)xs[o - 1] + be * (A)xs[o + 1]) + ihy * (bs_ * (A)xs[o - W] + bn * (A)xs[o + W]));
}

// FP64 (L u) at an own cell (gx, gy) of the finest level, the face
// coefficients from the FP64 density in global memory, u from the frame.
template <typename T, int W>
__device__ inline double lx_vc64(const T *xs, int o, const double *rho64, const Lay &L, const Bnd &B, int gx, int gy,
                                 double ihx, double ihy) {
#pragma clang fp contract(off)
  const long c = L.at(gx, gy, 0);
  const int nx = L.n[0], ny = L.n[1];
  const long sy = L.s[1];
  const double rc = rho64[c];
  double bw = 0.0, be = 0.0, bs_ = 0.0, bn = 0.0;
  if (B.periodic[0] || gx > 0) bw = face_beta<double>(rc, rho64[gx > 0 ? c - 1 : c + (nx - 1)]);
  if (B.periodic[0] || gx + 1 < nx) be = face_beta<double>(rc, rho64[gx + 1 < nx ? c + 1 : c - (nx - 1)]);
  if (B.periodic[1] || gy > 0) bs_ = face_beta<double>(rc, rho64[gy > 0 ? c - sy : c + (long)(ny - 1) * sy]);
  if (B.periodic[1] || gy + 1 < ny) bn = face_beta<double>(rc, rho64[gy + 1 < ny ? c + sy : c - (long)(ny - 1) * sy]);
  const double dg = ihx * (bw + be) + ihy * (bs_ + bn);
  return dg * (double)xs[o] - (ihx * (bw * (double)xs[o - 1] + be * (double)xs[o + 1]) +
                               ihy * (bs_ * (double)xs[o - W] + bn * (double)xs[o + W]));
}

// Variable-coefficient half-sweeps, same regions and colours as sweeps().
template <typename T, int W, int HH, int S0, int S1, int CSHIFT>
__device__ inline void sweeps_vc(T *xs, const T *bs, const T *fx, const T *fy, const T *ig, int p0, T ihx, T ihy,
                                 bool zero_first) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = S0; s <= S1; ++s) {
    const int color = (s + CSHIFT) & 1;
    const int w = W - 2 * s, rows = HH - 2 * s;
    const int half = w / 2;
    const int cnt = half * rows;
    const bool zn = zero_first && s == S0;
    for (int o = tid; o < cnt; o += kBlock) {
      const int ly = s + o / half;
      const int lx = s + 2 * (o % half) + ((color + p0 + ly + s) & 1);
      const int off = ly * W + lx;
      if (zn)
        xs[off] = bs[off] * ig[off];
      else
        xs[off] = gs_vc<T>(bs[off], xs[off - 1], xs[off + 1], xs[off - W], xs[off + W], fx[off], fx[off + 1], fy[off],
                           fy[off + W], ihx, ihy, ig[off]);
    }
    __syncthreads();
  }
}

// Down: [CG update] + NU red-black sweeps from zero + residual + restriction.
template <typename T, int NU, int TXT, int TYT, bool VC = false>
__global__ void __launch_bounds__(kBlock) k_mg_down2d(Down2DArgs<T> a) {
  static_assert((TXT * TYT) % kBlock == 0 && TXT % 2 == 0 && TYT % 2 == 0, "tile shape");
  constexpr int H = 2 * NU + 1;
  constexpr int W = TXT + 2 * H, HH = TYT + 2 * H;
  constexpr int WV = VC ? W * HH : 1;
  __shared__ T xs[W * HH];
  __shared__ T bs[W * HH];
  __shared__ T fx[WV], fy[WV], ig[WV];
  __shared__ double sh[kBlock / 64];
  if (a.sc->done) return;
  const int nx = a.Lf.n[0], ny = a.Lf.n[1];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int gx0 = (tile % a.tiles_x) * TXT - H, gy0 = (tile / a.tiles_x) * TYT - H;
  const int p0 = (gx0 + gy0) & 1;
  const int tid = threadIdx.x;
  const bool fast = frame_interior(a.B, gx0, gy0, W, HH, nx, ny);
  double alpha = 0.0, beta = 0.0;
  const bool cg = a.finest && a.k >= 1;
  if (cg && a.cgcg) {
    // gamma = r.u, delta = (A u).u, rr = r.r of iteration k-1: convergence
    // test, then alpha and beta of the single-reduction recurrence
    double cc, g, d, rr;
    sum_cc3(a.k, a.part_cc, a.np_cc, a.sc, a.part_g, a.part_g + a.np_g, a.part_g + 2 * a.np_g, a.np_g, cc, g, d, rr);
    const bool conv = (cc == 0.0) || (rr <= a.tol2 * cc);
    if (a.k == 1) {
      alpha = g / d;
    } else {
      beta = g / a.sc->rzh[(a.k - 2) & 1];
      alpha = g / (d - beta * g / a.sc->alh[(a.k - 2) & 1]);
    }
    const bool broken = !isfinite(rr) || !isfinite(alpha) || !isfinite(beta);
    if (blockIdx.x == 0 && tid == 0) {
      a.sc->rzh[(a.k - 1) & 1] = g;
      a.sc->alh[(a.k - 1) & 1] = alpha;
      a.sc->rr = rr;
      a.sc->cc = cc;
      a.sc->iters = a.k - 1;
      if (conv || broken) {
        a.sc->done = 1;
        a.sc->zero = (cc == 0.0);
        a.sc->nonconv = broken && !conv;
      }
    }
    if (conv || broken) return;
  } else if (cg) {
    const double pq = sum_all(a.part_pq, a.np_pq, sh);
    alpha = a.sc->rzh[(a.k - 1) & 1] / pq;
  }
  // right-hand side on the frame minus its outer ring; all loads of the
  // phase are issued before any is used (addresses of absent cells are
  // replaced by a valid one and the value discarded)
  constexpr int NPOS = W * HH;
  constexpr int NIT = (NPOS + kBlock - 1) / kBlock;
  long gi[NIT];
  bool ok[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int o = tid + it * kBlock;
    const int lx = o % W, ly = o / W;
    const bool ring = (lx == 0 || ly == 0 || lx == W - 1 || ly == HH - 1);
    const int gx = wrap_or_out(gx0 + lx, nx, a.B.periodic[0]);
    const int gy = wrap_or_out(gy0 + ly, ny, a.B.periodic[1]);
    ok[it] = o < NPOS && !ring && gx >= 0 && gy >= 0;
    gi[it] = ok[it] ? a.Lf.at(gx, gy, 0) : a.Lf.base;
  }
  if constexpr (VC) {
    // densities on the whole frame (ring included), 0 for missing cells
    // coefficients on the whole frame (ring included), 0 for missing cells;
    // x starts at 0 everywhere (missing cells stay 0)
    T gv[NIT], fv[NIT], hv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int o = tid + it * kBlock;
      const int gx = wrap_or_out(gx0 + o % W, nx, a.B.periodic[0]);
      const int gy = wrap_or_out(gy0 + o / W, ny, a.B.periodic[1]);
      const bool okr = o < NPOS && gx >= 0 && gy >= 0;
      const long id = okr ? a.Lf.at(gx, gy, 0) : a.Lf.base;
      gv[it] = a.cig[id];
      fv[it] = a.cfx[id];
      hv[it] = a.cfy[id];
      if (!okr) gv[it] = fv[it] = hv[it] = T(0);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int o = tid + it * kBlock;
      if (o < NPOS) {
        ig[o] = gv[it];
        fx[o] = fv[it];
        fy[o] = hv[it];
        xs[o] = T(0);
      }
    }
  }
  if (a.finest && cg && a.cgcg) {
    // r_k = r_{k-1} - alpha (w + beta s_{k-2}) on the frame
    const double *rb = (const double *)a.b;
    const bool old = a.k >= 2;
    double rv[NIT], wv[NIT], sv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      rv[it] = rb[gi[it]];
      wv[it] = a.w[gi[it]];
      sv[it] = old ? a.s_old[gi[it]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int o = tid + it * kBlock;
      if (o < NPOS) bs[o] = ok[it] ? (T)(rv[it] - alpha * (wv[it] + beta * sv[it])) : T(0);
    }
    // own cells: p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
    constexpr int NOWN = TXT * TYT / kBlock;
    long oi[NOWN];
    double ro[NOWN], wo[NOWN], so[NOWN], xo[NOWN], po[NOWN];
    T uo[NOWN];
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      const int o = tid + u * kBlock;
      oi[u] = a.Lf.at(gx0 + H + o % TXT, gy0 + H + o / TXT, 0);
    }
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      ro[u] = rb[oi[u]];
      wo[u] = a.w[oi[u]];
      so[u] = old ? a.s_old[oi[u]] : 0.0;
      po[u] = old ? a.p_io[oi[u]] : 0.0;
      xo[u] = a.x[oi[u]];
      uo[u] = a.u[oi[u]];
    }
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      const double pn = (double)uo[u] + beta * po[u];
      const double sn = wo[u] + beta * so[u];
      a.p_io[oi[u]] = pn;
      a.s_new[oi[u]] = sn;
      a.x[oi[u]] = xo[u] + alpha * pn;
      a.rnew[oi[u]] = ro[u] - alpha * (wo[u] + beta * so[u]);
    }
  } else if (a.finest) {
    const double *rb = (const double *)a.b;
    double rv[NIT], qv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      rv[it] = rb[gi[it]];
      qv[it] = cg ? a.q[gi[it]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int o = tid + it * kBlock;
      if (o < NPOS) bs[o] = ok[it] ? (T)(rv[it] - alpha * qv[it]) : T(0);
    }
    if (cg) {  // CG update of the tile's own cells
      constexpr int NOWN = TXT * TYT / kBlock;
      long oi[NOWN];
      double ro[NOWN], qo[NOWN], xo[NOWN], po[NOWN];
#pragma unroll
      for (int u = 0; u < NOWN; ++u) {
        const int o = tid + u * kBlock;
        oi[u] = a.Lf.at(gx0 + H + o % TXT, gy0 + H + o / TXT, 0);
      }
#pragma unroll
      for (int u = 0; u < NOWN; ++u) {
        ro[u] = rb[oi[u]];
        qo[u] = a.q[oi[u]];
        xo[u] = a.x[oi[u]];
        po[u] = a.p[oi[u]];
      }
#pragma unroll
      for (int u = 0; u < NOWN; ++u) {
        a.rnew[oi[u]] = ro[u] - alpha * qo[u];
        a.x[oi[u]] = xo[u] + alpha * po[u];
      }
    }
  } else {
    const T *bb = (const T *)a.b;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) v[it] = bb[gi[it]];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int o = tid + it * kBlock;
      if (o < NPOS) bs[o] = ok[it] ? v[it] : T(0);
    }
  }
  __syncthreads();
  // zero initial guess: the first (red) half-sweep reads no neighbours, and
  // every later half-sweep only reads cells updated before it
  if constexpr (VC) {
    sweeps_vc<T, W, HH, 1, 2 * NU, 1>(xs, bs, fx, fy, ig, p0, a.ihx, a.ihy, true);
  } else {
    sweeps<T, W, HH, 1, 2 * NU, 1>(xs, bs, p0, gx0, gy0, nx, ny, a.B, a.ihx, a.ihy, a.idg, fast, true);
  }
  for (int o = tid; o < TXT * TYT; o += kBlock) {
    const int lx = H + o % TXT, ly = H + o / TXT;
    a.xpre[a.Lf.at(gx0 + lx, gy0 + ly, 0)] = xs[ly * W + lx];
  }
  for (int o = tid; o < (TXT / 2) * (TYT / 2); o += kBlock) {
    const int cx = o % (TXT / 2), cy = o / (TXT / 2);
    T acc = T(0);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int lx = H + 2 * cx + dx, ly = H + 2 * cy + dy;
        const int off = ly * W + lx;
        T Lx;
        if constexpr (VC)
          Lx = lx_vc<T, W>(xs, fx, fy, off, a.ihx, a.ihy);
        else if (fast)
          Lx = (T(2) * (a.ihx + a.ihy)) * xs[off] - (a.ihx * (xs[off - 1] + xs[off + 1]) + a.ihy * (xs[off - W] + xs[off + W]));
        else
          Lx = lx_general<T, W>(xs, off, gx0 + lx, gy0 + ly, nx, ny, a.B, a.ihx, a.ihy);
        acc += bs[off] - Lx;
      }
    const int Cx = (gx0 + H) / 2 + cx, Cy = (gy0 + H) / 2 + cy;
    a.bc[a.Lc.at(Cx, Cy, 0)] = acc * T(0.25);
  }
}

// Up: prolongation + NU black-red sweeps; finest level: r.z, r.r partials.
// With EXTRA = 1 the frame carries one more halo ring, so the smoothed u is
// valid one cell beyond the tile and w = A u is formed for the tile
// (single-reduction CG: partials of r.u, w.u and r.r).
template <typename T, int NU, int EXTRA, int TXT, int TYT, bool VC = false>
__global__ void __launch_bounds__(kBlock) k_mg_up2d(Up2DArgs<T> a) {
  static_assert((TXT * TYT) % kBlock == 0 && TXT % 2 == 0 && TYT % 2 == 0, "tile shape");
  constexpr int H = 2 * NU + EXTRA;
  constexpr int W = TXT + 2 * H, HH = TYT + 2 * H;
  constexpr int WV = VC ? W * HH : 1;
  __shared__ T xs[W * HH];
  __shared__ T bs[W * HH];
  __shared__ T fx[WV], fy[WV], ig[WV];
  if (a.sc->done) return;
  const int nx = a.Lf.n[0], ny = a.Lf.n[1];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int gx0 = (tile % a.tiles_x) * TXT - H, gy0 = (tile / a.tiles_x) * TYT - H;
  const int p0 = (gx0 + gy0) & 1;
  const int tid = threadIdx.x;
  const bool fast = frame_interior(a.B, gx0, gy0, W, HH, nx, ny);
  constexpr int NPOS = W * HH;
  constexpr int NIT = (NPOS + kBlock - 1) / kBlock;
  long gi[NIT], ci[NIT];
  bool okx[NIT], okb[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int o = tid + it * kBlock;
    const int lx = o % W, ly = o / W;
    const int gx = wrap_or_out(gx0 + lx, nx, a.B.periodic[0]);
    const int gy = wrap_or_out(gy0 + ly, ny, a.B.periodic[1]);
    const bool ring = (lx == 0 || ly == 0 || lx == W - 1 || ly == HH - 1);
    okx[it] = o < NPOS && gx >= 0 && gy >= 0;
    okb[it] = okx[it] && !ring;
    gi[it] = okx[it] ? a.Lf.at(gx, gy, 0) : a.Lf.base;
    ci[it] = okx[it] ? a.Lc.at(gx >> 1, gy >> 1, 0) : a.Lc.base;
  }
  constexpr int NV = VC ? NIT : 1;
  T xv[NIT], cv[NIT], bv[NIT], gv[NV], fv[NV], hv[NV];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    xv[it] = a.xpre[gi[it]];
    cv[it] = a.xc[ci[it]];
    bv[it] = a.finest ? (T)((const double *)a.b)[gi[it]] : ((const T *)a.b)[gi[it]];
    if constexpr (VC) {
      gv[it] = a.cig[gi[it]];
      fv[it] = a.cfx[gi[it]];
      hv[it] = a.cfy[gi[it]];
    }
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int o = tid + it * kBlock;
    if (o < NPOS) {
      xs[o] = okx[it] ? xv[it] + cv[it] : T(0);
      bs[o] = okb[it] ? bv[it] : T(0);
      if constexpr (VC) {
        ig[o] = okx[it] ? gv[it] : T(0);
        fx[o] = okx[it] ? fv[it] : T(0);
        fy[o] = okx[it] ? hv[it] : T(0);
      }
    }
  }
  __syncthreads();
  // regions shrink from the frame edge, so with the extra ring the last
  // half-sweep leaves u valid on the tile plus one cell
  if constexpr (VC) {
    sweeps_vc<T, W, HH, 1, 2 * NU, 0>(xs, bs, fx, fy, ig, p0, a.ihx, a.ihy, false);
  } else {
    sweeps<T, W, HH, 1, 2 * NU, 0>(xs, bs, p0, gx0, gy0, nx, ny, a.B, a.ihx, a.ihy, a.idg, fast, false);
  }
  double rz = 0.0, rr = 0.0, rzo = 0.0;
  constexpr int NOWN = TXT * TYT / kBlock;
  long oi[NOWN];
  T zv[NOWN];
#pragma unroll
  for (int u = 0; u < NOWN; ++u) {
    const int o = tid + u * kBlock;
    const int lx = H + o % TXT, ly = H + o / TXT;
    oi[u] = a.Lf.at(gx0 + lx, gy0 + ly, 0);
    zv[u] = xs[ly * W + lx];
    a.xout[oi[u]] = zv[u];
  }
  if (EXTRA && a.finest) {
    double rv[NOWN];
#pragma unroll
    for (int u = 0; u < NOWN; ++u) rv[u] = ((const double *)a.b)[oi[u]];
    double ru = 0.0, wu = 0.0;
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      const int o = tid + u * kBlock;
      const int lx = H + o % TXT, ly = H + o / TXT;
      const int off = ly * W + lx;
      double Lu;
      if constexpr (VC) {
        if constexpr (sizeof(T) == 8)
          Lu = lx_vc<T, W, double>(xs, fx, fy, off, a.dihx, a.dihy);
        else
          Lu = lx_vc64<T, W>(xs, off, a.rho64, a.Lf, a.B, gx0 + lx, gy0 + ly, a.dihx, a.dihy);
      } else if (fast) {
        Lu = (2.0 * (a.dihx + a.dihy)) * (double)xs[off] -
             (a.dihx * ((double)xs[off - 1] + (double)xs[off + 1]) + a.dihy * ((double)xs[off - W] + (double)xs[off + W]));
      } else {
        Lu = lx_general<T, W, double>(xs, off, gx0 + lx, gy0 + ly, nx, ny, a.B, a.dihx, a.dihy);
      }
      const double wv = Lu;
      a.w[oi[u]] = wv;
      ru += rv[u] * (double)zv[u];
      wu += wv * (double)zv[u];
      rr += rv[u] * rv[u];
    }
    double v3[3] = {ru, wu, rr};
    block_allsum_n<3>(v3);
    if (linear_tid() == 0) {
      a.part_rz[blockIdx.x] = v3[0];
      a.part_rz[a.np + blockIdx.x] = v3[1];
      a.part_rz[2 * a.np + blockIdx.x] = v3[2];
    }
    return;
  }
  if (a.finest) {
    double rv[NOWN];
    T zo[NOWN];
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      rv[u] = ((const double *)a.b)[oi[u]];
      zo[u] = a.zold ? a.zold[oi[u]] : T(0);
    }
#pragma unroll
    for (int u = 0; u < NOWN; ++u) {
      rz += rv[u] * (double)zv[u];
      rr += rv[u] * rv[u];
      rzo += rv[u] * (double)zo[u];
    }
  }
  if (a.finest) {
    double v3[3] = {rz, rr, rzo};  // rzo stays 0 without z_old
    block_allsum_n<3>(v3);
    if (linear_tid() == 0) {
      a.part_rz[blockIdx.x] = v3[0];
      a.part_rz[a.np + blockIdx.x] = v3[1];
      a.part_rz[2 * a.np + blockIdx.x] = v3[2];
    }
  }
}

// ---------------------------------------------------------------------------
// One-block coarse V-cycle in LDS
// ---------------------------------------------------------------------------
constexpr int kCoarseLds = 5504;  // cells of all coarse levels together (4096 + 1024 + ... in 2D)
constexpr int kCoarseLoads = 4;   // cells per thread of the first coarse level (<= 4 x 1024)
constexpr int kCoarseLev = 8;     // coarse levels handled by the one-block kernel, at most

template <typename T>
struct CoarseArgs {
  int l0, nlev, nu;
  Bnd B;
  int n[kMaxLev][3];
  int off[kMaxLev];        // LDS offset of each level (compact, x fastest)
  int lg[kMaxLev][2];      // log2(n[0]/2), log2(n[1]) or -1 when not a power of two
  Ih2<T> ih2[kMaxLev];
  T idg[kCoarseLev][8];    // 1/diagonal of coarse level l0 + q, by neighbour code
  Lay L0;                  // global layout of level l0
  const void *b0;          // global right-hand side of level l0
  int b0_double;
  T *x0;                   // global output: correction of level l0
  const T *pinv;           // dense pseudo-inverse of the coarsest level
  const T *rho_c;          // variable coefficients: densities of levels l0.., packed at off[]
  int met = 0;             // stretched 2D grid: rho_c holds dx/dy (face_coef)
  // stretched 2D grid: per level l >= l0 at toff[l] the cell widths wx[n0],
  // wy[n1] and the face factors gx[n0], gy[n1] (g = 2 / (sum of the two
  // widths across the face; the last face wraps when periodic, else 0)
  const T *mtab = nullptr;
  int mtab_n = 0;
  int toff[kMaxLev];
};

// Stretched 2D grid: the four face coefficients (west, east, south, north)
// of cell (i, j) of a level from its 1D tables: an x-face carries the
// cell height over the distance between the two centres, dy_j 2/(dx_a +
// dx_b), a y-face dx_i 2/(dy_a + dy_b), each times the level's scale.
// Faces on a wall get 0 from the table.
template <typename T>
__device__ inline void m_faces(const T *tab, int toff, int n0, int n1, int i, int j, T ihx, T ihy, T cf[4]) {
  const T *wx = tab + toff, *wy = wx + n0, *gx = wy + n1, *gy = gx + n0;
  const int im = i > 0 ? i - 1 : n0 - 1, jm = j > 0 ? j - 1 : n1 - 1;
  const T ay = ihx * wy[j], ax = ihy * wx[i];
  cf[0] = ay * gx[im];
  cf[1] = ay * gx[i];
  cf[2] = ax * gy[jm];
  cf[3] = ax * gy[j];
}

template <int DIM, typename T>
__device__ inline void c_decode(const int n[3], int t, int &i, int &j, int &k) {
  const int n0 = n[0], n1 = n[1];
  int row;
  if ((n0 & (n0 - 1)) == 0) {
    i = t & (n0 - 1);
    row = t >> __builtin_ctz(n0);
  } else {
    row = t / n0;
    i = t - row * n0;
  }
  if (DIM == 3) {
    if ((n1 & (n1 - 1)) == 0) {
      j = row & (n1 - 1);
      k = row >> __builtin_ctz(n1);
    } else {
      k = row / n1;
      j = row - k * n1;
    }
  } else {
    j = row;
    k = 0;
  }
}

// Sum of the neighbours of cell c = (i, j, k), each scaled by 1/h_d^2, with
// no branches: a missing neighbour (a non-periodic side) is read at c and
// weighted 0. code gets bit d set when both neighbours along d exist; the
// diagonal of the cell is sum_d ih2[d] (1 + bit d), tabulated as 1/diag.
template <int DIM, typename T>
__device__ inline T c_nbs(const int n[3], const Bnd &B, const T ih2[3], const T *x, int i, int j, int k, int c,
                          int &code) {
  const int q[3] = {i, j, k};
  const int st[3] = {1, n[0], n[0] * n[1]};
  T v[2 * DIM], w[2 * DIM];
  code = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool per = B.periodic[d] != 0;
    const bool lo = q[d] > 0, hi = q[d] + 1 < n[d];
    const int cm = lo ? c - st[d] : (per ? c + (n[d] - 1) * st[d] : c);
    const int cp = hi ? c + st[d] : (per ? c - (n[d] - 1) * st[d] : c);
    v[2 * d] = x[cm];
    v[2 * d + 1] = x[cp];
    w[2 * d] = (lo || per) ? T(1) : T(0);
    w[2 * d + 1] = (hi || per) ? T(1) : T(0);
    code |= ((lo || per) && (hi || per)) ? (1 << d) : 0;
  }
  T nbs = T(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) nbs += ih2[d] * (w[2 * d] * v[2 * d] + w[2 * d + 1] * v[2 * d + 1]);
  return nbs;
}

// q = t / n, r = t % n with a shift when lg >= 0 (n = 2^lg).
__device__ inline int c_divmod(int t, int n, int lg, int &r) {
  if (lg >= 0) {
    r = t & (n - 1);
    return t >> lg;
  }
  const int q = t / n;
  r = t - q * n;
  return q;
}

// Cell of colour `color` number t of level l (even n[0]): the cells of one
// colour are enumerated directly, i = 2m + ((colour + j + k) & 1).
template <int DIM, typename T>
__device__ inline int c_colour_cell(const CoarseArgs<T> &a, int l, int color, int t, int &i, int &j, int &k) {
  const int *n = a.n[l];
  int m;
  k = 0;
  const int row = c_divmod(t, n[0] >> 1, a.lg[l][0], m);
  if (DIM == 3)
    k = c_divmod(row, n[1], a.lg[l][1], j);
  else
    j = row;
  i = 2 * m + ((color + j + k) & 1);
  return i + n[0] * (j + n[1] * k);
}

// The cells of one colour of level l that this thread updates (at most
// two: a level has at most kCoarseCells cells, 2 x 1024 per colour), with
// the LDS indices of their neighbours and their inverse diagonals, set up
// once per level and reused by every sweep. A missing neighbour (a
// non-periodic side) points at a zero slot of the LDS array.
template <int DIM, typename T>
struct CSet {
  int c[2];             // LDS index of the cell, -1 when the slot is empty
  int nb[2][2 * DIM];   // LDS indices of the neighbours (-d, +d per direction)
  T idg[2];             // 1 / diagonal
  int ij[2];            // stretched grid: i | j << 16 of the cell
};

// beta / h_d^2 of the face between LDS cells ia and ib, from the densities
// rs in LDS (ib == zero_slot: no face). Evaluated where it is used (the
// coarse levels are small and their sweeps latency bound), so the cell sets
// hold no coefficients and stay in registers.
template <typename T>
__device__ inline T c_face(const T *rs, int ia, int ib, int zero_slot, T ih2, int d, int met) {
  return ib == zero_slot ? T(0) : ih2 * face_coef<T>(rs[ia], rs[ib], d, met);
}

template <int DIM, typename T, bool VC = false, bool MET = false>
__device__ inline void c_set(const CoarseArgs<T> &a, const T *idg_s, const T *rs, int l, int color, int zero_slot,
                             CSet<DIM, T> &s, int tid) {
  const int *n = a.n[l];
  const int N = (n[0] >> 1) * n[1] * n[2];
  const int off = a.off[l];
  const int st[3] = {1, n[0], n[0] * n[1]};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int t = tid + q * blockDim.x;
    s.c[q] = -1;
    if (t >= N) continue;
    int i, j, k;
    const int c = c_colour_cell<DIM, T>(a, l, color, t, i, j, k);
    const int qd[3] = {i, j, k};
    int code = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool per = a.B.periodic[d] != 0;
      const bool lo = qd[d] > 0, hi = qd[d] + 1 < n[d];
      s.nb[q][2 * d] = lo ? off + c - st[d] : (per ? off + c + (n[d] - 1) * st[d] : zero_slot);
      s.nb[q][2 * d + 1] = hi ? off + c + st[d] : (per ? off + c - (n[d] - 1) * st[d] : zero_slot);
      code |= ((lo || per) && (hi || per)) ? (1 << d) : 0;
    }
    s.c[q] = off + c;
    if constexpr (MET) {
      T cf[4];
      m_faces<T>(rs, a.toff[l], n[0], n[1], i, j, a.ih2[l].v[0], a.ih2[l].v[1], cf);
      s.idg[q] = T(1) / (((cf[0] + cf[1]) + cf[2]) + cf[3]);
      s.ij[q] = i | (j << 16);
    } else if constexpr (VC) {
      T dg = T(0);
#pragma unroll
      for (int m = 0; m < 2 * DIM; ++m)
        dg += c_face<T>(rs, off + c, s.nb[q][m], zero_slot, a.ih2[l].v[m >> 1], m >> 1, a.met);
      s.idg[q] = T(1) / dg;
    } else {
      s.idg[q] = idg_s[8 * (l - a.l0) + code];
    }
  }
}

// One red/black half-sweep over a cell set: x = (b + sum of neighbours) /
// diag, all LDS reads of the thread issued before the arithmetic.
// (A missing neighbour is the zero slot: x = 0 there, so its term vanishes
// whatever the coefficient.)
template <int DIM, typename T, bool VC = false, bool MET = false>
__device__ inline void c_sweep(T *xs, const T *bs, const T *rs, const CSet<DIM, T> &s, const T ih2[3],
                               bool zero_init, int met, int toff = 0, int n0 = 0, int n1 = 0) {
  if constexpr (MET) {
    // stretched 2D grid: coefficients from the level's 1D tables
    T v[2][4] = {}, bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (s.c[q] < 0) continue;
      if (!zero_init)
#pragma unroll
        for (int m = 0; m < 4; ++m) v[q][m] = xs[s.nb[q][m]];
      bv[q] = bs[s.c[q]];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (s.c[q] < 0) continue;
      T cf[4];
      m_faces<T>(rs, toff, n0, n1, s.ij[q] & 0xffff, s.ij[q] >> 16, ih2[0], ih2[1], cf);
      T nbs = ((cf[0] * v[q][0] + cf[1] * v[q][1]) + cf[2] * v[q][2]) + cf[3] * v[q][3];
      if (zero_init) nbs = T(0);
      xs[s.c[q]] = (bv[q] + nbs) * s.idg[q];
    }
    __syncthreads();
    return;
  }
  if constexpr (VC && DIM == 3) {
    // one cell at a time (fewer live registers); cells of one colour read
    // only the other colour, so each result is stored at once
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (s.c[q] < 0) continue;
      const T rc = rs[s.c[q]];
      T nbs = T(0);
#pragma unroll
      for (int m = 0; m < 2 * DIM; ++m) {
        const int nb = s.nb[q][m];
        nbs += (ih2[m >> 1] * face_coef<T>(rc, rs[nb], m >> 1, met)) * xs[nb];
      }
      if (zero_init) nbs = T(0);
      xs[s.c[q]] = (bs[s.c[q]] + nbs) * s.idg[q];
    }
    __syncthreads();
    return;
  }
  T v[2][2 * DIM] = {}, bv[2], rv[2][VC ? 2 * DIM + 1 : 1];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (s.c[q] < 0) continue;
    if (!zero_init)  // a sweep from zero reads no neighbours
#pragma unroll
      for (int m = 0; m < 2 * DIM; ++m) v[q][m] = xs[s.nb[q][m]];
    bv[q] = bs[s.c[q]];
    if constexpr (VC) {
#pragma unroll
      for (int m = 0; m < 2 * DIM; ++m) rv[q][m] = rs[s.nb[q][m]];
      rv[q][2 * DIM] = rs[s.c[q]];
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (s.c[q] < 0) continue;
    T nbs = T(0);
    if constexpr (VC) {
#pragma unroll
      for (int m = 0; m < 2 * DIM; ++m)
        nbs += (ih2[m >> 1] * face_coef<T>(rv[q][2 * DIM], rv[q][m], m >> 1, met)) * v[q][m];
    } else {
#pragma unroll
      for (int d = 0; d < DIM; ++d) nbs += ih2[d] * (v[q][2 * d] + v[q][2 * d + 1]);
    }
    if (zero_init) nbs = T(0);
    xs[s.c[q]] = (bv[q] + nbs) * s.idg[q];
  }
  __syncthreads();
}

// The V-cycle over levels l0 .. nlev-1 out of LDS: the right-hand side of
// level l0 is in bs at off[l0] (the coarser levels' parts are written
// here), the correction of every level ends in xs, that of level l0 at
// off[l0]. rs holds the levels' densities (VC), idg_s the inverse
// diagonals by neighbour code; xs[zero_slot] = 0; tid is threadIdx.x (a
// caller that runs the cycle in a loop passes it through an opaque copy,
// so the per-level cell sets are recomputed, not held across iterations).
// Ends with a barrier.
template <int DIM, typename T, bool VC, bool MET = false>
__device__ __attribute__((always_inline)) inline void coarse_cycle(const CoarseArgs<T> &a, T *xs, T *bs, const T *rs,
                                                                   const T *idg_s, int zero_slot,
                                                                   int tid) {
  const int last = a.nlev - 1;
  for (int l = a.l0; l < last; ++l) {
    {
      CSet<DIM, T> red, black;
      c_set<DIM, T, VC, MET>(a, idg_s, rs, l, 0, zero_slot, red, tid);
      c_set<DIM, T, VC, MET>(a, idg_s, rs, l, 1, zero_slot, black, tid);
      for (int s = 0; s < a.nu; ++s) {
        c_sweep<DIM, T, VC, MET>(xs, bs, rs, red, a.ih2[l].v, s == 0, a.met, a.toff[l], a.n[l][0], a.n[l][1]);
        c_sweep<DIM, T, VC, MET>(xs, bs, rs, black, a.ih2[l].v, false, a.met, a.toff[l], a.n[l][0], a.n[l][1]);
      }
    }
    const int *nf = a.n[l], *nc = a.n[l + 1];
    const int Nc = nc[0] * nc[1] * nc[2];
    const T *x = xs + a.off[l];
    const T *b = bs + a.off[l];

    // After the last black half-sweep the black cells' residuals vanish
    // (each was just solved for with its red neighbours final), so only the
    // red children (dx + dy + dz even) are summed (nu >= 1 always).
    for (int t = tid; t < Nc; t += blockDim.x) {
      int I, J, K;
      c_decode<DIM, T>(nc, t, I, J, K);
      T acc = T(0);
      constexpr int kUnroll = VC ? 1 : 2;
#pragma unroll kUnroll
      for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll kUnroll
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = (dy + dz) & 1; dx < 2; dx += 2) {
            const int i = 2 * I + dx, j = 2 * J + dy, k = DIM == 3 ? 2 * K + dz : 0;
            const int c = i + nf[0] * (j + nf[1] * k);
            if constexpr (MET) {
              const int off = a.off[l];
              const bool pxp = a.B.periodic[0] != 0, pyp = a.B.periodic[1] != 0;
              const int iw = i > 0 ? off + c - 1 : (pxp ? off + c + nf[0] - 1 : zero_slot);
              const int ie = i + 1 < nf[0] ? off + c + 1 : (pxp ? off + c - (nf[0] - 1) : zero_slot);
              const int is = j > 0 ? off + c - nf[0] : (pyp ? off + c + (nf[1] - 1) * nf[0] : zero_slot);
              const int in = j + 1 < nf[1] ? off + c + nf[0] : (pyp ? off + c - (nf[1] - 1) * nf[0] : zero_slot);
              T cf[4];
              m_faces<T>(rs, a.toff[l], nf[0], nf[1], i, j, a.ih2[l].v[0], a.ih2[l].v[1], cf);
              const T nbs = ((cf[0] * xs[iw] + cf[1] * xs[ie]) + cf[2] * xs[is]) + cf[3] * xs[in];
              const T dg = ((cf[0] + cf[1]) + cf[2]) + cf[3];
              acc += b[c] - (dg * x[c] - nbs);
            } else if constexpr (VC) {
              // same neighbour rules and coefficients as c_set
              const int q[3] = {i, j, k};
              const int st[3] = {1, nf[0], nf[0] * nf[1]};
              const int off = a.off[l];
              T nbs = T(0), dg = T(0);
#pragma unroll
              for (int d = 0; d < DIM; ++d) {
                const bool per = a.B.periodic[d] != 0;
                const bool lo = q[d] > 0, hi = q[d] + 1 < nf[d];
                const int im = lo ? off + c - st[d] : (per ? off + c + (nf[d] - 1) * st[d] : zero_slot);
                const int ip = hi ? off + c + st[d] : (per ? off + c - (nf[d] - 1) * st[d] : zero_slot);
                const T bm = c_face<T>(rs, off + c, im, zero_slot, a.ih2[l].v[d], d, a.met);
                const T bp = c_face<T>(rs, off + c, ip, zero_slot, a.ih2[l].v[d], d, a.met);
                nbs += bm * xs[im] + bp * xs[ip];
                dg += bm + bp;
              }
              acc += b[c] - (dg * x[c] - nbs);
            } else {
              int code;
              const T nbs = c_nbs<DIM, T>(nf, a.B, a.ih2[l].v, x, i, j, k, c, code);
              T dg = T(0);
#pragma unroll
              for (int d = 0; d < DIM; ++d) dg += a.ih2[l].v[d] * ((code >> d) & 1 ? T(2) : T(1));
              acc += b[c] - (dg * x[c] - nbs);
            }
          }
      bs[a.off[l + 1] + t] = acc * (DIM == 3 ? T(0.125) : T(0.25));
    }
    __syncthreads();
  }
  {
    // x = pinv b on the coarsest level: 16 lanes per row, each summing a
    // strided quarter-row share (coalesced: a wavefront reads four row
    // segments), then a 16-lane xor-shuffle sum; rows beyond the block's
    // 64 groups of 16 are taken in further rounds.
    const int *n = a.n[last];
    const int N = n[0] * n[1] * n[2];
    const T *bl = bs + a.off[last];
    const int part = tid & 15, ngroups = blockDim.x >> 4;
    for (int r = tid >> 4; r - (tid >> 4) < N; r += ngroups) {  // uniform trip count per wavefront
      T acc = T(0);
      if (r < N) {
        const T *row = a.pinv + (long)r * N;
        for (int col = part; col < N; col += 16) acc += row[col] * bl[col];
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
      if (part == 0 && r < N) xs[a.off[last] + r] = acc;
    }
    __syncthreads();
  }
  for (int l = last - 1; l >= a.l0; --l) {
    const int *nf = a.n[l], *nc = a.n[l + 1];
    const int N = nf[0] * nf[1] * nf[2];
    {
      // piecewise-constant prolongation to the red cells: the first
      // post-smoothing half-sweep solves every black cell from its red
      // neighbours, so the black cells' corrected values would be discarded
      const int Nr = N >> 1;
      T xf[2], xc[2];
      int cf_[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int t = tid + q * blockDim.x;
        cf_[q] = -1;
        if (t >= Nr) continue;
        int i, j, k;
        const int c = c_colour_cell<DIM, T>(a, l, 0, t, i, j, k);
        const int pc = (i >> 1) + nc[0] * ((j >> 1) + nc[1] * (DIM == 3 ? (k >> 1) : 0));
        cf_[q] = a.off[l] + c;
        xf[q] = xs[cf_[q]];
        xc[q] = xs[a.off[l + 1] + pc];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (cf_[q] >= 0) xs[cf_[q]] = xf[q] + xc[q];
    }
    __syncthreads();
    CSet<DIM, T> red, black;
    c_set<DIM, T, VC, MET>(a, idg_s, rs, l, 0, zero_slot, red, tid);
    c_set<DIM, T, VC, MET>(a, idg_s, rs, l, 1, zero_slot, black, tid);
    for (int s = 0; s < a.nu; ++s) {
      c_sweep<DIM, T, VC, MET>(xs, bs, rs, black, a.ih2[l].v, false, a.met, a.toff[l], a.n[l][0], a.n[l][1]);
      c_sweep<DIM, T, VC, MET>(xs, bs, rs, red, a.ih2[l].v, false, a.met, a.toff[l], a.n[l][0], a.n[l][1]);
    }
  }
}

template <int DIM, typename T, bool VC = false, bool MET = false>
__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(CoarseArgs<T> a, const SolverScalars *sc) {
  __shared__ T xs[kCoarseLds + 1];     // all coarse levels, then a zero slot
  __shared__ T bs[kCoarseLds];
  __shared__ T idg_s[kCoarseLev * 8];  // inverse diagonals, read with a per-cell index
  __shared__ T rs[VC ? kCoarseLds + 1 : 1];  // densities of all coarse levels (variable coefficients)
  if (sc->done) return;
  const int last = a.nlev - 1;
  const int zero_slot = kCoarseLds;
  (void)last;
  if (threadIdx.x < kCoarseLev * 8) idg_s[threadIdx.x] = a.idg[threadIdx.x >> 3][threadIdx.x & 7];
  if (threadIdx.x == 0) xs[zero_slot] = T(0);
  if constexpr (MET) {
    for (int t = threadIdx.x; t < a.mtab_n; t += blockDim.x) rs[t] = a.mtab[t];
  } else if constexpr (VC) {
    const int ntot = a.off[last] + a.n[last][0] * a.n[last][1] * a.n[last][2];
    for (int t = threadIdx.x; t < ntot; t += blockDim.x) rs[t] = a.rho_c[t];
    if (threadIdx.x == 0) rs[zero_slot] = T(1);
  }
  {
    // all loads of the right-hand side issued before any is used
    const int *n = a.n[a.l0];
    const int N = n[0] * n[1] * n[2];
    T v[kCoarseLoads];
#pragma unroll
    for (int q = 0; q < kCoarseLoads; ++q) {
      const int t = threadIdx.x + q * blockDim.x;
      v[q] = T(0);
      if (t < N) {
        int i, j, k;
        c_decode<DIM, T>(n, t, i, j, k);
        const long g = a.L0.at(i, j, k);
        v[q] = a.b0_double ? (T)((const double *)a.b0)[g] : ((const T *)a.b0)[g];
      }
    }
#pragma unroll
    for (int q = 0; q < kCoarseLoads; ++q) {
      const int t = threadIdx.x + q * blockDim.x;
      if (t < N) bs[a.off[a.l0] + t] = v[q];
    }
    __syncthreads();
  }
  coarse_cycle<DIM, T, VC, MET>(a, xs, bs, rs, idg_s, zero_slot, threadIdx.x);
  {
    const int *n = a.n[a.l0];
    const int N = n[0] * n[1] * n[2];
#pragma unroll
    for (int q = 0; q < kCoarseLoads; ++q) {
      const int t = threadIdx.x + q * blockDim.x;
      if (t >= N) continue;
      int i, j, k;
      c_decode<DIM, T>(n, t, i, j, k);
      a.x0[a.L0.at(i, j, k)] = xs[a.off[a.l0] + t];
    }
  }
}

}  // namespace lm
