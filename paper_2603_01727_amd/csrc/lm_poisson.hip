// Pressure Poisson solver: preconditioned conjugate gradients on the
// singular, symmetric operator L = -A, A P = sum_d delta_1 delta_1 P (the
// discrete continuity constraint Eq 3.24 with the face flux of Eq 3.23;
// zero flux through non-periodic sides, section 3.3). The preconditioner is
// one symmetric geometric multigrid V-cycle: red-black Gauss-Seidel
// (red-black down, black-red up), 2^d-cell averaging restriction,
// piecewise-constant prolongation, rediscretised coarse operators and an
// exact pseudo-inverse on the coarsest grid, so the zero-mean solution is
// obtained as with the augmented-matrix method the paper uses. In mixed mode
// the V-cycle runs in FP32 and CG (flexible, Polak-Ribiere beta) in FP64.
//
// Every iteration is a fixed sequence of kernels that reads a device-side
// `done` flag and exits at once when it is set; scalars (alpha, beta, norms)
// stay on the device and are finished by the last block of each reduction.
// The host enqueues iterations in batches and reads the flag once per batch.
#include <cmath>
#include <vector>

#include "lm_device.h"

namespace lm {

constexpr int kCoarseThreads = 1024;

Lay make_layout(int ndim, const int n[3], int elem_bytes) {
  Lay L;
  L.ndim = ndim;
  const int align = 128 / elem_bytes;  // elements per 128-byte line
  for (int d = 0; d < 3; ++d) L.n[d] = d < ndim ? n[d] : 1;
  const long px = ((long)(L.n[0] + 2) + align - 1) / align * align;
  const long py = L.n[1] + 2;
  L.s[0] = 1;
  L.s[1] = px;
  L.s[2] = ndim == 3 ? px * py : 0;
  const long planes = ndim == 3 ? L.n[2] + 2 : 1;
  long b0 = 1 + px + (ndim == 3 ? L.s[2] : 0);
  const long shift = (align - (b0 % align)) % align;
  L.base = b0 + shift;
  L.total = shift + px * py * planes + align;
  return L;
}

// ---------------------------------------------------------------------------
// Operator pieces: neighbour sum and diagonal of L = -A at one cell
// ---------------------------------------------------------------------------
template <int DIM, typename A, typename T>
__device__ inline void op_parts(const Lay &L, const Bnd &B, const A ih2[3], const T *x, int i, int j, int k,
                                long c, A &nbsum, A &diag) {
  nbsum = A(0);
  diag = A(0);
  const int q[3] = {i, j, k};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    A s = A(0);
    int cnt = 0;
    const long lo = (q[d] > 0) ? c - L.s[d] : (B.periodic[d] ? c + (long)(L.n[d] - 1) * L.s[d] : -1);
    const long hi = (q[d] + 1 < L.n[d]) ? c + L.s[d] : (B.periodic[d] ? c - (long)(L.n[d] - 1) * L.s[d] : -1);
    if (lo >= 0) {
      s += (A)x[lo];
      ++cnt;
    }
    if (hi >= 0) {
      s += (A)x[hi];
      ++cnt;
    }
    nbsum += ih2[d] * s;
    diag += ih2[d] * (A)cnt;
  }
}

// ---------------------------------------------------------------------------
// CG kernels (FP64 vectors on the fine layout)
// ---------------------------------------------------------------------------
struct CGArgs {
  Lay L;
  Bnd B;
  double ih2[3], ih[3];
  const double *b, *x0;
  double *x, *r, *pold, *pnew, *q;
  const void *z, *zold;
  double *partials;
  SolverScalars *sc;
  double tol2;
  int maxit;
};

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cg_init(CGArgs a) {
  __shared__ double sh[kBlock / 64];
  CellPos p;
  double cc = 0.0, rr = 0.0, sx = 0.0;
  SolverScalars *sc = a.sc;
  if (cell_of_thread(a.L, p)) {
    const long c = p.c;
    const double xv = a.x0 ? a.x0[c] : 0.0;
    a.x[c] = xv;
    double bb = a.b[c] - sc->mean_b;
    const int q[3] = {p.i, p.j, p.k};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (a.B.kind[d][0] == LM_SIDE_OUTFLOW && q[d] == 0) bb -= sc->outflow_c * a.ih[d];
      if (a.B.kind[d][1] == LM_SIDE_OUTFLOW && q[d] == a.L.n[d] - 1) bb -= sc->outflow_c * a.ih[d];
    }
    const double cv = -bb;
    double Lx = 0.0;
    if (a.x0) {
      double nbs, dg;
      op_parts<DIM, double, double>(a.L, a.B, a.ih2, a.x0, p.i, p.j, p.k, c, nbs, dg);
      Lx = dg * xv - nbs;
    }
    const double rv = cv - Lx;
    a.r[c] = rv;
    cc = cv * cv;
    rr = rv * rv;
    sx = xv;
  }
  const unsigned nb = num_blocks(), bid = linear_block();
  double s0 = block_sum(cc, sh);
  double s1 = block_sum(rr, sh);
  double s2 = block_sum(sx, sh);
  if (linear_tid() == 0) {
    a.partials[bid] = s0;
    a.partials[nb + bid] = s1;
    a.partials[2 * nb + bid] = s2;
  }
  if (arrive_last(&sc->counter)) {
    const double tc = sum_partials(a.partials, nb, sh);
    const double tr = sum_partials(a.partials + nb, nb, sh);
    const double tx = sum_partials(a.partials + 2 * nb, nb, sh);
    if (linear_tid() == 0) {
      sc->cc = tc;
      sc->rr = tr;
      sc->mean_x = tx / (double)a.L.ncells();
      sc->tol2 = a.tol2;
      sc->maxit = a.maxit;
      sc->iters = 0;
      sc->first = 1;
      sc->beta = 0.0;
      sc->nonconv = 0;
      sc->zero = (tc == 0.0);
      sc->done = (tc == 0.0) || (tr <= a.tol2 * tc);
      if (!isfinite(tr)) {
        sc->done = 1;
        sc->nonconv = 1;
      }
      sc->counter = 0;
    }
  }
}

// r.z (and r.z_old in flexible mode); beta = r.z / r_old.z_old, or
// (r.z - r.z_old) / r_old.z_old (Polak-Ribiere) with an FP32 preconditioner.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cg_rz(CGArgs a) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  CellPos p;
  double rz = 0.0, rzo = 0.0;
  const TZ *z = (const TZ *)a.z;
  const TZ *zo = (const TZ *)a.zold;
  if (cell_of_thread(a.L, p)) {
    const double rv = a.r[p.c];
    rz = rv * (double)z[p.c];
    if (zo) rzo = rv * (double)zo[p.c];
  }
  const unsigned nb = num_blocks(), bid = linear_block();
  double s0 = block_sum(rz, sh);
  double s1 = zo ? block_sum(rzo, sh) : 0.0;
  if (linear_tid() == 0) {
    a.partials[bid] = s0;
    a.partials[nb + bid] = s1;
  }
  if (arrive_last(&sc->counter)) {
    const double t0 = sum_partials(a.partials, nb, sh);
    const double t1 = zo ? sum_partials(a.partials + nb, nb, sh) : 0.0;
    if (linear_tid() == 0) {
      if (sc->first) {
        sc->beta = 0.0;
        sc->first = 0;
      } else {
        sc->beta = (zo ? (t0 - t1) : t0) / sc->rz;
      }
      sc->rz = t0;
      if (!isfinite(t0) || !isfinite(sc->beta)) {
        sc->done = 1;
        sc->nonconv = 1;
      }
      sc->counter = 0;
    }
  }
}

// p_new = z + beta p_old; q = L p_new; alpha = r.z / p.q.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cg_pq(CGArgs a) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  CellPos p;
  double pq = 0.0;
  const TZ *z = (const TZ *)a.z;
  const double beta = sc->beta;
  if (cell_of_thread(a.L, p)) {
    const long c = p.c;
    auto pv = [&](long m) -> double { return beta != 0.0 ? (double)z[m] + beta * a.pold[m] : (double)z[m]; };
    const double pc = pv(c);
    double nbs = 0.0, dg = 0.0;
    const int q[3] = {p.i, p.j, p.k};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0;
      int cnt = 0;
      const long lo = (q[d] > 0) ? c - a.L.s[d] : (a.B.periodic[d] ? c + (long)(a.L.n[d] - 1) * a.L.s[d] : -1);
      const long hi = (q[d] + 1 < a.L.n[d]) ? c + a.L.s[d]
                                            : (a.B.periodic[d] ? c - (long)(a.L.n[d] - 1) * a.L.s[d] : -1);
      if (lo >= 0) {
        s += pv(lo);
        ++cnt;
      }
      if (hi >= 0) {
        s += pv(hi);
        ++cnt;
      }
      nbs += a.ih2[d] * s;
      dg += a.ih2[d] * (double)cnt;
    }
    const double qv = dg * pc - nbs;
    a.pnew[c] = pc;
    a.q[c] = qv;
    pq = pc * qv;
  }
  const unsigned nb = num_blocks(), bid = linear_block();
  double s0 = block_sum(pq, sh);
  if (linear_tid() == 0) a.partials[bid] = s0;
  if (arrive_last(&sc->counter)) {
    const double t0 = sum_partials(a.partials, nb, sh);
    if (linear_tid() == 0) {
      sc->pq = t0;
      sc->alpha = sc->rz / t0;
      if (!(t0 > 0.0) || !isfinite(sc->alpha)) {
        sc->done = 1;
        sc->nonconv = (sc->rr > sc->tol2 * sc->cc);
      }
      sc->counter = 0;
    }
  }
}

// x += alpha p; r -= alpha q; convergence test on ||r||^2 <= tol^2 ||c||^2.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cg_update(CGArgs a) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  CellPos p;
  double rr = 0.0, sx = 0.0;
  const double alpha = sc->alpha;
  if (cell_of_thread(a.L, p)) {
    const long c = p.c;
    const double xv = a.x[c] + alpha * a.pnew[c];
    const double rv = a.r[c] - alpha * a.q[c];
    a.x[c] = xv;
    a.r[c] = rv;
    rr = rv * rv;
    sx = xv;
  }
  const unsigned nb = num_blocks(), bid = linear_block();
  double s0 = block_sum(rr, sh);
  double s1 = block_sum(sx, sh);
  if (linear_tid() == 0) {
    a.partials[bid] = s0;
    a.partials[nb + bid] = s1;
  }
  if (arrive_last(&sc->counter)) {
    const double t0 = sum_partials(a.partials, nb, sh);
    const double t1 = sum_partials(a.partials + nb, nb, sh);
    if (linear_tid() == 0) {
      sc->rr = t0;
      sc->mean_x = t1 / (double)a.L.ncells();
      sc->iters += 1;
      if (!isfinite(t0)) {
        sc->done = 1;
        sc->nonconv = 1;
      } else if (t0 <= sc->tol2 * sc->cc) {
        sc->done = 1;
      } else if (sc->iters >= sc->maxit) {
        sc->done = 1;
        sc->nonconv = 1;
      }
      sc->counter = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Multigrid kernels (x in TX, right-hand side in TB)
// ---------------------------------------------------------------------------
template <typename T>
struct Ih2 {
  T v[3];
};

// One red (color 0) or black (color 1) half-sweep of Gauss-Seidel on
// L x = b. With zero_init the previous iterate is zero (first half-sweep
// of the pre-smoother): red cells take b/diag without reading x.
template <int DIM, typename TX, typename TB>
__global__ void __launch_bounds__(kBlock) k_mg_smooth(Lay L, Bnd B, Ih2<TX> ih2, TX *x, const TB *b, int color,
                                                      int zero_init, const SolverScalars *sc) {
  if (sc->done) return;
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  if (((p.i + p.j + p.k) & 1) != color) return;
  TX nbs, dg;
  if (zero_init) {
    op_parts<DIM, TX, TX>(L, B, ih2.v, x, p.i, p.j, p.k, p.c, nbs, dg);
    if (color == 0) nbs = TX(0);
  } else {
    op_parts<DIM, TX, TX>(L, B, ih2.v, x, p.i, p.j, p.k, p.c, nbs, dg);
  }
  x[p.c] = ((TX)b[p.c] + nbs) / dg;
}

// Coarse right-hand side: average over the 2^DIM children of b - L x.
template <int DIM, typename TX, typename TB>
__global__ void __launch_bounds__(kBlock) k_mg_restrict(Lay Lf, Lay Lc, Bnd B, Ih2<TX> ih2, const TX *x,
                                                        const TB *b, TX *bc, const SolverScalars *sc) {
  if (sc->done) return;
  CellPos p;
  if (!cell_of_thread(Lc, p)) return;
  TX acc = TX(0);
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int i = 2 * p.i + dx, j = 2 * p.j + dy, k = DIM == 3 ? 2 * p.k + dz : 0;
        const long c = Lf.at(i, j, k);
        TX nbs, dg;
        op_parts<DIM, TX, TX>(Lf, B, ih2.v, x, i, j, k, c, nbs, dg);
        acc += ((TX)b[c] - (dg * x[c] - nbs));
      }
  bc[p.c] = acc * (DIM == 3 ? TX(0.125) : TX(0.25));
}

// x_fine += x_coarse(parent) (piecewise-constant prolongation).
template <int DIM, typename TX>
__global__ void __launch_bounds__(kBlock) k_mg_prolong(Lay Lf, Lay Lc, TX *xf, const TX *xc,
                                                       const SolverScalars *sc) {
  if (sc->done) return;
  CellPos p;
  if (!cell_of_thread(Lf, p)) return;
  xf[p.c] += xc[Lc.at(p.i >> 1, p.j >> 1, DIM == 3 ? (p.k >> 1) : 0)];
}

// Coarse part of the V-cycle in one block: levels l0 .. nlev-1, with the
// dense pseudo-inverse on the coarsest level.
template <typename T>
struct CoarseArgs {
  int l0, nlev, nu, ndim;
  Bnd B;
  Lay L[kMaxLev];
  T *x[kMaxLev];
  const void *b[kMaxLev];
  Ih2<T> ih2[kMaxLev];
  const T *pinv;
  int b0_double;  // level l0 right-hand side is FP64 (the CG residual)
};

template <int DIM, typename T>
__device__ inline void cs_decode(const Lay &L, long t, int &i, int &j, int &k) {
  i = (int)(t % L.n[0]);
  j = (int)((t / L.n[0]) % L.n[1]);
  k = DIM == 3 ? (int)(t / ((long)L.n[0] * L.n[1])) : 0;
}

template <int DIM, typename T>
__device__ inline T cs_b(const CoarseArgs<T> &a, int l, long c) {
  if (l == a.l0 && a.b0_double) return (T)((const double *)a.b[l])[c];
  return ((const T *)a.b[l])[c];
}

template <int DIM, typename T>
__device__ void cs_half_sweep(const CoarseArgs<T> &a, int l, int color, int zero_init) {
  const Lay &L = a.L[l];
  T *x = a.x[l];
  const long N = L.ncells();
  for (long t = threadIdx.x; t < N; t += blockDim.x) {
    int i, j, k;
    cs_decode<DIM, T>(L, t, i, j, k);
    if (((i + j + k) & 1) != color) continue;
    const long c = L.at(i, j, k);
    T nbs, dg;
    op_parts<DIM, T, T>(L, a.B, a.ih2[l].v, x, i, j, k, c, nbs, dg);
    if (zero_init && color == 0) nbs = T(0);
    x[c] = (cs_b<DIM, T>(a, l, c) + nbs) / dg;
  }
  __syncthreads();
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(CoarseArgs<T> a, const SolverScalars *sc) {
  if (sc->done) return;
  const int last = a.nlev - 1;
  for (int l = a.l0; l < last; ++l) {
    for (int s = 0; s < a.nu; ++s) {
      cs_half_sweep<DIM, T>(a, l, 0, s == 0);
      cs_half_sweep<DIM, T>(a, l, 1, 0);
    }
    const Lay &Lf = a.L[l], &Lc = a.L[l + 1];
    const long Nc = Lc.ncells();
    for (long t = threadIdx.x; t < Nc; t += blockDim.x) {
      int I, J, K;
      cs_decode<DIM, T>(Lc, t, I, J, K);
      T acc = T(0);
      for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int i = 2 * I + dx, j = 2 * J + dy, k = DIM == 3 ? 2 * K + dz : 0;
            const long c = Lf.at(i, j, k);
            T nbs, dg;
            op_parts<DIM, T, T>(Lf, a.B, a.ih2[l].v, a.x[l], i, j, k, c, nbs, dg);
            acc += cs_b<DIM, T>(a, l, c) - (dg * a.x[l][c] - nbs);
          }
      ((T *)a.b[l + 1])[Lc.at(I, J, K)] = acc * (DIM == 3 ? T(0.125) : T(0.25));
    }
    __syncthreads();
  }
  {
    const Lay &L = a.L[last];
    const long N = L.ncells();
    for (long row = threadIdx.x; row < N; row += blockDim.x) {
      T acc = T(0);
      for (long col = 0; col < N; ++col) {
        int i, j, k;
        cs_decode<DIM, T>(L, col, i, j, k);
        acc += a.pinv[row * N + col] * cs_b<DIM, T>(a, last, L.at(i, j, k));
      }
      int i, j, k;
      cs_decode<DIM, T>(L, row, i, j, k);
      a.x[last][L.at(i, j, k)] = acc;
    }
    __syncthreads();
  }
  for (int l = last - 1; l >= a.l0; --l) {
    const Lay &Lf = a.L[l], &Lc = a.L[l + 1];
    const long N = Lf.ncells();
    for (long t = threadIdx.x; t < N; t += blockDim.x) {
      int i, j, k;
      cs_decode<DIM, T>(Lf, t, i, j, k);
      a.x[l][Lf.at(i, j, k)] += a.x[l + 1][Lc.at(i >> 1, j >> 1, DIM == 3 ? (k >> 1) : 0)];
    }
    __syncthreads();
    for (int s = 0; s < a.nu; ++s) {
      cs_half_sweep<DIM, T>(a, l, 1, 0);
      cs_half_sweep<DIM, T>(a, l, 0, 0);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool poisson_plan(PoissonWS &ws, Carver &cv, const Lay &fine, const Bnd &B, const double h[3], int mixed,
                  int nu, std::string *err) {
  ws.lay = fine;
  ws.bnd = B;
  ws.mixed = mixed;
  ws.nu = nu;
  const int ndim = fine.ndim;
  const int eb = mixed ? 4 : 8;
  int n[3] = {fine.n[0], fine.n[1], fine.n[2]};
  double hh[3] = {h[0], h[1], h[2]};
  int nl = 0;
  while (true) {
    MGLevel &m = ws.lev[nl];
    m.lay = nl == 0 ? fine : make_layout(ndim, n, eb);
    for (int d = 0; d < 3; ++d) m.ih2[d] = d < ndim ? 1.0 / (hh[d] * hh[d]) : 0.0;
    ++nl;
    long N = (long)n[0] * n[1] * n[2];
    bool even = true;
    for (int d = 0; d < ndim; ++d) even = even && (n[d] % 2 == 0) && (n[d] / 2 >= 2);
    if (!even || N <= 16 || nl == kMaxLev) break;
    for (int d = 0; d < ndim; ++d) {
      n[d] /= 2;
      hh[d] *= 2.0;
    }
  }
  ws.nlev = nl;
  const long ncoarsest = ws.lev[nl - 1].lay.ncells();
  if (ncoarsest > kMaxCoarsest) {
    if (err) *err = "grid does not coarsen to <= 1024 cells (need even sizes down to the coarse grid)";
    return false;
  }
  ws.lc = 0;
  while (ws.lc < nl - 1 && ws.lev[ws.lc].lay.ncells() > kCoarseCells) ++ws.lc;
  const size_t fbytes = (size_t)fine.total * 8;
  ws.x = (double *)cv.take(fbytes);
  ws.r = (double *)cv.take(fbytes);
  ws.p[0] = (double *)cv.take(fbytes);
  ws.p[1] = (double *)cv.take(fbytes);
  ws.q = (double *)cv.take(fbytes);
  ws.z[0] = cv.take((size_t)fine.total * eb);
  ws.z[1] = mixed ? cv.take((size_t)fine.total * eb) : ws.z[0];
  ws.lev[0].x = ws.z[0];
  ws.lev[0].b = ws.r;
  for (int l = 1; l < nl; ++l) {
    ws.lev[l].x = cv.take((size_t)ws.lev[l].lay.total * eb);
    ws.lev[l].b = cv.take((size_t)ws.lev[l].lay.total * eb);
  }
  ws.pinv = cv.take((size_t)ncoarsest * ncoarsest * eb);
  ws.partials = (double *)cv.take((size_t)4 * nblocks_for(fine) * 8 + 64);
  ws.sc = (SolverScalars *)cv.take(sizeof(SolverScalars));
  ws.pflip = 0;
  ws.zflip = 0;
  return true;
}

// Pseudo-inverse of the coarsest operator: (L + J/N)^{-1} - J/N, where J is
// the all-ones matrix (L is singular with the constants as null space).
hipError_t poisson_setup(hipStream_t st, PoissonWS &ws, const double h0[3]) {
  (void)h0;
  const MGLevel &m = ws.lev[ws.nlev - 1];
  const Lay &L = m.lay;
  const long N = L.ncells();
  std::vector<double> A((size_t)N * N, 0.0), I((size_t)N * N, 0.0);
  auto idx = [&](int i, int j, int k) { return (long)i + (long)L.n[0] * (j + (long)L.n[1] * k); };
  for (int k = 0; k < L.n[2]; ++k)
    for (int j = 0; j < L.n[1]; ++j)
      for (int i = 0; i < L.n[0]; ++i) {
        const long r = idx(i, j, k);
        const int q[3] = {i, j, k};
        for (int d = 0; d < L.ndim; ++d) {
          for (int dir = -1; dir <= 1; dir += 2) {
            int qq[3] = {q[0], q[1], q[2]};
            qq[d] += dir;
            if (qq[d] < 0 || qq[d] >= L.n[d]) {
              if (!ws.bnd.periodic[d]) continue;
              qq[d] = (qq[d] + L.n[d]) % L.n[d];
            }
            const long cidx = idx(qq[0], qq[1], qq[2]);
            A[r * N + r] += m.ih2[d];
            A[r * N + cidx] -= m.ih2[d];
          }
        }
      }
  for (long a = 0; a < N * N; ++a) A[a] += 1.0 / (double)N;
  for (long a = 0; a < N; ++a) I[a * N + a] = 1.0;
  // Gauss-Jordan with partial pivoting
  for (long col = 0; col < N; ++col) {
    long piv = col;
    for (long r = col + 1; r < N; ++r)
      if (std::fabs(A[r * N + col]) > std::fabs(A[piv * N + col])) piv = r;
    if (piv != col)
      for (long c = 0; c < N; ++c) {
        std::swap(A[col * N + c], A[piv * N + c]);
        std::swap(I[col * N + c], I[piv * N + c]);
      }
    const double d = A[col * N + col];
    for (long c = 0; c < N; ++c) {
      A[col * N + c] /= d;
      I[col * N + c] /= d;
    }
    for (long r = 0; r < N; ++r) {
      if (r == col) continue;
      const double f = A[r * N + col];
      if (f == 0.0) continue;
      for (long c = 0; c < N; ++c) {
        A[r * N + c] -= f * A[col * N + c];
        I[r * N + c] -= f * I[col * N + c];
      }
    }
  }
  for (long a = 0; a < N * N; ++a) I[a] -= 1.0 / (double)N;
  hipError_t e;
  if (ws.mixed) {
    std::vector<float> f(I.begin(), I.end());
    e = hipMemcpyAsync(ws.pinv, f.data(), f.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  } else {
    e = hipMemcpyAsync(ws.pinv, I.data(), I.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  return e;
}

template <int DIM, typename T>
static void vcycle(hipStream_t st, PoissonWS &ws, void *z) {
  const Bnd &B = ws.bnd;
  const int nu = ws.nu;
  const SolverScalars *sc = ws.sc;
  auto ih2 = [&](int l) {
    Ih2<T> v;
    for (int d = 0; d < 3; ++d) v.v[d] = (T)ws.lev[l].ih2[d];
    return v;
  };
  // fine levels: multi-block kernels
  for (int l = 0; l < ws.lc; ++l) {
    const Lay &L = ws.lev[l].lay;
    T *x = l == 0 ? (T *)z : (T *)ws.lev[l].x;
    dim3 g = grid_for(L), b(kBX, kBY);
    for (int s = 0; s < nu; ++s) {
      if (l == 0) {
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, b, 0, st, L, B, ih2(l), x, (const double *)ws.r, 0,
                           s == 0, sc);
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, b, 0, st, L, B, ih2(l), x, (const double *)ws.r, 1,
                           0, sc);
      } else {
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, b, 0, st, L, B, ih2(l), x, (const T *)ws.lev[l].b, 0,
                           s == 0, sc);
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, b, 0, st, L, B, ih2(l), x, (const T *)ws.lev[l].b, 1, 0,
                           sc);
      }
    }
    const Lay &Lc = ws.lev[l + 1].lay;
    dim3 gc = grid_for(Lc);
    if (l == 0)
      hipLaunchKernelGGL((k_mg_restrict<DIM, T, double>), gc, b, 0, st, L, Lc, B, ih2(l), x, (const double *)ws.r,
                         (T *)ws.lev[l + 1].b, sc);
    else
      hipLaunchKernelGGL((k_mg_restrict<DIM, T, T>), gc, b, 0, st, L, Lc, B, ih2(l), x, (const T *)ws.lev[l].b,
                         (T *)ws.lev[l + 1].b, sc);
  }
  // coarse levels in one block
  CoarseArgs<T> ca;
  ca.l0 = ws.lc;
  ca.nlev = ws.nlev;
  ca.nu = nu;
  ca.ndim = DIM;
  ca.B = B;
  for (int l = 0; l < ws.nlev; ++l) {
    ca.L[l] = ws.lev[l].lay;
    ca.x[l] = l == 0 ? (T *)z : (T *)ws.lev[l].x;
    ca.b[l] = l == 0 ? (const void *)ws.r : ws.lev[l].b;
    ca.ih2[l] = ih2(l);
  }
  ca.pinv = (const T *)ws.pinv;
  ca.b0_double = (ws.lc == 0);
  hipLaunchKernelGGL((k_mg_coarse<DIM, T>), dim3(1), dim3(kCoarseThreads), 0, st, ca, sc);
  // back up the fine levels
  for (int l = ws.lc - 1; l >= 0; --l) {
    const Lay &L = ws.lev[l].lay, &Lc = ws.lev[l + 1].lay;
    T *x = l == 0 ? (T *)z : (T *)ws.lev[l].x;
    dim3 g = grid_for(L), b(kBX, kBY);
    hipLaunchKernelGGL((k_mg_prolong<DIM, T>), g, b, 0, st, L, Lc, x, (const T *)ws.lev[l + 1].x, sc);
    for (int s = 0; s < nu; ++s) {
      if (l == 0) {
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, b, 0, st, L, B, ih2(l), x, (const double *)ws.r, 1,
                           0, sc);
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, b, 0, st, L, B, ih2(l), x, (const double *)ws.r, 0,
                           0, sc);
      } else {
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, b, 0, st, L, B, ih2(l), x, (const T *)ws.lev[l].b, 1, 0,
                           sc);
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, b, 0, st, L, B, ih2(l), x, (const T *)ws.lev[l].b, 0, 0,
                           sc);
      }
    }
  }
}

template <int DIM, typename T>
static void cg_iteration_kernels(hipStream_t st, PoissonWS &ws, CGArgs a, bool with_pq) {
  dim3 g = grid_for(ws.lay), b(kBX, kBY);
  if (with_pq) {
    a.pold = ws.p[ws.pflip];
    a.pnew = ws.p[ws.pflip ^ 1];
    a.z = ws.z[ws.zflip];
    hipLaunchKernelGGL((k_cg_pq<DIM, T>), g, b, 0, st, a);
    hipLaunchKernelGGL((k_cg_update<DIM>), g, b, 0, st, a);
    ws.pflip ^= 1;
    if (ws.mixed) ws.zflip ^= 1;
  }
  void *z = ws.z[ws.zflip];
  vcycle<DIM, T>(st, ws, z);
  a.z = z;
  a.zold = ws.mixed && with_pq ? ws.z[ws.zflip ^ 1] : nullptr;
  hipLaunchKernelGGL((k_cg_rz<DIM, T>), g, b, 0, st, a);
}

template <int DIM>
static hipError_t solve_dim(hipStream_t st, PoissonWS &ws, const double *bvec, const double *x0, double rtol,
                            int maxit, int expect, int *iters, double *relres, int *converged) {
  CGArgs a;
  a.L = ws.lay;
  a.B = ws.bnd;
  for (int d = 0; d < 3; ++d) {
    a.ih2[d] = ws.lev[0].ih2[d];
    a.ih[d] = std::sqrt(ws.lev[0].ih2[d]);
  }
  a.b = bvec;
  a.x0 = x0;
  a.x = ws.x;
  a.r = ws.r;
  a.q = ws.q;
  a.pold = a.pnew = nullptr;
  a.z = a.zold = nullptr;
  a.partials = ws.partials;
  a.sc = ws.sc;
  a.tol2 = rtol * rtol;
  a.maxit = maxit;
  dim3 g = grid_for(ws.lay), b(kBX, kBY);
  hipLaunchKernelGGL((k_cg_init<DIM>), g, b, 0, st, a);
  const bool mixed = ws.mixed;
  if (mixed)
    cg_iteration_kernels<DIM, float>(st, ws, a, false);
  else
    cg_iteration_kernels<DIM, double>(st, ws, a, false);
  int done_iters = 0;
  int batch = expect > 0 ? expect : 4;
  hipError_t e = hipSuccess;
  while (true) {
    for (int k = 0; k < batch; ++k) {
      if (mixed)
        cg_iteration_kernels<DIM, float>(st, ws, a, true);
      else
        cg_iteration_kernels<DIM, double>(st, ws, a, true);
    }
    done_iters += batch;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ws.host_sc, ws.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (ws.host_sc->done) break;
    if (done_iters >= maxit + 2) break;
    batch = 2;
  }
  const SolverScalars &h = *ws.host_sc;
  *iters = h.iters;
  *relres = h.cc > 0 ? std::sqrt(h.rr / h.cc) : 0.0;
  *converged = h.done && !h.nonconv;
  return hipSuccess;
}

hipError_t poisson_solve(hipStream_t st, PoissonWS &ws, const double *b, const double *x0, double rtol,
                         int maxit, int expect_iters, int *iters, double *relres, int *converged) {
  if (ws.lay.ndim == 3) return solve_dim<3>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged);
  return solve_dim<2>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged);
}

}  // namespace lm
