// Pressure Poisson solver: preconditioned conjugate gradients on the
// singular, symmetric operator L = -A, A P = sum_d delta_1 delta_1 P (the
// discrete continuity constraint Eq 3.24 with the face flux of Eq 3.23;
// zero flux through non-periodic sides, section 3.3). The preconditioner is
// one symmetric geometric multigrid V-cycle: red-black Gauss-Seidel
// (red-black down, black-red up), 2^d-cell averaging restriction,
// piecewise-constant prolongation, rediscretised coarse operators and an
// exact pseudo-inverse on the coarsest grid, so the zero-mean solution is
// obtained as with the augmented-matrix method the paper uses. The V-cycle
// runs in FP64, or in FP32 (mixed modes) with FP64 residuals, operator,
// updates and dot products.
//
// CG. Single-reduction CG (Chronopoulos-Gear: one global reduction per
// iteration, s = A p carried by recurrence and w = A u formed on the finest
// level of the V-cycle) in FP64 and in the default mixed mode; flexible CG
// (Polak-Ribiere beta, q = A p formed explicitly) in the flexible mixed
// mode. Scalars never leave the device. A reduction kernel writes one
// partial sum per block; the next kernel that needs the total has every
// block sum those partials in the same fixed order (no atomics, no grid-wide
// fences, bitwise reproducible). The convergence test runs on the device and
// raises a flag that turns every later kernel into an immediate return; the
// host queues iterations in batches and reads the flag once per batch.
//
// Levels. 2D levels whose sizes are multiples of the tile run one LDS tile
// kernel per level and direction with temporal blocking (nu red-black sweeps
// from a zero guess, residual and restriction on the way down; prolongation
// and nu black-red sweeps on the way up; on the finest level also the CG
// update, w = A u and the CG partial sums). Large fully periodic 3D levels
// run the z-marching equivalent (lm_mg3d.h). Levels of at most kCoarseCells
// cells are solved by one block in LDS; the remaining levels run one kernel
// per half-sweep.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "lm_device.h"

namespace lm {

constexpr int kCoarseThreads = 1024;
constexpr int kRedBlocks = 1024;   // grid of the grid-stride reduction kernels
// 2D tiles of the fused multigrid kernels: 64 x 16 preferred on the finest
// level (bandwidth), 32 x 8 below it (latency bound: shorter phases), 16 x 16
// for sizes that neither divides.
constexpr int TX = 64, TY = 16;
constexpr int TXS = 32, TYS = 8;
constexpr long kFused3DMinCells = 1L << 15;  // smaller 3D levels run the per-half-sweep kernels

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
// Small device helpers
// ---------------------------------------------------------------------------

// Block-wide sums of NV values, identical in every thread: wavefront
// shuffles, one exchange through LDS, then every thread adds the
// per-wavefront sums in wavefront order (the tree of block_sum, so the
// values are bitwise those of block_sum).
template <int NV>
__device__ inline void block_allsum_n(double (&v)[NV]) {
  __shared__ double shn[NV][16];
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
  const int t = linear_tid();
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
  __syncthreads();  // an earlier call may still be reading shn
  if ((t & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) shn[q][t >> 6] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += shn[q][w];
    v[q] = s;
  }
}

// This thread's share of the sum of np partials: loads issued four at a
// time so their latencies overlap.
__device__ inline double partial_share(const double *part, int np) {
  const int t = linear_tid();
  const int nt = blockDim.x * blockDim.y * blockDim.z;
  double s = 0.0;
  for (int q0 = 0; q0 < np; q0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * nt + t;
      v[u] = part[q < np ? q : 0];
      if (q >= np) v[u] = 0.0;
    }
    s += (v[0] + v[1]) + (v[2] + v[3]);
  }
  return s;
}

// Sum of np partials, identical in every block and thread.
__device__ inline double sum_all(const double *part, int np, double *) {
  double v[1] = {partial_share(part, np)};
  block_allsum_n<1>(v);
  return v[0];
}

// Sums of three partial arrays of np entries each (one combined pass).
__device__ inline void sum_all3(const double *p0, const double *p1, const double *p2, int np, double *,
                                double &s0, double &s1, double &s2) {
  double v[3] = {partial_share(p0, np), partial_share(p1, np), p2 ? partial_share(p2, np) : 0.0};
  block_allsum_n<3>(v);
  s0 = v[0];
  s1 = v[1];
  s2 = v[2];
}

// ||c||^2 (the partials of the solve's right-hand side on the first
// iteration, the value stored by block 0 afterwards) together with the
// three sums of sum_all3, in one pass.
__device__ inline void sum_cc3(int k, const double *part_cc, int np_cc, const SolverScalars *sc, const double *p0,
                               const double *p1, const double *p2, int np, double &cc, double &s0, double &s1,
                               double &s2) {
  if (k == 1) {
    double v[4] = {partial_share(part_cc, np_cc), partial_share(p0, np), partial_share(p1, np),
                   p2 ? partial_share(p2, np) : 0.0};
    block_allsum_n<4>(v);
    cc = v[0];
    s0 = v[1];
    s1 = v[2];
    s2 = v[3];
  } else {
    cc = sc->cc;
    double v[3] = {partial_share(p0, np), partial_share(p1, np), p2 ? partial_share(p2, np) : 0.0};
    block_allsum_n<3>(v);
    s0 = v[0];
    s1 = v[1];
    s2 = v[2];
  }
}

template <int DIM>
__device__ inline void decode(const Lay &L, long t, int &i, int &j, int &k);

// Grid-stride loops run over 64 x 4 tiles of cells (one wavefront per row):
// one 32-bit division per tile instead of per cell.
__device__ inline int ntiles_of(const Lay &L) { return ((L.n[0] + 63) >> 6) * ((L.n[1] + 3) >> 2) * L.n[2]; }

__device__ inline bool tile_cell(const Lay &L, int tile, int &i, int &j, int &k) {
  const int tx = (L.n[0] + 63) >> 6, ty = (L.n[1] + 3) >> 2;
  const int txy = tx * ty;
  k = tile / txy;
  const int rem = tile - k * txy;
  const int y = rem / tx;
  const int x = rem - y * tx;
  i = (x << 6) + (threadIdx.x & 63);
  j = (y << 2) + (threadIdx.x >> 6);
  return i < L.n[0] && j < L.n[1];
}

template <int DIM>
__device__ inline void decode(const Lay &L, long t, int &i, int &j, int &k) {
  i = (int)(t % L.n[0]);
  j = (int)((t / L.n[0]) % L.n[1]);
  k = DIM == 3 ? (int)(t / ((long)L.n[0] * L.n[1])) : 0;
}

// Neighbour sum and diagonal of L = -A at one cell (periodic wrap, zero
// flux through non-periodic sides).
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

template <typename T>
struct Ih2 {
  T v[3];
};

// Face coefficient of the variable-coefficient operator: beta = 1/rho_f
// with rho_f = (rho_a + rho_b)/2 the two-point face average (Eq 3.20,
// n = 1). Symmetric in its arguments bit for bit.
template <typename T>
__device__ inline T face_beta(T ra, T rb) {
  return T(2) / (ra + rb);
}

// Face coefficient along direction d. On a stretched 2D grid (met) the
// volume-weighted operator dV A has, on an x-face, dy / (distance between
// the two centres) = 2 / (dx_a/dy + dx_b/dy), i.e. face_beta of the cell
// ratio dx/dy, and on a y-face face_beta of dy/dx: the cell array holds
// dx/dy and y-faces take its reciprocals.
template <typename T>
__device__ inline T face_coef(T ra, T rb, int d, int met) {
  if (met && d == 1) return face_beta<T>(T(1) / ra, T(1) / rb);
  return face_beta<T>(ra, rb);
}

// Neighbour sum and diagonal of L = -A_beta at one cell, beta = 1/rho_f
// (same neighbour rules as op_parts).
template <int DIM, typename A, typename T, typename R>
__device__ inline void op_parts_vc(const Lay &L, const Bnd &B, const A ih2[3], const R *rho, const T *x, int i, int j,
                                   int k, long c, A &nbsum, A &diag, int met = 0) {
#pragma clang fp contract(off)
  nbsum = A(0);
  diag = A(0);
  const int q[3] = {i, j, k};
  const A rc = (A)rho[c];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    A s = A(0), sb = A(0);
    const long lo = (q[d] > 0) ? c - L.s[d] : (B.periodic[d] ? c + (long)(L.n[d] - 1) * L.s[d] : -1);
    const long hi = (q[d] + 1 < L.n[d]) ? c + L.s[d] : (B.periodic[d] ? c - (long)(L.n[d] - 1) * L.s[d] : -1);
    if (lo >= 0) {
      const A bt = face_coef<A>(rc, (A)rho[lo], d, met);
      s += bt * (A)x[lo];
      sb += bt;
    }
    if (hi >= 0) {
      const A bt = face_coef<A>(rc, (A)rho[hi], d, met);
      s += bt * (A)x[hi];
      sb += bt;
    }
    nbsum += ih2[d] * s;
    diag += ih2[d] * sb;
  }
}


// ---------------------------------------------------------------------------
// CG kernels (FP64 vectors on the fine layout, grid-stride over cells)
// ---------------------------------------------------------------------------
struct CGArgs {
  Lay L;
  Bnd B;
  double ih2[3], ih[3];
  const double *b, *x0;
  double *x;
  double *rold, *rnew;    // r_{k-1}, r_k
  double *pold, *pnew;    // p_{k-1}, p_k
  double *q;
  const void *z, *zold;   // z_{k-1}, z_{k-2} (flexible)
  double *part_cc, *part_pq, *part_rz;  // part_rz: [rz | rr | rzo] x np_rz
  int np_rz, np_pq;
  SolverScalars *sc;
  double tol2;
  int k;
  int flexible;
  const double *rho;      // density of beta = 1/rho_f; NULL: beta = 1
  int met = 0;                   // stretched 2D grid: rho holds dx/dy (face_coef)
  const double *vol = nullptr;   // stretched: cell volumes (the right-hand side is dV b)
};

// x = x0; r_0 = c - L x0 with c = -(b - mean(b) - outflow shift); ||c||^2
// partials, one per block (one thread per cell: the stencil of x0 reads
// planes a patch plane apart, still in L2).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cg_init(CGArgs a, double *partials) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (a.rho && sc->rho_bad) {  // invalid density: the solve ends at once
    if (linear_block() == 0 && linear_tid() == 0) {
      sc->done = 1;
      sc->nonconv = 1;
    }
    return;
  }
  double cc = 0.0;
  CellPos p;
  if (cell_of_thread(a.L, p)) {
    const int i = p.i, j = p.j, k = p.k;
    const long c = p.c;
    const double mb = sc->mean_b, oc = sc->outflow_c;
    const double xv = a.x0 ? a.x0[c] : 0.0;
    a.x[c] = xv;
    double bb = a.b[c] - mb;
    const int q[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (a.B.kind[d][0] == LM_SIDE_OUTFLOW && q[d] == 0) bb -= oc * a.ih[d];
      if (a.B.kind[d][1] == LM_SIDE_OUTFLOW && q[d] == a.L.n[d] - 1) bb -= oc * a.ih[d];
    }
    const double cv = a.vol ? -(bb * a.vol[c]) : -bb;  // stretched: dV (b - mean)
    double Lx = 0.0;
    if (a.x0) {
      double nbs, dg;
      if (a.rho)
        op_parts_vc<DIM, double, double, double>(a.L, a.B, a.ih2, a.rho, a.x0, i, j, k, c, nbs, dg, a.met);
      else
        op_parts<DIM, double, double>(a.L, a.B, a.ih2, a.x0, i, j, k, c, nbs, dg);
      Lx = dg * xv - nbs;
    }
    a.rnew[c] = cv - Lx;
    cc = cv * cv;
  }
  const double s = block_sum(cc, sh);
  if (linear_tid() == 0) partials[linear_block()] = s;
}

// Folds nb per-block partials into gridDim.x partials, each the fixed-order
// sum of a contiguous run.
__global__ void __launch_bounds__(kBlock) k_fold_partials(const double *in, long nb, double *out) {
  __shared__ double sh[kBlock / 64];
  const long per = (nb + gridDim.x - 1) / gridDim.x;
  const long q0 = (long)blockIdx.x * per, q1 = q0 + per < nb ? q0 + per : nb;
  double s = 0.0;
  for (long q = q0 + threadIdx.x; q < q1; q += blockDim.x) s += in[q];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// Convergence test on r_{k-1}; beta_k; p_k = z_{k-1} + beta_k p_{k-1};
// q = L p_k; partials of p_k.q.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cg_pq(CGArgs a, int np_cc) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  const int k = a.k;
  double cc, rz, rr, rzo;
  sum_cc3(k, a.part_cc, np_cc, sc, a.part_rz, a.part_rz + a.np_rz, a.flexible ? a.part_rz + 2 * a.np_rz : nullptr,
          a.np_rz, cc, rz, rr, rzo);
  const bool converged = (cc == 0.0) || (rr <= a.tol2 * cc);
  const bool broken = !isfinite(rr) || !isfinite(rz);
  double beta = 0.0;
  if (k > 1) beta = (a.flexible ? rz - rzo : rz) / sc->rzh[(k - 2) & 1];
  if (linear_block() == 0 && linear_tid() == 0) {
    sc->rzh[(k - 1) & 1] = rz;
    sc->rr = rr;
    sc->cc = cc;
    sc->iters = k - 1;
    if (converged || broken) {
      sc->done = 1;
      sc->zero = (cc == 0.0);
      sc->nonconv = broken && !converged;
    }
  }
  if (converged || broken) return;
  const TZ *z = (const TZ *)a.z;
  double pq = 0.0;
  for (int tile = blockIdx.x; tile < ntiles_of(a.L); tile += gridDim.x) {
    int i, j, kk;
    if (!tile_cell(a.L, tile, i, j, kk)) continue;
    const long c = a.L.at(i, j, kk);
    auto pv = [&](long m) -> double { return k > 1 ? (double)z[m] + beta * a.pold[m] : (double)z[m]; };
    const double pc = pv(c);
    double nbs = 0.0, dg = 0.0;
    const int q[3] = {i, j, kk};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double s = 0.0, sb = 0.0;
      const long lo = (q[d] > 0) ? c - a.L.s[d] : (a.B.periodic[d] ? c + (long)(a.L.n[d] - 1) * a.L.s[d] : -1);
      const long hi = (q[d] + 1 < a.L.n[d]) ? c + a.L.s[d]
                                            : (a.B.periodic[d] ? c - (long)(a.L.n[d] - 1) * a.L.s[d] : -1);
      if (lo >= 0) {
        const double bt = a.rho ? face_coef<double>(a.rho[c], a.rho[lo], d, a.met) : 1.0;
        s += bt * pv(lo);
        sb += bt;
      }
      if (hi >= 0) {
        const double bt = a.rho ? face_coef<double>(a.rho[c], a.rho[hi], d, a.met) : 1.0;
        s += bt * pv(hi);
        sb += bt;
      }
      nbs += a.ih2[d] * s;
      dg += a.ih2[d] * sb;
    }
    const double qv = dg * pc - nbs;
    a.pnew[c] = pc;
    a.q[c] = qv;
    pq += pc * qv;
  }
  const double s = block_sum(pq, sh);
  if (linear_tid() == 0) a.part_pq[blockIdx.x] = s;
}

// alpha_k = rho_{k-1}/(p_k.q); x += alpha p_k; r_k = r_{k-1} - alpha q.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_cg_update(CGArgs a) {
  __shared__ double sh[kBlock / 64];
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  const double pq = sum_all(a.part_pq, a.np_pq, sh);
  const double alpha = sc->rzh[(a.k - 1) & 1] / pq;
  for (int tile = blockIdx.x; tile < ntiles_of(a.L); tile += gridDim.x) {
    int i, j, k;
    if (!tile_cell(a.L, tile, i, j, k)) continue;
    const long c = a.L.at(i, j, k);
    a.x[c] += alpha * a.pnew[c];
    a.rnew[c] = a.rold[c] - alpha * a.q[c];
  }
}

// Partials of r.z, r.r (and r.z_old) for the unfused finest level.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cg_rz(CGArgs a) {
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  const TZ *z = (const TZ *)a.z;
  const TZ *zo = (const TZ *)a.zold;
  double rz = 0.0, rr = 0.0, rzo = 0.0;
  for (int tile = blockIdx.x; tile < ntiles_of(a.L); tile += gridDim.x) {
    int i, j, k;
    if (!tile_cell(a.L, tile, i, j, k)) continue;
    const long c = a.L.at(i, j, k);
    const double rv = a.rnew[c];
    rz += rv * (double)z[c];
    rr += rv * rv;
    if (zo) rzo += rv * (double)zo[c];
  }
  double v3[3] = {rz, rr, rzo};  // rzo stays 0 without z_old
  block_allsum_n<3>(v3);
  if (linear_tid() == 0) {
    a.part_rz[blockIdx.x] = v3[0];
    a.part_rz[a.np_rz + blockIdx.x] = v3[1];
    a.part_rz[2 * a.np_rz + blockIdx.x] = v3[2];
  }
}

// Single-reduction CG (Chronopoulos-Gear) for an unfused finest level.
// Step k: convergence test on r_{k-1}; beta = g_{k-1}/g_{k-2},
// alpha = g_{k-1} / (d_{k-1} - beta g_{k-1}/alpha_{k-2}) with g = r.u and
// d = (A u).u; p = u + beta p; s = w + beta s; x += alpha p; r -= alpha s.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cgcg_update(CGArgs a, int np_cc, const double *w, const double *s_old,
                                                        double *s_new) {
  SolverScalars *sc = a.sc;
  if (sc->done) return;
  const int k = a.k;
  double cc, g, d, rr;
  sum_cc3(k, a.part_cc, np_cc, sc, a.part_rz, a.part_rz + a.np_rz, a.part_rz + 2 * a.np_rz, a.np_rz, cc, g, d, rr);
  const bool conv = (cc == 0.0) || (rr <= a.tol2 * cc);
  double alpha, beta = 0.0;
  if (k == 1) {
    alpha = g / d;
  } else {
    beta = g / sc->rzh[(k - 2) & 1];
    alpha = g / (d - beta * g / sc->alh[(k - 2) & 1]);
  }
  const bool broken = !isfinite(rr) || !isfinite(alpha) || !isfinite(beta);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rzh[(k - 1) & 1] = g;
    sc->alh[(k - 1) & 1] = alpha;
    sc->rr = rr;
    sc->cc = cc;
    sc->iters = k - 1;
    if (conv || broken) {
      sc->done = 1;
      sc->zero = (cc == 0.0);
      sc->nonconv = broken && !conv;
    }
  }
  if (conv || broken) return;
  const TZ *u = (const TZ *)a.z;
  const bool old = k >= 2;
  for (int tile = blockIdx.x; tile < ntiles_of(a.L); tile += gridDim.x) {
    int i, j, kk;
    if (!tile_cell(a.L, tile, i, j, kk)) continue;
    const long c = a.L.at(i, j, kk);
    const double so = old ? s_old[c] : 0.0;
    const double pn = (double)u[c] + (old ? beta * a.pnew[c] : 0.0);
    const double sn = w[c] + beta * so;
    a.pnew[c] = pn;
    s_new[c] = sn;
    a.x[c] += alpha * pn;
    a.rnew[c] = a.rold[c] - alpha * sn;
  }
}

// w = A u (u = M r) and partials of r.u, w.u, r.r for the unfused finest level.
template <int DIM, typename TZ>
__global__ void __launch_bounds__(kBlock) k_cgcg_w(CGArgs a, double *w) {
  if (a.sc->done) return;
  const TZ *u = (const TZ *)a.z;
  double ru = 0.0, wu = 0.0, rr = 0.0;
  for (int tile = blockIdx.x; tile < ntiles_of(a.L); tile += gridDim.x) {
    int i, j, k;
    if (!tile_cell(a.L, tile, i, j, k)) continue;
    const long c = a.L.at(i, j, k);
    double nbs, dg;
    if (a.rho)
      op_parts_vc<DIM, double, TZ, double>(a.L, a.B, a.ih2, a.rho, u, i, j, k, c, nbs, dg, a.met);
    else
      op_parts<DIM, double, TZ>(a.L, a.B, a.ih2, u, i, j, k, c, nbs, dg);
    const double uc = (double)u[c];
    const double wv = dg * uc - nbs;
    const double rv = a.rnew[c];
    w[c] = wv;
    ru += rv * uc;
    wu += wv * uc;
    rr += rv * rv;
  }
  double v3[3] = {ru, wu, rr};
  block_allsum_n<3>(v3);
  if (linear_tid() == 0) {
    a.part_rz[blockIdx.x] = v3[0];
    a.part_rz[a.np_rz + blockIdx.x] = v3[1];
    a.part_rz[2 * a.np_rz + blockIdx.x] = v3[2];
  }
}

// Sum of x into partials (mean of the final solution).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_sum_x(Lay L, const double *x, double *part, const double *vol) {
  __shared__ double sh[kBlock / 64];
  // four tiles' loads in flight per trip, four running sums combined in a
  // fixed order
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const int nt = ntiles_of(L);
  for (int t0 = blockIdx.x; t0 < nt; t0 += 4 * gridDim.x) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tile = t0 + u * gridDim.x;
      int i, j, k;
      if (tile < nt && tile_cell(L, tile, i, j, k)) {
        const long c = L.at(i, j, k);
        s[u] += vol ? x[c] * vol[c] : x[c];   // stretched: the integral of x
      }
    }
  }
  const double r = block_sum((s[0] + s[1]) + (s[2] + s[3]), sh);
  if (linear_tid() == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_fin_mean_x(const double *part, int np, double ncells, SolverScalars *sc) {
  __shared__ double sh[kBlock / 64];
  const double s = sum_all(part, np, sh);
  if (threadIdx.x == 0) sc->mean_x = s / ncells;
}

// ---------------------------------------------------------------------------
// Unfused multigrid kernels (any dimension, ragged sizes)
// ---------------------------------------------------------------------------

// One red (color 0) or black (color 1) half-sweep of Gauss-Seidel on
// L x = b. With zero_init the previous iterate is zero (first half-sweep
// of the pre-smoother): red cells take b/diag without reading x.
template <int DIM, typename TX, typename TB>
__global__ void __launch_bounds__(kBlock) k_mg_smooth(Lay L, Bnd B, Ih2<TX> ih2, TX *x, const TB *b, int color,
                                                      int zero_init, const SolverScalars *sc, const TX *rho,
                                                      int met) {
  if (sc->done) return;
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  if (((p.i + p.j + p.k) & 1) != color) return;
  TX nbs, dg;
  if (rho)
    op_parts_vc<DIM, TX, TX, TX>(L, B, ih2.v, rho, x, p.i, p.j, p.k, p.c, nbs, dg, met);
  else
    op_parts<DIM, TX, TX>(L, B, ih2.v, x, p.i, p.j, p.k, p.c, nbs, dg);
  if (zero_init && color == 0) nbs = TX(0);
  x[p.c] = ((TX)b[p.c] + nbs) / dg;
}

// Coarse right-hand side: average over the 2^DIM children of b - L x.
template <int DIM, typename TX, typename TB>
__global__ void __launch_bounds__(kBlock) k_mg_restrict(Lay Lf, Lay Lc, Bnd B, Ih2<TX> ih2, const TX *x,
                                                        const TB *b, TX *bc, const SolverScalars *sc, const TX *rho,
                                                        int met) {
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
        if (rho)
          op_parts_vc<DIM, TX, TX, TX>(Lf, B, ih2.v, rho, x, i, j, k, c, nbs, dg, met);
        else
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

// ---------------------------------------------------------------------------
// Variable-coefficient set-up (once per solve with beta = 1/rho_f)
// ---------------------------------------------------------------------------

// Flags a density that is not positive and finite; converts the finest
// density to the multigrid precision (rt NULL: used as is).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_vc_rho0(Lay L, const double *r64, T *rt, SolverScalars *sc) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const double r = r64[p.c];
  if (!(r > 0.0) || !isfinite(r)) sc->rho_bad = 1;
  if (rt) rt[p.c] = (T)r;
}

// Density of the next coarser level: mean of the 2^DIM children.
template <int DIM, typename TS, typename TD>
__global__ void __launch_bounds__(kBlock) k_vc_rho_down(Lay Lf, Lay Lc, const TS *rf, TD *rc) {
  CellPos p;
  if (!cell_of_thread(Lc, p)) return;
  double acc = 0.0;
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx)
        acc += (double)rf[Lf.at(2 * p.i + dx, 2 * p.j + dy, DIM == 3 ? 2 * p.k + dz : 0)];
  rc[p.c] = (TD)(acc * (DIM == 3 ? 0.125 : 0.25));
}

// Face coefficients of a tiled 2D level: beta of each cell's west and south
// faces (0 through a non-periodic side) and 1/diagonal of L (the same
// operations as op_parts_vc, so the same bits).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vc_coef2d(Lay L, Bnd B, T ihx, T ihy, const T *rho, T *fx, T *fy,
                                                      T *ig) {
#pragma clang fp contract(off)
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  const int nx = L.n[0], ny = L.n[1];
  const long c = p.c, sy = L.s[1];
  const T rc = rho[c];
  T bw = T(0), be = T(0), bs = T(0), bn = T(0);
  if (B.periodic[0] || p.i > 0) bw = face_beta<T>(rc, rho[p.i > 0 ? c - 1 : c + (nx - 1)]);
  if (B.periodic[0] || p.i + 1 < nx) be = face_beta<T>(rc, rho[p.i + 1 < nx ? c + 1 : c - (nx - 1)]);
  if (B.periodic[1] || p.j > 0) bs = face_beta<T>(rc, rho[p.j > 0 ? c - sy : c + (long)(ny - 1) * sy]);
  if (B.periodic[1] || p.j + 1 < ny) bn = face_beta<T>(rc, rho[p.j + 1 < ny ? c + sy : c - (long)(ny - 1) * sy]);
  fx[c] = bw;
  fy[c] = bs;
  ig[c] = T(1) / (ihx * (bw + be) + ihy * (bs + bn));
}

// Density of a coarse-kernel level packed x fastest (the kernel's LDS order).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock) k_vc_pack(Lay L, const T *r, T *out) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  out[p.i + (long)L.n[0] * (p.j + (long)L.n[1] * p.k)] = r[p.c];
}

}  // namespace lm

#include "lm_mg_kernels.h"
#include "lm_mg3d.h"
#include "lm_pcg_block.h"

namespace lm {

// Pseudo-inverse of the coarsest variable-coefficient operator,
// (L + J/N)^{-1} - J/N with J the all-ones matrix: L + J/N is symmetric
// positive definite (L is singular with the constants as null space), so
// Gauss-Jordan elimination without pivoting inverts it in place in LDS.
// UNIT: beta = 1 on every face (no densities read).
constexpr int kPinvThreads = 256;
template <int DIM, typename T, bool UNIT = false>
__global__ void __launch_bounds__(kPinvThreads) k_vc_pinv(CoarseArgs<T> a, T *pinv) {
  __shared__ double M[kVcCoarsest * kVcCoarsest];
  __shared__ double rk[kVcCoarsest], ck[kVcCoarsest];
  const int last = a.nlev - 1;
  const int *n = a.n[last];
  const int N = n[0] * n[1] * n[2];
  const T *rho = UNIT ? nullptr : a.rho_c + a.off[last];
  const int t = threadIdx.x;
  const double jn = 1.0 / (double)N;
  for (int e = t; e < N * N; e += blockDim.x) M[e] = jn;
  __syncthreads();
  if (t < N) {
    int i, j, k;
    c_decode<DIM, T>(n, t, i, j, k);
    const int q[3] = {i, j, k};
    const int st[3] = {1, n[0], n[0] * n[1]};
    const double rc = UNIT ? 1.0 : (double)rho[t];
    for (int d = 0; d < DIM; ++d) {
      const bool per = a.B.periodic[d] != 0;
      const double ih2 = (double)a.ih2[last].v[d];
      for (int side = 0; side < 2; ++side) {
        const bool in = side == 0 ? q[d] > 0 : q[d] + 1 < n[d];
        if (!in && !per) continue;
        const int m = side == 0 ? (in ? t - st[d] : t + (n[d] - 1) * st[d]) : (in ? t + st[d] : t - (n[d] - 1) * st[d]);
        const double w = UNIT ? ih2 : ih2 * face_coef<double>(rc, (double)rho[m], d, a.met);
        M[t * N + t] += w;
        M[t * N + m] -= w;
      }
    }
  }
  __syncthreads();
  // thread t owns column j = t % N of rows t / N + R p (R = rows per pass)
  const int R = blockDim.x / N;
  const int j = t % N, i0 = t / N;
  const bool active = i0 < R;
  constexpr int kPass = (kVcCoarsest + kPinvThreads / kVcCoarsest - 1) / (kPinvThreads / kVcCoarsest);
  for (int kk = 0; kk < N; ++kk) {
    if (t < N) {
      rk[t] = M[kk * N + t];
      ck[t] = M[t * N + kk];
    }
    __syncthreads();
    const double ip = 1.0 / rk[kk];
    const double rj = rk[j] * ip;
    if (active) {
#pragma unroll
      for (int p = 0; p < kPass; ++p) {
        const int i = i0 + R * p;
        if (i >= N) break;
        double v;
        if (i == kk)
          v = (j == kk) ? ip : rj;
        else if (j == kk)
          v = -ck[i] * ip;
        else
          v = M[i * N + j] - ck[i] * rj;
        M[i * N + j] = v;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < N * N; e += blockDim.x) pinv[e] = (T)(M[e] - jn);
}

static_assert(kCoarseCells <= (long)kCoarseLoads * kCoarseThreads, "coarse loads per thread");
static_assert(kVcCoarsest <= kPinvThreads, "one thread per coarsest cell");
}  // namespace lm

namespace lm {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int tile_x(const PoissonWS &ws, int l) { return ws.vc ? ws.vtx[l] : ws.tx[l]; }
static int tile_y(const PoissonWS &ws, int l) { return ws.vc ? ws.vty[l] : ws.ty[l]; }

// Tile of 2D level l (< lc), or 0 x 0 when no tile divides it.
static void choose_tile(PoissonWS &ws, int l) {
  const Lay &L = ws.lev[l].lay;
  ws.tx[l] = ws.ty[l] = 0;
  if (L.ndim != 2 || ws.nu < 1 || ws.nu > 3 || l >= ws.lc) return;
  const int cand[3][2] = {{TX, TY}, {TXS, TYS}, {16, 16}};
  for (int q = (l == 0 ? 0 : 1); q < 3; ++q)
    if (L.n[0] % cand[q][0] == 0 && L.n[1] % cand[q][1] == 0) {
      ws.tx[l] = cand[q][0];
      ws.ty[l] = cand[q][1];
      return;
    }
}

// Tile of 2D level l (< lc) for the variable-coefficient kernels, whose
// frames carry three more LDS arrays (face coefficients, 1/diagonal): the
// small tiles only.
static void choose_tile_vc(PoissonWS &ws, int l) {
  const Lay &L = ws.lev[l].lay;
  ws.vtx[l] = ws.vty[l] = 0;
  if (!ws.vc_cap || ws.met || L.ndim != 2 || ws.nu < 1 || ws.nu > 3 || l >= ws.lc) return;
  const int cand[2][2] = {{TXS, TYS}, {16, 16}};
  for (int q = 0; q < 2; ++q)
    if (L.n[0] % cand[q][0] == 0 && L.n[1] % cand[q][1] == 0) {
      ws.vtx[l] = cand[q][0];
      ws.vty[l] = cand[q][1];
      return;
    }
}

// Fused 3D level kernels: the owned tile edge is the 32-cell frame less
// twice the x-y halo (down leg 2 nu; up leg 2 nu, plus one on the finest
// level of the single-reduction CG, which also forms w = A u; rounded up to
// even).
static int ti3(int nu, bool down, bool extra) {
  const int h = 2 * nu + ((!down && extra) ? 1 : 0);
  return kF3 - 2 * ((h + 1) & ~1);
}
static int tiles3(const Lay &L, int ti, int d) { return (L.n[d] + ti - 1) / ti; }

// Depth of the z chunk (a multiple of 4): the level is split into as many chunks as
// keep about one block per block slot of the chip (256 CUs, two 512-thread
// blocks each), but no chunk shallower than 16 planes: every chunk reads
// 2H halo planes beyond its own.
static int tz3_of(const Lay &L, int ti) {
  const long tiles = (long)tiles3(L, ti, 0) * tiles3(L, ti, 1);
  long nchunk = std::max(1L, 512L / tiles);
  int tz = (int)((L.n[2] + nchunk - 1) / nchunk);
  tz = std::max(16, (tz + 3) & ~3);  // chunks start on multiples of 4 (the kernels' LDS buffer order)
  return tz;
}

// Blocks of one fused 3D launch on layout L with owned tile edge ti.
static long blocks3d(const Lay &L, int ti) {
  const int tz = tz3_of(L, ti);
  return (long)tiles3(L, ti, 0) * tiles3(L, ti, 1) * ((L.n[2] + tz - 1) / tz);
}

// Level l runs the fused 3D kernels (fully periodic grids, even sizes).
static bool fused3d(const PoissonWS &ws, int l) {
  const Lay &L = ws.lev[l].lay;
  return !ws.vc && L.ndim == 3 && ws.bnd.all_periodic && ws.nu >= 1 && ws.nu <= 2 && l < ws.lc &&
         L.ncells() >= kFused3DMinCells && L.n[0] % 2 == 0 && L.n[1] % 2 == 0 && L.n[2] % 2 == 0 &&
         L.n[2] >= 16;
}

// Blocks of the finest level's up kernel with w = A u (its partials).
static long blocks3d_w(const PoissonWS &ws) { return blocks3d(ws.lev[0].lay, ti3(ws.nu, false, true)); }

static bool fused_level(const PoissonWS &ws, int l) { return tile_x(ws, l) > 0; }

bool poisson_plan(PoissonWS &ws, Carver &cv, const Lay &fine, const Bnd &B, const double h[3], int mixed, int flexible,
                  int nu, int vc_cap, std::string *err) {
  ws.lay = fine;
  ws.bnd = B;
  ws.mixed = mixed;
  ws.nu = nu;
  ws.vc_cap = vc_cap;
  ws.vc = 0;
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
    if (!even || N <= 64 || nl == kMaxLev) break;
    for (int d = 0; d < ndim; ++d) {
      n[d] /= 2;
      hh[d] *= 2.0;
    }
  }
  ws.nlev = nl;
  if (ws.met) {
    // volume-weighted operator: unit coefficients on the finest level, a
    // quarter per coarser level (the restriction averages the 4 children
    // of a residual whose coarse operator sums them)
    for (int l = 0; l < nl; ++l)
      for (int d = 0; d < 3; ++d) ws.lev[l].ih2[d] = d < ndim ? std::ldexp(1.0, -2 * l) : 0.0;
  }
  const long ncoarsest = ws.lev[nl - 1].lay.ncells();
  if (ncoarsest > kMaxCoarsest) {
    if (err) *err = "grid does not coarsen to <= 1024 cells (need even sizes down to the coarse grid)";
    return false;
  }
  ws.lc = 0;
  while (ws.lc < nl - 1 && ws.lev[ws.lc].lay.ncells() > kCoarseCells) ++ws.lc;
  long lds = 0;
  for (int l = ws.lc; l < nl; ++l) lds += ws.lev[l].lay.ncells();
  if (lds > kCoarseLds || nl - ws.lc > kCoarseLev) {
    if (err) *err = "coarse grid too large for the one-block coarse solver";
    return false;
  }
  if (vc_cap && ncoarsest > kVcCoarsest) {
    if (err) *err = "the variable-coefficient solve needs a grid that coarsens to <= 128 cells";
    return false;
  }
  const size_t fbytes = (size_t)fine.total * 8;
  ws.x = (double *)cv.take(fbytes);
  ws.r[0] = (double *)cv.take(fbytes);
  ws.r[1] = (double *)cv.take(fbytes);
  ws.p[0] = (double *)cv.take(fbytes);
  ws.p[1] = (double *)cv.take(fbytes);
  ws.q = (double *)cv.take(fbytes);
  ws.cgcg = !flexible;
  // grids the one-block V-cycle covers from the finest level: the whole
  // single-reduction solve in one workgroup (LM_BLOCK_PCG=0 turns it off)
  {
    const char *env = std::getenv("LM_BLOCK_PCG");
    const bool off = env && env[0] == '0';
    ws.block_pcg = !off && ws.cgcg && ws.lc == 0 && fine.ncells() <= (long)kCoarseLoads * kCoarseThreads;
    // its scratch: 2 ndim + 1 coefficient vectors, p, s, w and r (compact cell order)
    ws.blk = ws.block_pcg ? (double *)cv.take((size_t)(2 * fine.ndim + 5) * fine.ncells() * 8) : nullptr;
  }
  ws.w = (double *)cv.take(fbytes);
  ws.s[0] = (double *)cv.take(fbytes);
  ws.s[1] = (double *)cv.take(fbytes);
  ws.z[0] = cv.take((size_t)fine.total * eb);
  ws.z[1] = (mixed && !ws.cgcg) ? cv.take((size_t)fine.total * eb) : ws.z[0];  // z_old: flexible CG only
  ws.zpre = cv.take((size_t)fine.total * eb);
  ws.lev[0].x = nullptr;
  ws.lev[0].xpost = nullptr;
  ws.lev[0].b = nullptr;
  for (int l = 1; l < nl; ++l) {
    const size_t lb = (size_t)ws.lev[l].lay.total * eb;
    ws.lev[l].x = cv.take(lb);
    ws.lev[l].xpost = cv.take(lb);
    ws.lev[l].b = cv.take(lb);
  }
  ws.pinv = cv.take((size_t)ncoarsest * ncoarsest * eb);
  ws.rho64 = nullptr;
  ws.rho_c = ws.pinv_vc = nullptr;
  for (int l = 0; l < kMaxLev; ++l) ws.rho[l] = nullptr;
  if (vc_cap) {
    ws.rho64 = (double *)cv.take(fbytes);
    ws.rho[0] = mixed ? cv.take((size_t)fine.total * eb) : (void *)ws.rho64;
    for (int l = 1; l < nl; ++l) ws.rho[l] = cv.take((size_t)ws.lev[l].lay.total * eb);
    ws.rho_c = cv.take((size_t)(kCoarseLds + 1) * eb);
    ws.pinv_vc = cv.take((size_t)ncoarsest * ncoarsest * eb);
  }
  for (int l = 0; l < kMaxLev; ++l)
    for (int q = 0; q < 3; ++q) ws.cf[l][q] = nullptr;
  for (int l = 0; l < kMaxLev; ++l) {
    ws.tx[l] = ws.ty[l] = 0;
    ws.vtx[l] = ws.vty[l] = 0;
    if (l < nl) {
      choose_tile(ws, l);
      choose_tile_vc(ws, l);
    }
    if (ws.vtx[l] > 0)
      for (int q = 0; q < 3; ++q) ws.cf[l][q] = cv.take((size_t)ws.lev[l].lay.total * eb);
  }
  long npmax = kRedBlocks;
  if (ws.tx[0] > 0) npmax = std::max(npmax, (long)(fine.n[0] / ws.tx[0]) * (fine.n[1] / ws.ty[0]) + 1);
  if (ws.vtx[0] > 0) npmax = std::max(npmax, (long)(fine.n[0] / ws.vtx[0]) * (fine.n[1] / ws.vty[0]) + 1);
  if (fused3d(ws, 0) && blocks3d_w(ws) > npmax) npmax = blocks3d_w(ws);
  ws.np_max = npmax;
  ws.part_cc = (double *)cv.take((size_t)npmax * 8);
  ws.part_pq = (double *)cv.take((size_t)npmax * 8);
  ws.part_rz = (double *)cv.take((size_t)3 * npmax * 8);
  ws.partials = (double *)cv.take((size_t)(nblocks_for(fine) + kRedBlocks) * 8 + 64);
  ws.sc = (SolverScalars *)cv.take(sizeof(SolverScalars));
  ws.vol = nullptr;
  ws.met_w = nullptr;
  ws.met_tab = nullptr;
  if (ws.met) {
    long nw = 0, nt = 0;
    for (int l = 0; l < nl; ++l) nw += ws.lev[l].lay.n[0] + ws.lev[l].lay.n[1];
    for (int l = ws.lc; l < nl; ++l) nt += 2 * (ws.lev[l].lay.n[0] + ws.lev[l].lay.n[1]);
    if (nt > kCoarseLds) {
      if (err) *err = "stretched grid: the coarse levels' spacing tables exceed the one-block kernel's LDS";
      return false;
    }
    ws.vol = (double *)cv.take(fbytes);
    ws.met_w = (double *)cv.take((size_t)nw * 8);
    ws.met_tab = cv.take((size_t)nt * eb);
  }
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
  for (long col = 0; col < N; ++col) {  // Gauss-Jordan, partial pivoting
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

template <typename T>
static Ih2<T> ih2_of(const PoissonWS &ws, int l) {
  Ih2<T> v;
  for (int d = 0; d < 3; ++d) v.v[d] = (T)ws.lev[l].ih2[d];
  return v;
}

// Arrays of level l: input (pre-smoothed) and output (post-smoothed)
// corrections. Unfused levels smooth in place.
template <typename T>
static T *lev_xin(PoissonWS &ws, int l, void *z) {
  if (l == 0) return (fused_level(ws, 0) || fused3d(ws, 0)) ? (T *)ws.zpre : (T *)z;
  return (T *)ws.lev[l].x;
}
template <typename T>
static T *lev_xout(PoissonWS &ws, int l, void *z) {
  if (l == 0) return (T *)z;
  if (l >= ws.lc) return (T *)ws.lev[l].x;
  return ((fused_level(ws, l) || fused3d(ws, l)) ? (T *)ws.lev[l].xpost : (T *)ws.lev[l].x);
}

template <typename T>
static Fused3DArgs<T> f3_args(PoissonWS &ws, int l, const void *b, int b_double) {
  Fused3DArgs<T> a;
  const Lay &L = ws.lev[l].lay;
  a.Lf = L;
  a.Lc = ws.lev[l + 1].lay;
  a.ihx = (T)ws.lev[l].ih2[0];
  a.ihy = (T)ws.lev[l].ih2[1];
  a.ihz = (T)ws.lev[l].ih2[2];
  a.dihx = ws.lev[l].ih2[0];
  a.dihy = ws.lev[l].ih2[1];
  a.dihz = ws.lev[l].ih2[2];
  a.idg = (T)(1.0 / (2.0 * (ws.lev[l].ih2[0] + ws.lev[l].ih2[1] + ws.lev[l].ih2[2])));
  a.tiles_x = a.tiles_y = a.tz = 0;  // set by launch_3d for the leg
  a.b = b;
  a.b_double = b_double;
  a.xpre = nullptr;
  a.xc = nullptr;
  a.xout = nullptr;
  a.bc = (T *)ws.lev[l + 1].b;
  a.sc = ws.sc;
  return a;
}

// Launch with optional start/stop events bound to the dispatch itself: they
// bracket the kernel's execution, not the queueing gap before it.
template <typename K, typename A>
static void launch_ev(K kern, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const A &a) {
  if (e0)
    hipExtLaunchKernelGGL(kern, g, dim3(kBlock), 0, st, e0, e1, 0, a);
  else
    hipLaunchKernelGGL(kern, g, dim3(kBlock), 0, st, a);
}

template <typename T>
static void launch_3d(int nu, bool down, Fused3DArgs<T> &a, hipStream_t st, bool extra = false,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const int ti = ti3(nu, down, extra);
  a.tiles_x = tiles3(a.Lf, ti, 0);
  a.tiles_y = tiles3(a.Lf, ti, 1);
  a.tz = tz3_of(a.Lf, ti);
  const dim3 g((unsigned)blocks3d(a.Lf, ti));
  const dim3 bl(kF3Threads);
  // FP64 right-hand side in FP32 kernels only on the finest level
  const bool bd = a.b_double && sizeof(T) == 4;
  if (down) {
    auto k = nu == 1 ? (bd ? &k_mg_down3d<T, 1, true> : &k_mg_down3d<T, 1, false>)
                     : (bd ? &k_mg_down3d<T, 2, true> : &k_mg_down3d<T, 2, false>);
    if (e0)
      hipExtLaunchKernelGGL(k, g, bl, 0, st, e0, e1, 0, a);
    else
      hipLaunchKernelGGL(k, g, bl, 0, st, a);
  } else {
    auto k = extra ? (nu == 1 ? (bd ? &k_mg_up3d<T, 1, 1, true> : &k_mg_up3d<T, 1, 1, false>)
                              : (bd ? &k_mg_up3d<T, 2, 1, true> : &k_mg_up3d<T, 2, 1, false>))
                   : (nu == 1 ? (bd ? &k_mg_up3d<T, 1, 0, true> : &k_mg_up3d<T, 1, 0, false>)
                              : (bd ? &k_mg_up3d<T, 2, 0, true> : &k_mg_up3d<T, 2, 0, false>));
    if (e0)
      hipExtLaunchKernelGGL(k, g, bl, 0, st, e0, e1, 0, a);
    else
      hipLaunchKernelGGL(k, g, bl, 0, st, a);
  }
}

// The finest 3D up kernel forms w = A u and the single-reduction CG partials.
static bool w_in_up3d(const PoissonWS &ws) { return ws.cgcg && fused3d(ws, 0); }

template <typename T, int TXT, int TYT>
static void launch_nu_t(int nu, Down2DArgs<T> &a, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (nu == 1) launch_ev(&k_mg_down2d<T, 1, TXT, TYT>, g, st, e0, e1, a);
  else if (nu == 2) launch_ev(&k_mg_down2d<T, 2, TXT, TYT>, g, st, e0, e1, a);
  else launch_ev(&k_mg_down2d<T, 3, TXT, TYT>, g, st, e0, e1, a);
}
template <typename T, int TXT, int TYT>
static void launch_nu_t(int nu, Up2DArgs<T> &a, dim3 g, hipStream_t st, bool extra) {
  if (extra) {
    if (nu == 1) hipLaunchKernelGGL((k_mg_up2d<T, 1, 1, TXT, TYT>), g, dim3(kBlock), 0, st, a);
    else if (nu == 2) hipLaunchKernelGGL((k_mg_up2d<T, 2, 1, TXT, TYT>), g, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_mg_up2d<T, 3, 1, TXT, TYT>), g, dim3(kBlock), 0, st, a);
    return;
  }
  if (nu == 1) hipLaunchKernelGGL((k_mg_up2d<T, 1, 0, TXT, TYT>), g, dim3(kBlock), 0, st, a);
  else if (nu == 2) hipLaunchKernelGGL((k_mg_up2d<T, 2, 0, TXT, TYT>), g, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_mg_up2d<T, 3, 0, TXT, TYT>), g, dim3(kBlock), 0, st, a);
}
template <typename T, int TXT, int TYT>
static void launch_nu_vc(int nu, Down2DArgs<T> &a, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (nu == 1) launch_ev(&k_mg_down2d<T, 1, TXT, TYT, true>, g, st, e0, e1, a);
  else if (nu == 2) launch_ev(&k_mg_down2d<T, 2, TXT, TYT, true>, g, st, e0, e1, a);
  else launch_ev(&k_mg_down2d<T, 3, TXT, TYT, true>, g, st, e0, e1, a);
}
template <typename T, int TXT, int TYT>
static void launch_nu_vc(int nu, Up2DArgs<T> &a, dim3 g, hipStream_t st, bool extra) {
  if (extra) {
    if (nu == 1) hipLaunchKernelGGL((k_mg_up2d<T, 1, 1, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
    else if (nu == 2) hipLaunchKernelGGL((k_mg_up2d<T, 2, 1, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL((k_mg_up2d<T, 3, 1, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
    return;
  }
  if (nu == 1) hipLaunchKernelGGL((k_mg_up2d<T, 1, 0, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
  else if (nu == 2) hipLaunchKernelGGL((k_mg_up2d<T, 2, 0, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL((k_mg_up2d<T, 3, 0, TXT, TYT, true>), g, dim3(kBlock), 0, st, a);
}
// Level 0 runs the large tile, coarser levels the small one; the
// variable-coefficient kernels run the small tiles only.
template <typename T>
static void launch_nu(const PoissonWS &ws, int l, int nu, Down2DArgs<T> &a, hipStream_t st, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr) {
  const int tx = tile_x(ws, l), ty = tile_y(ws, l);
  const dim3 g((a.Lf.n[0] / tx) * (a.Lf.n[1] / ty));
  if (ws.vc) {
    if (tx == TXS && ty == TYS)
      launch_nu_vc<T, TXS, TYS>(nu, a, g, st, e0, e1);
    else
      launch_nu_vc<T, 16, 16>(nu, a, g, st, e0, e1);
    return;
  }
  if (tx == TX && ty == TY)
    launch_nu_t<T, TX, TY>(nu, a, g, st, e0, e1);
  else if (tx == TXS && ty == TYS)
    launch_nu_t<T, TXS, TYS>(nu, a, g, st, e0, e1);
  else
    launch_nu_t<T, 16, 16>(nu, a, g, st, e0, e1);
}
template <typename T>
static void launch_nu(const PoissonWS &ws, int l, int nu, Up2DArgs<T> &a, hipStream_t st, bool extra) {
  const int tx = tile_x(ws, l), ty = tile_y(ws, l);
  const dim3 g((a.Lf.n[0] / tx) * (a.Lf.n[1] / ty));
  if (ws.vc) {
    if (tx == TXS && ty == TYS)
      launch_nu_vc<T, TXS, TYS>(nu, a, g, st, extra);
    else
      launch_nu_vc<T, 16, 16>(nu, a, g, st, extra);
    return;
  }
  if (tx == TX && ty == TY)
    launch_nu_t<T, TX, TY>(nu, a, g, st, extra);
  else if (tx == TXS && ty == TYS)
    launch_nu_t<T, TXS, TYS>(nu, a, g, st, extra);
  else
    launch_nu_t<T, 16, 16>(nu, a, g, st, extra);
}

template <typename T>
static Down2DArgs<T> down_args(PoissonWS &ws, int l, int k, const void *b, T *xpre, double *x, const double *p,
                               const double *q, double *rnew) {
  Down2DArgs<T> a;
  const Lay &L = ws.lev[l].lay;
  a.Lf = L;
  a.Lc = ws.lev[l + 1].lay;
  a.B = ws.bnd;
  a.ihx = (T)ws.lev[l].ih2[0];
  a.ihy = (T)ws.lev[l].ih2[1];
  a.idg = (T)(1.0 / (2.0 * ws.lev[l].ih2[0] + 2.0 * ws.lev[l].ih2[1]));
  a.finest = (l == 0);
  a.k = k;
  a.b = b;
  a.xpre = xpre;
  a.bc = (T *)ws.lev[l + 1].b;
  a.x = x;
  a.p = p;
  a.q = q;
  a.rnew = rnew;
  a.part_pq = ws.part_pq;
  a.np_pq = kRedBlocks;
  a.sc = ws.sc;
  a.tiles_x = L.n[0] / tile_x(ws, l);
  // single-reduction CG (finest level, FP64)
  a.cgcg = ws.cgcg && l == 0;
  a.u = (const T *)ws.z[0];
  a.w = ws.w;
  a.s_old = ws.s[k & 1];
  a.s_new = ws.s[(k + 1) & 1];
  a.p_io = ws.p[0];
  a.part_g = ws.part_rz;
  a.part_cc = ws.part_cc;
  a.np_g = fused_level(ws, 0) ? (ws.lay.n[0] / tile_x(ws, 0)) * (ws.lay.n[1] / tile_y(ws, 0)) : 0;
  a.np_cc = kRedBlocks;
  a.tol2 = ws.tol2;
  a.cfx = ws.vc ? (const T *)ws.cf[l][0] : nullptr;
  a.cfy = ws.vc ? (const T *)ws.cf[l][1] : nullptr;
  a.cig = ws.vc ? (const T *)ws.cf[l][2] : nullptr;
  return a;
}

template <typename T>
static Up2DArgs<T> up_args(PoissonWS &ws, int l, const T *xpre, const T *xc, const void *b, T *xout,
                           const T *zold) {
  Up2DArgs<T> a;
  const Lay &L = ws.lev[l].lay;
  a.Lf = L;
  a.Lc = ws.lev[l + 1].lay;
  a.B = ws.bnd;
  a.ihx = (T)ws.lev[l].ih2[0];
  a.ihy = (T)ws.lev[l].ih2[1];
  a.dihx = ws.lev[l].ih2[0];
  a.dihy = ws.lev[l].ih2[1];
  a.idg = (T)(1.0 / (2.0 * ws.lev[l].ih2[0] + 2.0 * ws.lev[l].ih2[1]));
  a.xpre = xpre;
  a.xc = xc;
  a.b = b;
  a.xout = xout;
  a.finest = (l == 0);
  a.zold = zold;
  a.part_rz = ws.part_rz;
  a.np = (L.n[0] / tile_x(ws, l)) * (L.n[1] / tile_y(ws, l));
  a.sc = ws.sc;
  a.tiles_x = L.n[0] / tile_x(ws, l);
  a.w = ws.w;
  a.cfx = ws.vc ? (const T *)ws.cf[l][0] : nullptr;
  a.cfy = ws.vc ? (const T *)ws.cf[l][1] : nullptr;
  a.cig = ws.vc ? (const T *)ws.cf[l][2] : nullptr;
  a.rho64 = ws.vc ? ws.rho64 : nullptr;
  return a;
}

template <typename T>
static CoarseArgs<T> coarse_args(PoissonWS &ws, void *z, const double *r) {
  CoarseArgs<T> ca;
  ca.l0 = ws.lc;
  ca.nlev = ws.nlev;
  ca.nu = ws.nu;
  ca.B = ws.bnd;
  int off = 0;
  auto lg2 = [](int v) {
    int q = 0;
    while ((1 << q) < v) ++q;
    return (1 << q) == v ? q : -1;
  };
  for (int l = 0; l < ws.nlev; ++l) {
    for (int d = 0; d < 3; ++d) ca.n[l][d] = ws.lev[l].lay.n[d];
    ca.lg[l][0] = lg2(ws.lev[l].lay.n[0] / 2);
    ca.lg[l][1] = lg2(ws.lev[l].lay.n[1]);
    ca.ih2[l] = ih2_of<T>(ws, l);
    ca.off[l] = l >= ws.lc ? off : 0;
    if (l >= ws.lc) off += (int)ws.lev[l].lay.ncells();
  }
  for (int q = 0; q < kCoarseLev; ++q) {
    const int l = ws.lc + q;
    for (int code = 0; code < 8; ++code) {
      double dg = 0.0;
      if (l < ws.nlev)
        for (int d = 0; d < ws.lay.ndim; ++d) dg += ws.lev[l].ih2[d] * (((code >> d) & 1) ? 2.0 : 1.0);
      ca.idg[q][code] = dg > 0.0 ? (T)(1.0 / dg) : T(0);
    }
  }
  ca.L0 = ws.lev[ws.lc].lay;
  ca.b0 = ws.lc == 0 ? (const void *)r : ws.lev[ws.lc].b;
  ca.b0_double = (ws.lc == 0);
  ca.x0 = ws.lc == 0 ? (T *)z : (T *)ws.lev[ws.lc].x;
  ca.pinv = (const T *)(ws.vc ? ws.pinv_vc : ws.pinv);
  ca.rho_c = ws.vc ? (const T *)ws.rho_c : nullptr;
  ca.met = ws.met;
  int toff = 0;
  for (int l = 0; l < kMaxLev; ++l) {
    ca.toff[l] = toff;
    if (ws.met && l >= ws.lc && l < ws.nlev) toff += 2 * (ws.lev[l].lay.n[0] + ws.lev[l].lay.n[1]);
  }
  ca.mtab = ws.met ? (const T *)ws.met_tab : nullptr;
  ca.mtab_n = ws.met ? toff : 0;
  return ca;
}

// In-step timing: events for this launch when it is the next timed launch
// of the selected kernel class (0 finest down, 1 finest up, 2 CG update);
// the caller records the iteration after launching.
static bool timed_launch(const PoissonWS &ws, int which, hipEvent_t &e0, hipEvent_t &e1) {
  e0 = e1 = nullptr;
  if (ws.twhich != which || ws.tcount >= ws.tcap) return false;
  e0 = ws.tev[2 * ws.tcount];
  e1 = ws.tev[2 * ws.tcount + 1];
  return true;
}

// V-cycle of iteration k on b = r_k (finest), writing z = z_k.
template <int DIM, typename T>
static void vcycle(hipStream_t st, PoissonWS &ws, int k, const CGArgs &cg) {
  const Bnd &B = ws.bnd;
  const int nu = ws.nu;
  const SolverScalars *sc = ws.sc;
  void *z = ws.z[k & 1];
  const double *r = ws.r[k & 1];
  const double *rprev = ws.r[(k + 1) & 1];
  dim3 bb(kBX, kBY);
  for (int l = 0; l < ws.lc; ++l) {
    const Lay &L = ws.lev[l].lay, &Lc = ws.lev[l + 1].lay;
    T *xin = lev_xin<T>(ws, l, z);
    if (fused_level(ws, l)) {
      const void *b = l == 0 ? (k >= 1 ? (const void *)rprev : (const void *)r) : ws.lev[l].b;
      Down2DArgs<T> a = down_args<T>(ws, l, k, b, xin, cg.x, cg.pnew, cg.q, ws.r[k & 1]);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool timed = l == 0 && timed_launch(ws, 0, e0, e1);
      launch_nu<T>(ws, l, nu, a, st, e0, e1);
      if (timed) ws.tk[ws.tcount++] = k;
    } else if (fused3d(ws, l)) {
      Fused3DArgs<T> a = f3_args<T>(ws, l, l == 0 ? (const void *)r : ws.lev[l].b, l == 0);
      a.xout = xin;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool timed = l == 0 && timed_launch(ws, 0, e0, e1);
      launch_3d<T>(nu, true, a, st, false, e0, e1);
      if (timed) ws.tk[ws.tcount++] = k;
    } else {
      dim3 g = grid_for(L);
      const T *rl = ws.vc ? (const T *)ws.rho[l] : nullptr;
      for (int s = 0; s < nu; ++s) {
        for (int color = 0; color < 2; ++color) {
          if (l == 0)
            hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, bb, 0, st, L, B, ih2_of<T>(ws, l), xin, r, color,
                               s == 0 && color == 0, sc, rl, ws.met);
          else
            hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, bb, 0, st, L, B, ih2_of<T>(ws, l), xin,
                               (const T *)ws.lev[l].b, color, s == 0 && color == 0, sc, rl, ws.met);
        }
      }
      if (l == 0)
        hipLaunchKernelGGL((k_mg_restrict<DIM, T, double>), grid_for(Lc), bb, 0, st, L, Lc, B, ih2_of<T>(ws, l),
                           xin, r, (T *)ws.lev[l + 1].b, sc, rl, ws.met);
      else
        hipLaunchKernelGGL((k_mg_restrict<DIM, T, T>), grid_for(Lc), bb, 0, st, L, Lc, B, ih2_of<T>(ws, l), xin,
                           (const T *)ws.lev[l].b, (T *)ws.lev[l + 1].b, sc, rl, ws.met);
    }
  }
  if (DIM == 2 && ws.met)
    hipLaunchKernelGGL((k_mg_coarse<DIM, T, true, DIM == 2>), dim3(1), dim3(kCoarseThreads), 0, st,
                       coarse_args<T>(ws, z, r), sc);
  else if (ws.vc)
    hipLaunchKernelGGL((k_mg_coarse<DIM, T, true>), dim3(1), dim3(kCoarseThreads), 0, st, coarse_args<T>(ws, z, r), sc);
  else
    hipLaunchKernelGGL((k_mg_coarse<DIM, T>), dim3(1), dim3(kCoarseThreads), 0, st, coarse_args<T>(ws, z, r), sc);
  for (int l = ws.lc - 1; l >= 0; --l) {
    const Lay &L = ws.lev[l].lay, &Lc = ws.lev[l + 1].lay;
    T *xin = lev_xin<T>(ws, l, z);
    T *xout = lev_xout<T>(ws, l, z);
    const T *xc = lev_xout<T>(ws, l + 1, z);
    if (fused_level(ws, l)) {
      const T *zold = (l == 0 && !ws.cgcg && k >= 1) ? (const T *)ws.z[(k + 1) & 1] : nullptr;
      Up2DArgs<T> a = up_args<T>(ws, l, xin, xc, l == 0 ? (const void *)r : ws.lev[l].b, xout, zold);
      launch_nu<T>(ws, l, nu, a, st, ws.cgcg && l == 0);
    } else if (fused3d(ws, l)) {
      Fused3DArgs<T> a = f3_args<T>(ws, l, l == 0 ? (const void *)r : ws.lev[l].b, l == 0);
      a.xpre = xin;
      a.xc = xc;
      a.xout = xout;
      const bool extra = l == 0 && w_in_up3d(ws);
      a.w = ws.w;
      a.part_rz = ws.part_rz;
      a.np = (int)blocks3d(L, ti3(nu, false, extra));
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool timed = l == 0 && timed_launch(ws, 1, e0, e1);
      launch_3d<T>(nu, false, a, st, extra, e0, e1);
      if (timed) ws.tk[ws.tcount++] = k;
    } else {
      dim3 g = grid_for(L);
      const T *rl = ws.vc ? (const T *)ws.rho[l] : nullptr;
      hipLaunchKernelGGL((k_mg_prolong<DIM, T>), g, bb, 0, st, L, Lc, xin, xc, sc);
      for (int s = 0; s < nu; ++s) {
        for (int cc = 0; cc < 2; ++cc) {
          const int color = 1 - cc;
          if (l == 0)
            hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), g, bb, 0, st, L, B, ih2_of<T>(ws, l), xin, r, color, 0,
                               sc, rl, ws.met);
          else
            hipLaunchKernelGGL((k_mg_smooth<DIM, T, T>), g, bb, 0, st, L, B, ih2_of<T>(ws, l), xin,
                               (const T *)ws.lev[l].b, color, 0, sc, rl, ws.met);
        }
      }
    }
  }
  if (!fused_level(ws, 0)) {
    CGArgs a = cg;
    a.rnew = ws.r[k & 1];
    a.z = z;
    a.zold = (!ws.cgcg && k >= 1) ? ws.z[(k + 1) & 1] : nullptr;
    a.np_rz = kRedBlocks;
    if (ws.cgcg) {
      if (!w_in_up3d(ws)) hipLaunchKernelGGL((k_cgcg_w<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, a, ws.w);
    } else
      hipLaunchKernelGGL((k_cg_rz<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, a);
  }
}

static int np_rz_of(const PoissonWS &ws) {
  if (fused_level(ws, 0)) return (ws.lay.n[0] / tile_x(ws, 0)) * (ws.lay.n[1] / tile_y(ws, 0));
  if (w_in_up3d(ws)) return (int)blocks3d_w(ws);
  return kRedBlocks;
}

template <int DIM, typename T>
static void iteration(hipStream_t st, PoissonWS &ws, CGArgs a, int k) {
  a.k = k;
  if (ws.cgcg) {
    // single-reduction CG: the update runs in the finest down kernel, or
    // in its own kernel when that level is not tiled
    if (!fused_level(ws, 0)) {
      a.z = ws.z[0];
      a.pnew = ws.p[0];
      a.rold = ws.r[(k - 1) & 1];
      a.rnew = ws.r[k & 1];
      a.np_rz = np_rz_of(ws);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool timed = timed_launch(ws, 2, e0, e1);
      if (timed)
        hipExtLaunchKernelGGL((k_cgcg_update<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, e0, e1, 0, a,
                              kRedBlocks, (const double *)ws.w, (const double *)ws.s[k & 1], ws.s[(k + 1) & 1]);
      else
        hipLaunchKernelGGL((k_cgcg_update<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, a, kRedBlocks,
                           (const double *)ws.w, (const double *)ws.s[k & 1], ws.s[(k + 1) & 1]);
      if (timed) ws.tk[ws.tcount++] = k;
    }
    vcycle<DIM, T>(st, ws, k, a);
    return;
  }
  // pq(k): p_k = z_{k-1} + beta p_{k-1}
  a.z = ws.z[(k - 1) & 1];
  a.pold = ws.p[(k - 1) & 1];
  a.pnew = ws.p[k & 1];
  a.np_rz = np_rz_of(ws);
  a.flexible = !ws.cgcg;
  hipLaunchKernelGGL((k_cg_pq<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, a, kRedBlocks);
  a.np_pq = kRedBlocks;
  if (!fused_level(ws, 0)) {
    a.rold = ws.r[(k - 1) & 1];
    a.rnew = ws.r[k & 1];
    hipLaunchKernelGGL((k_cg_update<DIM>), dim3(kRedBlocks), dim3(kBlock), 0, st, a);
  }
  vcycle<DIM, T>(st, ws, k, a);
}

// The whole solve as one k_pcg_block launch (ws.block_pcg). With a log the
// outcome is left on the device for the caller to read later; without one
// this waits for it.
template <int DIM, typename T>
static hipError_t solve_block(hipStream_t st, PoissonWS &ws, const double *bvec, const double *x0, double rtol,
                              int maxit, int *iters, double *relres, int *converged, SolveLog *log) {
  BlockPCGArgs<T> pa;
  pa.ca = coarse_args<T>(ws, ws.z[0], ws.r[0]);
  pa.L = ws.lay;
  pa.B = ws.bnd;
  for (int d = 0; d < 3; ++d) {
    pa.ih2[d] = ws.lev[0].ih2[d];
    pa.ih[d] = std::sqrt(ws.lev[0].ih2[d]);
  }
  pa.b = bvec;
  pa.x0 = x0;
  pa.x = ws.x;
  pa.rho = ws.vc ? ws.rho64 : nullptr;
  pa.met = ws.met;
  pa.vol = ws.met ? ws.vol : nullptr;
  pa.mean_w = ws.met ? ws.volume : (double)ws.lay.ncells();
  pa.tol2 = rtol * rtol;
  pa.maxit = maxit;
  pa.cf = ws.blk;
  pa.sc = ws.sc;
  pa.log = log;
  ws.tol2 = pa.tol2;
  if (DIM == 2 && ws.met)
    hipLaunchKernelGGL((k_pcg_block<DIM, T, true, DIM == 2>), dim3(1), dim3(kCoarseThreads), 0, st, pa);
  else if (ws.vc)
    hipLaunchKernelGGL((k_pcg_block<DIM, T, true>), dim3(1), dim3(kCoarseThreads), 0, st, pa);
  else
    hipLaunchKernelGGL((k_pcg_block<DIM, T, false>), dim3(1), dim3(kCoarseThreads), 0, st, pa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || log) return e;
  e = hipMemcpyAsync(ws.host_sc, ws.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const SolverScalars &h = *ws.host_sc;
  *iters = h.iters;
  *relres = h.cc > 0 ? std::sqrt(h.rr / h.cc) : 0.0;
  *converged = h.done && !h.nonconv;
  return hipSuccess;
}

template <int DIM, typename T>
static hipError_t solve_dim(hipStream_t st, PoissonWS &ws, const double *bvec, const double *x0, double rtol,
                            int maxit, int expect, int *iters, double *relres, int *converged, SolveLog *log) {
  if (ws.block_pcg) return solve_block<DIM, T>(st, ws, bvec, x0, rtol, maxit, iters, relres, converged, log);
  if (log) return hipErrorInvalidValue;
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
  a.rold = nullptr;
  a.rnew = ws.r[0];
  a.pold = a.pnew = nullptr;
  a.q = ws.q;
  a.z = a.zold = nullptr;
  a.part_cc = ws.part_cc;
  a.part_pq = ws.part_pq;
  a.part_rz = ws.part_rz;
  a.np_rz = np_rz_of(ws);
  a.np_pq = kRedBlocks;
  a.sc = ws.sc;
  a.tol2 = rtol * rtol;
  ws.tol2 = a.tol2;
  a.k = 0;
  a.flexible = !ws.cgcg;
  a.rho = ws.vc ? ws.rho64 : nullptr;
  a.met = ws.met;
  a.vol = ws.met ? ws.vol : nullptr;
  ws.tsolve0 = ws.tcount;
  hipError_t e = hipMemsetAsync(&ws.sc->done, 0, 4 * sizeof(int), st);  // done, iters, zero, nonconv
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cg_init<DIM>), grid_for(ws.lay), dim3(kBX, kBY), 0, st, a, ws.partials);
  hipLaunchKernelGGL(k_fold_partials, dim3(kRedBlocks), dim3(kBlock), 0, st, (const double *)ws.partials,
                     nblocks_for(ws.lay), ws.part_cc);
  vcycle<DIM, T>(st, ws, 0, a);
  int k = 1;
  int batch = expect > 0 ? expect + 1 : 4;
  while (true) {
    for (int q = 0; q < batch && k <= maxit + 1; ++q, ++k) iteration<DIM, T>(st, ws, a, k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ws.host_sc, ws.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (ws.host_sc->done || k > maxit + 1) break;
    batch = 2;
  }
  const SolverScalars &h = *ws.host_sc;
  *iters = h.iters;
  // timed launches of this solve that did the full work of a CG iteration
  // with a previous direction: iterations 2 .. iters (iteration 0 has no
  // CG update, iteration 1 no old p and s; later ones found the solve done)
  for (int q = ws.tsolve0; q < ws.tcount; ++q)
    if (ws.tk[q] < 2 || ws.tk[q] > h.iters) ws.tk[q] = -1;
  *relres = h.cc > 0 ? std::sqrt(h.rr / h.cc) : 0.0;
  *converged = h.done && !h.nonconv;
  // mean of the solution (the stored pressure is zero-mean)
  hipLaunchKernelGGL((k_sum_x<DIM>), dim3(kRedBlocks), dim3(kBlock), 0, st, ws.lay, (const double *)ws.x,
                     ws.partials, ws.met ? (const double *)ws.vol : (const double *)nullptr);
  hipLaunchKernelGGL(k_fin_mean_x, dim3(1), dim3(kBlock), 0, st, (const double *)ws.partials, kRedBlocks,
                     ws.met ? ws.volume : (double)ws.lay.ncells(), ws.sc);
  return hipGetLastError();
}

hipError_t poisson_solve(hipStream_t st, PoissonWS &ws, const double *b, const double *x0, double rtol,
                         int maxit, int expect_iters, int *iters, double *relres, int *converged, SolveLog *log) {
  if (ws.lay.ndim == 3)
    return ws.mixed ? solve_dim<3, float>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged, log)
                    : solve_dim<3, double>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged, log);
  return ws.mixed ? solve_dim<2, float>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged, log)
                  : solve_dim<2, double>(st, ws, b, x0, rtol, maxit, expect_iters, iters, relres, converged, log);
}

// ---------------------------------------------------------------------------
// Variable-coefficient set-up
// ---------------------------------------------------------------------------
template <int DIM, typename T>
static hipError_t set_beta_dim(hipStream_t st, PoissonWS &ws) {
  const dim3 bb(kBX, kBY);
  const bool cast = sizeof(T) != 8;
  hipLaunchKernelGGL((k_vc_rho0<DIM, T>), grid_for(ws.lay), bb, 0, st, ws.lay, (const double *)ws.rho64,
                     cast ? (T *)ws.rho[0] : (T *)nullptr, ws.sc);
  for (int l = 0; l + 1 < ws.nlev; ++l) {
    const Lay &Lf = ws.lev[l].lay, &Lc = ws.lev[l + 1].lay;
    if (l == 0)
      hipLaunchKernelGGL((k_vc_rho_down<DIM, double, T>), grid_for(Lc), bb, 0, st, Lf, Lc,
                         (const double *)ws.rho64, (T *)ws.rho[1]);
    else
      hipLaunchKernelGGL((k_vc_rho_down<DIM, T, T>), grid_for(Lc), bb, 0, st, Lf, Lc, (const T *)ws.rho[l],
                         (T *)ws.rho[l + 1]);
  }
  if (DIM == 2)
    for (int l = 0; l < ws.lc; ++l)
      if (ws.vtx[l] > 0)
        hipLaunchKernelGGL((k_vc_coef2d<T>), grid_for(ws.lev[l].lay), bb, 0, st, ws.lev[l].lay, ws.bnd,
                           (T)ws.lev[l].ih2[0], (T)ws.lev[l].ih2[1], (const T *)ws.rho[l], (T *)ws.cf[l][0],
                           (T *)ws.cf[l][1], (T *)ws.cf[l][2]);
  const int vc = ws.vc;
  ws.vc = 1;
  CoarseArgs<T> ca = coarse_args<T>(ws, ws.z[0], ws.r[0]);
  ws.vc = vc;
  for (int l = ws.lc; l < ws.nlev; ++l)
    hipLaunchKernelGGL((k_vc_pack<DIM, T>), grid_for(ws.lev[l].lay), bb, 0, st, ws.lev[l].lay,
                       (const T *)ws.rho[l], (T *)ws.rho_c + ca.off[l]);
  hipLaunchKernelGGL((k_vc_pinv<DIM, T>), dim3(1), dim3(kPinvThreads), 0, st, ca, (T *)ws.pinv_vc);
  return hipGetLastError();
}

// Stretched 2D grid: the cell ratio dx/dy of every cell of a level (the
// cell array face_coef turns into the volume-weighted face coefficients)
// and, on the finest level, the cell volumes.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_met_level(Lay L, const double *wx, const double *wy, T *ratio,
                                                      double *vol) {
  CellPos p;
  if (!cell_of_thread(L, p)) return;
  ratio[p.c] = (T)(wx[p.i] / wy[p.j]);
  if (vol) vol[p.c] = wx[p.i] * wy[p.j];
}

template <typename T>
static hipError_t set_metric_t(hipStream_t st, PoissonWS &ws) {
  const dim3 bb(kBX, kBY);
  long off = 0;
  for (int l = 0; l < ws.nlev; ++l) {
    const Lay &L = ws.lev[l].lay;
    const double *wx = ws.met_w + off, *wy = wx + L.n[0];
    off += L.n[0] + L.n[1];
    if (l == 0) {
      hipLaunchKernelGGL((k_met_level<double>), grid_for(L), bb, 0, st, L, wx, wy, ws.rho64, ws.vol);
      if (sizeof(T) != 8)
        hipLaunchKernelGGL((k_met_level<T>), grid_for(L), bb, 0, st, L, wx, wy, (T *)ws.rho[0], (double *)nullptr);
    } else {
      hipLaunchKernelGGL((k_met_level<T>), grid_for(L), bb, 0, st, L, wx, wy, (T *)ws.rho[l], (double *)nullptr);
    }
  }
  ws.vc = 1;
  CoarseArgs<T> ca = coarse_args<T>(ws, ws.z[0], ws.r[0]);
  for (int l = ws.lc; l < ws.nlev; ++l)
    hipLaunchKernelGGL((k_vc_pack<2, T>), grid_for(ws.lev[l].lay), bb, 0, st, ws.lev[l].lay, (const T *)ws.rho[l],
                       (T *)ws.rho_c + ca.off[l]);
  hipLaunchKernelGGL((k_vc_pinv<2, T>), dim3(1), dim3(kPinvThreads), 0, st, ca, (T *)ws.pinv_vc);
  return hipGetLastError();
}

hipError_t poisson_set_metric(hipStream_t st, PoissonWS &ws, const double *wx, const double *wy) {
  if (!ws.met || ws.lay.ndim != 2 || ws.lev[ws.nlev - 1].lay.ncells() > kVcCoarsest) return hipErrorInvalidValue;
  // widths of every level: a coarse cell spans its two children
  std::vector<double> all;
  std::vector<double> cx(wx, wx + ws.lay.n[0]), cy(wy, wy + ws.lay.n[1]);
  double V = 0.0;
  {
    double sx = 0.0, sy = 0.0;
    for (double v : cx) sx += v;
    for (double v : cy) sy += v;
    V = sx * sy;
  }
  for (int l = 0; l < ws.nlev; ++l) {
    all.insert(all.end(), cx.begin(), cx.end());
    all.insert(all.end(), cy.begin(), cy.end());
    std::vector<double> nx(cx.size() / 2), ny(cy.size() / 2);
    for (size_t q = 0; q < nx.size(); ++q) nx[q] = cx[2 * q] + cx[2 * q + 1];
    for (size_t q = 0; q < ny.size(); ++q) ny[q] = cy[2 * q] + cy[2 * q + 1];
    cx.swap(nx);
    cy.swap(ny);
  }
  ws.volume = V;
  // the coarse kernel's tables: per level l >= lc the widths and the face
  // factors 2 / (w_a + w_b) (the last face wraps when periodic, else 0)
  std::vector<double> tab;
  {
    size_t off = 0;
    for (int l = 0; l < ws.nlev; ++l) {
      const int n0 = ws.lev[l].lay.n[0], n1 = ws.lev[l].lay.n[1];
      if (l >= ws.lc) {
        const double *lx = all.data() + off, *ly = lx + n0;
        auto faces = [&](const double *w, int n, int periodic) {
          for (int q = 0; q < n; ++q) {
            if (q + 1 < n)
              tab.push_back(2.0 / (w[q] + w[q + 1]));
            else
              tab.push_back(periodic ? 2.0 / (w[q] + w[0]) : 0.0);
          }
        };
        tab.insert(tab.end(), lx, lx + n0);
        tab.insert(tab.end(), ly, ly + n1);
        faces(lx, n0, ws.bnd.periodic[0]);
        faces(ly, n1, ws.bnd.periodic[1]);
      }
      off += n0 + n1;
    }
  }
  hipError_t e = hipMemcpyAsync(ws.met_w, all.data(), all.size() * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && ws.mixed) {
    std::vector<float> tf(tab.begin(), tab.end());
    e = hipMemcpyAsync(ws.met_tab, tf.data(), tf.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  } else if (e == hipSuccess) {
    e = hipMemcpyAsync(ws.met_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) return e;
  return ws.mixed ? set_metric_t<float>(st, ws) : set_metric_t<double>(st, ws);
}

hipError_t poisson_setup_device(hipStream_t st, PoissonWS &ws) {
  if (ws.lev[ws.nlev - 1].lay.ncells() > kVcCoarsest) return hipErrorInvalidValue;
  const bool three = ws.lay.ndim == 3;
  if (ws.mixed) {
    CoarseArgs<float> ca = coarse_args<float>(ws, ws.z[0], ws.r[0]);
    if (three)
      hipLaunchKernelGGL((k_vc_pinv<3, float, true>), dim3(1), dim3(kPinvThreads), 0, st, ca, (float *)ws.pinv);
    else
      hipLaunchKernelGGL((k_vc_pinv<2, float, true>), dim3(1), dim3(kPinvThreads), 0, st, ca, (float *)ws.pinv);
  } else {
    CoarseArgs<double> ca = coarse_args<double>(ws, ws.z[0], ws.r[0]);
    if (three)
      hipLaunchKernelGGL((k_vc_pinv<3, double, true>), dim3(1), dim3(kPinvThreads), 0, st, ca, (double *)ws.pinv);
    else
      hipLaunchKernelGGL((k_vc_pinv<2, double, true>), dim3(1), dim3(kPinvThreads), 0, st, ca, (double *)ws.pinv);
  }
  return hipGetLastError();
}

hipError_t poisson_set_beta(hipStream_t st, PoissonWS &ws) {
  if (!ws.vc_cap) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(&ws.sc->rho_bad, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  if (ws.lay.ndim == 3) return ws.mixed ? set_beta_dim<3, float>(st, ws) : set_beta_dim<3, double>(st, ws);
  return ws.mixed ? set_beta_dim<2, float>(st, ws) : set_beta_dim<2, double>(st, ws);
}

// ---------------------------------------------------------------------------
// Timing hook: one launch of a kernel class on scratch arrays
// ---------------------------------------------------------------------------
template <int DIM, typename T>
static hipError_t bench_launch_dim(hipStream_t st, PoissonWS &ws, int which) {
  CGArgs a;
  a.L = ws.lay;
  a.B = ws.bnd;
  for (int d = 0; d < 3; ++d) {
    a.ih2[d] = ws.lev[0].ih2[d];
    a.ih[d] = std::sqrt(ws.lev[0].ih2[d]);
  }
  a.b = ws.r[0];
  a.x0 = nullptr;
  a.x = ws.x;
  a.rold = ws.r[0];
  a.rnew = ws.r[1];
  a.pold = ws.p[0];
  a.pnew = ws.p[1];
  a.q = ws.q;
  a.z = ws.z[0];
  a.zold = nullptr;
  a.part_cc = ws.part_cc;
  a.part_pq = ws.part_pq;
  a.part_rz = ws.part_rz;
  a.np_rz = np_rz_of(ws);
  a.np_pq = kRedBlocks;
  a.sc = ws.sc;
  a.tol2 = 0.0;
  a.k = 2;
  a.flexible = 0;
  a.rho = nullptr;
  switch (which) {
    case 0: {  // finest-level down kernel (fused) or one half-sweep
      if (fused_level(ws, 0)) {
        Down2DArgs<T> d = down_args<T>(ws, 0, 2, ws.r[1], (T *)ws.zpre, ws.x, ws.p[0], ws.q, ws.r[0]);
        d.tol2 = 0.0;  // never converged: time the full kernel
        launch_nu<T>(ws, 0, ws.nu, d, st);
      } else {
        hipLaunchKernelGGL((k_mg_smooth<DIM, T, double>), grid_for(ws.lay), dim3(kBX, kBY), 0, st, ws.lay, ws.bnd,
                           ih2_of<T>(ws, 0), (T *)ws.z[0], (const double *)ws.r[0], 1, 0, ws.sc, (const T *)nullptr, 0);
      }
      break;
    }
    case 2: hipLaunchKernelGGL((k_cg_pq<DIM, T>), dim3(kRedBlocks), dim3(kBlock), 0, st, a, kRedBlocks); break;
    case 3: {  // finest-level up kernel (fused) or restriction
      if (ws.lc == 0) return hipErrorInvalidValue;
      if (fused_level(ws, 0)) {
        Up2DArgs<T> u = up_args<T>(ws, 0, (const T *)ws.zpre, lev_xout<T>(ws, 1, ws.z[0]), ws.r[0], (T *)ws.z[0],
                                   nullptr);
        launch_nu<T>(ws, 0, ws.nu, u, st, ws.cgcg);
      } else {
        hipLaunchKernelGGL((k_mg_restrict<DIM, T, double>), grid_for(ws.lev[1].lay), dim3(kBX, kBY), 0, st,
                           ws.lay, ws.lev[1].lay, ws.bnd, ih2_of<T>(ws, 0), (const T *)ws.z[0],
                           (const double *)ws.r[0], (T *)ws.lev[1].b, ws.sc, (const T *)nullptr, 0);
      }
      break;
    }
    case 4: hipLaunchKernelGGL((k_cg_update<DIM>), dim3(kRedBlocks), dim3(kBlock), 0, st, a); break;
    case 5:
      hipLaunchKernelGGL((k_mg_coarse<DIM, T>), dim3(1), dim3(kCoarseThreads), 0, st,
                         coarse_args<T>(ws, ws.z[0], ws.r[0]), ws.sc);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t poisson_bench_launch(hipStream_t st, PoissonWS &ws, int which) {
  if (ws.lay.ndim == 3)
    return ws.mixed ? bench_launch_dim<3, float>(st, ws, which) : bench_launch_dim<3, double>(st, ws, which);
  return ws.mixed ? bench_launch_dim<2, float>(st, ws, which) : bench_launch_dim<2, double>(st, ws, which);
}

}  // namespace lm
