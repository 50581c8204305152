// The whole pressure solve in one workgroup, for grids whose finest level
// the one-block coarse V-cycle already covers (at most kCoarseCells cells):
// the single-reduction preconditioned CG of the multi-kernel path (same
// recurrences, same stopping rule, FP64 vectors) with the CG vectors in
// registers (at most kCoarseLoads cells per thread) and the V-cycle out of
// LDS. One launch per solve instead of three per iteration and no host
// round trip between iterations: on such grids every kernel is a few
// microseconds of work, so launches and waits, not bytes, set the time.
// Included by lm_solver.hip only.
#pragma once

namespace lm {

template <typename T>
struct BlockPCGArgs {
  CoarseArgs<T> ca;         // the V-cycle from level 0 (ca.l0 == 0)
  Lay L;                    // finest layout of the global vectors
  Bnd B;
  double ih2[3], ih[3];     // finest 1/h^2, 1/h (FP64 operator)
  const double *b, *x0;     // right-hand side; warm start (NULL: zero)
  double *x;                // solution (fine layout)
  const double *rho;        // variable coefficients / cell ratios (FP64, fine layout), or NULL
  int met;                  // stretched grid: rho holds dx/dy
  const double *vol;        // stretched grid: cell volumes, else NULL
  double mean_w;            // weight of the solution mean: volume or cell count
  double tol2;
  int maxit;
  double *cf;               // scratch, compact cell order: variable coefficients (2 DIM face
                            // coefficients and the diagonal, N each), then p, s, w and r (N each)
  SolverScalars *sc;
  SolveLog *log;            // optional copy of the outcome (deferred checks)
};

// Neighbours of compact cell t = (i, j, k) of level 0 along d: LDS index
// or the zero slot when the side is a wall (no periodic wrap).
template <int DIM>
__device__ inline void pb_nbrs(const int n[3], const Bnd &B, int i, int j, int k, int t, int zero_slot,
                               int nb[2 * DIM]) {
  const int q[3] = {i, j, k};
  const int st[3] = {1, n[0], n[0] * n[1]};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool per = B.periodic[d] != 0;
    nb[2 * d] = q[d] > 0 ? t - st[d] : (per ? t + (n[d] - 1) * st[d] : zero_slot);
    nb[2 * d + 1] = q[d] + 1 < n[d] ? t + st[d] : (per ? t - (n[d] - 1) * st[d] : zero_slot);
  }
}

template <int DIM, typename T, bool VC, bool MET = false>
__global__ void __launch_bounds__(kCoarseThreads) k_pcg_block(BlockPCGArgs<T> a) {
#pragma clang fp contract(off)
  __shared__ T xs[kCoarseLds + 1];
  __shared__ T bs[kCoarseLds];
  __shared__ T idg_s[kCoarseLev * 8];
  __shared__ T rs[VC ? kCoarseLds + 1 : 1];
  constexpr int NC = kCoarseLoads;
  constexpr int NF = 2 * DIM;
  SolverScalars *sc = a.sc;
  const CoarseArgs<T> &ca = a.ca;
  const int zero_slot = kCoarseLds;
  const int tid = threadIdx.x;
  if (a.rho && sc->rho_bad) {  // invalid density: the solve ends at once
    if (tid == 0) {
      sc->done = 1;
      sc->iters = 0;
      sc->nonconv = 1;
      sc->zero = 0;
      if (a.log) {
        a.log->done = 1;
        a.log->nonconv = 1;
        a.log->iters = 0;
        a.log->rr = 0.0;
        a.log->cc = 0.0;
        a.log->mean_b = sc->mean_b;
      }
    }
    return;
  }
  const int last = ca.nlev - 1;
  if (tid < kCoarseLev * 8) idg_s[tid] = ca.idg[tid >> 3][tid & 7];
  if (tid == 0) xs[zero_slot] = T(0);
  if constexpr (MET) {
    for (int t = tid; t < ca.mtab_n; t += blockDim.x) rs[t] = ca.mtab[t];
  } else if constexpr (VC) {
    const int ntot = ca.off[last] + ca.n[last][0] * ca.n[last][1] * ca.n[last][2];
    for (int t = tid; t < ntot; t += blockDim.x) rs[t] = ca.rho_c[t];
    if (tid == 0) rs[zero_slot] = T(1);
  }
  const int *n = ca.n[0];
  const int N = n[0] * n[1] * n[2];
  const double mb = sc->mean_b, oc = sc->outflow_c;

  // No per-cell state stays in registers across the V-cycle (which needs
  // them all): p, s, w and r live in scratch (compact order, L2-resident;
  // in FP64 r is also the level-0 right-hand side in LDS, which the cycle
  // leaves intact), the solution in a.x; the FP64 face coefficients of a
  // variable-coefficient operator are computed once here and read back
  // from scratch; neighbour indices are recomputed where used.
  double *const pv = a.cf + (long)(NF + 1) * N;
  double *const sv = pv + N;
  double *const wv = sv + N;
  double *const rg = wv + N;
  auto r_of = [&](int t) -> double {
    if constexpr (sizeof(T) == 8)
      return (double)bs[t];
    else
      return rg[t];
  };
  double cc = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int t = tid + q * blockDim.x;
    if (t >= N) continue;
    int i, j, k;
    c_decode<DIM, T>(n, t, i, j, k);
    const long g = a.L.at(i, j, k);
    const int qd[3] = {i, j, k};
    if constexpr (VC) {
      const double rc = a.rho[g];
      double dg = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const bool per = a.B.periodic[d] != 0;
        const long gl = qd[d] > 0 ? g - a.L.s[d] : (per ? g + (long)(n[d] - 1) * a.L.s[d] : -1);
        const long gh = qd[d] + 1 < n[d] ? g + a.L.s[d] : (per ? g - (long)(n[d] - 1) * a.L.s[d] : -1);
        const double bl = gl >= 0 ? face_coef<double>(rc, a.rho[gl], d, a.met) : 0.0;
        const double bh = gh >= 0 ? face_coef<double>(rc, a.rho[gh], d, a.met) : 0.0;
        double sb = 0.0;
        if (gl >= 0) sb += bl;
        if (gh >= 0) sb += bh;
        dg += a.ih2[d] * sb;
        a.cf[(2 * d) * N + t] = bl;
        a.cf[(2 * d + 1) * N + t] = bh;
      }
      a.cf[NF * N + t] = dg;
    }
    // r_0 = c - L x0 with c the mean-free (volume-weighted) right-hand side
    double bb = a.b[g] - mb;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (a.B.kind[d][0] == LM_SIDE_OUTFLOW && qd[d] == 0) bb -= oc * a.ih[d];
      if (a.B.kind[d][1] == LM_SIDE_OUTFLOW && qd[d] == n[d] - 1) bb -= oc * a.ih[d];
    }
    const double cv = a.vol ? -(bb * a.vol[g]) : -bb;
    double Lx = 0.0, xv = 0.0;
    if (a.x0) {
      double nbs, dd;
      xv = a.x0[g];
      if constexpr (VC)
        op_parts_vc<DIM, double, double, double>(a.L, a.B, a.ih2, a.rho, a.x0, i, j, k, g, nbs, dd, a.met);
      else
        op_parts<DIM, double, double>(a.L, a.B, a.ih2, a.x0, i, j, k, g, nbs, dd);
      Lx = dd * xv - nbs;
    }
    a.x[g] = xv;
    const double r0 = cv - Lx;
    bs[t] = (T)r0;
    if constexpr (sizeof(T) != 8) rg[t] = r0;
    cc += cv * cv;
  }

  // u = M r (V-cycle), w = L u, and the three inner products of the
  // single-reduction recurrence
  auto precondition = [&](double &gam, double &del, double &rr) {
    // opaque copies: everything the cycle derives from the thread index is
    // recomputed per iteration instead of held in registers across them
    int tv = tid, zs = zero_slot;
    asm volatile("" : "+v"(tv), "+s"(zs));
    __syncthreads();
    coarse_cycle<DIM, T, VC, MET>(ca, xs, bs, rs, idg_s, zs, tv);
    gam = del = rr = 0.0;
#pragma unroll 1
    for (int q = 0; q < NC; ++q) {
      const int t = tv + q * blockDim.x;
      if (t >= N) continue;
      int i, j, k;
      c_decode<DIM, T>(n, t, i, j, k);
      int nb[NF];
      pb_nbrs<DIM>(n, a.B, i, j, k, t, zs, nb);
      double v[NF];
#pragma unroll
      for (int m = 0; m < NF; ++m) v[m] = (double)xs[nb[m]];
      const double uc = (double)xs[t];
      double nbs = 0.0, dg = 0.0;
      if constexpr (VC) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
          nbs += a.ih2[d] * (a.cf[(2 * d) * N + t] * v[2 * d] + a.cf[(2 * d + 1) * N + t] * v[2 * d + 1]);
        dg = a.cf[NF * N + t];
      } else {
        const int qd[3] = {i, j, k};
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const bool per = a.B.periodic[d] != 0;
          const int cnt = (qd[d] > 0 || per) + (qd[d] + 1 < n[d] || per);
          nbs += a.ih2[d] * (v[2 * d] + v[2 * d + 1]);
          dg += a.ih2[d] * (double)cnt;
        }
      }
      const double wq = dg * uc - nbs, rq = r_of(t);
      wv[t] = wq;
      gam += rq * uc;
      del += wq * uc;
      rr += rq * rq;
    }
  };

  double gam, del, rr;
  precondition(gam, del, rr);
  {
    double v4[4] = {cc, gam, del, rr};
    block_allsum_n<4>(v4);
    cc = v4[0];
    gam = v4[1];
    del = v4[2];
    rr = v4[3];
  }
  double g_prev = 0.0, al_prev = 0.0, alpha = 0.0, beta = 0.0;
  int iters = 0, done = 0, nonconv = 0;
  for (int k = 1; k <= a.maxit + 1; ++k) {
    const bool conv = (cc == 0.0) || (rr <= a.tol2 * cc);
    beta = 0.0;
    if (k == 1) {
      alpha = gam / del;
    } else {
      beta = gam / g_prev;
      alpha = gam / (del - beta * gam / al_prev);
    }
    const bool broken = !isfinite(rr) || !isfinite(alpha) || !isfinite(beta);
    iters = k - 1;
    if (conv || broken) {
      done = 1;
      nonconv = broken && !conv;
      break;
    }
    if (k == a.maxit + 1) break;  // out of iterations: not converged
    g_prev = gam;
    al_prev = alpha;
    // p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
    int tu = tid;
    asm volatile("" : "+v"(tu));
#pragma unroll 1
    for (int q = 0; q < NC; ++q) {
      const int t = tu + q * blockDim.x;
      if (t >= N) continue;
      int i, j, kk;
      c_decode<DIM, T>(n, t, i, j, kk);
      const long g = a.L.at(i, j, kk);
      const double uc = (double)xs[t];
      const double pn = uc + (k >= 2 ? beta * pv[t] : 0.0);
      const double sn = wv[t] + (k >= 2 ? beta * sv[t] : 0.0);
      pv[t] = pn;
      sv[t] = sn;
      a.x[g] += alpha * pn;
      const double rn = r_of(t) - alpha * sn;
      if constexpr (sizeof(T) != 8) rg[t] = rn;
      bs[t] = (T)rn;
    }
    precondition(gam, del, rr);  // its first barrier follows every read of u
    double v3[3] = {gam, del, rr};
    block_allsum_n<3>(v3);
    gam = v3[0];
    del = v3[1];
    rr = v3[2];
  }

  // the (volume-weighted) mean of the solution
  double sx = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int t = tid + q * blockDim.x;
    if (t >= N) continue;
    int i, j, k;
    c_decode<DIM, T>(n, t, i, j, k);
    const long g = a.L.at(i, j, k);
    sx += a.vol ? a.x[g] * a.vol[g] : a.x[g];
  }
  {
    double v1[1] = {sx};
    block_allsum_n<1>(v1);
    sx = v1[0];
  }
  if (tid == 0) {
    sc->rr = rr;
    sc->cc = cc;
    sc->iters = iters;
    sc->done = done;
    sc->zero = (cc == 0.0);
    sc->nonconv = nonconv;
    sc->mean_x = sx / a.mean_w;
    if (a.log) {
      a.log->rr = rr;
      a.log->cc = cc;
      a.log->mean_b = sc->mean_b;
      a.log->iters = iters;
      a.log->done = done;
      a.log->nonconv = nonconv;
    }
  }
}

}  // namespace lm
