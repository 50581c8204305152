// Fused 3D multigrid level kernels for fully periodic grids: one launch per
// level and direction of the V-cycle. A block owns a TXT x TYT column of
// cells over tz planes and marches through its planes in z, keeping a ring
// of planes in LDS: the red-black half-sweeps of the level run as a
// pipeline, half-sweep s one plane behind half-sweep s-1 (temporal blocking
// in z), and the x-y frame carries a halo that shrinks by one cell per
// half-sweep (temporal blocking in x-y), so each level is read and written
// once per leg instead of once per half-sweep. Included by lm_solver.hip.
#pragma once

namespace lm {

template <typename T>
struct Fused3DArgs {
  Lay Lf, Lc;
  T ihx, ihy, ihz, idg;   // 1/h^2 per direction, 1/diag
  double dihx, dihy, dihz;  // FP64 1/h^2: w = A u is formed in FP64 whatever T is
  int tiles_x, tiles_y, tz;
  const void *b;          // right-hand side of the level (FP64 on the finest level)
  int b_double;
  const T *xpre;          // up: pre-smoothed correction
  const T *xc;            // up: coarse correction
  T *xout;                // down: pre-smoothed correction; up: post-smoothed
  T *bc;                  // down: coarse right-hand side
  const SolverScalars *sc;
  double *w;              // up with EXTRA: A u on the owned cells
  double *part_rz;        // up with EXTRA: [r.u | w.u | r.r] x np
  int np;
};

__device__ inline int wrap_p(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }

// Gauss-Seidel value (b + sum of the six neighbours scaled by 1/h^2) / diag
// from v = {b, x-, x+, y-, y+, z-, z+}. A cell is updated by its owner and
// by the halos of its neighbours' blocks, and all of them must get the same
// bits (the single-reduction CG needs w = A u consistent with the stored u):
// in FP32 the expression is evaluated exactly as written, with no
// contraction into fused multiply-adds that could differ between the
// unrolled copies. (FP64 differences would sit at the 1e-16 level.)
template <typename T>
__device__ inline T gs7(const T (&v)[7], T ihx, T ihy, T ihz, T idg) {
  return (v[0] + (ihx * (v[1] + v[2]) + ihy * (v[3] + v[4]) + ihz * (v[5] + v[6]))) * idg;
}
template <>
__device__ inline float gs7<float>(const float (&v)[7], float ihx, float ihy, float ihz, float idg) {
#pragma clang fp contract(off)
  return (v[0] + (ihx * (v[1] + v[2]) + ihy * (v[3] + v[4]) + ihz * (v[5] + v[6]))) * idg;
}

// One red/black half-sweep on plane slot xcur of a W x HH frame over the
// region [s, W-s) x [s, HH-s); xm / xp are the planes below and above.
// A thread takes at most two cells; all their LDS reads are issued before
// the arithmetic (the cells of one colour never read each other).
template <typename T, int W, int HH>
__device__ inline void hs_plane(T *xcur, const T *xm, const T *xp, const T *b, int s, int color, int p0, T ihx,
                                T ihy, T ihz, T idg, bool zero) {
  static_assert(((W - 2) / 2) * (HH - 2) <= 2 * kBlock, "two cells per thread");
  const int w = W - 2 * s, rows = HH - 2 * s;
  const int half = w / 2;
  const int cnt = half * rows;
  int off[2];
  bool on[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int o = threadIdx.x + u * kBlock;
    on[u] = o < cnt;
    const int oo = on[u] ? o : 0;
    const int ly = s + oo / half;
    const int lx = s + 2 * (oo % half) + ((color + p0 + ly + s) & 1);
    off[u] = ly * W + lx;
  }
  if (zero) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (on[u]) xcur[off[u]] = b[off[u]] * idg;
    return;
  }
  T v[2][7];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int c = off[u];
    v[u][0] = b[c];
    v[u][1] = xcur[c - 1];
    v[u][2] = xcur[c + 1];
    v[u][3] = xcur[c - W];
    v[u][4] = xcur[c + W];
    v[u][5] = xm[c];
    v[u][6] = xp[c];
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (on[u]) xcur[off[u]] = gs7<T>(v[u], ihx, ihy, ihz, idg);
}

// Down leg: NU red-black sweeps from zero, then residual and restriction.
template <typename T, int NU, int TXT, int TYT>
__global__ void __launch_bounds__(kBlock) k_mg_down3d(Fused3DArgs<T> a) {
  static_assert(TXT * TYT == kBlock && TXT % 2 == 0 && TYT % 2 == 0, "tile shape");
  constexpr int H = 2 * NU + 1;
  constexpr int W = TXT + 2 * H, HH = TYT + 2 * H, P = W * HH;
  constexpr int NX = 2 * NU + 2, NB = 2 * NU + 1;
  constexpr int NIT = (P + kBlock - 1) / kBlock;
  __shared__ T xr[NX][P];
  __shared__ T br[NB][P];
  if (a.sc->done) return;
  const int nx = a.Lf.n[0], ny = a.Lf.n[1], nz = a.Lf.n[2];
  const int ntile = a.tiles_x * a.tiles_y;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = lb % ntile, chunk = lb / ntile;
  const int gx0 = (tile % a.tiles_x) * TXT - H, gy0 = (tile / a.tiles_x) * TYT - H;
  const int z0 = chunk * a.tz;
  const int zf0 = z0 - H, zf1 = z0 + a.tz + H;  // frame planes [zf0, zf1)
  const int tid = threadIdx.x;
  // frame positions of this thread and their x-y offsets in the level
  long goff[NIT];
  bool inner[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int o = tid + it * kBlock;
    const int lx = o % W, ly = o / W;
    inner[it] = o < P && lx > 0 && ly > 0 && lx < W - 1 && ly < HH - 1;
    goff[it] = (long)wrap_p(gx0 + lx, nx) + (long)wrap_p(gy0 + ly, ny) * a.Lf.s[1];
  }
  auto plane_base = [&](int t) { return a.Lf.base + (long)wrap_p(t, nz) * a.Lf.s[2]; };
  T bnext[NIT];
  auto fetch = [&](int t) {
    const long pb = plane_base(t);
    const bool ring = (t == zf0 || t == zf1 - 1);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      T v = T(0);
      if (inner[it] && !ring)
        v = a.b_double ? (T)((const double *)a.b)[pb + goff[it]] : ((const T *)a.b)[pb + goff[it]];
      bnext[it] = v;
    }
  };
  fetch(zf0);
  // coarse cell of this thread (restriction): accumulated over two planes
  const int cxl = tid % (TXT / 2), cyl = tid / (TXT / 2);
  const bool has_coarse = tid < (TXT / 2) * (TYT / 2);
  T racc = T(0);
  const int tlast = z0 + a.tz - 1 + 2 * NU;
  for (int t = zf0; t <= tlast; ++t) {
    if (t < zf1) {
      T *xs = xr[(t - zf0) % NX];
      T *bs = br[(t - zf0) % NB];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int o = tid + it * kBlock;
        if (o < P) {
          xs[o] = T(0);
          bs[o] = bnext[it];
        }
      }
      if (t + 1 < zf1) fetch(t + 1);  // in flight during this step's sweeps
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= 2 * NU; ++s) {
      const int q = t - (s - 1);
      if (q >= zf0 + s && q < zf1 - s) {
        const int p0 = (gx0 + gy0 + wrap_p(q, nz)) & 1;
        hs_plane<T, W, HH>(xr[(q - zf0) % NX], xr[(q - 1 - zf0) % NX], xr[(q + 1 - zf0) % NX],
                           br[(q - zf0) % NB], s, (s + 1) & 1, p0, a.ihx, a.ihy, a.ihz, a.idg, s == 1);
      }
      __syncthreads();
    }
    const int q = t - 2 * NU;
    if (q >= z0 && q < z0 + a.tz) {
      const T *xs = xr[(q - zf0) % NX];
      const T *xm = xr[(q - 1 - zf0) % NX];
      const T *xp = xr[(q + 1 - zf0) % NX];
      const T *bs = br[(q - zf0) % NB];
      const long pb = plane_base(q);
      {
        const int lx = H + tid % TXT, ly = H + tid / TXT;
        a.xout[pb + (long)(gx0 + lx) + (long)(gy0 + ly) * a.Lf.s[1]] = xs[ly * W + lx];
      }
      if (has_coarse) {
        T acc = T(0);
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int lx = H + 2 * cxl + dx, ly = H + 2 * cyl + dy;
            const int off = ly * W + lx;
            const T Lx = (T(2) * (a.ihx + a.ihy + a.ihz)) * xs[off] -
                         (a.ihx * (xs[off - 1] + xs[off + 1]) + a.ihy * (xs[off - W] + xs[off + W]) +
                          a.ihz * (xm[off] + xp[off]));
            acc += bs[off] - Lx;
          }
        racc += acc;
        if (q & 1) {
          const int Cx = (gx0 + H) / 2 + cxl, Cy = (gy0 + H) / 2 + cyl;
          a.bc[a.Lc.at(Cx, Cy, q >> 1)] = racc * T(0.125);
          racc = T(0);
        }
      }
    }
    __syncthreads();
  }
}

// Up leg: prolongation of the coarse correction, then NU black-red sweeps.
// With EXTRA = 1 (finest level of the FP64 single-reduction CG) the frame
// carries one more halo ring and plane, so the smoothed u is valid one
// cell around the owned column: w = A u is formed for the owned cells with
// the partials of r.u, w.u and r.r (r = the level's right-hand side).
template <typename T, int NU, int EXTRA, int TXT, int TYT>
__global__ void __launch_bounds__(kBlock) k_mg_up3d(Fused3DArgs<T> a) {
  static_assert(TXT * TYT == kBlock && TXT % 2 == 0 && TYT % 2 == 0, "tile shape");
  constexpr int H = 2 * NU + EXTRA;
  constexpr int W = TXT + 2 * H, HH = TYT + 2 * H, P = W * HH;
  constexpr int NX = 2 * NU + 2 + EXTRA, NB = 2 * NU + 1 + EXTRA;
  constexpr int NIT = (P + kBlock - 1) / kBlock;
  __shared__ T xr[NX][P];
  __shared__ T br[NB][P];
  if (a.sc->done) return;
  const int nx = a.Lf.n[0], ny = a.Lf.n[1], nz = a.Lf.n[2];
  const int ntile = a.tiles_x * a.tiles_y;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = lb % ntile, chunk = lb / ntile;
  const int gx0 = (tile % a.tiles_x) * TXT - H, gy0 = (tile / a.tiles_x) * TYT - H;
  const int z0 = chunk * a.tz;
  const int zf0 = z0 - H, zf1 = z0 + a.tz + H;
  const int tid = threadIdx.x;
  long goff[NIT], coff[NIT];
  bool inner[NIT], valid[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int o = tid + it * kBlock;
    const int lx = o % W, ly = o / W;
    const int gx = wrap_p(gx0 + lx, nx), gy = wrap_p(gy0 + ly, ny);
    valid[it] = o < P;
    inner[it] = valid[it] && lx > 0 && ly > 0 && lx < W - 1 && ly < HH - 1;
    goff[it] = (long)gx + (long)gy * a.Lf.s[1];
    coff[it] = (long)(gx >> 1) + (long)(gy >> 1) * a.Lc.s[1];
  }
  T xn[NIT], cn[NIT], bn[NIT];
  auto fetch = [&](int t) {
    const int gz = wrap_p(t, nz);
    const long pb = a.Lf.base + (long)gz * a.Lf.s[2];
    const long pc = a.Lc.base + (long)(gz >> 1) * a.Lc.s[2];
    const bool ring = (t == zf0 || t == zf1 - 1);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      xn[it] = valid[it] ? a.xpre[pb + goff[it]] : T(0);
      cn[it] = valid[it] ? a.xc[pc + coff[it]] : T(0);
      T v = T(0);
      if (inner[it] && !ring)
        v = a.b_double ? (T)((const double *)a.b)[pb + goff[it]] : ((const T *)a.b)[pb + goff[it]];
      bn[it] = v;
    }
  };
  fetch(zf0);
  double ru = 0.0, wu = 0.0, rr = 0.0;
  const int tlast = z0 + a.tz - 1 + 2 * NU + EXTRA;
  for (int t = zf0; t <= tlast; ++t) {
    if (t < zf1) {
      T *xs = xr[(t - zf0) % NX];
      T *bs = br[(t - zf0) % NB];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int o = tid + it * kBlock;
        if (o < P) {
          xs[o] = xn[it] + cn[it];
          bs[o] = bn[it];
        }
      }
      if (t + 1 < zf1) fetch(t + 1);
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= 2 * NU; ++s) {
      const int q = t - s;
      if (q >= zf0 + s && q < zf1 - s) {
        const int p0 = (gx0 + gy0 + wrap_p(q, nz)) & 1;
        hs_plane<T, W, HH>(xr[(q - zf0) % NX], xr[(q - 1 - zf0) % NX], xr[(q + 1 - zf0) % NX],
                           br[(q - zf0) % NB], s, s & 1, p0, a.ihx, a.ihy, a.ihz, a.idg, false);
      }
      __syncthreads();
    }
    const int q = t - 2 * NU - EXTRA;
    if (q >= z0 && q < z0 + a.tz) {
      const T *xs = xr[(q - zf0) % NX];
      const long pb = a.Lf.base + (long)wrap_p(q, nz) * a.Lf.s[2];
      const int lx = H + tid % TXT, ly = H + tid / TXT;
      const int off = ly * W + lx;
      const long g = pb + (long)(gx0 + lx) + (long)(gy0 + ly) * a.Lf.s[1];
      const T u = xs[off];
      a.xout[g] = u;
      if (EXTRA) {
        const T *xm = xr[(q - 1 - zf0) % NX];
        const T *xp = xr[(q + 1 - zf0) % NX];
        const double Lu = (2.0 * (a.dihx + a.dihy + a.dihz)) * (double)u -
                          (a.dihx * ((double)xs[off - 1] + (double)xs[off + 1]) +
                           a.dihy * ((double)xs[off - W] + (double)xs[off + W]) +
                           a.dihz * ((double)xm[off] + (double)xp[off]));
        // r in FP64 from the level's right-hand side (the LDS copy is in T)
        const double rv = a.b_double ? ((const double *)a.b)[g] : (double)br[(q - zf0) % NB][off];
        a.w[g] = Lu;
        ru += rv * (double)u;
        wu += Lu * (double)u;
        rr += rv * rv;
      }
    }
    // with EXTRA the next plane's slots are the ones read just above
    if (EXTRA) __syncthreads();
  }
  if (EXTRA) {
    double v3[3] = {ru, wu, rr};
    block_allsum_n<3>(v3);
    if (tid == 0) {
      a.part_rz[blockIdx.x] = v3[0];
      a.part_rz[a.np + blockIdx.x] = v3[1];
      a.part_rz[2 * a.np + blockIdx.x] = v3[2];
    }
  }
}

}  // namespace lm
