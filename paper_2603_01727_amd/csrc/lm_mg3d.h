// Fused 3D multigrid level kernels for fully periodic grids: one launch per
// level and leg of the V-cycle, each level read and written once per leg.
//
// A block of 512 threads owns a 32 x 32 x-y frame and marches through a
// chunk of planes in z. Each thread holds an x-adjacent pair of columns of
// the frame in registers over a ring of planes: on every plane the pair has
// one red and one black cell, so every half-sweep updates exactly one cell
// per thread. The red-black half-sweeps run as a pipeline one plane apart:
// at step t, stage s works on plane t - lag(s), lag(s) = s (down leg: s - 1,
// its first half-sweep starts from zero and needs no neighbours). Every
// value a stage reads was made at an earlier step or earlier in the same
// thread's step:
//  - z neighbours are the thread's own registers (stage s - 1 reached plane
//    q + 1 in this step, before stage s, in program order);
//  - the x neighbour outside the pair is the adjacent lane's register, one
//    DPP row shift away (a frame row is one 16-lane row of a wavefront);
//  - the y neighbours are the cells the previous stage updated, which every
//    thread publishes to an LDS half plane one step earlier.
// So one barrier per step separates the LDS writes of a step from the reads
// of the next. The frame's outer H cells are halo whose values go stale by
// one cell per stage that reads neighbours; the block writes its
// (32 - 2H)^2 interior, and the chunk's H halo planes at either end are
// read but not written. Included by lm_solver.hip.
#pragma once

#include <type_traits>

namespace lm {

constexpr int kF3 = 32;                    // x-y frame of a block, cells
constexpr int kF3Threads = kF3 / 2 * kF3;  // one thread per x-adjacent pair

template <typename T>
struct Fused3DArgs {
  Lay Lf, Lc;
  T ihx, ihy, ihz, idg;     // 1/h^2 per direction, 1/diag
  double dihx, dihy, dihz;  // FP64 1/h^2: w = A u is formed in FP64 whatever T is
  int tiles_x, tiles_y, tz; // owned tiles per direction; z chunk (even)
  const void *b;            // right-hand side of the level (FP64 on the finest level)
  int b_double;             // b is FP64 (the launch picks the kernel instance)
  const T *xpre;            // up: pre-smoothed correction
  const T *xc;              // up: coarse correction
  T *xout;                  // down: pre-smoothed correction; up: post-smoothed
  T *bc;                    // down: coarse right-hand side
  const SolverScalars *sc;
  double *w;                // up with EXTRA: A u on the owned cells
  double *part_rz;          // up with EXTRA: [r.u | w.u | r.r] x np
  int np;
};

__device__ inline int wrap_p(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }
// Plane index of the loads, which stay within [-n, 2n) on the fused levels
// (chunks reach at most 13 planes past either end; levels have >= 16).
__device__ inline int wrap_any(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }

// The pair's two right-hand-side values at offset g: FP64 (the finest
// level's r, or any FP64 level) or the level's own precision.
template <typename T, bool BD>
__device__ inline void load_b_pair(const void *b, long g, T &b0, T &b1) {
  if constexpr (BD || sizeof(T) == 8) {
    const double2 v = *(const double2 *)((const double *)b + g);
    b0 = (T)v.x;
    b1 = (T)v.y;
  } else {
    const float2 v = *(const float2 *)((const float *)b + g);
    b0 = v.x;
    b1 = v.y;
  }
}

// Gauss-Seidel value (b + sum of the six neighbours scaled by 1/h^2) / diag.
// A cell is updated by its owner and by the halos of its neighbours'
// blocks, and all of them must get the same bits (the single-reduction CG
// needs w = A u consistent with the stored u): in FP32 the expression is
// evaluated exactly as written, with no contraction into fused
// multiply-adds. (FP64 differences would sit at the 1e-16 level.)
template <typename T>
__device__ inline T gs7(T b, T xl, T xr, T yl, T yr, T zl, T zr, T ihx, T ihy, T ihz, T idg) {
  return (b + (ihx * (xl + xr) + ihy * (yl + yr) + ihz * (zl + zr))) * idg;
}
template <>
__device__ inline float gs7<float>(float b, float xl, float xr, float yl, float yr, float zl, float zr, float ihx,
                                   float ihy, float ihz, float idg) {
#pragma clang fp contract(off)
  return (b + (ihx * (xl + xr) + ihy * (yl + yr) + ihz * (zl + zr))) * idg;
}

// Value of the same register in the lane one to the left (SHR) or right
// (SHL) within a 16-lane row; the row's end lanes read 0 (frame halo).
template <bool SHL>
__device__ inline double row_shift(double v) {
  constexpr int ctrl = SHL ? 0x101 : 0x111;  // row_shl:1 / row_shr:1
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffLL), ctrl, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <bool SHL>
__device__ inline float row_shift(float v) {
  constexpr int ctrl = SHL ? 0x101 : 0x111;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xf, 0xf, true));
}

// The x neighbour outside the pair of the pair's cell `cell` (0: the left
// lane's cell 1, 1: the right lane's cell 0); `other` is the register that
// holds, in every lane, the pair's cell of the other colour (which is the
// neighbour's colour). Within a frame row every lane has the same `cell`.
template <typename T>
__device__ inline T outside_x(int cell, T other) {
  const T l = row_shift<false>(other), r = row_shift<true>(other);
  return cell ? r : l;
}

// Placement of a block: the owned tile [tx0, tx0 + TI) x [ty0, ty0 + TI)
// (clipped to the level), the frame origin (tile minus the halo H), the z
// chunk, and the thread's pair.
struct Place3 {
  int nx, ny, nz;
  int gx0, gy0, tx0, ty0, z0, zc;
  int px, ly, lx0;
  long xy;       // offset of the pair's cell 0 (wrapped) within a plane
  int bpar;      // parity of (x + y) of the pair's cell 0
  bool own;      // the pair lies in the owned tile
};
template <int H, int TI>
__device__ inline Place3 place3(const Lay &L, int tiles_x, int tiles_y, int tz) {
  Place3 p;
  p.nx = L.n[0];
  p.ny = L.n[1];
  p.nz = L.n[2];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = tiles_x * tiles_y;
  const int tile = lb % ntile, chunk = lb / ntile;
  p.tx0 = (tile % tiles_x) * TI;
  p.ty0 = (tile / tiles_x) * TI;
  p.gx0 = p.tx0 - H;
  p.gy0 = p.ty0 - H;
  p.z0 = chunk * tz;
  p.zc = min(tz, p.nz - p.z0);
  p.px = threadIdx.x & 15;
  p.ly = threadIdx.x >> 4;
  p.lx0 = 2 * p.px;
  const int gx = wrap_p(p.gx0 + p.lx0, p.nx), gy = wrap_p(p.gy0 + p.ly, p.ny);
  p.xy = (long)gx + (long)gy * L.s[1];
  p.bpar = (p.gx0 + p.gy0 + p.ly) & 1;
  p.own = p.lx0 >= H && p.lx0 < H + TI && p.gx0 + p.lx0 < p.nx && p.ly >= H && p.ly < H + TI &&
          p.gy0 + p.ly < p.ny;
  return p;
}

__device__ inline int clamp_row(int r) { return r < 0 ? 0 : (r >= kF3 ? kF3 - 1 : r); }

// c ? a : b on values (a conditional on two array elements would select
// their addresses and keep the register ring in memory)
template <typename T>
__device__ inline T pick(bool c, T a, T b) {
  return c ? a : b;
}

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time
// (the plane-ring registers are indexed by constants only).
template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

// Plane ring of the pipeline: R slots hold planes t-R+1 .. t; slot of the
// plane D steps behind the one in slot U.
template <int R, int U, int D>
struct Slot {
  static constexpr int v = ((U - D) % R + R) % R;
};

// The pair's registers hold its cells by colour: XR / XB (BR / BB for the
// right-hand side) are the red and black cells of each plane slot; the red
// cell of plane q is the pair's cell cr = (bpar + q) & 1. A red cell's z
// neighbours, x partner and outside x neighbour are all black, and a black
// cell's red, so a half-sweep reads and writes its colour's registers with
// no per-lane choice; the choice of cell order happens only where cells are
// loaded and stored.

// Down leg: NU red-black sweeps from zero (red first), then the residual
// restricted to the coarse level (2x2x2 average). After the last (black)
// half-sweep the black cells' residual is zero: each black cell's equation
// was just solved with its red neighbours' final values, so only the red
// cells contribute. Stage s (1 .. 2 NU) runs at lag s - 1, the residual at
// lag 2 NU. Halo H = 2 NU: stage 1 needs no neighbours, stages 2 .. 2 NU and
// the residual one ring each; it is even, so the pairs sit on (even, odd)
// global columns and a coarse cell's x-children are one pair.
template <typename T, int NU, bool BD>
__global__ void __launch_bounds__(kF3Threads, 4) k_mg_down3d(Fused3DArgs<T> a) {
  constexpr int S = 2 * NU;
  constexpr int H = S, TI = kF3 - 2 * H;
  constexpr int kRing = S + 2;  // the residual reads planes t-S-1 .. t-S+1
  constexpr int D = kRing / 2;  // planes of b in flight ahead of the step that uses them
  static_assert(kRing % D == 0, "prefetch slots follow the ring");
  __shared__ T pub[S][2][kF3][kF3 / 2];
  if (a.sc->done) return;
  const Place3 p = place3<H, TI>(a.Lf, a.tiles_x, a.tiles_y, a.tz);
  const long s2 = a.Lf.s[2];
  const int t0 = p.z0 - H;
  const int nstep = p.zc + 2 * H;   // planes [z0 - H, z0 + zc + H); the residual lags H steps
  const int yd = clamp_row(p.ly - 1), yu = clamp_row(p.ly + 1);
  const T diag = T(2) * (a.ihx + a.ihy + a.ihz);
  T XR[kRing], XB[kRing], BR[kRing], BB[kRing];
#pragma unroll
  for (int k = 0; k < kRing; ++k) XR[k] = XB[k] = BR[k] = BB[k] = T(0);
  // b of planes t + 1 .. t + D in flight, slot (plane - t0) % D
  T F0[D], F1[D];
  // (issued unconditionally: past the chunk's last plane the loads read
  // planes that are never used, so no branch joins pending loads)
  auto fetch = [&](int t, T &f0, T &f1) __attribute__((always_inline)) {
    load_b_pair<T, BD>(a.b, a.Lf.base + (long)wrap_any(t, p.nz) * s2 + p.xy, f0, f1);
  };
  static_for<0, D>([&](auto J) __attribute__((always_inline)) {
    constexpr int j = decltype(J)::value;
    fetch(t0 + j, F0[j], F1[j]);
  });
  T racc = T(0);
  auto step = [&](auto U, int ts) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    constexpr int f = u % D;
    const int t = t0 + ts;
    // LDS buffers of this step (written) and of the last (read): z0 is a
    // multiple of 4 and the ring even, so the parity of t is u + H's
    constexpr int wb = (u + H) & 1, rb = wb ^ 1;
    // stage 1 on plane t: the red cell from zero, x = b / diag
    {
      const T b0 = F0[f], b1 = F1[f];
      fetch(t + D, F0[f], F1[f]);
      const int cr = (p.bpar + t) & 1;
      BR[u] = pick<T>(cr, b1, b0);
      BB[u] = pick<T>(cr, b0, b1);
      XR[u] = BR[u] * a.idg;
      XB[u] = T(0);
      pub[0][wb][p.ly][p.px] = XR[u];
    }
    // stages 2 .. S on plane t - s + 1: black for even s, red for odd s
    static_for<2, S + 1>([&](auto Sc) __attribute__((always_inline)) {
      constexpr int s = decltype(Sc)::value;
      constexpr bool red = (s & 1) != 0;
      const int q = t - (s - 1);
      constexpr int k = Slot<kRing, u, s - 1>::v;
      constexpr int km = Slot<kRing, u, s>::v, kp = Slot<kRing, u, s - 2>::v;
      T *Xo = red ? XB : XR;  // the other colour (compile-time choice)
      const int cell = ((p.bpar + q) & 1) ^ (red ? 0 : 1);  // pair cell of the updated colour
      const T yl = pub[s - 2][rb][yd][p.px], yr = pub[s - 2][rb][yu][p.px];
      const T v = gs7<T>(red ? BR[k] : BB[k], Xo[k], outside_x<T>(cell, Xo[k]), yl, yr, Xo[km], Xo[kp], a.ihx,
                         a.ihy, a.ihz, a.idg);
      if (red)
        XR[k] = v;
      else
        XB[k] = v;
      pub[s - 1][wb][p.ly][p.px] = v;
    });
    // residual on plane q = t - S at the red cell, restriction, output
    {
      const int q = t - S;
      constexpr int k = Slot<kRing, u, S>::v;
      constexpr int km = Slot<kRing, u, S + 1>::v, kp = Slot<kRing, u, S - 1>::v;
      const int cr = (p.bpar + q) & 1;
      const T xo = outside_x<T>(cr, XB[k]);
      const T yl = pub[S - 1][rb][yd][p.px], yr = pub[S - 1][rb][yu][p.px];
      const T r = BR[k] - (diag * XR[k] - (a.ihx * (XB[k] + xo) + a.ihy * (yl + yr) + a.ihz * (XB[km] + XB[kp])));
      // coarse cell: x-children = the pair, y-children = rows ly, ly ^ 1
      // (lanes 16 apart), z-children = planes q, q + 1 (even q first)
      T rs = r + __shfl_xor(r, 16, 64);
      const bool in_chunk = q >= p.z0 && q < p.z0 + p.zc;
      if ((q & 1) == 0) {
        racc = rs;
      } else {
        racc += rs;
        if (in_chunk && p.own && (p.ly & 1) == 0) {
          const int Cx = (p.gx0 + p.lx0) >> 1, Cy = (p.gy0 + p.ly) >> 1;
          a.bc[a.Lc.at(Cx, Cy, q >> 1)] = racc * T(0.125);
        }
      }
      if (in_chunk && p.own) {
        T *o = a.xout + a.Lf.base + (long)q * s2 + p.xy;
        o[0] = pick<T>(cr, XB[k], XR[k]);
        o[1] = pick<T>(cr, XR[k], XB[k]);
      }
    }
    // one barrier: the next step reads what this one wrote
    __syncthreads();
  };
  // whole rounds of the ring (no branch between the unrolled steps: a step
  // past the last one works on planes outside the chunk and writes nothing)
  for (int tb = 0; tb < nstep; tb += kRing)
    static_for<0, kRing>([&](auto U) __attribute__((always_inline)) { step(U, tb + decltype(U)::value); });
}

// Up leg: prolongation of the coarse correction (piecewise constant) added
// to the pre-smoothed correction, then NU black-red sweeps (black first).
// Stage s (1 .. 2 NU) runs at lag s. With EXTRA = 1 (finest level of the
// FP64 single-reduction CG) a last stage at lag 2 NU + 1 forms w = A u on
// the owned cells in FP64 with the partials of r.u, w.u and r.r (r = the
// level's right-hand side, read in FP64). Halo 2 NU + EXTRA planes in z; in x and y
// rounded up to even, so the pairs sit on (even, odd) columns and never
// straddle the periodic seam.
template <typename T, int NU, int EXTRA, bool BD>
__global__ void __launch_bounds__(kF3Threads, 4) k_mg_up3d(Fused3DArgs<T> a) {
  constexpr int S = 2 * NU;
  constexpr int HZ = S + EXTRA;                       // stages that read neighbours: z halo
  constexpr int H = (HZ + 1) & ~1, TI = kF3 - 2 * H;  // x-y halo, even: pairs on (even, odd) columns
  // >= the last stage's planes t-S-EXTRA-1 .. t; even, a multiple of 4 with
  // EXTRA (the four-buffer ring below follows it)
  constexpr int kRing = EXTRA ? ((S + EXTRA + 5) & ~3) : ((S + 3) & ~1);
  constexpr int D = 2;  // planes of inputs in flight ahead of their step
  static_assert(kRing % D == 0, "prefetch slots follow the ring");
  // published half planes: stage 0 (red) and every half-sweep; with EXTRA
  // the last black half-sweep's is read two steps later (four buffers)
  __shared__ T pub[S + 1][2][kF3][kF3 / 2];
  __shared__ T pubB[EXTRA ? 4 : 1][kF3][kF3 / 2];
  if (a.sc->done) return;
  const Place3 p = place3<H, TI>(a.Lf, a.tiles_x, a.tiles_y, a.tz);
  const long s2 = a.Lf.s[2];
  const int t0 = p.z0 - HZ;
  const int nstep = p.zc + 2 * HZ;  // planes [z0 - HZ, z0 + zc + HZ); the last stage lags HZ steps
  const int yd = clamp_row(p.ly - 1), yu = clamp_row(p.ly + 1);
  // b in FP64 where it is FP64 (the finest level)
  using TB = typename std::conditional<BD || sizeof(T) == 8, double, T>::type;
  T XR[kRing], XB[kRing];
  TB BR[kRing], BB[kRing];
#pragma unroll
  for (int k = 0; k < kRing; ++k) {
    XR[k] = XB[k] = T(0);
    BR[k] = BB[k] = TB(0);
  }
  // coarse cell of the pair (both cells share it)
  const int gxw = wrap_p(p.gx0 + p.lx0, p.nx), gyw = wrap_p(p.gy0 + p.ly, p.ny);
  const long cxy = (long)(gxw >> 1) + (long)(gyw >> 1) * a.Lc.s[1];
  // inputs of planes t + 1 .. t + D in flight, slot (plane - t0) % D
  T FX0[D], FX1[D], FC[D];
  TB FB0[D], FB1[D];
  // (issued unconditionally: past the chunk's last plane the loads read
  // planes that are never used, so no branch joins pending loads)
  auto fetch = [&](int t, auto F) __attribute__((always_inline)) {
    constexpr int f = decltype(F)::value;
    const int gz = wrap_any(t, p.nz);
    const long g = a.Lf.base + (long)gz * s2 + p.xy;
    const T *xp = a.xpre + g;
    FX0[f] = xp[0];
    FX1[f] = xp[1];
    FC[f] = a.xc[a.Lc.base + (long)(gz >> 1) * a.Lc.s[2] + cxy];
    load_b_pair<TB, BD>(a.b, g, FB0[f], FB1[f]);
  };
  static_for<0, D>([&](auto J) __attribute__((always_inline)) { fetch(t0 + decltype(J)::value, J); });
  double ru = 0.0, wu = 0.0, rr = 0.0;
  // EXTRA: r of the w stage's next plane, in flight one step ahead
  double rn0 = 0.0, rn1 = 0.0;
  auto fetch_r = [&](int q) __attribute__((always_inline)) {
    const double2 v = *(const double2 *)((const double *)a.b + a.Lf.base + (long)wrap_any(q, p.nz) * s2 + p.xy);
    rn0 = v.x;
    rn1 = v.y;
  };
  if (EXTRA) fetch_r(t0 - S - 1);
  auto step = [&](auto U, int ts) __attribute__((always_inline)) {
    constexpr int u = decltype(U)::value;
    const int t = t0 + ts;
    // LDS buffers of this step (written) and of earlier ones (read): z0 is a
    // multiple of 4 and the ring a multiple of 4 (of 2 without EXTRA), so t
    // mod 4 (mod 2) is that of u - HZ: every buffer index is a constant and
    // the compiler sees that a step's reads and writes never overlap
    constexpr int wb = ((u - HZ) % 2 + 2) % 2, rb = wb ^ 1;
    constexpr int wb4 = ((u - HZ) % 4 + 4) % 4, rb4 = (wb4 + 2) % 4;  // values this step publishes
    // stage 0 on plane t: x = pre-smoothed + coarse correction; publish red
    {
      constexpr int f = u % D;
      const int cr = (p.bpar + t) & 1;
      const T x0 = FX0[f] + FC[f], x1 = FX1[f] + FC[f];
      XR[u] = pick<T>(cr, x1, x0);
      XB[u] = pick<T>(cr, x0, x1);
      BR[u] = pick<TB>(cr, FB1[f], FB0[f]);
      BB[u] = pick<TB>(cr, FB0[f], FB1[f]);
      fetch(t + D, std::integral_constant<int, f>());
      pub[0][wb][p.ly][p.px] = XR[u];
    }
    // half-sweeps s = 1 .. S on plane t - s: black for odd s, red for even s
    static_for<1, S + 1>([&](auto Sc) __attribute__((always_inline)) {
      constexpr int s = decltype(Sc)::value;
      constexpr bool red = (s & 1) == 0;
      const int q = t - s;
      constexpr int k = Slot<kRing, u, s>::v;
      constexpr int km = Slot<kRing, u, s + 1>::v, kp = Slot<kRing, u, s - 1>::v;
      T *Xo = red ? XB : XR;
      const int cell = ((p.bpar + q) & 1) ^ (red ? 0 : 1);
      const T yl = pub[s - 1][rb][yd][p.px], yr = pub[s - 1][rb][yu][p.px];
      const T v = gs7<T>((T)(red ? BR[k] : BB[k]), Xo[k], outside_x<T>(cell, Xo[k]), yl, yr, Xo[km], Xo[kp],
                         a.ihx, a.ihy, a.ihz, a.idg);
      if (red)
        XR[k] = v;
      else
        XB[k] = v;
      pub[s][wb][p.ly][p.px] = v;
      if (EXTRA && s == S - 1) pubB[EXTRA ? wb4 : 0][p.ly][p.px] = v;
      // stages stay in order in the schedule: hoisting later stages' work
      // above this one only adds live registers (the FP64 kernel with the w
      // stage would spill)
      __builtin_amdgcn_sched_barrier(0);
      if (!EXTRA && s == S && q >= p.z0 && q < p.z0 + p.zc && p.own) {
        // both cells final on plane q: black after S - 1, red after S
        const int cr = (p.bpar + q) & 1;
        T *o = a.xout + a.Lf.base + (long)q * s2 + p.xy;
        o[0] = pick<T>(cr, XB[k], XR[k]);
        o[1] = pick<T>(cr, XR[k], XB[k]);
      }
    });
    if (EXTRA) {
      // w = A u on plane q = t - S - 1, both cells, in FP64
      const int q = t - S - 1;
      const double r0 = rn0, r1 = rn1;
      fetch_r(q + 1);
      constexpr int k = Slot<kRing, u, S + 1>::v;
      constexpr int km = Slot<kRing, u, S + 2>::v, kp = Slot<kRing, u, S>::v;
      if (q >= p.z0 && q < p.z0 + p.zc) {
        const int cr = (p.bpar + q) & 1;  // pair cell of the red cell
        // the red cell's neighbours are black: y from the last black
        // half-sweep (two steps ago); the black cell's are red: y from the
        // last red half-sweep (one step ago)
        const T ybl = pubB[EXTRA ? rb4 : 0][yd][p.px], ybu = pubB[EXTRA ? rb4 : 0][yu][p.px];
        const T yrl = pub[S][rb][yd][p.px], yru = pub[S][rb][yu][p.px];
        const double dg = 2.0 * (a.dihx + a.dihy + a.dihz);
        const double uR = (double)XR[k], uB = (double)XB[k];
        const double wR = dg * uR - (a.dihx * ((double)XB[k] + (double)outside_x<T>(cr, XB[k])) +
                                     a.dihy * ((double)ybl + (double)ybu) +
                                     a.dihz * ((double)XB[km] + (double)XB[kp]));
        const double wB = dg * uB - (a.dihx * ((double)XR[k] + (double)outside_x<T>(cr ^ 1, XR[k])) +
                                     a.dihy * ((double)yrl + (double)yru) +
                                     a.dihz * ((double)XR[km] + (double)XR[kp]));
        if (p.own) {
          const long g = a.Lf.base + (long)q * s2 + p.xy;
          T *o = a.xout + g;
          o[0] = pick<T>(cr, XB[k], XR[k]);
          o[1] = pick<T>(cr, XR[k], XB[k]);
          *(double2 *)(a.w + g) = make_double2(pick<double>(cr, wB, wR), pick<double>(cr, wR, wB));
          const double rR = pick<double>(cr, r1, r0), rB = pick<double>(cr, r0, r1);
          ru += rR * uR + rB * uB;
          wu += wR * uR + wB * uB;
          rr += rR * rR + rB * rB;
        }
      }
    }
    // one barrier: the next steps read what this one wrote
    __syncthreads();
  };
  // whole rounds of the ring (no branch between the unrolled steps: a step
  // past the last one works on planes outside the chunk and writes nothing)
  for (int tb = 0; tb < nstep; tb += kRing)
    static_for<0, kRing>([&](auto U) __attribute__((always_inline)) { step(U, tb + decltype(U)::value); });
  if (EXTRA) {
    double v3[3] = {ru, wu, rr};
    block_allsum_n<3>(v3);
    if (threadIdx.x == 0) {
      a.part_rz[blockIdx.x] = v3[0];
      a.part_rz[a.np + blockIdx.x] = v3[1];
      a.part_rz[2 * a.np + blockIdx.x] = v3[2];
    }
  }
}

}  // namespace lm
