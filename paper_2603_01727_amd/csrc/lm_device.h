// Device helpers shared by the kernels of liblowmach: cell indexing with
// periodic wrap, block reductions over 64-wide wavefronts, the single-pass
// "last block finishes the reduction" pattern, and the flame-sheet
// temperature map.
#pragma once

#include "lm_internal.h"

namespace lm {

// Linear block id and cell coordinates of the 2D-tiled launch (64 x 4 blocks,
// grid z = planes). Returns false for threads past the ragged edge.
struct CellPos {
  int i, j, k;
  long c;
};

__device__ inline unsigned linear_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ inline unsigned num_blocks() { return gridDim.x * gridDim.y * gridDim.z; }

// Workgroups are dealt to the 8 XCDs round robin (linear block b runs on
// XCD b mod 8), and each XCD has its own L2. Remapping block b to logical
// block (b mod 8) q + b / 8 (q = blocks per XCD) gives XCD j the j-th
// contiguous eighth of the domain, so tiles whose stencils overlap share an
// L2. Blocks of an incomplete last round keep their index.
constexpr unsigned kXCD = 8;
__device__ inline unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb / kXCD;
  if (b >= q * kXCD) return b;
  return (b % kXCD) * q + b / kXCD;
}

// 3D launches (grid z = planes) walk up the planes inside patches of a few
// tile rows across the whole x extent: consecutive blocks cover one patch
// plane after another, so the planes above and below that a stencil reads
// were loaded one patch plane earlier and are still in L2; with the XCD
// remap a patch's column of planes stays on one XCD.
constexpr unsigned kPatchRows = 8;
__device__ inline bool cell_of_thread(const Lay &L, CellPos &p) {
  const unsigned b = xcd_remap(linear_block(), num_blocks());
  unsigned bx, by, bz;
  if (gridDim.z > 1) {
    const unsigned tx = gridDim.x, ty = gridDim.y, nz = gridDim.z;
    unsigned py = kPatchRows;
    while (ty % py) py >>= 1;  // patch rows divide the tile rows
    const unsigned pp = tx * py;  // blocks of one patch plane
    const unsigned patch = b / (pp * nz), rem = b - patch * (pp * nz);
    bz = rem / pp;
    const unsigned t = rem - bz * pp;
    by = patch * py + t / tx;
    bx = t % tx;
  } else {
    bx = b % gridDim.x;
    const unsigned byz = b / gridDim.x;
    by = byz % gridDim.y;
    bz = byz / gridDim.y;
  }
  p.i = bx * kBX + threadIdx.x;
  p.j = by * kBY + threadIdx.y;
  p.k = bz;
  if (p.i >= L.n[0] || p.j >= L.n[1]) return false;
  p.c = L.at(p.i, p.j, p.k);
  return true;
}
__device__ inline int linear_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }

// Index of the neighbour of cell (coord q along d) at offset +-1 with
// periodic wrap; returns -1 when the neighbour lies outside a non-periodic
// side.
__device__ inline long nbr(const Lay &L, const Bnd &B, long c, int q, int d, int dir) {
  if (dir > 0) {
    if (q + 1 < L.n[d]) return c + L.s[d];
    return B.periodic[d] ? c - (long)(L.n[d] - 1) * L.s[d] : -1;
  }
  if (q > 0) return c - L.s[d];
  return B.periodic[d] ? c + (long)(L.n[d] - 1) * L.s[d] : -1;
}

__device__ inline int coord(const CellPos &p, int d) { return d == 0 ? p.i : (d == 1 ? p.j : p.k); }

// Sum over a block of kBlock threads; the result is valid in thread 0.
// Fixed reduction tree, so results are bitwise reproducible.
__device__ inline double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int t = linear_tid();
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
  __syncthreads();
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int w = 0; w < nw; ++w) s += sh[w];
  return s;
}

__device__ inline double block_max(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int t = linear_tid();
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
  __syncthreads();
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double s = -1.0;
  if (t == 0)
    for (int w = 0; w < nw; ++w) s = fmax(s, sh[w]);
  return s;
}

// Sum of nb partials written by an earlier kernel (fixed order, whole block
// participates); valid in thread 0. Partial sums are always consumed by a
// later kernel: no grid-wide fence is ever needed.
__device__ inline double sum_partials(const double *part, unsigned nb, double *sh) {
  const unsigned t = linear_tid();
  const unsigned nt = blockDim.x * blockDim.y * blockDim.z;
  // four independent running sums per thread (loads in flight together),
  // combined in a fixed order
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  unsigned q = t;
  for (; q + 3 * nt < nb; q += 4 * nt) {
    s0 += part[q];
    s1 += part[q + nt];
    s2 += part[q + 2 * nt];
    s3 += part[q + 3 * nt];
  }
  for (; q < nb; q += nt) s0 += part[q];
  return block_sum((s0 + s1) + (s2 + s3), sh);
}

// ---- stretched grids (section 3.2.1) ---------------------------------------
// Spacing arrays of direction d on a stretched grid, packed direction after
// direction: inverse cell widths on the padded cells (n + 2), then per face
// between padded cells p and p + 1 (n + 1 each) the inverse distance
// between the two centres and the Eq 3.20 (n = 1) weights of the lower and
// the upper centre, then per interior cell the inverse distance between its
// two neighbours' centres (Eq 3.21, n = 2; n entries). Interior cell i is
// padded cell i + 1; its high face is face i + 1, its low face face i.
struct MetView {
  const double *iwid, *idfc, *wlo, *whi, *id2;
};
__device__ inline MetView met_view(const double *met, const Lay &L, int d) {
  const double *p = met;
  for (int e = 0; e < d; ++e) p += 5 * (long)L.n[e] + 5;
  const long n = L.n[d];
  return {p, p + n + 2, p + 2 * n + 3, p + 3 * n + 4, p + 4 * n + 5};
}

// ---- flame sheet: T(Z, H), section 3.5 -------------------------------------

__device__ inline double lncosh(double x) {
  const double ax = fabs(x);
  return ax + log1p(exp(-2.0 * ax)) - 0.69314718055994530942;
}

// Regularised F of Eq 3.41 translated by fshift (F~(0) = -1).
__device__ inline double f_tilde(const Phys &P, double Z) {
  const double S = P.S, k = P.k;
  const double fe = (-(S + 1.0) * lncosh(k * (Z - 1.0)) / k + (S - 1.0) * (Z - 1.0)) / (2.0 * S);
  return fe + P.fshift;
}

// Eq 3.42; without reaction Z = 0 and F(0) = -1 (Eq 3.37).
__device__ inline double temperature(const Phys &P, double Z, double H) {
  if (!P.reacting) return P.qs * (H - 1.0);
  return P.qs * (f_tilde(P, Z) + H);
}

__device__ inline double theta_eps(const Phys &P, double Z) { return 0.5 * (1.0 + tanh(P.k * (Z - 1.0))); }

// Conductivity (= viscosity, Eq 2.49-2.50) of temperature: T^sigma, or
// Sutherland's law T^{3/2} (1 + C)/(T + C) (Eq 4.12).
__device__ inline double kappa_of(const Phys &P, double T) {
  if (P.suth_C > 0.0) {
    const double C = P.suth_C;
    return T * sqrt(T) * (1.0 + C) / (T + C);
  }
  return pow(T, P.sigma);
}

}  // namespace lm
