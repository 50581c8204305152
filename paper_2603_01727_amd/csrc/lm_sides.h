// Side data and ghost rules of non-periodic sides (section 3.6): the rule
// each field follows on each side and the prescribed side values. Shared by
// the forward step and its adjoint. Included after lm_device.h.
#pragma once

#include "lm_device.h"

namespace lm {

// ---------------------------------------------------------------------------
// Side data and ghost rules
// ---------------------------------------------------------------------------

// Compact index of the side cell that holds position p on a side normal to d
// (other coordinates clamped into the interior).
__device__ inline long side_index(const Lay &L, int d, int i, int j, int k) {
  i = min(max(i, 0), L.n[0] - 1);
  j = min(max(j, 0), L.n[1] - 1);
  k = min(max(k, 0), L.n[2] - 1);
  if (d == 0) return (long)k * L.n[1] + j;
  if (d == 1) return (long)k * L.n[0] + i;
  return (long)j * L.n[0] + i;
}

enum { R_PER = 0, R_DIR = 1, R_NEU = 2, R_EXT = 3 };

// A wall side with a given scalar (only H: an isothermal wall) takes it as
// a Dirichlet value (Eq 3.43); otherwise wall scalars are zero-gradient.
__device__ inline bool wall_scalar(const SideData &q, int f) { return (f == 4 && q.H) || (f == 3 && q.Z); }

// Ghost rule of field f (0..2 velocity components, 3 Z, 4 H) on side (d, s)
// at position (i, j, k) (used for the solid footprint of inflow sides).
__device__ inline int ghost_rule(const Bnd &B, const Sides &sd, const Lay &L, int d, int s, int f, int i, int j,
                                 int k) {
  const int kind = B.kind[d][s];
  switch (kind) {
    case LM_SIDE_PERIODIC: return R_PER;
    case LM_SIDE_OUTFLOW: return R_EXT;
    case LM_SIDE_INFLOW: {
      const unsigned char *w = sd.s[d][s].wall;
      if (f >= 3 && w && w[side_index(L, d, i, j, k)]) return R_NEU;
      return R_DIR;
    }
    case LM_SIDE_NOSLIP: return (f < 3 || wall_scalar(sd.s[d][s], f)) ? R_DIR : R_NEU;
    default: return (f == d || wall_scalar(sd.s[d][s], f)) ? R_DIR : R_NEU;  // slip wall
  }
}

// Isothermal wall: the highest direction in which (i, j, k) lies outside
// the box on a slip / no-slip side with a wall H (false if none).
template <int DIM>
__device__ inline bool isothermal_ghost(const Lay &L, const Bnd &B, const Sides &sd, int i, int j, int k, int &dw,
                                        int &sw) {
  const int q[3] = {i, j, k};
  for (int d = DIM - 1; d >= 0; --d) {
    if (q[d] >= 0 && q[d] < L.n[d]) continue;
    const int s = q[d] < 0 ? 0 : 1;
    const int kind = B.kind[d][s];
    if ((kind == LM_SIDE_SLIP || kind == LM_SIDE_NOSLIP) && sd.s[d][s].H) {
      dw = d;
      sw = s;
      return true;
    }
  }
  return false;
}

__device__ inline double side_value(const Sides &sd, const Lay &L, int d, int s, int f, int i, int j,
                                    int k) {
  const SideData &q = sd.s[d][s];
  const double *a = f < 3 ? q.v[f] : (f == 3 ? q.Z : q.H);
  if (!a) return 0.0;
  return a[side_index(L, d, i, j, k)];
}

}  // namespace lm
