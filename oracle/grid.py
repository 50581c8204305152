"""Uniform collocated Cartesian grid, ghost cells and boundary rules.

TEST INFRASTRUCTURE ONLY (see the package header).

Cell-centred variables live on an (n_d) grid per direction with one ghost layer
(section 3.2, Fig 1); face fluxes F_d live on the n_d + 1 faces normal to d.
Ghost values follow section 3.6: Dirichlet (Eq 3.43), Neumann (Eq 3.44),
periodic (Eq 3.45) and quadratic extrapolation (Eq 3.46 with the
coefficients of Eq 3.28).
"""
from __future__ import annotations

import numpy as np

SIDE_KINDS = ("periodic", "slip", "noslip", "inflow", "outflow")


class Grid:
    """Uniform grid: ``n`` cells and length ``L`` per direction, and per
    direction a pair (lo, hi) of side kinds from SIDE_KINDS. ``bnd`` maps
    (d, side) to boundary data: for inflow sides a dict with optional keys
    'v' (list per component), 'Z', 'H', 'F' (normal mass flux), each an array
    over the side's cells (interior shape without axis d) or a scalar; for
    wall sides (slip, no-slip) optional 'Z', 'H': wall values that make the
    scalar Dirichlet on that wall (an isothermal wall, Eq 4.16a-b) instead
    of Neumann 0 (adiabatic, Eq 4.16c)."""

    def __init__(self, n, L, bc=None, bnd=None):
        self.ndim = len(n)
        self.n = tuple(int(q) for q in n)
        self.L = tuple(float(q) for q in L[: self.ndim])
        self.h = tuple(self.L[d] / self.n[d] for d in range(self.ndim))
        if bc is None:
            bc = (("periodic", "periodic"),) * self.ndim
        self.bc = tuple(tuple(b) for b in bc[: self.ndim])
        for d in range(self.ndim):
            lo, hi = self.bc[d]
            assert lo in SIDE_KINDS and hi in SIDE_KINDS
            assert (lo == "periodic") == (hi == "periodic")
        self.bnd = dict(bnd or {})
        self.shape = tuple(reversed(self.n))
        self.pshape = tuple(q + 2 for q in self.shape)
        self.dV = float(np.prod(self.h))
        self.volume = float(np.prod(self.L))

    def axis(self, d):
        return self.ndim - 1 - d

    def periodic(self, d):
        return self.bc[d][0] == "periodic"

    @property
    def all_periodic(self):
        return all(self.periodic(d) for d in range(self.ndim))

    # -- slicing helpers ---------------------------------------------------
    def S(self, Ap, face_dir=None, off=None):
        """View of padded array ``Ap``. Along ``face_dir`` the view has
        n_d + 1 entries starting at padded index 0 (the cells left of each
        face); along the other directions it covers the interior. ``off``
        shifts the view by a cell offset per direction."""
        idx = [None] * self.ndim
        for d in range(self.ndim):
            o = 0 if off is None else off[d]
            if d == face_dir:
                idx[self.axis(d)] = slice(o, o + self.n[d] + 1)
            else:
                idx[self.axis(d)] = slice(1 + o, 1 + o + self.n[d])
        return Ap[tuple(idx)]

    def e(self, d, s=1):
        o = [0] * self.ndim
        o[d] = s
        return tuple(o)

    def plus(self, G, d):
        """Face array G (n_d + 1 along d) restricted to the high face of each cell."""
        idx = [slice(None)] * self.ndim
        idx[self.axis(d)] = slice(1, None)
        return G[tuple(idx)]

    def minus(self, G, d):
        idx = [slice(None)] * self.ndim
        idx[self.axis(d)] = slice(0, -1)
        return G[tuple(idx)]

    def face_index(self, d, f):
        """Index tuple selecting face f (0..n_d) of a face array along d."""
        idx = [slice(None)] * self.ndim
        idx[self.axis(d)] = f
        return tuple(idx)

    def pad(self, a):
        p = np.zeros(self.pshape, dtype=np.result_type(a, np.float64))
        p[tuple(slice(1, -1) for _ in range(self.ndim))] = a
        return p

    def interior(self, Ap):
        return Ap[tuple(slice(1, -1) for _ in range(self.ndim))]

    def bvalue(self, d, side, key, comp=None, default=0.0):
        data = self.bnd.get((d, side), {})
        val = data.get(key, None)
        if val is not None and comp is not None:
            val = val[comp]
        return default if val is None else val


def _side_index(g: Grid, d, pos, upto):
    """Index tuple of a hyperplane at padded position ``pos`` along axis d:
    directions e < d span the full padded range, e > d the interior."""
    idx = [None] * g.ndim
    for e in range(g.ndim):
        if e == d:
            idx[g.axis(e)] = pos
        elif e < upto:
            idx[g.axis(e)] = slice(None)
        else:
            idx[g.axis(e)] = slice(1, -1)
    return tuple(idx)


def _extend(g: Grid, d, val):
    """Broadcast a boundary-value array given over the interior cells of a
    side (C order, axis d removed) to the hyperplane used by ``_side_index``:
    edge values are repeated into the ghost positions of directions e < d."""
    if np.isscalar(val):
        return val
    dirs = [e for e in reversed(range(g.ndim)) if e != d]   # C-order axes of val
    pw = [(1, 1) if e < d else (0, 0) for e in dirs]
    return np.pad(np.asarray(val), pw, mode="edge")


def fill_ghosts(g: Grid, Ap, rules):
    """Fill the ghost layer of padded array ``Ap`` in place.

    ``rules[d] = (rule_lo, rule_hi)`` with each rule one of
    ('periodic',), ('dirichlet', value), ('neumann', value), ('extrap',).
    Directions are filled in order d = 0, 1, 2; pass d covers the full padded
    extent of the directions already filled and the interior of the others,
    so edge and corner ghosts take the rule of the highest direction."""
    for d in range(g.ndim):
        n = g.n[d]
        h = g.h[d]
        for side in (0, 1):
            rule = rules[d][side]
            gpos = 0 if side == 0 else n + 1
            i1 = 1 if side == 0 else n          # first interior cell
            i2 = 2 if side == 0 else n - 1
            i3 = 3 if side == 0 else n - 2
            G = _side_index(g, d, gpos, d)
            kind = rule[0]
            if kind == "periodic":
                src = n if side == 0 else 1      # Eq 3.45
                Ap[G] = Ap[_side_index(g, d, src, d)]
            elif kind == "dirichlet":           # Eq 3.43, mirrored ghost
                Ap[G] = 2.0 * _extend(g, d, rule[1]) - Ap[_side_index(g, d, i1, d)]
            elif kind == "dirichlet_or_wall":   # Eq 3.43 on inflow cells, Eq 3.44 (zero) on wall cells
                inner = Ap[_side_index(g, d, i1, d)]
                wall = _extend(g, d, np.asarray(rule[2], dtype=bool))
                Ap[G] = np.where(wall, inner, 2.0 * _extend(g, d, rule[1]) - inner)
            elif kind == "neumann":             # Eq 3.44, Phi = outward-normal derivative
                Ap[G] = Ap[_side_index(g, d, i1, d)] + h * _extend(g, d, rule[1])
            elif kind == "extrap":              # Eq 3.46 / 3.28 on a uniform grid: A=3, B=-3, C=1
                Ap[G] = (3.0 * Ap[_side_index(g, d, i1, d)] - 3.0 * Ap[_side_index(g, d, i2, d)]
                         + Ap[_side_index(g, d, i3, d)])
            else:
                raise ValueError(kind)
    return Ap


def extrap_coeffs(x0, x1, x2, x3):
    """Quadratic-extrapolation weights of Eq 3.28 for general positions."""
    A = (x2 - x0) * (x3 - x0) / ((x2 - x1) * (x3 - x1))
    B = (x1 - x0) * (x3 - x0) / ((x1 - x2) * (x3 - x2))
    C = (x1 - x0) * (x2 - x0) / ((x1 - x3) * (x2 - x3))
    return A, B, C


def field_rules(g: Grid, field, comp=None):
    """Ghost rules for a field given the side kinds.

    field: 'v' (component ``comp``), 'Z', 'H', 'P'.
    periodic: Eq 3.45 for every field.
    slip wall: normal velocity Dirichlet 0, tangential velocity and scalars
      Neumann 0.
    no-slip wall: velocity Dirichlet 0, scalars Neumann 0.
    on either wall a scalar with a value in the side data is Dirichlet
      with that value (Eq 3.43) instead.
    inflow: velocity and scalars Dirichlet with the side's given values;
      cells flagged 'wall' in the side data (a solid footprint on the
      side) take Neumann 0 for the scalars instead.
    outflow: velocity and scalars by quadratic extrapolation (Eq 3.46).
    P: quadratic extrapolation at every non-periodic side (Eq 3.27-3.28).
    """
    rules = []
    for d in range(g.ndim):
        pair = []
        for side in (0, 1):
            kind = g.bc[d][side]
            if kind == "periodic":
                pair.append(("periodic",))
            elif field == "P":
                pair.append(("extrap",))
            elif kind == "outflow":
                pair.append(("extrap",))
            elif kind == "inflow":
                wall = g.bvalue(d, side, "wall", default=None)
                if field == "v":
                    pair.append(("dirichlet", g.bvalue(d, side, "v", comp)))
                elif wall is not None:
                    pair.append(("dirichlet_or_wall", g.bvalue(d, side, field), wall))
                else:
                    pair.append(("dirichlet", g.bvalue(d, side, field)))
            elif field in ("Z", "H") and g.bvalue(d, side, field, default=None) is not None:
                pair.append(("dirichlet", g.bvalue(d, side, field)))
            elif kind == "noslip":
                pair.append(("dirichlet", 0.0) if field == "v" else ("neumann", 0.0))
            elif kind == "slip":
                if field == "v" and comp == d:
                    pair.append(("dirichlet", 0.0))
                else:
                    pair.append(("neumann", 0.0))
            else:
                raise ValueError(kind)
        rules.append(tuple(pair))
    return rules
