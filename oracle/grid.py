"""Collocated Cartesian grid (uniform or stretched), ghost cells and
boundary rules.

TEST INFRASTRUCTURE ONLY (see the package header).

Cell-centred variables live on an (n_d) grid per direction with one ghost layer
(section 3.2, Fig 1); face fluxes F_d live on the n_d + 1 faces normal to d.
Ghost values follow section 3.6: Dirichlet (Eq 3.43), Neumann (Eq 3.44),
periodic (Eq 3.45) and quadratic extrapolation (Eq 3.46 with the
coefficients of Eq 3.28).

A stretched grid gives the face coordinates of each direction; the cell
centre is the midpoint of its two faces (the centroid), a ghost cell
mirrors the first interior cell at a wall (the spacing Eq 3.43 assumes)
and repeats the wrapped cell's width on a periodic direction. The spacing
arrays below feed the interpolation and difference operators of Eq 3.20
and 3.21 (section 3.2.1); on a uniform grid they hold h, 2h and 1/2
exactly, so the uniform arithmetic is unchanged.
"""
from __future__ import annotations

import numpy as np

SIDE_KINDS = ("periodic", "slip", "noslip", "inflow", "outflow")


class Grid:
    """Grid of ``n`` cells and length ``L`` per direction (uniform, or with
    the face coordinates ``faces[d]``, n_d + 1 increasing values from 0 to
    L_d, on a stretched direction), and per direction a pair (lo, hi) of
    side kinds from SIDE_KINDS. ``bnd`` maps
    (d, side) to boundary data: for inflow sides a dict with optional keys
    'v' (list per component), 'Z', 'H', 'F' (normal mass flux), each an array
    over the side's cells (interior shape without axis d) or a scalar; for
    wall sides (slip, no-slip) optional 'Z', 'H': wall values that make the
    scalar Dirichlet on that wall (an isothermal wall, Eq 4.16a-b) instead
    of Neumann 0 (adiabatic, Eq 4.16c)."""

    def __init__(self, n, L, bc=None, bnd=None, faces=None):
        self.ndim = len(n)
        self.n = tuple(int(q) for q in n)
        self.L = tuple(float(q) for q in L[: self.ndim])
        self.h = tuple(self.L[d] / self.n[d] for d in range(self.ndim))
        faces = list(faces or [None] * self.ndim)[: self.ndim]
        self.faces = [None if f is None else np.asarray(f, dtype=np.float64) for f in faces]
        for d, f in enumerate(self.faces):
            if f is not None:
                assert f.shape == (self.n[d] + 1,) and np.all(np.diff(f) > 0), "faces: n + 1 increasing values"
                assert abs(f[0]) < 1e-15 and abs(f[-1] - self.L[d]) < 1e-12 * self.L[d], "faces span [0, L]"
        self.stretched = any(f is not None for f in self.faces)
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
        self._spacings()

    # -- spacings (Eq 3.20-3.21 on the padded cells) --------------------------
    def _spacings(self):
        """Per direction, along the padded cells 0..n+1: ``wid`` the cell
        widths, ``dfc`` the distances between the centres of cells p and
        p+1 (one per face, n + 1), ``wlo``/``whi`` the weights of Eq 3.20
        (n = 1) that interpolate from those two centres to their face, and
        ``d2`` the distance between the centres of cells p-1 and p+1 for the
        interior cells (Eq 3.21, n = 2)."""
        self.wid, self.dfc, self.wlo, self.whi, self.d2 = [], [], [], [], []
        for d in range(self.ndim):
            n, h, f = self.n[d], self.h[d], self.faces[d]
            if f is None:
                self.wid.append(np.full(n + 2, h))
                self.dfc.append(np.full(n + 1, h))
                self.wlo.append(np.full(n + 1, 0.5))
                self.whi.append(np.full(n + 1, 0.5))
                self.d2.append(np.full(n, 2.0 * h))
                continue
            w = np.diff(f)
            lo, hi = (w[-1], w[0]) if self.periodic(d) else (w[0], w[-1])
            wid = np.concatenate([[lo], w, [hi]])
            self.wid.append(wid)
            self.dfc.append(0.5 * (wid[:-1] + wid[1:]))
            self.wlo.append(wid[1:] / (wid[:-1] + wid[1:]))
            self.whi.append(wid[:-1] / (wid[:-1] + wid[1:]))
            self.d2.append(0.5 * wid[:-2] + wid[1:-1] + 0.5 * wid[2:])

    def along(self, d, a):
        """1D array ``a`` reshaped to broadcast along direction d."""
        shp = [1] * self.ndim
        shp[self.axis(d)] = -1
        return np.reshape(a, shp)

    def cell_volumes(self):
        """Cell volumes Delta V (Eq 3.22) on the interior cells."""
        out = np.ones(self.shape)
        for d in range(self.ndim):
            out = out * self.along(d, self.wid[d][1:-1])
        return out

    def integral(self, a):
        """Midpoint-rule integral of a cell field (Eq 3.22)."""
        if not self.stretched:
            return np.sum(a) * self.dV
        return np.sum(a * self.cell_volumes())

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
                # the ghost and first interior centres are one cell width apart
                Ap[G] = Ap[_side_index(g, d, i1, d)] + g.wid[d][i1] * _extend(g, d, rule[1])
            elif kind == "extrap":              # Eq 3.46 / 3.28 (uniform grid: A=3, B=-3, C=1)
                A, B, C = ghost_extrap_coeffs(g, d, side)
                Ap[G] = (A * Ap[_side_index(g, d, i1, d)] + B * Ap[_side_index(g, d, i2, d)]
                         + C * Ap[_side_index(g, d, i3, d)])
            else:
                raise ValueError(kind)
    return Ap


def extrap_coeffs(x0, x1, x2, x3):
    """Quadratic-extrapolation weights of Eq 3.28 for general positions."""
    A = (x2 - x0) * (x3 - x0) / ((x2 - x1) * (x3 - x1))
    B = (x1 - x0) * (x3 - x0) / ((x1 - x2) * (x3 - x2))
    C = (x1 - x0) * (x2 - x0) / ((x1 - x3) * (x2 - x3))
    return A, B, C


def side_centres(g: Grid, d, side):
    """Distances from the boundary face of side (d, side) to the centres of
    the first three interior cells, inward."""
    w = g.wid[d]
    if side == 0:
        a, b, c = w[1], w[2], w[3]
    else:
        a, b, c = w[-2], w[-3], w[-4]
    return 0.5 * a, a + 0.5 * b, a + b + 0.5 * c


def ghost_extrap_coeffs(g: Grid, d, side):
    """Eq 3.28 for the mirrored ghost centre (half a first-cell width
    outside the boundary face) from the first three interior centres;
    exactly 3, -3, 1 on a uniform spacing."""
    if g.faces[d] is None:
        return 3.0, -3.0, 1.0
    x1, x2, x3 = side_centres(g, d, side)
    return extrap_coeffs(-x1, x1, x2, x3)


def face_extrap_coeffs(g: Grid, d, side):
    """Quadratic extrapolation from the first three interior centres to the
    boundary face itself (Eq 3.28 with x_0 at the face); 15/8, -10/8, 3/8
    on a uniform spacing."""
    if g.faces[d] is None:
        return 15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0
    return extrap_coeffs(0.0, *side_centres(g, d, side))


def tanh_faces(n, m, L=1.0):
    """Face coordinates of the tanh stretching of Eq 4.18 on [0, L], read as
    x~ = (1 + tanh(alpha (x - 1/2)) / tanh(alpha / 2)) / 2 (the printed form
    does not map 0 to 0), at the uniform faces x = k/n, with alpha chosen so
    that the largest cell is m times the smallest (the spacing ratio by
    which section 4.4 sets alpha). m = 1 gives the uniform faces."""
    x = np.arange(n + 1) / n
    if m == 1.0:
        return L * x

    def faces(a):
        return 0.5 * (1.0 + np.tanh(a * (x - 0.5)) / np.tanh(0.5 * a))

    def ratio(a):
        w = np.diff(faces(a))
        return w.max() / w.min()

    lo, hi = 1e-8, 1.0
    while ratio(hi) < m:
        hi *= 2.0
    for _ in range(200):                      # bisection on the monotone ratio
        mid = 0.5 * (lo + hi)
        if ratio(mid) < m:
            lo = mid
        else:
            hi = mid
    f = L * faces(0.5 * (lo + hi))
    f[0], f[-1] = 0.0, L
    return f


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
