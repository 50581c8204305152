"""Exact zero-mean solution of the discrete pressure Poisson problem.

TEST INFRASTRUCTURE ONLY (see the package header).

The discrete operator is A P = sum_d delta_1(beta delta_1 P)/delta_1 x_d, the
composition of the face difference (Eq 3.21, n = 1) with itself that the
discrete continuity equation Eq 3.24 produces once the face flux of Eq 3.23 is
inserted. The paper's step has beta = 1; a face coefficient beta is accepted
for the variable-coefficient form, beta = 1/rho_f for div(grad P / rho)
(beta_inv_rho). Boundary faces of non-periodic sides carry
a prescribed mass flux, so A has zero flux there (a pure Neumann problem,
section 3.3). The singular system is closed by the augmented-matrix method of
section 3.3: [A 1; 1^T 0][P; lam] = [b; 0], whose solution is the zero-mean P,
with lam = mean(b) absorbing any compatibility residue. With beta = 1 the
operator is separable on every uniform grid: the Fourier modes diagonalise
it along periodic directions and the cosine modes of the DCT-II along the
zero-flux ones, so the same zero-mean solution is obtained by transforming
b, dividing by the eigenvalues (the constant mode, eigenvalue 0, is
dropped: that removes mean(b) and fixes the mean of P at 0) and
transforming back. With a face coefficient beta the augmented matrix is
factored by sparse LU.

On a stretched grid the differences of Eq 3.21 use the local spacings and
the operator is symmetric only after weighting each cell's row by its
volume: K = Delta V A has face coefficients area_f / (distance between the
two centres). The solve takes K P = Delta V (b - lam) with the constraint
sum(Delta V P) = 0 (the discrete integral of P, Eq 3.22, vanishes), i.e. the
augmented system [K dV; dV^T 0][P; lam] = [dV b; 0], whose lam is the
volume-weighted mean of b.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Grid

# threads of the scipy.fft transforms (the elementwise NumPy work runs on one)
FFT_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def face_grad(g: Grid, P, d):
    """delta_1 P / delta_1 x_d on the n_d + 1 faces normal to d, with periodic
    wrap on periodic directions and zero on boundary faces otherwise."""
    ax = g.axis(d)
    dfc = g.dfc[d]                              # h on a uniform grid
    if g.periodic(d):
        Pm = np.roll(P, 1, axis=ax)             # cell f-1 for face f = 0..n-1
        inner = (P - Pm) / g.along(d, dfc[:-1])
        first = np.take(inner, [0], axis=ax)
        return np.concatenate([inner, first], axis=ax)
    grad = np.diff(P, axis=ax) / g.along(d, dfc[1:-1])
    shp = list(P.shape)
    shp[ax] = 1
    z = np.zeros(shp, dtype=P.dtype)
    return np.concatenate([z, grad, z], axis=ax)


def laplacian(g: Grid, P, beta=None):
    """A P = sum_d [ (beta grad)_{f+1} - (beta grad)_f ] / h_d."""
    out = np.zeros_like(P)
    for d in range(g.ndim):
        G = face_grad(g, P, d)
        if beta is not None:
            G = G * beta[d]
        out = out + (g.plus(G, d) - g.minus(G, d)) / g.along(d, g.wid[d][1:-1])
    return out


def beta_inv_rho(g: Grid, rho):
    """Face coefficient beta = 1/rho_f of the variable-coefficient form
    div(grad P / rho), with rho_f the face value of the cell density by the
    two-point average of Eq 3.20 (n = 1), on the n_d + 1 faces normal to d
    (face f between cells f-1 and f, periodic wrap on periodic directions).
    Boundary faces of non-periodic sides carry no flux; their entry is 0."""
    out = []
    for d in range(g.ndim):
        ax = g.axis(d)
        if g.periodic(d):
            rm = np.roll(rho, 1, axis=ax)             # cell f-1 for face f = 0..n-1
            inner = 1.0 / (0.5 * (rho + rm))
            first = np.take(inner, [0], axis=ax)
            out.append(np.concatenate([inner, first], axis=ax))
            continue
        lo = np.take(rho, np.arange(0, g.n[d] - 1), axis=ax)
        hi = np.take(rho, np.arange(1, g.n[d]), axis=ax)
        inner = 1.0 / (0.5 * (lo + hi))
        shp = list(rho.shape)
        shp[ax] = 1
        z = np.zeros(shp)
        out.append(np.concatenate([z, inner, z], axis=ax))
    return out


def transform_eigenvalues(g: Grid):
    """Eigenvalues of A (beta = 1) on the separable modes of any uniform
    grid: along a periodic direction the Fourier mode k has
    -(4/h_d^2) sin^2(pi k / n_d); along a zero-flux direction the cosine
    mode cos(pi m (i + 1/2) / n_d) of the DCT-II has
    -(4/h_d^2) sin^2(pi m / (2 n_d))."""
    lam = np.zeros(g.shape)
    for d in range(g.ndim):
        k = np.arange(g.n[d])
        den = g.n[d] if g.periodic(d) else 2 * g.n[d]
        ld = -(4.0 / g.h[d] ** 2) * np.sin(np.pi * k / den) ** 2
        shp = [1] * g.ndim
        shp[g.axis(d)] = g.n[d]
        lam = lam + ld.reshape(shp)
    return lam


def periodic_eigenvalues(g: Grid):
    """Eigenvalues of A (beta = 1) on the Fourier modes of a periodic grid:
    lam(k) = -sum_d (4/h_d^2) sin^2(pi k_d / n_d)."""
    lam = np.zeros(g.shape)
    for d in range(g.ndim):
        k = np.arange(g.n[d])
        ld = -(4.0 / g.h[d] ** 2) * np.sin(np.pi * k / g.n[d]) ** 2
        shp = [1] * g.ndim
        shp[g.axis(d)] = g.n[d]
        lam = lam + ld.reshape(shp)
    return lam


class PoissonSolver:
    """Solves A P = b for the zero-mean P; returns (P, mean(b)).

    beta None: transform solve (FFT along periodic directions, DCT-II along
    the others); ``method="lu"`` forces the sparse LU of the augmented
    matrix instead. A face coefficient beta always takes the LU."""

    def __init__(self, g: Grid, beta=None, method=None):
        self.g = g
        self.beta = beta
        self.transform = beta is None and method != "lu" and not g.stretched
        self.fft = self.transform and g.all_periodic
        if self.transform:
            self.per_axes = [g.axis(d) for d in range(g.ndim) if g.periodic(d)]
            self.neu_axes = [g.axis(d) for d in range(g.ndim) if not g.periodic(d)]
            lam = transform_eigenvalues(g)
            if self.per_axes:
                # the real FFT keeps n//2 + 1 modes along its last axis
                last = self.per_axes[-1]
                lam = np.take(lam, np.arange(lam.shape[last] // 2 + 1), axis=last)
            lam.flat[0] = 1.0
            self.inv = 1.0 / lam
            self.inv.flat[0] = 0.0       # constant mode: zero mean
        else:
            self.lu = spla.splu(self._augmented().tocsc())

    def _augmented(self):
        g = self.g
        N = int(np.prod(g.shape))
        cols = []
        # assemble A column by column from its action on face differences
        idx = np.arange(N).reshape(g.shape)
        rows, cidx, vals = [], [], []
        vol = g.cell_volumes() if g.stretched else None
        for d in range(g.ndim):
            ax = g.axis(d)
            h2 = g.h[d] ** 2
            n = g.n[d]
            if g.stretched:
                # face areas of the d-faces: cell volume over the d-width
                area = vol / g.along(d, g.wid[d][1:-1])
            for f in range(n + 1):
                # face f between cells f-1 and f along d
                if f == 0 or f == n:
                    if not g.periodic(d):
                        continue
                    if f == n:
                        continue           # periodic face n is face 0
                    left = np.take(idx, n - 1, axis=ax)
                else:
                    left = np.take(idx, f - 1, axis=ax)
                right = np.take(idx, f % n, axis=ax)
                w = np.ones(left.shape) / h2
                if g.stretched:
                    # K = dV A: area_f / (distance between the two centres)
                    w = np.take(area, f % n, axis=ax) / g.dfc[d][f]
                if self.beta is not None:
                    bf = np.take(self.beta[d], f, axis=ax)
                    w = w * bf if g.stretched else bf / h2
                l, r, w = left.ravel(), right.ravel(), np.asarray(w).ravel()
                # flux w (P_r - P_l) leaves cell l through its high face and
                # enters cell r through its low face
                rows += [l, l, r, r]
                cidx += [r, l, l, r]
                vals += [w, -w, w, -w]
        rows = np.concatenate(rows)
        cidx = np.concatenate(cidx)
        vals = np.concatenate(vals)
        A = sp.coo_matrix((vals, (rows, cidx)), shape=(N, N)).tocsr()
        one = sp.csr_matrix((vol.ravel() if g.stretched else np.ones(N)).reshape(N, 1))
        aug = sp.bmat([[A, one], [one.T, None]])
        del cols
        return aug

    def _transform_solve(self, b):
        c = b
        if self.neu_axes:
            c = sfft.dctn(c, type=2, axes=self.neu_axes, norm="ortho", workers=FFT_WORKERS)
        if self.per_axes:
            c = sfft.rfftn(c, axes=self.per_axes, workers=FFT_WORKERS)
            c = c * self.inv
            s = [b.shape[a] for a in self.per_axes]
            c = sfft.irfftn(c, s=s, axes=self.per_axes, workers=FFT_WORKERS)
        else:
            c = c * self.inv
        if self.neu_axes:
            c = sfft.idctn(c, type=2, axes=self.neu_axes, norm="ortho", workers=FFT_WORKERS)
        return c

    def solve(self, b):
        g = self.g
        if g.stretched:
            vol = g.cell_volumes()
            rhs = np.concatenate([(vol * b).ravel(), [0.0]])
            if np.iscomplexobj(rhs):
                x = self.lu.solve(rhs.real) + 1j * self.lu.solve(rhs.imag)
            else:
                x = self.lu.solve(rhs)
            return x[: b.size].reshape(g.shape), x[b.size]
        lam = np.mean(b)
        if self.transform:
            if np.iscomplexobj(b):
                # the solve is a real-linear map: apply it to both parts
                # separately so that rounding of the real part never leaks
                # into the imaginary part (complex-step derivatives)
                return self.solve(b.real)[0] + 1j * self.solve(b.imag)[0], lam
            return self._transform_solve(np.asarray(b, dtype=np.float64)), lam
        N = b.size
        rhs = np.concatenate([b.ravel(), [0.0]])
        if np.iscomplexobj(rhs):
            x = self.lu.solve(rhs.real) + 1j * self.lu.solve(rhs.imag)
        else:
            x = self.lu.solve(rhs)
        return x[:N].reshape(g.shape), x[N]
