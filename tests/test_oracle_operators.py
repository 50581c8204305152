"""Oracle pins for the spatial operators (section 3.2, Eq 3.20-3.26) and the
ghost rules (section 3.6).

Each discrete term is compared with the continuous operator applied to smooth
periodic fields; the continuous value is obtained by spectral differentiation
(exact to round-off for these band-limited inputs up to products), an
independent route. Second-order convergence pins every coefficient: a
dropped term, a wrong sign, a wrong index or a wrong 2/3 leaves an O(1) error.
"""
import math

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, fill_ghosts
from oracle.grid import extrap_coeffs, field_rules
from workloads import cell_centres

TWO_PI = 2 * math.pi


def spec_d(f, g, d):
    """Spectral derivative along direction d on a periodic grid."""
    ax = g.axis(d)
    n = g.n[d]
    k = np.fft.fftfreq(n, d=g.h[d]) * TWO_PI
    shp = [1] * g.ndim
    shp[ax] = n
    return np.real(np.fft.ifft(1j * k.reshape(shp) * np.fft.fft(f, axis=ax), axis=ax))


def face_values(g, d, fn):
    cs = cell_centres(g.n, g.L)
    fc = list(cs)
    shp = [1] * g.ndim
    shp[g.axis(d)] = g.n[d] + 1
    fc[d] = (np.arange(g.n[d] + 1) * g.h[d]).reshape(shp)
    full = tuple(g.n[d] + 1 if a == g.axis(d) else g.shape[a] for a in range(g.ndim))
    return np.broadcast_to(fn(*fc), full).copy()


def periodic_pad(g, a):
    p = g.pad(a)
    fill_ghosts(g, p, [(("periodic",),) * 2] * g.ndim)
    return p


def fields2d():
    phi = lambda x, y: np.sin(x) * np.cos(2 * y) + 0.3 * np.cos(x + y)
    kap = lambda x, y: 1.5 + 0.4 * np.sin(x + 2 * y)
    F = [lambda x, y: 1.0 + 0.5 * np.cos(y) * np.sin(x), lambda x, y: 0.7 * np.sin(2 * x) - 0.2 * np.cos(y)]
    v = [lambda x, y: np.sin(x) * np.cos(y) + 0.2 * np.cos(2 * x),
         lambda x, y: np.cos(2 * x) * np.sin(y) + 0.3 * np.sin(x)]
    return phi, kap, F, v


def fields3d():
    phi = lambda x, y, z: np.sin(x) * np.cos(2 * y) + 0.3 * np.cos(x + z)
    kap = lambda x, y, z: 1.5 + 0.4 * np.sin(x + 2 * y - z)
    F = [lambda x, y, z: 1.0 + 0.5 * np.cos(y) * np.sin(x + z),
         lambda x, y, z: 0.7 * np.sin(2 * x) - 0.2 * np.cos(y + z),
         lambda x, y, z: 0.4 * np.cos(x - y) + 0.1 * np.sin(z)]
    v = [lambda x, y, z: np.sin(x) * np.cos(y) + 0.2 * np.cos(2 * z),
         lambda x, y, z: np.cos(2 * x) * np.sin(y) + 0.3 * np.sin(z + x),
         lambda x, y, z: np.cos(y) * np.sin(2 * z) - 0.1 * np.cos(x)]
    return phi, kap, F, v


def errors(ndim, n):
    g = Grid((n,) * ndim, (TWO_PI,) * ndim)
    cs = cell_centres(g.n, g.L)
    phi, kap, Ff, vf = fields2d() if ndim == 2 else fields3d()
    full = lambda f: np.broadcast_to(f(*cs), g.shape).copy()
    o = Oracle(g, Params())
    P = full(phi)
    K = full(kap)
    V = [full(f) for f in vf]
    F = [face_values(g, d, Ff[d]) for d in range(ndim)]
    Fc = [full(Ff[d]) for d in range(ndim)]
    adv, dif = o._scalar_terms(periodic_pad(g, P), periodic_pad(g, K), F)
    adv_t = sum(Fc[d] * spec_d(P, g, d) for d in range(ndim))
    dif_t = sum(spec_d(K * spec_d(P, g, d), g, d) for d in range(ndim))
    conv, visc = o._momentum_terms([periodic_pad(g, a) for a in V], periodic_pad(g, K), F)
    D = [[spec_d(V[c], g, k) for c in range(ndim)] for k in range(ndim)]   # D[k][c] = d v_c / d x_k
    div = sum(D[k][k] for k in range(ndim))
    errs = [np.max(np.abs(adv - adv_t)), np.max(np.abs(dif - dif_t))]
    for i in range(ndim):
        conv_t = sum(spec_d(Fc[d] * V[i], g, d) for d in range(ndim))
        visc_t = 0.0
        for d in range(ndim):
            tau = D[d][i] + D[i][d] - (2.0 / 3.0 if i == d else 0.0) * div
            visc_t = visc_t + spec_d(K * tau, g, d)
        errs += [np.max(np.abs(conv[i] - conv_t)), np.max(np.abs(visc[i] - visc_t))]
    return np.array(errs)


@pytest.mark.parametrize("ndim,ns", [(2, (16, 32, 64)), (3, (10, 20, 40))])
def test_operators_second_order(ndim, ns):
    es = [errors(ndim, n) for n in ns]
    order = np.log2(es[-2] / es[-1])
    assert np.all(order > 1.85), (order, es[-1])
    assert np.all(order < 2.3), order


def test_extrapolation_coefficients_uniform():
    """Eq 3.28 at x0 = -h/2, x1..x3 = h/2, 3h/2, 5h/2: A, B, C = 3, -3, 1."""
    A, B, C = extrap_coeffs(-0.5, 0.5, 1.5, 2.5)
    assert (A, B, C) == (3.0, -3.0, 1.0)


def test_ghost_rules_reproduce_boundary_conditions():
    g = Grid((6, 5), (6.0, 5.0), bc=(("inflow", "outflow"), ("slip", "noslip")))
    x, y = cell_centres(g.n, g.L)
    q = np.broadcast_to(2.0 + 0.5 * x + 0.25 * x * x + 0 * y, g.shape).copy()
    p = g.pad(q)
    fill_ghosts(g, p, [(("dirichlet", 7.0), ("extrap",)), (("neumann", 0.0), ("neumann", 0.0))])
    # Dirichlet: face average equals the value (Eq 3.43)
    assert np.allclose(0.5 * (p[1:-1, 0] + p[1:-1, 1]), 7.0)
    # extrapolation is exact for a quadratic in x (Eq 3.46)
    xg = g.L[0] + 0.5 * g.h[0]
    assert np.allclose(p[1:-1, -1], 2.0 + 0.5 * xg + 0.25 * xg * xg)
    # zero Neumann: ghost equals first interior value, corners included
    assert np.array_equal(p[0, :], p[1, :])
    assert np.array_equal(p[-1, :], p[-2, :])


@pytest.mark.parametrize("side", [0, 1])
def test_outflow_face_flux_is_exact_for_quadratic_momentum(side):
    """The outflow face carries the cell momentum extrapolated to the face
    by the quadratic through the three nearest cells (the outflow closure
    of section 4.5 with the quadratic rule of Eq 3.28): for a momentum
    field quadratic in the outflow direction the face value is exact.
    The mirrored ghost averaged with the first cell (the interior face
    rule at a boundary) or a linear rule misses by c h^2 / 4 or more."""
    bc = (("periodic", "periodic"), ("outflow", "slip") if side == 0 else ("inflow", "outflow"))
    g = Grid((3, 10), (1.0, 2.0), bc=bc)
    x, y = cell_centres(g.n, g.L)
    a, b, c = 0.7, -1.3, 2.9
    m = lambda s: a + b * s + c * s * s
    M = [np.zeros(g.shape), np.broadcast_to(m(y) + 0 * x, g.shape).copy()]
    o = Oracle(g, Params())
    F = o.face_average_flux(M)
    yf = 0.0 if side == 0 else g.L[1]
    face = F[1][0, :] if side == 0 else F[1][-1, :]
    assert np.max(np.abs(face - m(yf))) < 1e-13
    # the interior faces stay two-point averages (Eq 3.20, n = 1)
    inner = 0.5 * (M[1][:-1, :] + M[1][1:, :])
    assert np.max(np.abs(F[1][1:-1, :] - inner)) < 1e-15
    # a plausible wrong rule: the average of the first cell and its
    # quadratically extrapolated ghost
    h = g.h[1]
    m1 = m(yf + (h / 2 if side == 0 else -h / 2))
    ghost = m(yf + (-h / 2 if side == 0 else h / 2))
    assert abs(0.5 * (m1 + ghost) - m(yf)) > 0.2 * c * h * h


def test_inflow_footprint_ghosts_mix_dirichlet_and_zero_gradient():
    """An inflow side partly covered by a solid footprint: on footprint
    cells the scalars take the zero-gradient ghost (Eq 3.44 with zero
    flux), elsewhere the mirrored Dirichlet ghost of the given value
    (Eq 3.43); the velocity is Dirichlet on every cell of the side."""
    g = Grid((8, 6), (1.0, 1.0), bc=(("periodic", "periodic"), ("inflow", "outflow")))
    wall = np.zeros(8, dtype=bool)
    wall[2:5] = True
    Zb = np.linspace(0.5, 1.2, 8)
    vb = [np.zeros(8), np.where(wall, 0.0, 0.3)]
    g.bnd[(1, 0)] = {"Z": Zb, "H": 2.5, "v": vb, "F": np.where(wall, 0.0, 0.3), "wall": wall}
    rng = np.random.default_rng(3)
    q = rng.standard_normal(g.shape)
    for field, val in (("Z", Zb), ("H", np.full(8, 2.5))):
        p = g.pad(q)
        fill_ghosts(g, p, field_rules(g, field))
        ghost, inner = p[0, 1:-1], p[1, 1:-1]
        assert np.array_equal(ghost[wall], inner[wall])                         # zero gradient
        assert np.max(np.abs(0.5 * (ghost[~wall] + inner[~wall]) - val[~wall])) < 1e-15   # face value
    for comp in (0, 1):
        p = g.pad(q)
        fill_ghosts(g, p, field_rules(g, "v", comp))
        assert np.max(np.abs(0.5 * (p[0, 1:-1] + p[1, 1:-1]) - vb[comp])) < 1e-15
