"""Pins of the oracle's stretched grids (section 3.2.1, Eq 3.20-3.22;
section 4.4, Eq 4.18): the tanh stretching against the spacings printed in
Tables 3-4, second-order truncation of every spatial operator on a smoothly
stretched grid, the volume-weighted Poisson solve against a manufactured
solution, discrete continuity after the projection, and the uniform limit."""
import math
import os

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, PoissonSolver
from oracle.grid import tanh_faces, fill_ghosts, field_rules
from oracle.poisson import laplacian

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tab34_max_spacing.txt")


def _rows():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            m, n, w, p0 = line.split()
            out.append((float(m), int(n), float(w), float(p0)))
    return out


def test_tanh_spacing_matches_tables_3_and_4():
    """Eq 4.18 read as x~ = (1 + tanh(alpha (x - 1/2)) / tanh(alpha/2)) / 2
    at the uniform faces, alpha set so that the largest cell is m times the
    smallest, gives every printed max(Delta x) to one unit in its last
    digit; alpha from the continuous derivative ratio cosh^2(alpha/2) = m
    instead misses the 64^2 rows by 10 and more units."""
    for m, n, w, _ in _rows():
        f = tanh_faces(n, m)
        d = np.diff(f)
        assert abs(d.max() / d.min() - m) < 1e-9
        assert abs(f[0]) == 0.0 and f[-1] == 1.0
        assert np.allclose(f + f[::-1], 1.0, atol=1e-15)       # symmetric about the centre
        assert abs(d.max() - w) <= 1.0e-5 + 1e-12, (m, n, d.max(), w)
    for m, n, w, _ in _rows():
        if n != 64:
            continue
        a = 2.0 * math.acosh(math.sqrt(m))
        x = np.arange(n + 1) / n
        fc = 0.5 * (1.0 + np.tanh(a * (x - 0.5)) / math.tanh(0.5 * a))
        assert abs(np.diff(fc).max() - w) > 1.0e-4


def _sine_faces(n, a=0.6):
    """Smooth periodic stretching of [0, 1]: x~ = x + a sin(2 pi x) / (2 pi),
    cells from (1 - a) to (1 + a) times the mean width."""
    x = np.arange(n + 1) / n
    f = x + a * np.sin(2.0 * np.pi * x) / (2.0 * np.pi)
    f[0], f[-1] = 0.0, 1.0
    return f


def _centres(g, d):
    if g.faces[d] is None:
        return (np.arange(g.n[d]) + 0.5) * g.h[d]
    f = g.faces[d]
    return 0.5 * (f[:-1] + f[1:])


def _fields(g, fn):
    X, Y = np.meshgrid(_centres(g, 0), _centres(g, 1))
    return fn(X, Y)


def _face_fields(g, d, fn):
    """Analytic values on the d-faces (n_d + 1 along d)."""
    xs = [_centres(g, 0), _centres(g, 1)]
    xs[d] = g.faces[d] if g.faces[d] is not None else np.arange(g.n[d] + 1) * g.h[d]
    X, Y = np.meshgrid(xs[0], xs[1])
    return fn(X, Y)


TWO_PI = 2.0 * np.pi


def _operator_errors(n):
    """Truncation errors (max over cells) of the scalar advection and
    diffusion terms and of the momentum convection and viscous terms on a
    periodic unit square stretched smoothly in both directions."""
    g = Grid((n, n), (1.0, 1.0), faces=[_sine_faces(n, 0.6), _sine_faces(n, 0.4)])
    o = Oracle(g, Params(Re=1.0, Pr=1.0))
    phi = lambda X, Y: np.sin(TWO_PI * X) * np.cos(TWO_PI * Y) + 0.3 * np.cos(TWO_PI * (X + 2 * Y))
    kap = lambda X, Y: 1.0 + 0.4 * np.sin(TWO_PI * X + 0.3) * np.cos(TWO_PI * Y)
    u = [lambda X, Y: 0.7 + np.sin(TWO_PI * Y) * np.cos(TWO_PI * X),
         lambda X, Y: -0.2 + 0.5 * np.sin(TWO_PI * (X - Y))]
    # exact derivatives (by hand) of the fields above
    k2 = TWO_PI

    def dphi(X, Y):
        return (k2 * np.cos(k2 * X) * np.cos(k2 * Y) - 0.3 * k2 * np.sin(k2 * (X + 2 * Y)),
                -k2 * np.sin(k2 * X) * np.sin(k2 * Y) - 0.6 * k2 * np.sin(k2 * (X + 2 * Y)))

    def dkap(X, Y):
        return (0.4 * k2 * np.cos(k2 * X + 0.3) * np.cos(k2 * Y), -0.4 * k2 * np.sin(k2 * X + 0.3) * np.sin(k2 * Y))

    def lap_phi(X, Y):
        return (-2 * k2 ** 2 * np.sin(k2 * X) * np.cos(k2 * Y) - 0.3 * 5 * k2 ** 2 * np.cos(k2 * (X + 2 * Y)))

    def du(X, Y):   # du[i][j] = d u_i / d x_j
        return [[-k2 * np.sin(k2 * Y) * np.sin(k2 * X), k2 * np.cos(k2 * Y) * np.cos(k2 * X)],
                [0.5 * k2 * np.cos(k2 * (X - Y)), -0.5 * k2 * np.cos(k2 * (X - Y))]]

    def d2u(X, Y):  # d2u[i][j][k] = d^2 u_i / dx_j dx_k
        a = [[-k2 ** 2 * np.sin(k2 * Y) * np.cos(k2 * X), -k2 ** 2 * np.cos(k2 * Y) * np.sin(k2 * X)],
             [-k2 ** 2 * np.cos(k2 * Y) * np.sin(k2 * X), -k2 ** 2 * np.sin(k2 * Y) * np.cos(k2 * X)]]
        s = -0.5 * k2 ** 2 * np.sin(k2 * (X - Y))
        b = [[s, -s], [-s, s]]
        return [a, b]

    P = _fields(g, phi)
    Pp = g.pad(P)
    fill_ghosts(g, Pp, field_rules(g, "H"))
    K = g.pad(_fields(g, kap))
    fill_ghosts(g, K, field_rules(g, "H"))
    F = [_face_fields(g, d, u[d]) for d in range(2)]
    adv, dif = o._scalar_terms(Pp, K, F)
    X, Y = np.meshgrid(_centres(g, 0), _centres(g, 1))
    gp, gk = dphi(X, Y), dkap(X, Y)
    U = [u[0](X, Y), u[1](X, Y)]
    adv_ex = U[0] * gp[0] + U[1] * gp[1]
    dif_ex = kap(X, Y) * lap_phi(X, Y) + gk[0] * gp[0] + gk[1] * gp[1]
    vp = []
    for i in range(2):
        a = g.pad(U[i])
        fill_ghosts(g, a, field_rules(g, "v", i))
        vp.append(a)
    conv, visc = o._momentum_terms(vp, K, F)
    D, DD = du(X, Y), d2u(X, Y)
    kc = kap(X, Y)
    div = D[0][0] + D[1][1]
    ddiv = [DD[0][0][j] + DD[1][1][j] for j in range(2)]
    conv_ex, visc_ex = [], []
    for i in range(2):
        # d_j (u_j u_i) and d_j tau_ij, tau_ij = kappa (d_j u_i + d_i u_j - 2/3 delta_ij div)
        conv_ex.append(sum(D[j][j] * U[i] + U[j] * D[i][j] for j in range(2)))
        v = 0.0
        for j in range(2):
            t = D[i][j] + D[j][i] - (2.0 / 3.0 * div if i == j else 0.0)
            dt = DD[i][j][j] + DD[j][i][j] - (2.0 / 3.0 * ddiv[j] if i == j else 0.0)
            v = v + gk[j] * t + kc * dt
        visc_ex.append(v)
    return (np.max(np.abs(adv - adv_ex)), np.max(np.abs(dif - dif_ex)),
            max(np.max(np.abs(conv[i] - conv_ex[i])) for i in range(2)),
            max(np.max(np.abs(visc[i] - visc_ex[i])) for i in range(2)))


def test_stretched_operators_are_second_order():
    """Advection (Eq 3.26b), diffusion, convection (Eq 3.26a) and the
    viscous stress (Eq 2.46) built from Eq 3.20-3.21 on a smoothly
    stretched periodic grid (cells 0.4 to 1.6 times the mean width):
    each truncation error falls by 4 per halving of the cells. Reading
    any spacing as uniform, or swapping the interpolation weights, leaves
    an O(1) error that does not fall."""
    e = [np.array(_operator_errors(n)) for n in (16, 32, 64)]
    for a, b in zip(e[:-1], e[1:]):
        order = np.log2(a / b)
        assert np.all(order > 1.85) and np.all(order < 2.3), (order, a, b)


def _poisson_case(n, m):
    g = Grid((n, n), (1.0, 1.0), bc=(("noslip", "noslip"), ("periodic", "periodic")),
             faces=[tanh_faces(n, m), _sine_faces(n, 0.5)])
    X, Y = np.meshgrid(_centres(g, 0), _centres(g, 1))
    P = np.cos(np.pi * X) * np.cos(TWO_PI * Y) + 0.5 * np.cos(2 * np.pi * X)
    b = -(np.pi ** 2 + TWO_PI ** 2) * np.cos(np.pi * X) * np.cos(TWO_PI * Y) - 2.0 * np.pi ** 2 * np.cos(2 * np.pi * X)
    return g, P, b


def test_stretched_poisson_manufactured_solution():
    """Zero-flux walls stretched by tanh (m = 3) in x, periodic y stretched
    smoothly: P = cos(pi x) cos(2 pi y) + cos(2 pi x)/2 from its exact
    Laplacian. The solve returns the solution with vanishing integral
    (Eq 3.22), lam = the volume-weighted mean of b, and converges at second
    order."""
    errs = []
    for n in (16, 32, 64):
        g, P, b = _poisson_case(n, 3.0)
        vol = g.cell_volumes()
        Pex = P - np.sum(vol * P) / np.sum(vol)
        sol, lam = PoissonSolver(g).solve(b)
        assert abs(np.sum(vol * sol)) < 1e-13
        assert abs(lam - np.sum(vol * b) / np.sum(vol)) < 1e-11 * np.max(np.abs(b))
        r = laplacian(g, sol) - (b - lam)
        assert np.max(np.abs(r)) < 1e-9 * np.max(np.abs(b))
        errs.append(np.max(np.abs(sol - Pex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), (errs, orders)


def test_stretched_operator_is_symmetric_after_volume_weighting():
    """K = dV A (the matrix the solve factors) is symmetric; A alone is
    not on a stretched grid."""
    g, _, _ = _poisson_case(8, 3.0)
    N = 64
    A = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        A[:, k] = laplacian(g, e.reshape(g.shape)).ravel()
    K = g.cell_volumes().ravel()[:, None] * A
    assert np.max(np.abs(K - K.T)) < 1e-13 * np.max(np.abs(K))
    assert np.max(np.abs(A - A.T)) > 1e-2 * np.max(np.abs(A))


def _box(n, m, bc):
    rng = np.random.default_rng(9)
    g = Grid((n, n), (1.0, 1.0), bc=bc, faces=[tanh_faces(n, m), tanh_faces(n, m)])
    X, Y = np.meshgrid(_centres(g, 0), _centres(g, 1))
    T = 1.0 + 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.6) ** 2) / 0.05) + 1e-3 * rng.standard_normal(g.shape)
    s = np.sin(np.pi * X) ** 2 * np.sin(np.pi * Y) ** 2
    v = [0.1 * s * np.cos(np.pi * Y), -0.1 * s * np.cos(np.pi * X)]
    return g, T, v


def test_stretched_projection_gives_discrete_continuity():
    """After each stage's projection on a stretched walled box (tanh, m = 2,
    gravity and isothermal walls), delta_1 F / delta_1 x + d_t rho equals
    the solve's constant lam in every cell (Eq 3.24 with the compatibility
    residue of section 3.3) to solver precision."""
    n = 24
    g, T, v = _box(n, 2.0, (("noslip", "noslip"), ("noslip", "noslip")))
    g.bnd[(0, 0)] = {"H": 1.0 + 1.2 / 0.6}
    g.bnd[(0, 1)] = {"H": 1.0 + 0.6 / 0.6}
    o = Oracle(g, Params(Re=50.0, Pr=0.71, inv_Fr2=2.0, qs=0.6, cfl=0.2))
    st = o.initial_state(T, v)
    for _ in range(3):
        rho_n = st.rho
        nxt = o.step(st)
        drho = (nxt.rho - rho_n) / o.dt if st.rho_prev is None else \
            (3.0 * nxt.rho - 4.0 * rho_n + st.rho_prev) / (2.0 * o.dt)
        div = sum((g.plus(nxt.F[d], d) - g.minus(nxt.F[d], d)) / g.along(d, g.wid[d][1:-1]) for d in range(2))
        res = div + drho
        lam = o.stats["corr_compat"]
        assert np.max(np.abs(res - lam)) < 1e-9 * np.max(np.abs(drho)), np.max(np.abs(res - lam))
        st = nxt


def test_uniform_faces_reproduce_the_uniform_grid():
    """Face coordinates given explicitly for a uniform spacing reproduce the
    uniform grid's step (walls, gravity) to rounding."""
    n = 20
    bc = (("noslip", "noslip"), ("slip", "slip"))
    gu = Grid((n, n), (1.0, 1.0), bc=bc)
    gs = Grid((n, n), (1.0, 1.0), bc=bc, faces=[np.arange(n + 1) / n, np.arange(n + 1) / n])
    rng = np.random.default_rng(4)
    T = 1.0 + 0.2 * rng.random((n, n))
    v = [0.05 * rng.standard_normal((n, n)), 0.05 * rng.standard_normal((n, n))]
    out = []
    for g in (gu, gs):
        o = Oracle(g, Params(Re=30.0, inv_Fr2=1.0, cfl=0.2))
        st = o.initial_state(T, v)
        for _ in range(3):
            st = o.step(st)
        out.append(st)
    a, b = out
    assert np.max(np.abs(a.T - b.T)) < 1e-12
    assert max(np.max(np.abs(x - y)) for x, y in zip(a.v, b.v)) < 1e-12
    assert np.max(np.abs((a.P - a.P.mean()) - (b.P - b.P.mean()))) < 1e-12


def test_extrapolation_weights_are_exact_for_quadratics():
    """Eq 3.28 on a stretched wall side: the weights that fill the mirrored
    ghost (P at walls, outflow fields) and those that carry a cell field to
    the boundary face reproduce any quadratic in x exactly, at both sides."""
    from oracle.grid import ghost_extrap_coeffs, face_extrap_coeffs
    n = 12
    g = Grid((n, 4), (1.0, 1.0), bc=(("noslip", "outflow"), ("periodic", "periodic")),
             faces=[tanh_faces(n, 5.0), None])
    f = g.faces[0]
    xc = 0.5 * (f[:-1] + f[1:])
    q = lambda x: 1.3 - 2.0 * x + 4.5 * x * x
    for side in (0, 1):
        A, B, C = ghost_extrap_coeffs(g, 0, side)
        cells = (xc[0], xc[1], xc[2]) if side == 0 else (xc[-1], xc[-2], xc[-3])
        wall = f[0] if side == 0 else f[-1]
        ghost = 2.0 * wall - cells[0]                     # mirrored centre
        assert abs(A * q(cells[0]) + B * q(cells[1]) + C * q(cells[2]) - q(ghost)) < 1e-12
        A, B, C = face_extrap_coeffs(g, 0, side)
        assert abs(A * q(cells[0]) + B * q(cells[1]) + C * q(cells[2]) - q(wall)) < 1e-12
    gu = Grid((n, 4), (1.0, 1.0), bc=g.bc)
    assert ghost_extrap_coeffs(gu, 0, 0) == (3.0, -3.0, 1.0)
    assert face_extrap_coeffs(gu, 0, 1) == (15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0)
