"""Oracle pins for the pressure Poisson problem (section 3.3, Eq 3.24)."""
import math

import numpy as np

from oracle import Grid, PoissonSolver, laplacian
from workloads import cell_centres


def test_laplacian_on_fourier_mode_matches_trig_identity():
    """cos(k(x+h)) + cos(k(x-h)) - 2 cos(kx) = -4 sin^2(kh/2) cos(kx)."""
    g = Grid((24, 18), (2 * math.pi, 3.0))
    x, y = cell_centres(g.n, g.L)
    kx, ky = 3 * 2 * math.pi / g.L[0], 2 * 2 * math.pi / g.L[1]
    u = np.cos(kx * x + ky * y) + 0 * x * y
    lam = -(4 / g.h[0] ** 2) * math.sin(kx * g.h[0] / 2) ** 2 \
          - (4 / g.h[1] ** 2) * math.sin(ky * g.h[1] / 2) ** 2
    assert np.max(np.abs(laplacian(g, u) - lam * u)) < 1e-11 * abs(lam)


def test_neumann_laplacian_on_cosine_mode():
    """Cell-centred zero-flux Laplacian: cos(pi m (i+1/2)/n) is an
    eigenvector with eigenvalue -(4/h^2) sin^2(pi m/(2n)) (DCT-II)."""
    g = Grid((20, 12), (1.0, 0.6), bc=(("slip", "slip"), ("noslip", "outflow")))
    i = np.arange(20)
    j = np.arange(12)
    u = np.cos(math.pi * 3 * (i[None, :] + 0.5) / 20) * np.cos(math.pi * 5 * (j[:, None] + 0.5) / 12)
    lam = -(4 / g.h[0] ** 2) * math.sin(math.pi * 3 / 40) ** 2 \
          - (4 / g.h[1] ** 2) * math.sin(math.pi * 5 / 24) ** 2
    assert np.max(np.abs(laplacian(g, u) - lam * u)) < 1e-10 * abs(lam)


def _check_solution(g, beta=None, seed=0):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(g.shape) + 0.3
    P, lam = PoissonSolver(g, beta).solve(b)
    assert abs(lam - b.mean()) < 1e-14
    assert abs(P.mean()) < 1e-12 * np.max(np.abs(P))
    r = laplacian(g, P, beta) - (b - b.mean())
    assert np.max(np.abs(r)) < 1e-9 * np.max(np.abs(b))


def test_fft_solution_satisfies_difference_equation():
    _check_solution(Grid((32, 16), (2 * math.pi, 1.0)))
    _check_solution(Grid((8, 12, 10), (1.0, 2.0, 3.0)))


def test_augmented_solution_satisfies_difference_equation():
    _check_solution(Grid((16, 20), (1.0, 1.25), bc=(("slip", "slip"), ("inflow", "outflow"))))
    _check_solution(Grid((12, 10), (1.0, 1.0), bc=(("periodic", "periodic"), ("noslip", "noslip"))))


def _beta_faces(g, fn):
    out = []
    for d in range(g.ndim):
        cs = cell_centres(g.n, g.L)
        fc = list(cs)
        h = g.h[d]
        f = np.arange(g.n[d] + 1) * h
        shp = [1] * g.ndim
        shp[g.axis(d)] = g.n[d] + 1
        fc[d] = f.reshape(shp)
        out.append(np.broadcast_to(fn(*fc), tuple(g.n[d] + 1 if a == g.axis(d) else g.shape[a]
                                                  for a in range(g.ndim))).copy())
    return out


def test_variable_coefficient_manufactured_second_order():
    """div(beta grad P) = b with beta = 1/rho(x): P = cos x sin 2y,
    rho = 2 + sin(x + y); error in P is O(h^2)."""
    errs = []
    for n in (16, 32, 64):
        g = Grid((n, n), (2 * math.pi, 2 * math.pi))
        x, y = cell_centres(g.n, g.L)
        rho = lambda x, y: 2 + np.sin(x + y)
        Pex = np.cos(x) * np.sin(2 * y)
        # b = d/dx(beta P_x) + d/dy(beta P_y), beta = 1/rho
        beta = 1 / rho(x, y)
        bx = -np.cos(x + y) / rho(x, y) ** 2          # d beta/dx = d beta/dy
        Px = -np.sin(x) * np.sin(2 * y)
        Py = 2 * np.cos(x) * np.cos(2 * y)
        Pxx = -np.cos(x) * np.sin(2 * y)
        Pyy = -4 * np.cos(x) * np.sin(2 * y)
        b = bx * Px + beta * Pxx + bx * Py + beta * Pyy
        bf = _beta_faces(g, lambda X, Y: 1 / rho(X, Y))
        P, _ = PoissonSolver(g, bf).solve(b)
        errs.append(math.sqrt(np.mean((P - (Pex - Pex.mean())) ** 2)))
    for a, c in zip(errs, errs[1:]):
        assert abs(math.log(a / c, 2) - 2) < 0.15, errs
