"""Oracle pins for the pressure Poisson problem (section 3.3, Eq 3.24)."""
import math

import numpy as np

from oracle import Grid, PoissonSolver, beta_inv_rho, laplacian
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


# ---------------------------------------------------------------------------
# Variable-coefficient form div(grad P / rho): beta = 1 / (face mean of rho)
# ---------------------------------------------------------------------------

def test_beta_inv_rho_constant_density_scales_the_fft_solution():
    """rho = c everywhere: A_beta = A / c, so P = c P_1 with P_1 the FFT
    solution of the constant-coefficient problem (independent solve)."""
    rng = np.random.default_rng(3)
    g = Grid((24, 16), (2 * math.pi, 1.5))
    b = rng.standard_normal(g.shape)
    P1, _ = PoissonSolver(g).solve(b)
    c = 2.75
    Pc, _ = PoissonSolver(g, beta_inv_rho(g, np.full(g.shape, c))).solve(b)
    assert np.max(np.abs(Pc - c * P1)) < 1e-11 * np.max(np.abs(c * P1))


def _separable_case(g, rho_axis_d, mode_d, k, periodic):
    """rho varies only along rho_axis_d, P only along mode_d != rho_axis_d:
    then no flux crosses faces normal to rho_axis_d, the faces normal to
    mode_d carry beta = 1/rho of their column, and A_beta P = lam_k P / rho
    with lam_k the 1D eigenvalue of the mode (Fourier or cosine)."""
    rng = np.random.default_rng(11 + rho_axis_d)
    shp = [1] * g.ndim
    shp[g.axis(rho_axis_d)] = g.n[rho_axis_d]
    rho = np.broadcast_to(rng.uniform(0.25, 1.0, g.n[rho_axis_d]).reshape(shp), g.shape).copy()
    n, h = g.n[mode_d], g.h[mode_d]
    i = np.arange(n)
    if periodic:
        m = np.cos(2 * math.pi * k * i / n)
        lam = -(4 / h ** 2) * math.sin(math.pi * k / n) ** 2
    else:
        m = np.cos(math.pi * k * (i + 0.5) / n)
        lam = -(4 / h ** 2) * math.sin(math.pi * k / (2 * n)) ** 2
    shp = [1] * g.ndim
    shp[g.axis(mode_d)] = n
    P = np.broadcast_to(m.reshape(shp), g.shape).copy()
    return rho, P, lam * P / rho


def test_beta_inv_rho_separable_closed_form():
    """Exact solutions of the discrete variable-coefficient problem: a mode
    along one direction with the density varying (arbitrarily) along
    another, periodic and zero-flux sides, 2D both ways round and 3D."""
    cases = [
        (Grid((20, 16), (2 * math.pi, 2.0)), 0, 1, 3, True),
        (Grid((20, 16), (2 * math.pi, 2.0)), 1, 0, 4, True),
        (Grid((12, 18), (1.0, 1.5), bc=(("slip", "slip"), ("noslip", "outflow"))), 0, 1, 5, False),
        (Grid((12, 18), (1.0, 1.5), bc=(("slip", "slip"), ("noslip", "outflow"))), 1, 0, 2, False),
        (Grid((8, 10, 12), (1.0, 2.0, 3.0)), 1, 2, 2, True),
    ]
    for g, da, dm, k, per in cases:
        rho, P, b = _separable_case(g, da, dm, k, per)
        beta = beta_inv_rho(g, rho)
        assert np.max(np.abs(laplacian(g, P, beta) - b)) < 1e-10 * np.max(np.abs(b))
        Ps, _ = PoissonSolver(g, beta).solve(b)
        assert np.max(np.abs(Ps - (P - P.mean()))) < 1e-9, (g.n, da, dm)


def test_beta_inv_rho_conserves_and_is_symmetric():
    """sum over cells of A_beta P is zero (fluxes telescope, zero-flux
    sides), and <A_beta u, w> = <u, A_beta w>."""
    rng = np.random.default_rng(5)
    for g in (Grid((16, 12), (1.0, 1.0)),
              Grid((10, 14), (1.0, 2.0), bc=(("slip", "slip"), ("inflow", "outflow"))),
              Grid((6, 8, 10), (1.0, 1.0, 1.0), bc=(("periodic", "periodic"), ("slip", "slip"),
                                                    ("noslip", "noslip")))):
        rho = rng.uniform(0.2, 1.5, g.shape)
        beta = beta_inv_rho(g, rho)
        u, w = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
        Au, Aw = laplacian(g, u, beta), laplacian(g, w, beta)
        assert abs(Au.sum()) < 1e-11 * np.abs(Au).sum()
        assert abs((Au * w).sum() - (u * Aw).sum()) < 1e-11 * np.abs(Au * w).sum()


def test_beta_inv_rho_manufactured_second_order():
    """The same manufactured problem as above with beta from the cell
    density by face averaging (what a solver given only rho uses):
    still O(h^2)."""
    errs = []
    for n in (16, 32, 64):
        g = Grid((n, n), (2 * math.pi, 2 * math.pi))
        x, y = cell_centres(g.n, g.L)
        rho = 2 + np.sin(x + y)
        Pex = np.cos(x) * np.sin(2 * y)
        bx = -np.cos(x + y) / rho ** 2
        b = (bx * (-np.sin(x) * np.sin(2 * y)) + (-np.cos(x) * np.sin(2 * y)) / rho
             + bx * (2 * np.cos(x) * np.cos(2 * y)) + (-4 * np.cos(x) * np.sin(2 * y)) / rho)
        P, _ = PoissonSolver(g, beta_inv_rho(g, rho)).solve(b)
        errs.append(math.sqrt(np.mean((P - (Pex - Pex.mean())) ** 2)))
    for a, c in zip(errs, errs[1:]):
        assert abs(math.log(a / c, 2) - 2) < 0.15, errs


def test_transform_solve_matches_augmented_matrix():
    """With beta = 1 the oracle solves by transforms (Fourier along
    periodic directions, DCT-II along zero-flux ones, section 3.3's
    zero-mean solution); the sparse LU of the augmented matrix
    [A 1; 1^T 0] gives the same P and lam = mean(b), on every mix of
    periodic and zero-flux sides, odd sizes included."""
    cases = [((16, 20), (("slip", "slip"), ("inflow", "outflow"))),
             ((12, 10), (("periodic", "periodic"), ("noslip", "noslip"))),
             ((9, 12), (("slip", "noslip"), ("periodic", "periodic"))),
             ((8, 6, 10), (("periodic", "periodic"), ("slip", "slip"), ("periodic", "periodic"))),
             ((7, 6, 5), (("slip", "slip"), ("outflow", "inflow"), ("noslip", "noslip"))),
             ((9, 7), None)]
    for n, bc in cases:
        g = Grid(n, (1.0, 1.3, 0.7)[:len(n)], bc=bc)
        b = np.random.default_rng(len(n) + n[0]).standard_normal(g.shape) + 0.3
        P, lam = PoissonSolver(g).solve(b)
        assert PoissonSolver(g).transform
        Pl, laml = PoissonSolver(g, method="lu").solve(b)
        assert abs(lam - laml) < 1e-13
        assert np.max(np.abs(P - Pl)) < 1e-13 * np.max(np.abs(Pl)), (n, bc)
        r = laplacian(g, P) - (b - b.mean())
        assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(b))


def test_transform_solve_on_zero_flux_cosine_mode():
    """A single cosine mode of the DCT-II on a box with zero-flux sides
    in x and periodic y is returned divided by its eigenvalue (the
    closed form of the Neumann eigenpair pinned above); a wrong
    eigenvalue (the periodic sin^2(pi m / n) along x) misses by O(1)."""
    g = Grid((24, 16), (1.0, 2.0), bc=(("slip", "outflow"), ("periodic", "periodic")))
    i = np.arange(24)
    j = np.arange(16)
    m, k = 5, 3
    u = np.cos(math.pi * m * (i[None, :] + 0.5) / 24) * np.cos(2 * math.pi * k * (j[:, None] + 0.5) / 16)
    lam = -(4 / g.h[0] ** 2) * math.sin(math.pi * m / 48) ** 2 - (4 / g.h[1] ** 2) * math.sin(math.pi * k / 16) ** 2
    P, mb = PoissonSolver(g).solve(u)
    assert abs(mb) < 1e-15
    assert np.max(np.abs(P - u / lam)) < 1e-13 * np.max(np.abs(u / lam))
    lam_wrong = -(4 / g.h[0] ** 2) * math.sin(math.pi * m / 24) ** 2 - (4 / g.h[1] ** 2) * math.sin(math.pi * k / 16) ** 2
    assert np.max(np.abs(P - u / lam_wrong)) > 0.1 * np.max(np.abs(u / lam))
