"""The C-ABI library loads and exports every symbol that include/lowmach.h
declares; argument checks that need no GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lowmach.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("lm_workspace_size", "lm_init_grid", "lm_set_fields", "lm_step", "lm_project",
                 "lm_get_fields", "lm_destroy", "lm_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2603_01727_amd import lib
    L = lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(lib.EXPORTS) == set(declared_functions())


def _grid_params(n=(64, 64), bc=None):
    from paper_2603_01727_amd import lib
    g = lib.lm_grid()
    g.ndim = len(n)
    for d in range(3):
        g.n[d] = n[d] if d < len(n) else 1
        g.L[d] = 1.0
        for s in range(2):
            g.bc[d][s] = 0 if bc is None else bc[d][s]
    p = lib.lm_params(Re=100.0, Pr=0.7, sigma=0.7, qs=1.0, S=1.0, eps=0.5, tol=1e-3, Le_F=1.0, Le_O=1.0,
                      p0=1.0, cfl=0.2, poisson_rtol=1e-10, poisson_maxit=100, mg_nu=2)
    return g, p


def test_workspace_size_scales_with_grid():
    from paper_2603_01727_amd import lib
    L = lib.load()
    sizes = []
    for n in ((64, 64), (128, 128), (32, 32, 32)):
        g, p = _grid_params(n)
        b = C.c_size_t()
        assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
        sizes.append(b.value)
    assert sizes[1] > 3.0 * sizes[0]
    # FP64 state: at least ~30 padded arrays of 8 bytes per cell
    assert sizes[0] > 30 * 64 * 64 * 8


def test_invalid_arguments_rejected_without_gpu():
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    g, p = _grid_params((64, 64))
    g.ndim = 4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    g, p = _grid_params((64, 64), bc=[(0, 1), (0, 0), (0, 0)])   # broken periodic pair
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    g, p = _grid_params((64, 64))
    p.poisson_rtol = 0.0
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    g, p = _grid_params((250, 250))   # coarsens to 125^2 > 1024 cells
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    ctx = C.c_void_p()
    g, p = _grid_params((64, 64))
    assert L.lm_init_grid(C.byref(g), C.byref(p), None, 0, None, C.byref(ctx)) == lib.LM_EINVAL


def test_degenerate_grids_and_params_rejected():
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    for n in ((2, 8), (0, 16), (8, 3)):
        g, p = _grid_params(n)
        assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL, n
        assert L.lm_last_error(None).decode()  # the reason is reported without a context
    g, p = _grid_params((64, 64))
    p.precision = 3
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    g, p = _grid_params((64, 64))
    p.with_adjoint = 1
    p.precision = lib.LM_MIXED          # the adjoint is FP64 only
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    g, p = _grid_params((64, 64))
    p.with_adjoint, p.reacting = 1, 1   # reacting flow has an adjoint
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    g, p = _grid_params((4, 4))       # smallest grid: one level, solved by the dense pseudo-inverse
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK


def test_variable_coefficient_reservation():
    """poisson_beta = LM_BETA_INV_RHO reserves the per-level densities and
    the coarsest inverse (more workspace), and needs a grid that coarsens
    to <= 128 cells; other values are rejected."""
    from paper_2603_01727_amd import lib
    L = lib.load()
    b0, b1 = C.c_size_t(), C.c_size_t()
    g, p = _grid_params((128, 96))
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b0)) == lib.LM_OK
    p.poisson_beta = lib.LM_BETA_INV_RHO
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b1)) == lib.LM_OK
    assert b1.value > b0.value + 128 * 96 * 8
    g, p = _grid_params((100, 60))    # coarsens to 25 x 15 = 375 cells
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b0)) == lib.LM_OK
    p.poisson_beta = lib.LM_BETA_INV_RHO
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b0)) == lib.LM_EUNSUPPORTED
    assert "128" in L.lm_last_error(None).decode()
    g, p = _grid_params((64, 64))
    p.poisson_beta = 2
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b0)) == lib.LM_EINVAL


def test_enclosed_system_checks_without_gpu():
    """p0_closed: gamma must exceed 1; reacting flow, inflow or outflow
    sides are not an enclosed system (reacting flow is a semi-enclosed
    one); the adjoint needs constant p0."""
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    g, p = _grid_params((64, 64))
    p.p0_closed, p.gamma = 1, 1.4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    p.gamma = 1.0
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.gamma, p.reacting = 1.4, 1
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    p.p0_closed = 2                          # Eq 2.38 carries the flame's heat
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    p.with_ib, p.Da_ib = 1, 1e-3             # but not the penalisation's
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    p.with_ib = 0
    p.p0_closed, p.reacting = 1, 0
    g, p = _grid_params((64, 64), bc=[(2, 2), (3, 4), (0, 0)])   # noslip x, inflow / outflow y
    p.p0_closed, p.gamma = 1, 1.4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    g, p = _grid_params((64, 64))
    p.p0_closed, p.gamma, p.with_adjoint = 1, 1.4, 1
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.p0_closed = 2
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL


def test_sutherland_checks_without_gpu():
    """sutherland_C must be >= 0 and finite (the adjoint takes it too)."""
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    g, p = _grid_params((64, 64))
    p.sutherland_C = 110.5 / 600.0
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    p.sutherland_C = -1.0
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.sutherland_C = float("nan")
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.sutherland_C, p.with_adjoint = 0.2, 1
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK


def test_adaptive_step_checks_without_gpu():
    """dt_tol must be >= 0 and finite and needs cfl > 0; not with the
    adjoint (EINVAL); enclosed systems take it."""
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    g, p = _grid_params((64, 64))
    p.dt_tol, p.cfl = 1e-6, 0.3
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    p.dt_tol = -1.0
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.dt_tol, p.cfl, p.dt = 1e-6, 0.0, 1e-3
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.cfl, p.with_adjoint = 0.3, 1
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL
    p.with_adjoint, p.p0_closed, p.gamma = 0, 1, 1.4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK


def test_semi_enclosed_checks_without_gpu():
    """p0_closed = 2 (Eq 2.38) takes inflow sides but no outflow side;
    values beyond 2 are rejected."""
    from paper_2603_01727_amd import lib
    L = lib.load()
    b = C.c_size_t()
    g, p = _grid_params((64, 64), bc=[(3, 2), (0, 0), (0, 0)])   # inflow / no-slip x, periodic y
    p.p0_closed, p.gamma = 2, 1.4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_OK
    p.p0_closed = 1
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    g, p = _grid_params((64, 64), bc=[(3, 4), (0, 0), (0, 0)])   # inflow / outflow
    p.p0_closed, p.gamma = 2, 1.4
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EUNSUPPORTED
    p.p0_closed = 3
    assert L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b)) == lib.LM_EINVAL


def test_stretched_grid_checks_without_gpu():
    """lm_grid.faces: n + 1 strictly increasing values from 0 to L, else
    LM_EINVAL; the stretched path covers 2D without outflow sides, the
    adjoint, a density-weighted pressure or the reacting form of p0, else
    LM_EUNSUPPORTED. A stretched grid reserves more than the uniform one
    (the packed spacing arrays)."""
    import numpy as np
    from paper_2603_01727_amd import lib
    from workloads import tanh_stretched_faces
    L = lib.load()
    b = C.c_size_t()
    f = tanh_stretched_faces(64, 2.0)
    keep = []

    def size(g, p, faces):
        for d in range(3):
            g.faces[d] = None
        for d, a in enumerate(faces):
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                keep.append(a)
                g.faces[d] = a.ctypes.data
        return L.lm_workspace_size(C.byref(g), C.byref(p), C.byref(b))

    walls = [(2, 2), (2, 2), (0, 0)]
    g, p = _grid_params((64, 64), bc=walls)
    assert size(g, p, []) == lib.LM_OK
    uniform = b.value
    assert size(g, p, [f, f]) == lib.LM_OK and b.value > uniform
    assert size(g, p, [None, f]) == lib.LM_OK
    for bad in (f[::-1], f * 1.01, np.concatenate([[0.0, 0.02, 0.01], f[3:]]), f - 1e-3):
        assert size(g, p, [bad, None]) == lib.LM_EINVAL
    g, p = _grid_params((64, 64), bc=[(2, 4), (2, 2), (0, 0)])      # an outflow side
    assert size(g, p, [f, None]) == lib.LM_EUNSUPPORTED
    g, p = _grid_params((64, 64, 64), bc=walls)
    assert size(g, p, [f, None, None]) == lib.LM_EUNSUPPORTED
    g, p = _grid_params((64, 64), bc=walls)
    p.with_adjoint = 1
    assert size(g, p, [f, f]) == lib.LM_EUNSUPPORTED
    p.with_adjoint, p.poisson_beta = 0, lib.LM_BETA_INV_RHO
    assert size(g, p, [f, f]) == lib.LM_EUNSUPPORTED
    g, p = _grid_params((64, 64))
    p.reacting, p.p0_closed, p.gamma = 1, 2, 1.4
    assert size(g, p, [f, f]) == lib.LM_EUNSUPPORTED
    p.p0_closed = 0
    assert size(g, p, [f, f]) == lib.LM_OK
