"""Edge cases on the GPU: the smallest grid, a vanishing right-hand side,
calls out of order, the largest 2D size tested and a non-cubic fused 3D
grid, each against the FP64 oracle where a field is produced."""
import math

import numpy as np
import pytest

from oracle import Grid, PoissonSolver
from workloads import Case, c2_case, fourier_temperature, solenoidal_velocity
from _cases import oracle_for, gpu_for, compare

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(errs, tol=TOL):
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"fields above {tol:g}: {bad} (all: {errs})"


def _periodic_case(n, seed, kmax=2, Re=100.0, m=32):
    nd = len(n)
    L = tuple(2 * math.pi for _ in range(nd))
    rng = np.random.default_rng(seed)
    T = fourier_temperature(n, L, rng, kmax, 2.0, m=m)
    v = solenoidal_velocity(n, L, rng, kmax, 0.1, m=m)
    return Case("edge", nd, tuple(n) + (1,) * (3 - nd), L + (1.0,) * (3 - nd),
                (("periodic", "periodic"),) * nd, dict(Re=Re, Pr=0.7, cfl=0.3), T, v)


def test_smallest_grid_4x4():
    """4 x 4 cells: a single multigrid level, solved by the dense
    pseudo-inverse inside the coarse block."""
    case = _periodic_case((4, 4), 21, kmax=1, m=4)
    print("4x4", flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 3)
    s = gpu_for(case)
    s.step(3)
    _check(compare(st, s.get(device=False)))


def test_zero_right_hand_side_gives_zero_pressure():
    from paper_2603_01727_amd import Solver
    s = Solver((64, 32), (2.0, 1.0), Re=10.0, dt=1e-3, poisson_rtol=1e-12)
    P, info = s.project(np.zeros((32, 64)))
    assert np.all(P == 0.0) and info["mean_b"] == 0.0
    # a constant right-hand side is all mean: removed, zero pressure
    P, info = s.project(np.full((32, 64), 3.5))
    assert np.max(np.abs(P)) == 0.0 and abs(info["mean_b"] - 3.5) < 1e-15


def test_calls_out_of_order_are_errors():
    from paper_2603_01727_amd import Solver, LowMachError
    from paper_2603_01727_amd import lib
    s = Solver((32, 32), (1.0, 1.0), Re=10.0, dt=1e-3)
    with pytest.raises(LowMachError) as e:
        s.step(1)                       # no state yet
    assert e.value.status == lib.LM_ESTATE
    with pytest.raises(LowMachError) as e:
        s.get(("rho",))
    assert e.value.status == lib.LM_ESTATE
    s.set(T=np.full((32, 32), 1.5), v=[np.zeros((32, 32)), np.zeros((32, 32))])
    st = s.step(0)                      # zero steps: nothing changes
    assert st["steps"] == 0
    with pytest.raises(LowMachError) as e:
        s.adjoint_seed_ke()             # adjoint arrays not reserved
    assert e.value.status == lib.LM_EUNSUPPORTED


def test_largest_2d_size_4096():
    """4096^2 (16.8M cells, six tiled multigrid levels above the coarse block),
    one step against the oracle."""
    case = c2_case(n=4096)
    print("4096^2", flush=True)
    o, st = oracle_for(case)
    st1 = o.step(st)
    s = gpu_for(case)
    s.step(1)
    errs = compare(st1, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


def test_noncubic_fused_3d():
    """256 x 128 x 64 (2^21 cells: the finest level runs the fused 3D
    kernels with 8-plane chunks), two steps against the oracle."""
    case = _periodic_case((256, 128, 64), 22, kmax=4, Re=300.0)
    case.L = (4 * math.pi, 2 * math.pi, math.pi)
    rng = np.random.default_rng(22)
    case.T = fourier_temperature((256, 128, 64), case.L, rng, 4, 3.0)
    case.v = solenoidal_velocity((256, 128, 64), case.L, rng, 4, 0.1)
    print("256x128x64", flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 2)
    s = gpu_for(case)
    s.step(2)
    errs = compare(st, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


def _reacting_3d_case(n, seed=23):
    """Periodic 3D flame-sheet box: smooth mixture fraction across the
    stoichiometric value (Z in [0, 3], the sheet at Z = 1), H near its
    uniform value, unequal Lewis numbers (the Z diffusion, its H coupling
    and T(Z, H) all in play)."""
    from workloads.ics import QS_C3
    L = (2 * math.pi,) * 3
    rng = np.random.default_rng(seed)
    S = 1.0 / 0.055 - 1.0
    w = fourier_temperature(n, L, rng, 2, 1.0, m=16)        # in [1, 2]
    Z = 3.0 * (w - w.min()) / (w.max() - w.min())
    H = 1.0 / QS_C3 + 1.0 + 0.02 * (fourier_temperature(n, L, rng, 2, 1.0, m=16) - 1.5)
    v = solenoidal_velocity(n, L, rng, 2, 0.1, m=16)
    params = dict(Re=150.0, Pr=0.7, Le_F=1.3, Le_O=0.9, reacting=1, S=S, qs=QS_C3, eps=0.5, tol=1e-3,
                  p0=1.0, dt=0.02)
    case = Case("react3d", 3, tuple(n), L, (("periodic", "periodic"),) * 3, params, None, v, Z=Z)
    case.H = H
    return case


@pytest.mark.parametrize("n", [(64, 8, 16), (24, 12, 10)])
def test_reacting_3d_matches_oracle(n):
    """The 3D stage with the flame sheet (Z diffusion at unequal Lewis
    numbers, its H coupling, T(Z, H))."""
    case = _reacting_3d_case(n)
    print("reacting 3d", n, flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 3)
    s = gpu_for(case)
    s.step(3)
    errs = compare(st, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)
