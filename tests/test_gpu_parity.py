"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs. Bar: relative L2 <= 1e-10 per field after the step
in FP64 (Poisson solved to 1e-13 so solver error stays below the bar)."""
import math

import numpy as np
import pytest

from oracle import Grid, Oracle, Params, PoissonSolver
from workloads import c1_case, c2_case, c4_case, c5_case, Case, cell_centres
from _cases import oracle_for, gpu_for, compare, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _check(errs, tol=TOL):
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"fields above {tol:g}: {bad} (all: {errs})"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("shape", [(64, 64), (96, 40), (48, 48, 32)])
def test_project_matches_exact_solution(shape):
    from paper_2603_01727_amd import Solver
    n = tuple(reversed(shape))
    nd = len(n)
    print("project", shape, flush=True)
    s = Solver(n, (2 * math.pi,) * nd, Re=100.0, dt=1e-3, poisson_rtol=1e-13)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(shape) + 0.25
    P, info = s.project(b)
    Pex, lam = PoissonSolver(Grid(n, (2 * math.pi,) * nd)).solve(b)
    assert abs(info["mean_b"] - lam) < 1e-14
    assert rel_l2(P, Pex) < 1e-11, (rel_l2(P, Pex), info)
    assert info["relres"] <= 1e-13


def test_c1_one_step():
    """Hot spot on a Taylor-Green vortex, 64^2, one Heun-start step."""
    case = c1_case()
    print("c1 one step", flush=True)
    o, st = oracle_for(case)
    st1 = o.step(st)
    s = gpu_for(case)
    assert abs(s.dt / o.dt - 1) < 1e-14
    s.step(1)
    errs = compare(st1, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


@pytest.mark.parametrize("n,steps", [(64, 4), (96, 3)])
def test_random_modes_multi_step(n, steps):
    """Random-mode density ratio 4 box (the 1024^2 workload shape at small
    size), several AB2/AM2 steps with BDF2 density derivative."""
    case = c2_case(n=n)
    print("random modes", n, steps, flush=True)
    o, st = oracle_for(case)
    for _ in range(steps):
        st = o.step(st)
    s = gpu_for(case)
    s.step(steps)
    errs = compare(st, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


def test_3d_random_modes():
    case = c4_case(n=24)
    print("3d random modes 24^3", flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 2)
    s = gpu_for(case)
    s.step(2)
    errs = compare(st, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


def test_ragged_sizes():
    """Sizes that are not multiples of the 64 x 4 block (ragged tails)."""
    for n in ((100, 36), (20, 132)):
        L = (2 * math.pi * n[0] / n[1], 2 * math.pi)
        rng = np.random.default_rng(3)
        from workloads import fourier_temperature, solenoidal_velocity
        T = fourier_temperature(n, L, rng, 4, 2.0)
        v = solenoidal_velocity(n, L, rng, 4, 0.2)
        case = Case("ragged", 2, n + (1,), L + (1.0,), (("periodic", "periodic"),) * 2,
                    dict(Re=200.0, Pr=0.7, cfl=0.3), T, v)
        print("ragged", n, flush=True)
        o, st = oracle_for(case)
        st = o.run(st, 2)
        s = gpu_for(case)
        s.step(2)
        errs = compare(st, s.get(device=False))
        _check(errs)


@pytest.mark.parametrize("precision", ["mixed", "mixed-flexible"])
def test_mixed_precision_matches_fp64_oracle(precision):
    """FP32 multigrid inside the FP64 single-reduction CG (mixed) or the FP64
    flexible CG (mixed-flexible) converges to the same FP64 solution: the
    per-field error against the FP64 oracle is stated here."""
    case = c2_case(n=128)
    print(precision, "128", flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 2)
    s = gpu_for(case, precision=precision)
    s.step(2)
    errs = compare(st, s.get(device=False))
    print("mixed-precision errors vs FP64 oracle:", errs, s.stats, flush=True)
    _check(errs)


def test_free_stream_preserved_on_gpu():
    from paper_2603_01727_amd import Solver
    s = Solver((32, 16), (2.0, 1.0), Re=10.0, dt=1e-2, poisson_rtol=1e-12)
    s.set(T=np.full((16, 32), 2.0), v=[np.full((16, 32), 0.3), np.full((16, 32), -0.2)])
    s.step(3)
    g = s.get(device=False)
    assert np.max(np.abs(g["v"][0] - 0.3)) < 1e-14
    assert np.max(np.abs(g["T"] - 2.0)) < 1e-14
    assert np.max(np.abs(g["P"])) < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed-flexible"])
def test_3d_fused_multigrid_128(precision):
    """128^3: the finest multigrid level runs the fused z-marching 3D
    kernels (FP64, or FP32 inside the flexible FP64 CG)."""
    case = c4_case(n=128)
    print("3d 128^3", precision, flush=True)
    o, st = oracle_for(case)
    st = o.run(st, 2)
    s = gpu_for(case, precision=precision)
    s.step(2)
    errs = compare(st, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


def test_taylor_green_spatial_orders_table1():
    """The GPU step on the Taylor-Green vortex (section 4.2, Re = 100, unit
    square) against the closed form: the observed L2 orders of v1 and of
    the interval-averaged pressure (Eq 4.7) between 20, 40, 80, 160 cells
    match Table 1's order rows (tests/golden/tab1_orders.txt); v1 and v2
    errors coincide (the table's notes)."""
    import os
    from paper_2603_01727_amd import Solver
    from workloads import taylor_green
    gold = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "tab1_orders.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            r = [float(x) for x in line.split()]
            gold[(int(r[0]), int(r[1]))] = r
    Re, dt, tend = 100.0, 5e-4, 0.1
    k = int(round(tend / dt))
    a = 16 * math.pi ** 2 / Re
    errs = {}
    for n in (20, 40, 80, 160):
        print("taylor-green", n, flush=True)
        v1, v2, _ = taylor_green((n, n), (1.0, 1.0), 0.0, Re)
        s = Solver((n, n), (1.0, 1.0), Re=Re, Pr=0.7, dt=dt, poisson_rtol=1e-13, poisson_maxit=400)
        s.set(T=np.ones((n, n)), v=[v1, v2])
        s.step(k)
        g = s.get(("v", "P"), device=False)
        e1, e2, pe = taylor_green((n, n), (1.0, 1.0), k * dt, Re)
        pbar = (math.exp(a * dt) - 1) / (a * dt) * pe
        rms = lambda x: math.sqrt(float(np.mean(x ** 2)))
        errs[n] = (rms(g["v"][0] - e1), rms(g["v"][1] - e2), rms(g["P"] / dt - pbar))
    for (c, f) in ((20, 40), (40, 80), (80, 160)):
        ov = math.log(errs[c][0] / errs[f][0]) / math.log(2)
        op = math.log(errs[c][2] / errs[f][2]) / math.log(2)
        print(c, f, ov, op, flush=True)
        assert abs(ov - gold[(c, f)][2]) < 0.05, ov
        assert abs(op - gold[(c, f)][3]) < 0.08, op
        assert abs(errs[f][0] / errs[f][1] - 1) < 1e-6


def _load_golden(name):
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _load_golden("tab2_temporal.txt"), ids=lambda r: f"{int(r[0])}-{r[1]:g}")
def test_taylor_green_table2_on_gpu(row):
    """Table 2 (section 4.2.2) from the GPU step: start from the exact
    vortex at 1.3 - 8 dt, take 8 steps (the first the Heun start), and
    compare the RMS differences between the predicted level (read back as
    LM_LEVEL_PREDICTED) and the corrected one of the last step with the
    printed entries (the round-off-limited entry the paper flags to 6 %)."""
    from paper_2603_01727_amd import Solver
    from workloads import taylor_green
    n, dt, eP, ev1, ev2 = row
    n = int(n)
    v1, v2, _ = taylor_green((n, n), (1.0, 1.0), 1.3 - 8 * dt, 100.0)
    s = Solver((n, n), (1.0, 1.0), Re=100.0, Pr=0.7, dt=dt, poisson_rtol=1e-14, poisson_maxit=400)
    s.set(T=np.ones((n, n)), v=[v1, v2])
    s.step(8)
    a = s.get(("v", "P"), device=False)
    b = s.get(("v", "P"), device=False, predicted=True)
    rms = lambda x: math.sqrt(float(np.mean(x ** 2)))
    d1, d2, dP = rms(b["v"][0] - a["v"][0]), rms(b["v"][1] - a["v"][1]), rms(b["P"] - a["P"])
    flagged = n == 400 and dt < 2e-5
    tol = 0.06 if flagged else 2.5e-3
    print(n, dt, d1 / ev1, dP / eP, flush=True)
    assert abs(d1 / ev1 - 1) < tol, (d1, ev1)
    assert abs(dP / eP - 1) < tol, (dP, eP)
    if not flagged:
        assert abs(d2 / ev2 - 1) < tol


def test_predicted_level_needs_a_step():
    from paper_2603_01727_amd import Solver, LowMachError, lib
    s = Solver((32, 32), (1.0, 1.0), Re=100.0, dt=1e-3)
    s.set(T=np.ones((32, 32)), v=[np.zeros((32, 32))] * 2)
    with pytest.raises(LowMachError) as e:
        s.get(("v",), predicted=True)
    assert e.value.status == lib.LM_ESTATE
