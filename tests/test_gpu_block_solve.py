"""The one-workgroup pressure solve (grids of at most 4096 cells: the whole
single-reduction MG-PCG in one launch, outcome checked after the step)
against the multi-kernel solve of the same context kinds (LM_BLOCK_PCG=0,
read when a context is created): same solutions to 1e-12, iteration counts
within one (the inner products are summed in another order), the same
step results, and the failure paths (iterations exhausted in lm_project
and inside lm_step, where the check is deferred to the end of the step)."""
import math
import os

import numpy as np
import pytest

from workloads import (c1_case, heated_cavity_case, tanh_stretched_faces, variable_coefficient_problem)
from _cases import gpu_for, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_env(value, make):
    old = os.environ.get("LM_BLOCK_PCG")
    if value is None:
        os.environ.pop("LM_BLOCK_PCG", None)
    else:
        os.environ["LM_BLOCK_PCG"] = value
    try:
        return make()
    finally:
        if old is None:
            os.environ.pop("LM_BLOCK_PCG", None)
        else:
            os.environ["LM_BLOCK_PCG"] = old


# (n, L, bc, faces, density): periodic, walls, outflow, 3D, variable
# density, stretched; the largest has 4096 cells
PROJECT_CASES = [
    ((64, 64), (2 * math.pi, 2 * math.pi), None, None, False),
    ((48, 32), (1.5, 1.0), [("noslip", "noslip"), ("slip", "slip")], None, False),
    ((32, 64), (1.0, 2.0), [("periodic", "periodic"), ("inflow", "outflow")], None, False),
    ((16, 16, 16), (2 * math.pi,) * 3, None, None, False),
    ((16, 8, 12), (1.0, 0.5, 0.75), [("noslip", "noslip"), ("periodic", "periodic"), ("slip", "slip")], None, False),
    ((64, 32), (2.0, 1.0), None, None, True),
    ((16, 16, 8), (1.0, 1.0, 0.5), [("noslip", "noslip"), ("slip", "slip"), ("periodic", "periodic")], None, True),
    ((64, 48), (1.5, 1.0), [("noslip", "noslip"), ("slip", "slip")], "tanh", False),
]


def _pid(c):
    return "x".join(map(str, c[0])) + ("-walls" if c[2] else "") + ("-rho" if c[4] else "") + ("-str" if c[3] else "")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", PROJECT_CASES, ids=[_pid(c) for c in PROJECT_CASES])
def test_block_solve_matches_multi_kernel_solve(case, precision):
    from paper_2603_01727_amd import Solver
    n, L, bc, faces, dens = case
    if faces == "tanh":
        faces = [tanh_stretched_faces(n[0], 3.0, L[0]), tanh_stretched_faces(n[1], 2.0, L[1])]
    rho, b = variable_coefficient_problem(n, L, seed=13 + len(n), kmax=4)
    print("block solve", n, bc, precision, "density" if dens else "", "stretched" if faces else "", flush=True)

    def make():
        return Solver(n, L, bc=bc, Re=10.0, dt=1e-3, precision=precision, poisson_rtol=1e-13, poisson_maxit=300,
                      variable_coefficient=dens, faces=faces)

    out = []
    for env in (None, "0"):
        s = _with_env(env, make)
        P, info = s.project(b, rho=rho if dens else None)
        out.append((P, info))
        s.close()
    (P1, i1), (P0, i0) = out
    print(i1, i0, rel_l2(P1, P0), flush=True)
    assert i1["relres"] <= 1e-13 and i0["relres"] <= 1e-13
    assert abs(i1["iters"] - i0["iters"]) <= 1, (i1, i0)
    assert abs(i1["mean_b"] - i0["mean_b"]) <= 1e-14 * max(1.0, abs(i0["mean_b"]))
    assert rel_l2(P1, P0) <= 1e-12


@pytest.mark.parametrize("which", ["c1", "cavity", "stretched"])
def test_block_solve_steps_match_multi_kernel_steps(which):
    if which == "c1":
        case = c1_case(n=64)
    else:
        case = heated_cavity_case(n=32, m=2.0 if which == "stretched" else 1.0)
    print("block steps", which, flush=True)
    fields, stats = [], []
    for env in (None, "0"):
        s = _with_env(env, lambda: gpu_for(case))
        st = s.step(5)
        fields.append(s.get(device=False))
        stats.append(st)
        s.close()
    (a, b) = fields
    for k in ("rho", "H", "T", "P"):
        assert rel_l2(a[k], b[k]) <= 1e-12, k
    for d in range(2):
        assert rel_l2(a["v"][d], b["v"][d]) <= 1e-12
        assert rel_l2(a["F"][d], b["F"][d]) <= 1e-12
    s1, s0 = stats
    assert abs(s1["p0"] - s0["p0"]) <= 1e-14
    for q in range(2):
        assert abs(s1["poisson_iters"][q] - s0["poisson_iters"][q]) <= 1
        assert s1["poisson_relres"][q] <= 1e-13
        assert abs(s1["compat"][q] - s0["compat"][q]) <= 1e-13
    assert abs(s1["total_poisson_iters"] - s0["total_poisson_iters"]) <= 10


def test_block_solve_out_of_iterations():
    """maxit too small for the tolerance: lm_project and lm_step report
    LM_ENOCONV; the failed step leaves the state at n untouched."""
    from paper_2603_01727_amd import LowMachError, Solver, lib
    n, L = (64, 64), (2 * math.pi, 2 * math.pi)
    _, b = variable_coefficient_problem(n, L, seed=3)
    s = Solver(n, L, Re=10.0, dt=1e-3, poisson_rtol=1e-14, poisson_maxit=2)
    with pytest.raises(LowMachError) as e:
        s.project(b)
    assert e.value.status == lib.LM_ENOCONV
    case = c1_case(n=64)
    s = Solver(case.n[:2], case.L[:2], Re=case.params["Re"], Pr=case.params["Pr"], cfl=case.params["cfl"],
               poisson_rtol=1e-14, poisson_maxit=2)
    s.set(T=case.T, v=case.v)
    g0 = s.get(device=False)
    with pytest.raises(LowMachError) as e:
        s.step(1)
    assert e.value.status == lib.LM_ENOCONV
    g1 = s.get(device=False)
    for k in ("T", "rho", "P"):
        assert np.array_equal(g0[k], g1[k]), k
    assert np.array_equal(g0["v"][0], g1["v"][0]) and np.array_equal(g0["F"][1], g1["F"][1])
    with pytest.raises(LowMachError) as e:       # the same again: still the state at n
        s.step(1)
    assert e.value.status == lib.LM_ENOCONV
