"""lm_project_static, the pressure solve that allocates nothing (its arrays
live in the library's static device buffer), against lm_project, the
same solve on a context and its caller-owned workspace: two calls in a
row on one GPU, the second smaller than the first (the buffer keeps the
first call's contents), in FP64 and mixed precision, from device and host
arrays. Bar: relative L2 <= 1e-10 between the two solutions (both solved
to 1e-13)."""
import math

import numpy as np
import pytest

from _cases import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rhs(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape) + 0.2


CASES = [  # (shape in C order, lengths, sides): larger first
    ((256, 256), (2 * math.pi, 2 * math.pi), None),
    ((48, 96), (2.0, 1.0), [("slip", "outflow"), ("inflow", "noslip")]),
    ((32, 24, 40), (1.0, 0.6, 0.8), [("periodic", "periodic"), ("slip", "slip"), ("periodic", "periodic")]),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_solve_matches_lm_project_twice_shrinking(precision):
    import torch
    from paper_2603_01727_amd import Solver, project_static
    for k, (shape, L, bc) in enumerate(CASES):
        print("project_static", precision, shape, flush=True)
        b = _rhs(shape, 40 + k)
        n = tuple(reversed(shape))
        s = Solver(n, L, bc=bc, Re=1.0, dt=1.0, precision=precision, poisson_rtol=1e-13, poisson_maxit=400)
        Pref, info_ref = s.project(torch.from_numpy(b).cuda())
        s.close()
        bt = torch.from_numpy(b).cuda()
        P = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        info = project_static(bt, L, P, bc=bc, rtol=1e-13, precision=precision)
        torch.cuda.synchronize()
        err = rel_l2(P.cpu().numpy(), Pref.cpu().numpy())
        print(info, info_ref, err, flush=True)
        assert info["relres"] <= 1e-13 and abs(info["mean_b"] - info_ref["mean_b"]) < 1e-13
        assert err <= 1e-10, err
        # host arrays through the same buffer
        Ph = np.full(shape, np.nan)
        project_static(b, L, Ph, bc=bc, rtol=1e-13, precision=precision)
        assert rel_l2(Ph, Pref.cpu().numpy()) <= 1e-10


def test_static_solve_rejects_oversized_and_unsupported_grids():
    from paper_2603_01727_amd import project_static, LowMachError, lib
    with pytest.raises(LowMachError) as e:
        project_static(np.zeros((2048, 2048)), (1.0, 1.0))
    assert e.value.status == lib.LM_ENOMEM and "64 MiB" in str(e.value)
    with pytest.raises(LowMachError) as e:       # coarsest level 5 x 45 cells
        project_static(np.zeros((90, 10)), (1.0, 9.0))
    assert e.value.status == lib.LM_EUNSUPPORTED
