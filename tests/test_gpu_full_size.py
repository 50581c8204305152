"""GPU parity at the workloads' full sizes and lengths: every field of the
HIP step against the FP64 oracle (exact transform Poisson solves) on the
same seeded inputs. Bar: relative L2 <= 1e-10 per field, the GPU Poisson
solves converged to 1e-13 (1e-12 on the slot flame: at 768 x 1536 with
walls, 1e-13 sits on the rounding floor of the CG recurrence, where even
the FP64 solve at times stalls for a dozen extra iterations); the
mixed-precision runs (FP32 V-cycle inside the FP64 single-reduction CG) are
held to the same bar.

 - 768 x 1536 slot flame: 3 steps (immersed burner with the fuel mass
   source, inflow with a solid footprint, slip sides, outflow closure,
   regularised flame sheet), FP64 and mixed;
 - 1024^2 random-mode box: after 1 step and after all 100 steps;
 - 256^3 random-mode box: after 1 and after 3 steps, FP64 and mixed.
After the first step the solves start from the previous pressure, and P
is held to the bound of the solver's stopping rule, kappa(A) rtol (see
warm_start_bound_P); every other field keeps the 1e-10 bar."""
import pytest

from workloads import c2_case, c3_case, c4_case
from _cases import oracle_for, gpu_for, compare

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(errs, tol=TOL, tol_P=None):
    tols = {k: (tol_P if (k == "P" and tol_P is not None) else tol) for k in errs}
    bad = {k: v for k, v in errs.items() if not (v <= tols[k])}
    assert not bad, f"fields above {tol:g} (P: {tols.get('P'):g}): {bad} (all: {errs})"


def periodic_condition_number(n, ndim):
    """kappa of the compact Laplacian on a periodic grid of n cells per
    direction (all directions alike): the largest eigenvalue, sin^2 = 1 in
    every direction, over the smallest non-zero one, one direction at the
    lowest mode: ndim / sin^2(pi / n)."""
    import math
    return ndim / math.sin(math.pi / n) ** 2


def warm_start_bound_P(n, ndim, rtol):
    """After steps whose solves start from the previous pressure, the
    solver controls the residual, ||b - A P|| <= rtol ||b||; the pressure
    itself is then known to kappa(A) rtol (relative), the bound of the
    stopping rule. The fields the step carries forward (velocity, face
    flux, density) see only delta P and stay at the 1e-10 bar."""
    return periodic_condition_number(n, ndim) * rtol


def _trajectory(case, marks):
    """Oracle states after each step count in ``marks``."""
    o, st = oracle_for(case)
    out = {}
    done = 0
    for m in sorted(marks):
        st = o.run(st, m - done)
        done = m
        out[m] = st
    return o, out


@pytest.fixture(scope="module")
def c3_oracle():
    print("oracle: slot flame 768x1536, 3 steps", flush=True)
    return _trajectory(c3_case(), (3,))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slot_flame_full_size_three_steps(c3_oracle, precision):
    o, traj = c3_oracle
    case = c3_case()
    print("slot flame 768x1536", precision, flush=True)
    s = gpu_for(case, rtol=1e-12, precision=precision)
    assert abs(s.dt / o.dt - 1) < 1e-13
    s.step(3)
    errs = compare(traj[3], s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)


@pytest.fixture(scope="module")
def c2_oracle():
    print("oracle: random modes 1024^2, 100 steps", flush=True)
    return _trajectory(c2_case(), (1, 100))


@pytest.mark.timeout(400)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_full_size_hundred_steps(c2_oracle, precision):
    """All 100 steps of the 1024^2 workload; also compared after the first
    (the Heun start)."""
    o, traj = c2_oracle
    case = c2_case()
    print("c2 1024^2", precision, flush=True)
    s = gpu_for(case, precision=precision)
    s.step(1)
    e1 = compare(traj[1], s.get(device=False))
    print("after 1 step", e1, s.stats, flush=True)
    _check(e1)
    s.step(99)
    e100 = compare(traj[100], s.get(device=False))
    bound = warm_start_bound_P(1024, 2, 1e-13)
    print("after 100 steps", e100, "P bound", bound, s.stats, flush=True)
    _check(e100, tol_P=bound)


@pytest.fixture(scope="module")
def c4_oracle():
    print("oracle: random modes 256^3, 3 steps", flush=True)
    return _trajectory(c4_case(), (1, 3))


@pytest.mark.timeout(400)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c4_full_size_three_steps(c4_oracle, precision):
    """256^3: the Heun start and two AB2/AM2 steps with BDF2 density
    derivatives, through the fused 3D multigrid levels."""
    o, traj = c4_oracle
    case = c4_case()
    print("c4 256^3", precision, flush=True)
    s = gpu_for(case, precision=precision)
    s.step(1)
    e1 = compare(traj[1], s.get(device=False))
    print("after 1 step", e1, s.stats, flush=True)
    _check(e1)
    s.step(2)
    e3 = compare(traj[3], s.get(device=False))
    bound = warm_start_bound_P(256, 3, 1e-13)
    print("after 3 steps", e3, "P bound", bound, s.stats, flush=True)
    _check(e3, tol_P=bound)
