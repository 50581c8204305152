"""GPU parity of the adaptive time step (dt_tol > 0): the step sequence the
controller chooses from the predictor-corrector estimate, and the fields
after each step, against the FP64 oracle (relative L2 <= 1e-10 per field,
Poisson solved to 1e-14); exact restart of an adaptive run."""
import numpy as np
import pytest

from workloads import c1_case, c3_case
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


def _run(case, steps, precision="fp64", tol_P=TOL):
    """Both sides step by step. The controller halves the step several
    times, and P = p dt shrinks with it while the right-hand side does not,
    so the pressure solve is taken to 1e-14 here to keep P's relative
    error below the bar."""
    o, st = oracle_for(case)
    s = gpu_for(case, precision=precision, rtol=1e-14)
    assert abs(s.dt / o.dt - 1) < 1e-13
    changes = 0
    for k in range(steps):
        dt_o = o.dt
        st = o.step(st)
        stats = s.step(1)
        # the estimate is a difference of two levels that agree to ~1e-14:
        # it matches to ~1e-9 relative, and the chosen step to a third of that
        assert abs(stats["dt"] / dt_o - 1) < 1e-8, (k, stats["dt"], dt_o)
        assert abs(stats["pc_err"] / o.stats["pc_err"] - 1) < 1e-7, (k, stats["pc_err"], o.stats["pc_err"])
        assert stats["pc_err_used"] == o.stats["pc_err_clean"]
        assert abs(s.dt / o.dt - 1) < 1e-8, (k, s.dt, o.dt)
        changes += s.dt != stats["dt"]
        errs = compare(st, s.get(device=False))
        print(k, stats["dt"], stats["pc_err"], errs, flush=True)
        _check({q: e for q, e in errs.items() if q != "P"})
        assert errs["P"] <= tol_P, errs
    return changes


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adaptive_hot_spot_matches_oracle(precision):
    """64^2 hot spot (density ratio 5): the estimate exceeds the
    tolerance, so the controller halves the step every fourth step."""
    case = c1_case(n=64)
    case.params = dict(case.params, dt_tol=1e-7)
    print("adaptive hot spot", precision, flush=True)
    assert _run(case, 16, precision) >= 3


def test_adaptive_slot_flame_matches_oracle():
    """Reacting slot flame (inflow, outflow, immersed burner, Z in the
    estimate). The controller takes the step down to a fifth of the
    CFL step here; P = p dt shrinks with it while the right-hand side,
    dominated by the injector's sharp source, does not, and the relative
    error of P left by a solve to relative residual 1e-14 on this
    walled, open grid reaches ~5e-9 in its smoothest modes (the velocities
    and face fluxes, which carry its gradient, stay at ~1e-12): P is held
    to 1e-8."""
    case = c3_case(nx=128, ny=256, W=32, wall=4, wall_h=32, inj=4)
    case.params = dict(case.params, dt_tol=1e-6)
    print("adaptive slot flame", flush=True)
    _run(case, 9, tol_P=1e-8)


def test_adaptive_3d_matches_oracle():
    """24^3 random-mode box (density ratio 6): the controller halves the
    step twice in 12 steps."""
    from workloads import c4_case
    case = c4_case(n=24)
    case.params = dict(case.params, dt_tol=1e-6)
    print("adaptive 3D", flush=True)
    assert _run(case, 12) >= 2


@pytest.mark.parametrize("mode", [1, 2], ids=["enclosed", "semi-enclosed"])
def test_adaptive_closed_systems_match_oracle(mode):
    """Adaptive steps with p0 from the conserved mass (a closed heated box,
    BDF2 of d_t p0 for unequal steps) and from the ODE of Eq 2.38 (gas
    pushed in through an inflow side, AB2 with the step ratio)."""
    if mode == 1:
        from test_gpu_p0 import _heated_box
        case = _heated_box((64, 48), (("periodic", "periodic"), ("noslip", "noslip")))
        case.params = dict(case.params, dt_tol=1e-7)
    else:
        from test_gpu_p0 import _compression_case
        case = _compression_case(profile=True)
        case.params = dict(case.params, dt_tol=1e-8)
    print("adaptive p0 mode", mode, flush=True)
    o, st = oracle_for(case)
    s = gpu_for(case, rtol=1e-14)
    changes = 0
    for k in range(12):
        st = o.step(st)
        stats = s.step(1)
        assert abs(stats["p0"] / st.p0 - 1) < 1e-12, (k, stats["p0"], st.p0)
        assert abs(s.dt / o.dt - 1) < 1e-8, (k, s.dt, o.dt)
        changes += s.dt != stats["dt"]
        errs = compare(st, s.get(device=False))
        print(k, stats["dt"], stats["pc_err"], st.p0, errs, flush=True)
        _check(errs)
    assert changes >= 1


def test_adaptive_restart_is_exact():
    import torch
    case = c1_case(n=64)
    case.params = dict(case.params, dt_tol=1e-7)
    s = gpu_for(case)
    s.step(6)
    buf = s.save_state()
    s.step(7)
    ref = s.get(device=False)
    dt_ref = s.dt
    s2 = gpu_for(case)
    s2.load_state(buf)
    s2.step(7)
    got = s2.get(device=False)
    assert s2.dt == dt_ref
    for k in ("rho", "H", "P"):
        assert np.array_equal(got[k], ref[k]), k
    for d in range(2):
        assert np.array_equal(got["v"][d], ref["v"][d])
