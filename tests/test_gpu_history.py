"""The level n-1 history through the C ABI and the standalone pressure
solve's isolation from the state, on the GPU.

 - lm_set_fields(level = 1): the fields of time n-1 give the history of the
   next step (rho^{n-1} and the level n-1 residuals), so a run restarted
   from two oracle levels takes the oracle's AB2 / BDF2 step (Eq 3.1, 3.3,
   3.10, 3.11) instead of the Heun start;
 - lm_project leaves the state alone: the pressure returned by
   lm_get_fields and the checkpoint bytes are the same before and after a
   solve, and the next step is bit for bit that of a run without it."""
import numpy as np
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


def _check(errs, tol=TOL):
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, f"fields above {tol:g}: {bad} (all: {errs})"


def _fields(st, reacting):
    d = dict(H=st.H, v=st.v, F=st.F, P=st.P)
    if reacting:
        d["Z"] = st.Z
    return d


@pytest.mark.parametrize("which", ["random-2d", "slot-flame", "random-3d"])
def test_restart_from_two_levels_takes_the_ab2_step(which):
    case = {"random-2d": lambda: c2_case(n=96), "slot-flame": lambda: c3_case(nx=128, ny=256, W=32, wall=4,
                                                                               wall_h=32, inj=4),
            "random-3d": lambda: c4_case(n=32)}[which]()
    print("level-1 restart", which, flush=True)
    o, st0 = oracle_for(case)
    st1 = o.step(st0)
    st3 = o.run(st1, 2)
    reacting = bool(case.params.get("reacting"))
    s = gpu_for(case, dt=o.dt)     # the oracle's step, fixed from the state at t0
    dt = s.dt
    # level 0 at t1, level 1 at t0 (H given: no T -> H round trip)
    s.set(ib=case.ib, **_fields(st1, reacting))
    prev = _fields(st0, reacting)
    prev.pop("P")
    s.set(level=1, **prev)
    assert abs(s.dt / dt - 1) < 1e-15
    s.step(2)
    errs = compare(st3, s.get(device=False))
    print(errs, s.stats, flush=True)
    _check(errs)
    # without the history the first step is a Heun start: a clear miss
    s.set(ib=case.ib, **_fields(st1, reacting))
    s.step(2)
    heun = compare(st3, s.get(device=False))
    assert max(heun.values()) > 1e3 * max(max(errs.values()), 1e-16), heun


def test_level_one_needs_level_zero_and_constant_p0():
    from paper_2603_01727_amd import Solver, LowMachError, lib
    s = Solver((32, 32), (1.0, 1.0), Re=10.0, dt=1e-3)
    one = np.ones((32, 32))
    with pytest.raises(LowMachError) as e:
        s.set(level=1, T=one, v=[0 * one, 0 * one])
    assert e.value.status == lib.LM_ESTATE
    with pytest.raises(LowMachError) as e:
        s.set(level=2, T=one, v=[0 * one, 0 * one])
    assert e.value.status == lib.LM_EUNSUPPORTED
    c = Solver((32, 32), (1.0, 1.0), bc=[("slip", "slip"), ("noslip", "noslip")], Re=10.0, dt=1e-3,
               p0_closed=True)
    c.set(T=one, v=[0 * one, 0 * one])
    with pytest.raises(LowMachError) as e:
        c.set(level=1, T=one, v=[0 * one, 0 * one])
    assert e.value.status == lib.LM_EUNSUPPORTED


def test_project_leaves_the_state_untouched():
    import torch
    case = c2_case(n=128)
    s = gpu_for(case)
    r = gpu_for(case)
    s.step(2)
    r.step(2)
    P0 = s.get(("P",), device=False)["P"]
    b0 = s.save_state().cpu().numpy().copy()
    b = np.random.default_rng(5).standard_normal(s.shape)
    P, info = s.project(b)
    assert info["relres"] <= 1e-13
    P1 = s.get(("P",), device=False)["P"]
    b1 = s.save_state().cpu().numpy()
    assert np.array_equal(P0, P1)
    assert np.array_equal(b0, b1)
    s.step(1)
    r.step(1)
    a, q = s.get(device=False), r.get(device=False)
    for k in ("rho", "H", "P"):
        assert np.array_equal(a[k], q[k]), k
    for d in range(2):
        assert np.array_equal(a["v"][d], q["v"][d]) and np.array_equal(a["F"][d], q["F"][d])
    torch.cuda.synchronize()
