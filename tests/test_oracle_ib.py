"""Oracle pin for the penalised immersed boundary (section 3.4, Eq 3.30):
Taylor-Couette flow between immersed cylinders against the exact annular
profile v_theta = (4 - r^2)/(3 r) (section 4.3), and the shifted mask of
Iwakami (body grown by the Brinkman length sqrt(Da)) against the cell-exact
one."""
import math

import numpy as np

from workloads import taylor_couette_case
from _cases import oracle_for


def _run(shifted, n=48, Da=1e-2, t_end=0.3):
    case = taylor_couette_case(n=n, Da=Da, shifted=shifted)
    o, st = oracle_for(case)
    for _ in range(int(math.ceil(t_end / o.dt))):
        st = o.step(st)
    a = case.annulus
    ex = case.exact_v
    err = [math.sqrt(np.mean((st.v[i][a] - ex[i][a]) ** 2) / np.mean(ex[i][a] ** 2)) for i in range(2)]
    return err, st


def test_taylor_couette_penalised_cylinders():
    """Re = 1, Da = 1e-2, 48^2 cells over [-2.5, 2.5]^2, run from the exact
    profile to t = 0.3 (three viscous decay times of the gap): with the
    shifted mask the annular velocity stays within a few per cent of the
    exact one, both components alike (the flow is symmetric); the cell-exact
    mask leaves the whole Brinkman layer inside the gap and misses by an
    order of magnitude more."""
    err_s, st = _run(True)
    err_u, _ = _run(False)
    assert max(err_s) < 0.03, err_s
    assert abs(err_s[0] - err_s[1]) < 0.1 * err_s[0]
    assert min(err_u) > 5 * max(err_s), (err_u, err_s)
    assert np.all(np.isfinite(st.P))


def _penalised_mixture_fraction(dt, t_end=2.0, Le=1.5, delta=1e-7):
    """A periodic, uniformly penalised box (chi = 1) of reacting gas at
    rest, with uniform Z a small delta above its target Z_ib and H at its
    target: only the scalar penalisation F_Z of Eq 3.31 acts, so
    d_t Z = -kappa (Z - Z_ib) / (rho Le Pe Da) (Eq 3.2), linearised about
    Z_ib: Z - Z_ib = delta exp(-c t) with c = kappa(T_ib) T_ib / (p0 Le Pe Da)
    (rho = p0/T, T_ib = T(Z_ib, H_ib) by Eq 3.42). Le_F = Le_O = Le makes
    the regularised Le_eps of Eq 3.35 equal Le exactly."""
    from oracle import Grid, Oracle, Params, temperature
    g = Grid((6, 4), (1.0, 1.0))
    p = Params(Re=10.0, Pr=0.7, sigma=0.7, reacting=True, S=2.0, qs=0.8, Le_F=Le, Le_O=Le, Da_ib=0.5, dt=dt)
    Zib, Hib = 0.3, 2.0
    ib = {"chi": np.ones(g.shape), "Z_ib": np.full(g.shape, Zib), "H_ib": np.full(g.shape, Hib)}
    o = Oracle(g, p, ib=ib)
    st = o.initial_state(None, [np.zeros(g.shape)] * 2, Z=np.full(g.shape, Zib + delta), H=np.full(g.shape, Hib))
    n = int(round(t_end / dt))
    st = o.run(st, n)
    assert np.ptp(st.Z) == 0.0 and np.ptp(st.H) == 0.0 and np.max(np.abs(st.v[0])) == 0.0
    T = float(temperature(np.float64(Zib), np.float64(Hib), p.flame()))
    c = T ** p.sigma * T / (p.p0 * Le * p.Pe * p.Da_ib)
    return float(np.mean(st.Z)) - Zib, delta * math.exp(-c * n * dt), delta * math.exp(-c * Le * n * dt)


def test_mixture_fraction_penalisation_relaxes_at_lewis_rate():
    """The Z penalisation (Eq 3.31) carries 1/(Le Pe Da): with Le = 1.5 the
    excess relaxes at the closed-form rate at second order in dt; dropping
    the Lewis factor (the F_H form of Eq 3.32) is an O(1) miss."""
    errs = []
    for dt in (0.2, 0.1, 0.05):
        got, ex, no_le = _penalised_mixture_fraction(dt)
        errs.append(abs(got - ex) / ex)
    assert errs[-1] < 2e-5, errs
    for a, b in zip(errs, errs[1:]):
        assert abs(math.log(a / b, 2) - 2.0) < 0.25, errs
    assert abs(no_le - ex) / ex > 1000 * errs[-1]
