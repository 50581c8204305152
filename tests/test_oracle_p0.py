"""Oracle pins for the thermodynamic pressure of an enclosed system
(Eq 2.40 with the zeta d_t p0 source of Eq 2.45 / 3.4b and the BDF
derivatives of Eq 3.5, 3.14)."""
import math

import numpy as np

from oracle import Grid, Oracle, Params
from workloads import fourier_temperature


def _uniform_heating(dt, t_end, gamma=1.4, T0=1.0, T_ib=2.0, Da=0.5, Re=10.0, Pr=0.7):
    """A closed, uniformly penalised box (chi = 1 everywhere) at rest with
    a uniform temperature: the mass fixes rho, so p0 = rho T rises with T,
    and d_t H = -gamma (H - H_ib) / (rho Pe Da) with kappa = 1 (sigma = 0):
    heating at constant volume is gamma times faster than the constant-p0
    law. Returns (T, p0) after t_end and the closed form."""
    g = Grid((8, 6), (1.0, 1.0))
    p = Params(Re=Re, Pr=Pr, sigma=0.0, Da_ib=Da, p0=1.0, dt=dt, p0_closed=True, gamma=gamma)
    ib = {"chi": np.ones(g.shape), "H_ib": np.full(g.shape, T_ib + 1.0)}
    o = Oracle(g, p, ib=ib)
    st = o.initial_state(np.full(g.shape, T0), [np.zeros(g.shape)] * 2)
    n = int(round(t_end / dt))
    for _ in range(n):
        st = o.step(st)
    rho0 = 1.0 / T0
    lam = gamma / (rho0 * p.Pe * Da)
    T_ex = T_ib + (T0 - T_ib) * math.exp(-lam * n * dt)
    return float(st.T.mean()), st.p0, T_ex, rho0 * T_ex, st


def test_uniform_heating_matches_constant_volume_law_second_order():
    errs = []
    for dt in (0.02, 0.01, 0.005):
        T, p0, T_ex, p0_ex, st = _uniform_heating(dt, 0.4)
        assert np.ptp(st.T) < 1e-14 and np.max(np.abs(st.v[0])) < 1e-14
        assert abs(p0 - st.rho.mean() * T) < 1e-14          # rho p0/T consistent
        errs.append(abs(T - T_ex))
        assert abs(p0 - p0_ex) < 5e-3
    for a, b in zip(errs, errs[1:]):
        assert abs(math.log(a / b, 2) - 2.0) < 0.25, errs
    # the constant-pressure law (zeta source dropped) is an O(1) miss
    T_cp = 2.0 + (1.0 - 2.0) * math.exp(-(1.0 / (1.0 * 7.0 * 0.5)) * 0.4)
    assert abs(T_cp - T_ex) > 100 * errs[-1]


def _closed_box(closed):
    g = Grid((24, 20), (1.0, 1.0), bc=(("slip", "noslip"), ("noslip", "slip")))
    rng = np.random.default_rng(4)
    T = fourier_temperature(g.n, g.L, rng, 3, 2.0, m=8)
    chi = np.zeros(g.shape)
    chi[8:12, 10:14] = 1.0                          # a hot body in the box
    ib = {"chi": chi, "H_ib": np.full(g.shape, 5.0)}
    p = Params(Re=50.0, Pr=0.7, Da_ib=1.0 / 24 ** 2, cfl=0.2, p0_closed=closed)
    o = Oracle(g, p, ib=ib)
    st = o.initial_state(T, [np.zeros(g.shape)] * 2)
    return g, o, st


def test_closed_box_conserves_mass_and_closes_the_poisson_balance():
    """With p0 from the conserved mass, sum(rho dV) stays m and the BDF
    d_t rho integrates to zero, so the compatibility residue mean(b) of
    both solves sits at rounding level; with p0 held constant the hot
    body's heating shows up as an O(1e-3) residue instead. p0 rises."""
    for closed in (True, False):
        g, o, st = _closed_box(closed)
        m = np.sum(st.rho) * g.dV
        for _ in range(6):
            st = o.step(st)
            res = max(abs(o.stats["pred_compat"]), abs(o.stats["corr_compat"]))
            if closed:
                assert abs(np.sum(st.rho) * g.dV - m) < 1e-13 * m
                assert res < 1e-11
        if closed:
            assert st.p0 > 1.0 + 1e-4
            assert abs(st.p0 - o.closed_p0(st.T)) == 0.0
        else:
            assert res > 1e-6 and st.p0 == 1.0


def test_bdf_start_up_and_history():
    """d_t p0 from the levels before: 0 with none (the first step takes the
    balance of balance_ddt_p0 instead), BDF1 with one, BDF2 with two."""
    g, o, st = _closed_box(True)
    dt = o.dt
    assert o.ddt_p0(1.3, ()) == 0.0
    assert abs(o.ddt_p0(1.3, (1.2,)) - 0.1 / dt) < 1e-12 / dt
    assert abs(o.ddt_p0(1.3, (1.2, 1.0)) - (3 * 1.3 - 4 * 1.2 + 1.0) / (2 * dt)) < 1e-12 / dt
    st1 = o.step(st)
    st2 = o.step(st1)
    assert st1.p0_hist == (st.p0,) and st2.p0_hist == (st1.p0, st.p0)
