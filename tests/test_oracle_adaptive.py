"""Pins of the oracle's adaptive time step: Adams-Bashforth 2 and BDF2 for
unequal steps, and the step controller driven by the predictor-corrector
difference (the local-error estimate of Tab 2, proposed by the paper for
adaptive stepping).

* Taylor-Green (section 4.2, Tab 2 set-up): for a smooth solution the
  predictor-corrector difference of one step of size dt after a step of
  size dt/w tends (h -> 0) to |d3v/dt3| dt^3 (1 + w)/(4 w): the AB2
  extrapolation error, (1/6 + 1/(4w)) dt^3 d3v/dt3, plus the trapezoid's,
  dt^3 d3v/dt3 / 12. With equal steps this is Appendix A's 0.044089 dt^3 at
  t = 1.3; here w = 2 and w = 1/2.
* A density wave carried by a uniform flow (Re -> large) on alternating
  steps tau, 1.6 tau converges at second order in time (ratio 4 of
  successive differences when tau halves); the equal-step coefficients on
  the same step sequence converge at first order only.
* The controller keeps the estimate near 0.9^3 dt_tol on a smooth flow,
  grows the step by at most 1.5 and never exceeds the CFL step."""
import math

import numpy as np

from oracle import Grid, Oracle, Params
from workloads import taylor_green, cell_centres

LAM = 8 * math.pi ** 2 / 100.0          # decay rate of the unit-square vortex at Re = 100


def _tg_pc_difference(n, dt1, dt2, k=6):
    """Predictor-corrector difference of v1 in a step of size dt2 that
    follows k steps of size dt1, ending at t = 1.3 (Taylor-Green, Re 100),
    as its signed component along the vortex mode (RMS units)."""
    g = Grid((n, n), (1.0, 1.0))
    o = Oracle(g, Params(Re=100.0, Pr=0.7, dt=dt1, dt_tol=1e30, cfl=1e30))
    v1, v2, _ = taylor_green((n, n), (1.0, 1.0), 1.3 - k * dt1 - dt2, 100.0)
    st = o.initial_state(np.ones((n, n)), [v1, v2])
    for _ in range(k):
        o.dt = dt1                       # override the controller: a fixed sequence
        st = o.step(st)
    o.dt = dt2
    out = o.step(st)
    d = o.last_predicted.v[0] - out.v[0]
    mode = taylor_green((n, n), (1.0, 1.0), 1.3, 100.0)[0]
    return float(np.mean(d * mode)) / math.sqrt(float(np.mean(mode * mode)))


def test_unequal_step_predictor_corrector_difference():
    """On the collocated grid the cell velocity keeps a non-solenoidal part
    of order h^2 dt (the projection subtracts delta_2 P with P = p dt), so
    a change of step adds an O(h^2 dt^2) term to the difference; the
    difference's component along the vortex mode is extrapolated to h = 0
    (Richardson over 100^2 and 200^2) before the comparison with the
    closed form (d3v/dt3 = -LAM^3 v: the predictor lies above the
    corrector along v)."""
    dt1 = 1e-3
    for w in (2.0, 0.5):
        dt2 = w * dt1
        a = _tg_pc_difference(100, dt1, dt2)
        b = _tg_pc_difference(200, dt1, dt2)
        got = b + (b - a) / 3.0
        # |d3v1/dt3| = LAM^3 |v1|, the RMS of v1 at t = 1.3 from Appendix A
        expect = LAM ** 3 * 0.5 * math.exp(-LAM * 1.3) * dt2 ** 3 * (1.0 + w) / (4.0 * w)
        assert abs(got / expect - 1.0) < 0.05, (w, a, b, got, expect)


def _wave(m, adaptive=True):
    """Density wave on 32^2 to t = 0.5 with steps alternating tau, 1.6 tau
    (m pairs). adaptive=False takes the equal-step coefficients."""
    n = 32
    U = (0.7, -0.4)
    g = Grid((n, n), (2 * math.pi, 2 * math.pi))
    x, y = cell_centres(g.n, g.L)
    T0 = 1.0 + 0.5 * np.sin(x) * np.cos(y) + 0.3 * np.cos(2 * y)
    tau = 0.5 / (2.6 * m)
    p = Params(Re=1e12, Pr=1.0, dt=tau, dt_tol=1e30 if adaptive else 0.0, cfl=1e30)
    o = Oracle(g, p)
    st = o.initial_state(np.broadcast_to(T0, g.shape).copy(), [np.full(g.shape, U[0]), np.full(g.shape, U[1])])
    for q in range(2 * m):
        o.dt = tau if q % 2 == 0 else 1.6 * tau
        st = o.step(st)
    return st


def test_unequal_steps_second_order_in_time():
    rms = lambda a: math.sqrt(float(np.mean(a * a)))
    for adaptive, lo, hi in ((True, 3.6, 4.4), (False, 1.6, 2.6)):
        a, b, c = (_wave(m, adaptive) for m in (8, 16, 32))
        e1 = rms(a.T - b.T) + rms(a.v[0] - b.v[0])
        e2 = rms(b.T - c.T) + rms(b.v[0] - c.v[0])
        assert lo < e1 / e2 < hi, (adaptive, e1, e2, e1 / e2)


def test_controller_tracks_tolerance_and_cfl():
    n = 64
    g = Grid((n, n), (1.0, 1.0))
    v1, v2, _ = taylor_green((n, n), (1.0, 1.0), 0.0, 100.0)
    for tol in (1e-11, 1e-9):
        o = Oracle(g, Params(Re=100.0, Pr=0.7, dt=1e-4, dt_tol=tol, cfl=0.3))
        st = o.initial_state(np.ones((n, n)), [v1, v2])
        rows = []
        for k in range(60):
            cap = o.cfl_dt(st)
            st = o.step(st)
            rows.append((o.stats["dt"], o.stats["pc_err"], o.stats["pc_err_clean"]))
            assert o.stats["dt"] <= cap * (1 + 1e-12)
        dts = [r[0] for r in rows]
        # growth by at most 1.5, and only after four steps of one size
        for q in range(1, len(dts)):
            if dts[q] != dts[q - 1]:
                assert dts[q] <= 1.5 * dts[q - 1] * (1 + 1e-12)
                assert rows[q - 1][2]
        clean = [r[1] for r in rows[30:] if r[2]]
        assert clean
        if tol == 1e-11:
            # the error estimate sets the step: it settles with the estimate
            # inside the controller's band
            assert len(set(dts[30:])) == 1
            assert all(0.55 * tol < e < 1.0 * tol for e in clean), clean
        else:
            # a loose tolerance: the step climbs to the CFL step
            assert dts[-1] > 0.85 * o.cfl_dt(st)
            assert all(e < tol for e in clean)


def _alternating(o, st, tau, m):
    for q in range(2 * m):
        o.dt = tau if q % 2 == 0 else 1.6 * tau
        st = o.step(st)
    return st


def test_enclosed_system_unequal_steps_second_order():
    """Enclosed system (Eq 2.40) on steps alternating tau, 1.6 tau: the
    uniformly penalised closed box heats at constant volume, T = T_ib +
    (T0 - T_ib) exp(-gamma t / (rho Pe Da)) in closed form; with the
    unequal-step BDF2 of d_t p0 (and of d_t rho, AB2) the error falls at
    second order; with the equal-step formulas on the same steps it does
    not fall at all (the derivatives of rho and p0 are then inconsistent)."""
    import math as _m
    g = Grid((8, 6), (1.0, 1.0))
    T0, T_ib, Da, Re, Pr, gam = 1.0, 2.0, 0.5, 10.0, 0.7, 1.4
    lam = gam / ((1.0 / T0) * Re * Pr * Da)
    for adaptive, lo, hi in ((True, 3.5, 4.5), (False, 0.0, 1.5)):
        errs = []
        for m in (4, 8, 16):
            tau = 0.4 / (2.6 * m)
            p = Params(Re=Re, Pr=Pr, sigma=0.0, Da_ib=Da, dt=tau, p0_closed=1, gamma=gam,
                       dt_tol=1e30 if adaptive else 0.0, cfl=1e30)
            o = Oracle(g, p, ib={"chi": np.ones(g.shape), "H_ib": np.full(g.shape, T_ib + 1.0)})
            st = o.initial_state(np.full(g.shape, T0), [np.zeros(g.shape)] * 2)
            st = _alternating(o, st, tau, m)
            errs.append(abs(float(st.T.mean()) - (T_ib + (T0 - T_ib) * _m.exp(-lam * 0.4))))
        ratios = [a / b for a, b in zip(errs, errs[1:])]
        assert all(lo < r < hi for r in ratios), (adaptive, errs, ratios)


def test_semi_enclosed_unequal_steps_second_order():
    """Semi-enclosed system (Eq 2.38): compression through an inflow side
    on alternating steps; p0 self-converges at second order with the
    unequal-step AB2 of the ODE."""
    n, ny, U = 16, 2, 0.5
    x = (np.arange(n) + 0.5) / n
    res = []
    for m in (8, 16, 32):
        tau = 0.2 / (2.6 * m)
        g = Grid((n, ny), (1.0, 0.125), bc=(("inflow", "noslip"), ("periodic", "periodic")),
                 bnd={(0, 0): dict(v=[U, 0.0], H=2.0, F=U)})
        o = Oracle(g, Params(Re=1e6, Pr=0.71, p0_closed=2, gamma=1.4, dt=tau, dt_tol=1e30, cfl=1e30))
        st = o.initial_state(np.ones((ny, n)), [np.broadcast_to(U * (1 - x), (ny, n)).copy(), np.zeros((ny, n))])
        res.append(_alternating(o, st, tau, m).p0)
    r = (res[0] - res[1]) / (res[1] - res[2])
    assert 3.5 < r < 4.5, (res, r)
