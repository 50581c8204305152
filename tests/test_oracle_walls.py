"""Pins of the oracle's isothermal walls (Eq 3.43 with the wall values of
Eq 4.16a-b), Sutherland's conductivity (Eq 4.12) and, through them, the
enclosed-system pressure (Eq 2.40) at a steady state.

A box with isothermal walls at x = 0 and x = 1, periodic in y and without
gravity relaxes to pure conduction: v = 0 and, in every row, the discrete
steady heat equation sum_f kappa_f delta_1 T = 0, i.e. the same heat flux q
through every x-face, with the wall faces at the wall conductivity and the
mirrored ghost T_g = 2 T_w - T. That steady state is solved here directly
(shooting on q, one scalar root per face) and the time-marched oracle must
reach it: every term of the step (walls, conductivity, the closed-system
p0 and its d_t p0 source, the projection) has to vanish there."""
import math

import numpy as np
from scipy.optimize import brentq

from oracle import Grid, Oracle, Params

C_SUTH = 110.5 / 600.0


def _kappa(T):
    return T ** 1.5 * (1.0 + C_SUTH) / (T + C_SUTH)


def _steady_conduction(n, TL, TR):
    """Cell temperatures and flux q of the discrete steady conduction
    problem on n cells of width 1/n between walls at TL and TR."""
    h = 1.0 / n

    def march(q):
        """Cell temperatures from the left wall for flux q (None once the
        flux cannot be carried at a positive temperature)."""
        T = [TL - q * h / (2.0 * _kappa(TL))]
        for _ in range(n - 1):
            a = T[-1]
            f = lambda b: 0.5 * (_kappa(a) + _kappa(b)) * (a - b) - q * h
            if a <= 1e-6 or f(1e-6) < 0.0:
                return None
            T.append(brentq(f, 1e-6, a, xtol=1e-15, rtol=1e-15))
        return np.array(T)

    def right_wall(q):
        T = march(q)
        if T is None:
            return -1e300
        return 2.0 * _kappa(TR) * (T[-1] - TR) / h - q

    # q between 0 and the flux of a wall-to-wall jump across one cell
    q = brentq(right_wall, 1e-9, (TL - TR) * _kappa(TL) / h * 0.999, xtol=1e-15, rtol=1e-15)
    return march(q), q


def test_steady_conduction_between_isothermal_walls():
    n, ny = 8, 2
    TL, TR = 1.6, 0.4
    g = Grid((n, ny), (1.0, 0.25), bc=(("noslip", "noslip"), ("periodic", "periodic")),
             bnd={(0, 0): dict(H=TL + 1.0), (0, 1): dict(H=np.full(ny, TR + 1.0))})
    p = Params(Re=2.0, Pr=0.71, sutherland_C=C_SUTH, p0_closed=True, gamma=1.4, cfl=0.3)
    o = Oracle(g, p)
    st = o.initial_state(np.ones((ny, n)), [np.zeros((ny, n)), np.zeros((ny, n))])
    mass = float(np.sum(st.rho) * g.dV)
    assert abs(mass - 0.25) < 1e-15
    st = o.run(st, 2200)
    T_ss, q = _steady_conduction(n, TL, TR)
    assert np.max(np.abs(st.T - T_ss[None, :])) < 1e-9, np.max(np.abs(st.T - T_ss[None, :]))
    for d in range(2):
        assert np.max(np.abs(st.v[d])) < 1e-9
    p0_ss = mass / float(np.sum(g.dV / np.broadcast_to(T_ss, (ny, n))))
    assert abs(st.p0 - p0_ss) < 1e-10, (st.p0, p0_ss)
    # mass is conserved exactly by p0 = m / sum(dV / T)
    assert abs(float(np.sum(st.rho) * g.dV) - mass) < 1e-14
    # the steady flux tends to the continuous one, integral of kappa dT
    # over [TR, TL], at second order (checked here at two resolutions)
    qc = _integral_kappa(TR, TL)
    e1 = abs(_steady_conduction(16, TL, TR)[1] - qc)
    e2 = abs(_steady_conduction(32, TL, TR)[1] - qc)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def _integral_kappa(a, b, m=20000):
    """Composite Simpson rule for the integral of kappa over [a, b]."""
    x = np.linspace(a, b, 2 * m + 1)
    w = np.ones_like(x)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return float(np.sum(w * _kappa(x)) * (b - a) / (6.0 * m))


def test_adiabatic_and_isothermal_walls():
    """A closed box without gravity and a perturbed temperature. With
    adiabatic (zero-gradient) walls everywhere its mass is conserved
    exactly and the temperature evens out; with the top wall isothermal at
    T = 1.5 the mass is still conserved and the top row heats up."""
    n = 8
    g_ad = Grid((n, n), (1.0, 1.0), bc=(("noslip", "noslip"), ("slip", "slip")))
    g_iso = Grid((n, n), (1.0, 1.0), bc=(("noslip", "noslip"), ("slip", "slip")),
                 bnd={(1, 1): dict(H=2.5)})
    x = (np.arange(n) + 0.5) / n
    T0 = 1.0 + 0.2 * np.cos(math.pi * x)[None, :] * np.cos(math.pi * x)[:, None]
    v0 = [np.zeros((n, n)), np.zeros((n, n))]
    p = Params(Re=5.0, Pr=0.71, sutherland_C=C_SUTH, p0_closed=True, gamma=1.4, cfl=0.3)
    for g in (g_ad, g_iso):
        o = Oracle(g, p)
        st = o.initial_state(T0, v0)
        mass = float(np.sum(st.rho) * g.dV)
        st = o.run(st, 150)
        assert abs(float(np.sum(st.rho) * g.dV) - mass) < 1e-13
        if g is g_ad:
            assert np.ptp(st.T) < 0.2 * np.ptp(T0)
        else:
            # the top wall heats the box towards T = 1.5
            assert st.T[-1].mean() > T0[-1].mean() + 0.05
            assert o.conductivity(o.padded_fields(st)[3])[-1, 1:-1].mean() > 0
