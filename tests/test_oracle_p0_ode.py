"""Pins of the oracle's semi-enclosed thermodynamic pressure: p0 from the
ordinary differential equation of Eq 2.38 (p0_closed = 2), integrated with
the step's AB2 predictor and trapezoid corrector, its rate the d_t p0 of
each level's excess-enthalpy residual (Eq 3.4b).

* Compression by an inflow side (a piston of gas): with a uniform gas at
  rest-like isentropic compression, a large Peclet number and the inflow
  normal velocity U over a unit length, Eq 2.38 reduces to
  d p0/dt = gamma U p0, so p0 = exp(gamma U t), and away from the inflow
  the temperature follows the isentrope T = p0^{(gamma-1)/gamma} (the
  zeta d_t p0 source of Eq 3.4b).
* An enclosed box with zero-gradient walls: both integrals of Eq 2.38
  vanish (the discrete diffusion telescopes to the boundary fluxes), so p0
  stays exactly constant while the temperature evens out.
* An enclosed box heated through an isothermal wall: Eq 2.38 and the
  mass form of Eq 2.40 are two discretisations of one p0(t); each
  converges at second order and their extrapolated limits agree."""
import math

import numpy as np

from oracle import Grid, Oracle, Params


def test_inflow_compression_follows_exponential_and_isentrope():
    n, ny, U, gam = 32, 4, 0.1, 1.4
    g = Grid((n, ny), (1.0, 0.125), bc=(("inflow", "noslip"), ("periodic", "periodic")),
             bnd={(0, 0): dict(v=[U, 0.0], H=2.0, F=U)})
    o = Oracle(g, Params(Re=1e6, Pr=0.71, p0_closed=2, gamma=gam, dt=1e-3))
    x = (np.arange(n) + 0.5) / n
    # the velocity of uniform compression: U at the inflow, 0 at the wall
    st = o.initial_state(np.ones((ny, n)), [np.broadcast_to(U * (1 - x), (ny, n)).copy(), np.zeros((ny, n))])
    st = o.run(st, 200)
    pe = math.exp(gam * U * 0.2)
    assert abs(st.p0 / pe - 1.0) < 5e-7, (st.p0, pe)
    far = st.T[:, n // 2:]
    assert np.ptp(far) < 1e-12
    assert abs(far.mean() / pe ** ((gam - 1) / gam) - 1.0) < 2e-7


def test_adiabatic_box_keeps_p0():
    n = 16
    g = Grid((n, n), (1.0, 1.0), bc=(("noslip", "slip"), ("noslip", "noslip")))
    x = (np.arange(n) + 0.5) / n
    T0 = 1.0 + 0.4 * np.cos(math.pi * x)[None, :] * np.cos(2 * math.pi * x)[:, None]
    o = Oracle(g, Params(Re=20.0, Pr=0.71, inv_Fr2=1.0, p0_closed=2, gamma=1.4, cfl=0.3))
    st = o.initial_state(T0, [np.zeros((n, n)), np.zeros((n, n))])
    st = o.run(st, 60)
    assert abs(st.p0 - 1.0) < 1e-14
    assert np.ptp(st.T) < 0.9 * np.ptp(T0)
    assert max(float(np.max(np.abs(a))) for a in st.v) > 1e-4     # the box is not at rest


def _heated_box_p0(n, mode):
    g = Grid((n, 2), (1.0, 2.0 / n), bc=(("noslip", "noslip"), ("periodic", "periodic")),
             bnd={(0, 0): dict(H=2.3)})
    x = (np.arange(n) + 0.5) / n
    T0 = np.broadcast_to(1.0 + 0.3 * (1 - x) ** 2, (2, n)).copy()   # matches the wall, zero slope at x = 1
    dt = 0.4 / n ** 2
    o = Oracle(g, Params(Re=5.0, Pr=0.71, p0_closed=mode, gamma=1.4, dt=dt, sutherland_C=110.5 / 600))
    st = o.initial_state(T0, [np.zeros((2, n)), np.zeros((2, n))])
    st = o.run(st, int(round(0.05 / dt)))
    return st.p0


def test_ode_and_mass_forms_converge_together():
    lim = {}
    for mode in (1, 2):
        a, b, c = (_heated_box_p0(n, mode) for n in (16, 32, 64))
        assert 3.3 < (a - b) / (b - c) < 4.7, (mode, a, b, c)      # second order
        assert c > 1.01                                             # the wall heated the box
        lim[mode] = c + (c - b) / 3.0
    assert abs(lim[1] - lim[2]) < 1e-7, lim


def _reacting_box_p0(n, eps):
    """Closed box with adiabatic walls and a mixture-fraction profile that
    crosses the flame level: the H integral of Eq 2.38 vanishes, so the whole
    rise of p0 comes from the N' term (the heat the flame releases)."""
    g = Grid((n, 2), (1.0, 2.0 / n), bc=(("noslip", "noslip"), ("periodic", "periodic")))
    x = (np.arange(n) + 0.5) / n
    Z = np.broadcast_to(0.2 + 2.0 * (1 - x) ** 2 * (1 + 2 * x), (2, n)).copy()   # zero slope at both walls
    dt = 0.4 / n ** 2
    o = Oracle(g, Params(Re=5.0, Pr=0.71, reacting=True, S=3.0, qs=0.5, eps=eps, tol=1e-3,
                         Le_F=0.7, Le_O=1.2, p0_closed=2, gamma=1.4, dt=dt))
    st = o.initial_state(None, [np.zeros((2, n)), np.zeros((2, n))], Z=Z, H=np.full((2, n), 3.0))
    m = o.mass
    st = o.run(st, int(round(0.05 / dt)))
    return st.p0, m / (float(np.sum(1.0 / st.T)) * g.dV)


def test_reacting_ode_matches_mass_form_up_to_regularisation():
    """Eq 2.38 with N' of Eq 2.39 against the mass form of Eq 2.40 taken from
    the same run (the box conserves mass). With the sharp Heaviside the two
    are one identity (N + N'/Le = N' on both sides of the flame, and N' is
    the slope of the T(Z, H) map); the regularisation of section 3.5 breaks
    it inside the flame layer only, so the gap between the two grid-converged
    limits is first order in eps and small against the rise of p0. A dropped
    or mis-signed N' term, or N in its place, leaves a gap of the order of
    the rise itself."""
    gap = {}
    for eps in (0.5, 0.25):
        r = [_reacting_box_p0(n, eps) for n in (32, 64, 128)]
        lim = []
        for k in (0, 1):
            a, b, c = (x[k] for x in r)
            assert 3.5 < (a - b) / (b - c) < 4.5, (eps, k, a, b, c)   # second order
            lim.append(c + (c - b) / 3.0)
        rise = lim[1] - 1.0
        assert rise > 0.04                                           # the flame heats the box
        gap[eps] = lim[0] - lim[1]
        assert abs(gap[eps]) < 0.01 * rise, (eps, lim)
    assert 0.4 < gap[0.25] / gap[0.5] < 0.6, gap                     # first order in eps
