"""Pins of the oracle's complex-step tangent-linear derivatives against
central finite differences of the oracle's own real-valued step (the
derivative of a smooth map is what its difference quotients converge to),
on tiny 2D periodic grids."""
import math

import numpy as np
import pytest

from oracle import Grid, Oracle, Params
from oracle import tangent as tg
from workloads.ics import c5_case, fd_directions


def _setup(n=24, nsteps=0):
    c = c5_case(n=n)
    g = Grid(c.n[:2], c.L[:2], bc=c.bc)
    o = Oracle(g, Params(Re=300.0, Pr=0.7, cfl=0.3))
    st = o.initial_state(c.T, c.v)
    p = Params(Re=300.0, Pr=0.7, dt=o.dt)
    return c, g, p


@pytest.mark.parametrize("nsteps", [1, 4])
def test_complex_step_matches_central_differences(nsteps):
    c, g, p = _setup()
    for d in fd_directions(c.T.shape, k=3, seed=7):
        cs = tg.ke_directional(g, p, c.T, c.v, d, nsteps)
        errs = []
        for h in (1e-3, 1e-4):
            jp = tg.final_kinetic_energy(g, p, c.T + h * d, c.v, nsteps)
            jm = tg.final_kinetic_energy(g, p, c.T - h * d, c.v, nsteps)
            errs.append(abs((jp - jm) / (2 * h) - cs) / abs(cs))
        # second-order convergence of the difference quotient towards cs
        assert errs[1] < 1e-7
        assert errs[1] < errs[0] / 30.0 or errs[1] < 1e-10


def test_complex_step_is_linear_in_the_direction():
    c, g, p = _setup()
    d1, d2 = fd_directions(c.T.shape, k=2, seed=8)
    a = tg.ke_directional(g, p, c.T, c.v, d1, 2)
    b = tg.ke_directional(g, p, c.T, c.v, d2, 2)
    ab = tg.ke_directional(g, p, c.T, c.v, d1 - 2.5 * d2, 2)
    assert abs(ab - (a - 2.5 * b)) <= 1e-12 * (abs(a) + 2.5 * abs(b))


def _history_state(o, c, nsteps=1):
    return tg.with_eos(o, o.run(o.initial_state(c.T, c.v), nsteps))


def _direction(g, rng, with_history):
    shape = g.shape
    dx = {"H": rng.normal(size=shape), "v": [rng.normal(size=shape) for _ in range(2)]}
    F = []
    for d in range(2):
        ax = g.axis(d)
        f = rng.normal(size=shape)
        # periodic face arrays: face 0 repeats face n
        F.append(np.concatenate([np.take(f, [-1], axis=ax), f], axis=ax))
    dx["F"] = F
    if with_history:
        dx["rho_prev"] = rng.normal(size=shape)
        dx["R_H"] = rng.normal(size=shape)
        dx["R_v"] = [rng.normal(size=shape) for _ in range(2)]
    return dx


def _flat(y):
    out = []
    for k in ("H", "v", "F", "rho_prev", "R_H", "R_v"):
        if k in y:
            x = y[k]
            out += [np.ravel(a) for a in x] if isinstance(x, list) else [np.ravel(x)]
    return np.concatenate(out)


@pytest.mark.parametrize("with_history", [False, True])
def test_step_tangent_matches_central_differences(with_history):
    c, g, p = _setup(n=20)
    o = Oracle(g, p)
    st = _history_state(o, c, 1) if with_history else tg.with_eos(o, o.initial_state(c.T, c.v))
    rng = np.random.default_rng(11)
    dx = _direction(g, rng, with_history)
    t = tg.step_tangent(o, st, dx)
    h = 1e-5

    def real_step(sign):
        s = st.copy()
        s.H = s.H + sign * h * dx["H"]
        s.v = [a + sign * h * dx["v"][d] for d, a in enumerate(s.v)]
        s.F = [a + sign * h * dx["F"][d] for d, a in enumerate(s.F)]
        if with_history:
            s.rho_prev = s.rho_prev + sign * h * dx["rho_prev"]
            s.R_prev = dict(s.R_prev)
            s.R_prev["H"] = s.R_prev["H"] + sign * h * dx["R_H"]
            s.R_prev["v"] = [a + sign * h * dx["R_v"][d] for d, a in enumerate(s.R_prev["v"])]
        tg.with_eos(o, s)
        out = o.step(s)
        return dict(H=out.H, v=out.v, F=out.F, rho_prev=out.rho_prev, R_H=out.R_prev["H"],
                    R_v=out.R_prev["v"])

    yp, ym = real_step(1.0), real_step(-1.0)
    fd = (_flat(yp) - _flat(ym)) / (2 * h)
    cs = _flat(t)
    assert np.linalg.norm(fd - cs) <= 1e-8 * np.linalg.norm(cs)
    # the output history is the input level: its tangent is the input's
    assert np.allclose(t["rho_prev"], -o.p.p0 / st.T ** 2 * o.p.qs * dx["H"], rtol=1e-12, atol=0)


def test_kinetic_energy_of_uniform_flow():
    """J = 1/2 rho |U|^2 |Omega| for a uniform state (closed form)."""
    g = Grid((8, 8), (2 * math.pi, 2 * math.pi), bc=(("periodic", "periodic"),) * 2)
    o = Oracle(g, Params(dt=0.01))
    st = o.initial_state(np.full(g.shape, 2.0), [np.full(g.shape, 0.3), np.full(g.shape, -0.4)])
    J = tg.kinetic_energy(g, st)
    assert abs(J - 0.5 * 0.5 * 0.25 * (2 * math.pi) ** 2) < 1e-13


@pytest.mark.parametrize("with_history", [False, True])
def test_reacting_step_tangent_matches_central_differences(with_history):
    """Reacting periodic mixture (Z spans the flame level, Le_F != Le_O):
    the complex-step tangent of one step, along directions in every input
    including Z and R_Z, against central differences of the real step."""
    from workloads.ics import reacting_periodic_case
    c = reacting_periodic_case((20, 16), seed=7)
    g = Grid(c.n[:2], c.L[:2], bc=c.bc)
    pr = dict(c.params)
    pr.pop("cfl")
    o = Oracle(g, Params(dt=0.02, **pr))
    st = o.initial_state(c.T, c.v, Z=c.Z)
    if with_history:
        st = o.step(st)
    st = tg.with_eos(o, st)
    rng = np.random.default_rng(12)
    dx = _direction(g, rng, with_history)
    dx["Z"] = 0.1 * rng.normal(size=g.shape)
    if with_history:
        dx["R_Z"] = rng.normal(size=g.shape)
    t = tg.step_tangent(o, st, dx)
    h = 1e-6

    def real_step(sign):
        s = st.copy()
        s.H = s.H + sign * h * dx["H"]
        s.Z = s.Z + sign * h * dx["Z"]
        s.v = [a + sign * h * dx["v"][d] for d, a in enumerate(s.v)]
        s.F = [a + sign * h * dx["F"][d] for d, a in enumerate(s.F)]
        if with_history:
            s.rho_prev = s.rho_prev + sign * h * dx["rho_prev"]
            s.R_prev = dict(s.R_prev)
            s.R_prev["H"] = s.R_prev["H"] + sign * h * dx["R_H"]
            s.R_prev["Z"] = s.R_prev["Z"] + sign * h * dx["R_Z"]
            s.R_prev["v"] = [a + sign * h * dx["R_v"][d] for d, a in enumerate(s.R_prev["v"])]
        tg.with_eos(o, s)
        out = o.step(s)
        return dict(H=out.H, Z=out.Z, v=out.v, F=out.F, rho_prev=out.rho_prev, R_H=out.R_prev["H"],
                    R_Z=out.R_prev["Z"], R_v=out.R_prev["v"])

    flat = lambda y: np.concatenate([_flat(y), np.ravel(y["Z"]), np.ravel(y["R_Z"])])
    fd = (flat(real_step(1.0)) - flat(real_step(-1.0))) / (2 * h)
    cs = flat(t)
    assert np.linalg.norm(fd - cs) <= 1e-7 * np.linalg.norm(cs)


def test_open_channel_step_tangent_matches_central_differences():
    """Inflow / outflow channel (section 3.6; the outflow closure of section
    3.3 sums the right-hand side over the domain): the complex-step tangent
    of one step along H, v and F against central differences of the real
    step, so the closure keeps the imaginary part of that sum."""
    from workloads.ics import fourier_temperature, solenoidal_velocity
    n, L = (24, 32), (2 * math.pi, 2.5 * math.pi)
    rng = np.random.default_rng(17)
    T = fourier_temperature(n, L, rng, 3, 2.0, m=16)
    v = solenoidal_velocity(n, L, rng, 3, 0.1, m=16)
    v[1] = v[1] + 0.5
    bnd = {(1, 0): dict(v=[np.zeros(n[0]), np.full(n[0], 0.5)], H=np.full(n[0], 2.5),
                        F=np.full(n[0], 0.5 / 1.5))}
    g = Grid(n, L, bc=(("periodic", "periodic"), ("inflow", "outflow")), bnd=bnd)
    o = Oracle(g, Params(Re=200.0, Pr=0.7, dt=0.02))
    st = tg.with_eos(o, o.step(o.initial_state(T, v)))
    dx = _direction(g, np.random.default_rng(18), True)
    t = tg.step_tangent(o, st, dx)
    h = 1e-6

    def real_step(sign):
        s = st.copy()
        s.H = s.H + sign * h * dx["H"]
        s.v = [a + sign * h * dx["v"][d] for d, a in enumerate(s.v)]
        s.F = [a + sign * h * dx["F"][d] for d, a in enumerate(s.F)]
        s.rho_prev = s.rho_prev + sign * h * dx["rho_prev"]
        s.R_prev = dict(s.R_prev)
        s.R_prev["H"] = s.R_prev["H"] + sign * h * dx["R_H"]
        s.R_prev["v"] = [a + sign * h * dx["R_v"][d] for d, a in enumerate(s.R_prev["v"])]
        tg.with_eos(o, s)
        out = o.step(s)
        return dict(H=out.H, v=out.v, F=out.F, rho_prev=out.rho_prev, R_H=out.R_prev["H"],
                    R_v=out.R_prev["v"])

    fd = (_flat(real_step(1.0)) - _flat(real_step(-1.0))) / (2 * h)
    cs = _flat(t)
    assert np.linalg.norm(fd - cs) <= 1e-7 * np.linalg.norm(cs)
