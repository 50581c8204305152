"""Step-level pins of the oracle: discrete continuity after projection
(Eq 3.24 with the source of Eq 3.33), global mass closure through inflow,
outflow and the immersed-boundary mass source, free-stream preservation and
convergence to an exact variable-density solution."""
import math

import numpy as np
import pytest

from oracle import Grid, Oracle, Params
from workloads import cell_centres, c1_case


def discrete_continuity(o, st_new, st_old, first):
    """sum_d delta_1 F_d + d_t rho - S_m at every cell."""
    g = o.g
    div = sum((g.plus(st_new.F[d], d) - g.minus(st_new.F[d], d)) / g.h[d] for d in range(g.ndim))
    if first:
        dr = (st_new.rho - st_old.rho) / o.dt
    else:
        dr = (3 * st_new.rho - 4 * st_old.rho + st_old.rho_prev) / (2 * o.dt)
    Sm = o.ib.get("Sm", 0.0)
    return div + dr - Sm


def test_projection_enforces_discrete_continuity_periodic():
    c = c1_case(n=32)
    g = Grid(c.n[:2], c.L[:2])
    o = Oracle(g, Params(Re=100.0, Pr=0.7, cfl=0.2))
    st0 = o.initial_state(c.T, c.v)
    st1 = o.step(st0)
    r1 = discrete_continuity(o, st1, st0, True)
    lam = o.stats["corr_compat"]
    assert np.max(np.abs(r1 - lam)) < 1e-9 * np.max(np.abs(st1.rho)) / o.dt
    st2 = o.step(st1)
    r2 = discrete_continuity(o, st2, st1, False)
    assert np.max(np.abs(r2 - o.stats["corr_compat"])) < 1e-9 / o.dt
    # the residue is the mass-rate mismatch of the non-conservative H update:
    # small, not zero
    assert abs(o.stats["corr_compat"]) < 1e-3 * np.max(np.abs(r2))  + 1e-2


def open_case(n=(24, 32), with_ib=True):
    """Channel: slip side walls, inflow at the bottom, outflow at the top,
    a small immersed injector with a mass source."""
    nx, ny = n
    h = 1.0 / 8
    L = (nx * h, ny * h)
    x, y = cell_centres(n, L)
    bnd = {(1, 0): dict(v=[np.zeros(nx), np.full(nx, 0.2)], H=None, F=np.full(nx, 0.2))}
    g = Grid(n, L, bc=(("slip", "slip"), ("inflow", "outflow")), bnd=bnd)
    ib = {}
    if with_ib:
        chi = np.zeros(g.shape)
        chi[2:4, 10:14] = 1.0
        Sm = np.zeros(g.shape)
        Sm[2:4, 10:14] = 0.5
        vib = [np.zeros(g.shape), np.where(chi > 0, 0.4, 0.0)]
        ib = dict(chi=chi, Sm=Sm, v_ib=vib, H_ib=np.where(chi > 0, 2.5, 0.0))
    p = Params(Re=50.0, Pr=0.7, Da_ib=h * h, cfl=0.2)
    # inflow enthalpy H = T + 1 with T = 1
    bnd[(1, 0)]["H"] = np.full(nx, 2.0)
    o = Oracle(g, p, ib=ib)
    T = np.broadcast_to(1.0 + 0.5 * np.exp(-((x - 1.5) ** 2 + (y - 2.0) ** 2)), g.shape).copy()
    v = [np.zeros(g.shape), np.full(g.shape, 0.2)]
    return o, o.initial_state(T, v)


def test_open_domain_mass_closure_and_continuity():
    o, st0 = open_case()
    st1 = o.step(st0)
    st2 = o.step(st1)
    # outflow correction closes the balance: no compatibility residue left
    assert abs(o.stats["pred_compat"]) < 1e-12
    assert abs(o.stats["corr_compat"]) < 1e-12
    r = discrete_continuity(o, st2, st1, False)
    assert np.max(np.abs(r)) < 1e-9
    # boundary fluxes: zero through the slip walls, the inflow value at the bottom
    assert np.all(st2.F[0][:, 0] == 0) and np.all(st2.F[0][:, -1] == 0)
    assert np.all(st2.F[1][0, :] == 0.2)
    # injected mass = sum S_m dV (closed form 2 rows x 4 cells x 0.5 x h^2)
    g = o.g
    inj = float(np.sum(o.ib["Sm"]) * g.dV)
    assert abs(inj - 8 * 0.5 * g.dV) < 1e-15
    dr = (3 * st2.rho - 4 * st1.rho + st1.rho_prev) / (2 * o.dt)
    out = float(np.sum(st2.F[1][-1, :]) * g.h[0])
    inn = float(np.sum(st2.F[1][0, :]) * g.h[0])
    assert abs(float(np.sum(dr) * g.dV) - (inj + inn - out)) < 1e-11


def test_free_stream_preserved():
    g = Grid((16, 12), (2.0, 1.5))
    o = Oracle(g, Params(Re=10.0, Pr=0.7, dt=1e-2))
    st = o.initial_state(np.full(g.shape, 2.0), [np.full(g.shape, 0.3), np.full(g.shape, -0.2)])
    st = o.run(st, 4)
    assert np.max(np.abs(st.v[0] - 0.3)) < 1e-14
    assert np.max(np.abs(st.v[1] + 0.2)) < 1e-14
    assert np.max(np.abs(st.T - 2.0)) < 1e-14
    assert np.max(np.abs(st.P)) < 1e-14


def test_advected_density_wave_converges_second_order():
    """Uniform velocity carrying a temperature (density) pattern is an exact
    inviscid solution: T(x, t) = T0(x - U t), p = const. With Re -> large
    the discrete solution converges at second order (dt proportional to h),
    which pins the EOS, the BDF2 density derivative in the Poisson right-hand
    side and the advective form of the H equation."""
    U = (0.7, -0.4)
    errs = []
    for n in (16, 32, 64):
        g = Grid((n, n), (TWO_PI := 2 * math.pi, TWO_PI))
        x, y = cell_centres(g.n, g.L)
        T0 = lambda x, y: 1.0 + 0.5 * np.sin(x) * np.cos(y) + 0.3 * np.cos(2 * y)
        dt = 0.4 / n
        o = Oracle(g, Params(Re=1e12, Pr=1.0, dt=dt))
        st = o.initial_state(np.broadcast_to(T0(x, y), g.shape).copy(),
                             [np.full(g.shape, U[0]), np.full(g.shape, U[1])])
        k = n // 2
        st = o.run(st, k)
        t = k * dt
        Tex = T0(x - U[0] * t, y - U[1] * t)
        errs.append(math.sqrt(np.mean((st.T - Tex) ** 2)) + math.sqrt(np.mean((st.v[0] - U[0]) ** 2)))
    for a, b in zip(errs, errs[1:]):
        assert abs(math.log2(a / b) - 2.0) < 0.2, errs


def test_slot_flame_mass_closure_and_injection_rate():
    """Slot burner (section 4.5 analogue): the injected fuel mass rate is
    sum(S_m) dV = sum(U) dx per unit depth in closed form; the outflow
    shift closes the global balance, so no compatibility residue remains
    (the augmented-matrix multiplier of section 3.3 vanishes)."""
    from workloads import c3_case
    from _cases import oracle_for
    case = c3_case(nx=64, ny=96, W=16, wall=4, wall_h=16, inj=4)
    o, st = oracle_for(case)
    g = o.g
    U = case.ib["v_ib"][1][0, :]
    assert abs(float(np.sum(case.ib["Sm"]) * g.dV) - float(np.sum(U)) * g.h[0]) < 1e-13
    assert abs(case.injected_rate - float(np.sum(U)) * g.h[0]) < 1e-13
    st1 = o.step(st)
    st2 = o.step(st1)
    for key in ("pred_compat", "corr_compat"):
        assert abs(o.stats[key]) < 1e-12
    r = discrete_continuity(o, st2, st1, False)
    assert np.max(np.abs(r)) < 1e-8
    # temperature stays within the flame-sheet bounds [1, 7]
    assert st2.T.min() > 0.99 and st2.T.max() < 7.0 + 1e-9


def _stratified_column(ny, inv_Fr2=4.0, dt=1e-3):
    """Gas at rest between isothermal slip walls (bottom T = 1, top
    T = 2.5), periodic in x, with the linear conduction profile
    T = 1 + 1.5 y and kappa = 1 (sigma = 0): the discrete diffusion of
    the linear H vanishes, so rho stays put and the only force is the
    buoyancy (1/Fr^2)(1 - rho) e_y of Eq 3.8b. Returns the oracle, the
    initial state and the predicted level of one step."""
    H0, s = 2.0, 1.5
    g = Grid((4, ny), (1.0, 1.0), bc=(("periodic", "periodic"), ("slip", "slip")),
             bnd={(1, 0): {"H": np.full(4, H0)}, (1, 1): {"H": np.full(4, H0 + s)}})
    x, y = cell_centres(g.n, g.L)
    H = np.broadcast_to(H0 + s * y + 0 * x, g.shape).copy()
    o = Oracle(g, Params(Re=50.0, Pr=0.7, sigma=0.0, inv_Fr2=inv_Fr2, dt=dt))
    st = o.initial_state(None, [np.zeros(g.shape)] * 2, H=H)
    o.step(st)
    return o, st, o.last_predicted, y[:, 0]


def test_buoyancy_gives_hydrostatic_pressure():
    """At rest, the projection balances buoyancy: the predicted face flux
    vanishes and P = p dt is the hydrostatic pressure,
    P(y) = dt (1/Fr^2) integral (1 - rho) dy (Eq 3.8b with Eq 3.23-3.24),
    exactly in its discrete form (the face difference of P equals the
    face average of the buoyancy momentum: the trapezoid rule over cell
    centres) and at second order against the integral of
    1 - 1/T(y) = 1 - 1/(1 + 1.5 y). A sign error, a misplaced 1/Fr^2, the
    force on the wrong component or a missing dt fails."""
    inv_Fr2, dt = 4.0, 1e-3
    errs = []
    for ny in (16, 32, 64):
        o, st, pr, yc = _stratified_column(ny, inv_Fr2, dt)
        g = o.g
        assert np.max(np.abs(pr.F[1])) < 1e-15 and np.max(np.abs(pr.F[0])) < 1e-15
        assert np.max(np.ptp(pr.P, axis=1)) == 0.0
        rho = st.rho[:, 0]
        dP = g.h[1] * dt * inv_Fr2 * (1.0 - 0.5 * (rho[1:] + rho[:-1]))
        Pd = np.concatenate([[0.0], np.cumsum(dP)])
        Pd -= Pd.mean()
        assert np.max(np.abs(pr.P[:, 0] - Pd)) < 1e-13 * np.max(np.abs(Pd))
        Pc = dt * inv_Fr2 * (yc - np.log(1.0 + 1.5 * yc) / 1.5)
        Pc -= Pc.mean()
        errs.append(np.max(np.abs(pr.P[:, 0] - Pc)) / np.max(np.abs(Pc)))
    assert errs[-1] < 1e-4
    for a, b in zip(errs, errs[1:]):
        assert abs(math.log(a / b, 2) - 2.0) < 0.1, errs
