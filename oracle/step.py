"""One predictor-corrector time step of the low-Mach fractional-step method.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows section 3.1 (Eq 3.1-3.19) with the spatial operators of section 3.2
(Eq 3.20-3.26), the projection of section 3.3, the penalisation immersed
boundary of section 3.4 (Eq 3.29-3.33) and the T(Z, H) map of section 3.5.
Readings where the paper is silent or garbled are listed in the docstrings of
the functions that take them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .flame import FlameParams, le_eps, n_eps, n_prime_eps, temperature, enthalpy_from_T
from .grid import Grid, face_extrap_coeffs, fill_ghosts, field_rules
from .poisson import PoissonSolver


def _real_or_complex(a):
    """Copy as float64, or complex128 for complex input (complex-step
    differentiation runs the same arithmetic on complex fields)."""
    return np.array(a, dtype=np.result_type(a, np.float64))


@dataclasses.dataclass
class Params:
    """Dimensionless parameters (section 2.2, Eq 2.12-2.21; section 4.1):
    Pe = Re Pr; kappa = T^sigma (Eq 2.50), or Sutherland's law
    kappa = T^{3/2} (1 + C)/(T + C) (Eq 4.12) when sutherland_C = C > 0;
    inv_Fr2 = 1/Fr^2 (Eq 2.43);
    Da_ib: immersed-boundary Darcy number (Eq 3.30); p0: thermodynamic
    pressure, constant for open and periodic systems (Eq 2.41), or its
    initial value when p0_closed is set: p0_closed = 1 (True), an enclosed
    system whose p0 follows from the conserved mass, p0 = m / integral(1/T)
    (Eq 2.40); p0_closed = 2, a semi-enclosed system whose p0 follows the
    ordinary differential equation of Eq 2.38 (see Oracle.p0_rate); both
    with the
    zeta d_t p0 source of the excess-enthalpy equation (Eq 2.45, 3.4b),
    zeta = (S+1)(gamma-1)/(gamma Q) = (gamma-1)/(gamma qs); dt = 0 asks for a
    step fixed once from the CFL number of the initial state; dt_tol > 0
    makes the step adaptive (see Oracle.next_dt)."""
    Re: float = 100.0
    Pr: float = 0.7
    sigma: float = 0.7
    inv_Fr2: float = 0.0
    reacting: bool = False
    S: float = 1.0
    qs: float = 1.0
    eps: float = 0.5
    tol: float = 1e-3
    Le_F: float = 1.0
    Le_O: float = 1.0
    Da_ib: float = 1.0
    p0: float = 1.0
    dt: float = 0.0
    cfl: float = 0.2
    p0_closed: int = 0
    gamma: float = 1.4
    sutherland_C: float = 0.0
    dt_tol: float = 0.0

    def kappa(self, T):
        """Conductivity (= viscosity) of temperature: T^sigma (Eq 2.50) or
        Sutherland's law (Eq 4.12)."""
        if self.sutherland_C > 0.0:
            C = self.sutherland_C
            return T * np.sqrt(T) * (1.0 + C) / (T + C)
        return T ** self.sigma

    @property
    def zeta(self):
        return (self.gamma - 1.0) / (self.gamma * self.qs)

    @property
    def Pe(self):
        return self.Re * self.Pr

    def flame(self):
        return FlameParams(S=self.S, qs=self.qs, eps=self.eps, tol=self.tol,
                           Le_F=self.Le_F, Le_O=self.Le_O, reacting=bool(self.reacting))


@dataclasses.dataclass
class State:
    rho: np.ndarray
    v: list
    Z: Optional[np.ndarray]
    H: np.ndarray
    T: np.ndarray
    P: np.ndarray
    F: list
    rho_prev: Optional[np.ndarray] = None     # rho^{n-1}
    R_prev: Optional[dict] = None             # residuals at level n-1
    nstep: int = 0
    p0: float = 1.0                           # thermodynamic pressure at level n
    p0_hist: tuple = ()                       # p0 at levels n-1, n-2 (closed systems)
    dt_prev: float = 0.0                      # step from level n-1 to n (adaptive steps)
    p0_rate_prev: Optional[float] = None      # d_t p0 at level n-1 (Eq 2.38 systems)
    dt_prev2: float = 0.0                     # step from level n-2 to n-1 (adaptive steps)
    nsame: int = 0                            # steps of that size in a row (adaptive steps)

    def copy(self):
        c = lambda a: None if a is None else a.copy()
        return State(c(self.rho), [a.copy() for a in self.v], c(self.Z), c(self.H), c(self.T),
                     c(self.P), [a.copy() for a in self.F], c(self.rho_prev),
                     None if self.R_prev is None else {k: ([a.copy() for a in v] if isinstance(v, list) else v.copy())
                                                       for k, v in self.R_prev.items()},
                     self.nstep, self.p0, tuple(self.p0_hist), dt_prev=self.dt_prev,
                     p0_rate_prev=self.p0_rate_prev, dt_prev2=self.dt_prev2, nsame=self.nsame)


class Oracle:
    """Holds grid, parameters, immersed-boundary data and a Poisson solver.

    ``ib``: dict with 'chi' (0/1 mask), 'v_ib' (list), 'Z_ib', 'H_ib', 'Sm'
    (mass source of Eq 3.33), any of which may be missing (= 0)."""

    def __init__(self, grid: Grid, params: Params, ib=None, beta=None):
        self.g = grid
        self.p = params
        self.fp = params.flame()
        self.ib = dict(ib or {})
        self.poisson = PoissonSolver(grid, beta)
        self.dt = params.dt
        self.stats = {}

    # -- set-up ------------------------------------------------------------
    def initial_state(self, T, v, Z=None, P=None, F=None, H=None):
        """State at level 0 from temperature (or excess enthalpy) and
        velocity (and Z).

        H is obtained by inverting Eq 3.42 when T is given; T is then
        re-evaluated from (Z, H) and rho = p0/T (Eq 2.49). Unless given, the
        face fluxes are the face average of rho v (Eq 3.20 with n = 1), not
        projected, and P = 0."""
        g, fp = self.g, self.fp
        if self.p.p0_closed:
            # an enclosed system: no mass crosses the sides or enters through
            # a source; the first-step balance takes the non-reacting map. A
            # semi-enclosed one (Eq 2.38) may also have inflow sides.
            banned = ("outflow",) if self.p.p0_closed == 2 else ("inflow", "outflow")
            open_side = any(g.bc[d][s] in banned for d in range(g.ndim) for s in (0, 1))
            reacting_closed = self.p.reacting and self.p.p0_closed == 1
            # Eq 2.38 has no term for the penalisation's heat (Eq 3.31-3.32)
            body_ode = self.p.p0_closed == 2 and self.ib.get("chi") is not None
            if open_side or self.ib.get("Sm") is not None or reacting_closed or body_ode:
                raise ValueError("p0_closed needs walls or periodic sides (or inflow sides for Eq 2.38) and "
                                 "no mass source; the enclosed form (1) also needs non-reacting flow, the ODE (2) no immersed body")
        Zs = None
        if self.p.reacting:
            Zs = np.zeros(g.shape) if Z is None else _real_or_complex(Z)
        if T is None:
            H = _real_or_complex(H)
        else:
            H = enthalpy_from_T(_real_or_complex(T), Zs if Zs is not None else 0.0, fp)
        T2 = temperature(Zs if Zs is not None else 0.0, H, fp)
        rho = self.p.p0 / T2
        # enclosed system: the mass of the initial state is conserved (Eq 2.40)
        self.mass = g.integral(rho)
        v = [_real_or_complex(a) for a in v]
        if F is None:
            F = self.face_average_flux([rho * a for a in v])
        Pz = np.zeros(g.shape) if P is None else _real_or_complex(P)
        st = State(rho, v, Zs, H, T2, Pz, F, p0=self.p.p0)
        if self.dt == 0.0:
            self.dt = self.cfl_dt(st)
        return st

    def cfl_dt(self, st: State):
        """Fixed time step from the initial state (a reading: the paper only
        bounds dt by C dx^2 and, with penalisation, by c Re Da):
        dt = CFL / max_cells[ sum_d |v_d|/h_d + 2 nu sum_d 1/h_d^2 + chi nu / Da ]
        with nu = max(Pr, 1, 1/Le_F, 1/Le_O) kappa / (Pe rho)."""
        g, p = self.g, self.p
        kap = p.kappa(st.T)
        nu = max(p.Pr, 1.0, 1.0 / p.Le_F, 1.0 / p.Le_O) * kap / (p.Pe * st.rho)
        wid = [g.along(d, g.wid[d][1:-1]) for d in range(g.ndim)]   # h on a uniform grid
        rate = sum(np.abs(st.v[d]) / wid[d] for d in range(g.ndim))
        rate = rate + 2.0 * nu * sum(1.0 / wid[d] ** 2 for d in range(g.ndim))
        chi = self.ib.get("chi")
        if chi is not None:
            rate = rate + chi * nu / p.Da_ib
        return p.cfl / float(np.max(rate))

    # -- operators -----------------------------------------------------------
    def face_average_flux(self, M):
        """Face average of cell momentum M_d on faces normal to d (Eq 3.20,
        n = 1); boundary faces of non-periodic sides take the side's mass
        flux (zero at walls, the given flux at inflow sides, the cell value
        extrapolated at outflow sides)."""
        g = self.g
        F = []
        for d in range(g.ndim):
            Mp = g.pad(M[d])
            fill_ghosts(g, Mp, [(("periodic",),) * 2 if g.periodic(e) else (("extrap",),) * 2
                                for e in range(g.ndim)])
            G = self._face_interp(Mp, d)
            self._boundary_faces(G, d, M[d], None)
            F.append(G)
        return F

    def _face_interp(self, Ap, d):
        """Eq 3.20 (n = 1) from the two cell centres to each d-face (the
        two-point mean on a uniform grid)."""
        g = self.g
        return (g.along(d, g.wlo[d]) * g.S(Ap, d, None) + g.along(d, g.whi[d]) * g.S(Ap, d, g.e(d)))

    def _boundary_faces(self, G, d, Md, corr):
        """Overwrite boundary faces normal to d with the prescribed flux."""
        g = self.g
        if g.periodic(d):
            return
        ax = g.axis(d)
        n = g.n[d]
        for side in (0, 1):
            kind = g.bc[d][side]
            f = 0 if side == 0 else n
            if kind in ("slip", "noslip"):
                G[g.face_index(d, f)] = 0.0
            elif kind == "inflow":
                G[g.face_index(d, f)] = g.bvalue(d, side, "F")
            elif kind == "outflow":
                # quadratic extrapolation of the cell momentum to the face
                if side == 1:
                    m1, m2, m3 = (np.take(Md, n - 1, axis=ax), np.take(Md, n - 2, axis=ax),
                                  np.take(Md, n - 3, axis=ax))
                else:
                    m1, m2, m3 = (np.take(Md, 0, axis=ax), np.take(Md, 1, axis=ax),
                                  np.take(Md, 2, axis=ax))
                if g.faces[d] is None:
                    Gf = (15.0 * m1 - 10.0 * m2 + 3.0 * m3) / 8.0
                else:
                    A, B, C = face_extrap_coeffs(g, d, side)
                    Gf = A * m1 + B * m2 + C * m3
                G[g.face_index(d, f)] = Gf + (0.0 if corr is None else corr)

    def padded_fields(self, st: State):
        """Ghost-filled copies of v, Z, H and T (T from Z, H at ghosts)."""
        g = self.g
        vp = []
        for i in range(g.ndim):
            a = g.pad(st.v[i])
            fill_ghosts(g, a, field_rules(g, "v", i))
            vp.append(a)
        Hp = g.pad(st.H)
        fill_ghosts(g, Hp, field_rules(g, "H"))
        Zp = None
        if self.p.reacting:
            Zp = g.pad(st.Z)
            fill_ghosts(g, Zp, field_rules(g, "Z"))
            # Ghost temperatures (used only for the boundary-face
            # conductivity) take Z clamped to its realizable range
            # [0, S+1]; a mirrored ghost of a small interior Z can otherwise
            # leave the range where the map of Eq 3.42 stays positive.
            Zc = np.clip(Zp, 0.0, self.p.S + 1.0)
            g.interior(Zc)[...] = st.Z
            Tp = temperature(Zc, Hp, self.fp)
        else:
            Tp = temperature(0.0, Hp, self.fp)
        return vp, Zp, Hp, Tp

    def conductivity(self, Tp):
        """Padded conductivity of the padded temperature. Ghosts take
        kappa of the ghost temperature, except at an isothermal wall (a slip
        or no-slip side with a wall H, Eq 4.16a-b), where the ghost is
        2 kappa(T_w) - kappa(T) of the adjacent cell, so that the wall
        face's two-cell mean is the conductivity of the wall temperature.
        (A reading: the mirrored ghost temperature 2 T_w - T is negative
        whenever T > 2 T_w, as at the cold wall of a cavity started from
        the mean temperature, and kappa is undefined there.)"""
        g, p = self.g, self.p
        iso = [(d, s) for d in range(g.ndim) for s in (0, 1)
               if g.bc[d][s] in ("slip", "noslip") and g.bvalue(d, s, "H", default=None) is not None]
        if not iso:
            return p.kappa(Tp)
        assert not p.reacting, "isothermal walls: non-reacting flow only"
        T = Tp.copy()

        def plane(d, pos, full):
            idx = [slice(None) if full else slice(1, -1)] * g.ndim
            idx[g.axis(d)] = pos
            return tuple(idx)

        for d, s in iso:
            T[plane(d, 0 if s == 0 else g.n[d] + 1, True)] = 1.0     # placeholder
        kapp = p.kappa(T)
        for d, s in iso:
            Tw = temperature(0.0, np.asarray(g.bvalue(d, s, "H"), dtype=float), self.fp)
            inner = Tp[plane(d, 1 if s == 0 else g.n[d], False)]
            kapp[plane(d, 0 if s == 0 else g.n[d] + 1, False)] = 2.0 * p.kappa(Tw) - p.kappa(inner)
        return kapp

    def _scalar_terms(self, phip, kapp, F):
        """Advective term of Eq 3.26b, sum_d avg_d(F_d delta_1 phi) (face to
        cell average, Eq 3.20 with n = 1), and the diffusive term
        sum_d delta_1(kappa_f delta_1 phi) with the face conductivity the
        arithmetic mean of the two cells (centred differences, section 3.2)."""
        g = self.g
        adv = 0.0
        dif = 0.0
        for d in range(g.ndim):
            dfc = g.along(d, g.dfc[d])               # centre distance across each face
            wid = g.along(d, g.wid[d][1:-1])         # cell width
            grad = (g.S(phip, d, g.e(d)) - g.S(phip, d, None)) / dfc
            kf = self._face_interp(kapp, d)
            Fg = F[d] * grad
            # face to centre: the centroid is midway between its faces
            adv = adv + 0.5 * (g.plus(Fg, d) + g.minus(Fg, d))
            q = kf * grad
            dif = dif + (g.plus(q, d) - g.minus(q, d)) / wid
        return adv, dif

    def _momentum_terms(self, vp, kapp, F):
        """Convective term of Eq 3.26a, sum_d delta_1(F_d avg_d v_i), with the
        velocity averaged along the face direction d (the printed superscript
        names x_i; only x_d puts v_i on a d-face), and the viscous term
        sum_d delta_1 tau_id of Eq 2.46 with tau_id evaluated on d-faces:
        tau_id = kappa_f [D_d v_i + D_i v_d - 2/3 delta_id sum_k D_k v_k],
        D_d the face difference across the face and D_k (k != d) the average
        of the two adjacent cells' centred differences (Eq 3.21, n = 2)."""
        g = self.g
        nd = g.ndim
        conv = [0.0] * nd
        visc = [0.0] * nd
        for d in range(nd):
            dfc = g.along(d, g.dfc[d])
            wid = g.along(d, g.wid[d][1:-1])
            wlo, whi = g.along(d, g.wlo[d]), g.along(d, g.whi[d])
            kf = self._face_interp(kapp, d)
            # derivative matrix D[k][c] = D_k v_c on d-faces
            D = [[None] * nd for _ in range(nd)]
            for c in range(nd):
                for k in range(nd):
                    if k == d:
                        D[k][c] = (g.S(vp[c], d, g.e(d)) - g.S(vp[c], d, None)) / dfc
                    else:
                        d2k = g.along(k, g.d2[k])    # Eq 3.21, n = 2, at the cells on either side
                        offp = g.e(k)
                        offm = g.e(k, -1)
                        offdp = tuple(a + b for a, b in zip(g.e(d), g.e(k)))
                        offdm = tuple(a + b for a, b in zip(g.e(d), g.e(k, -1)))
                        cl = (g.S(vp[c], d, offp) - g.S(vp[c], d, offm)) / d2k
                        cr = (g.S(vp[c], d, offdp) - g.S(vp[c], d, offdm)) / d2k
                        D[k][c] = wlo * cl + whi * cr
            div = sum(D[k][k] for k in range(nd))
            for i in range(nd):
                vf = self._face_interp(vp[i], d)
                fl = F[d] * vf
                conv[i] = conv[i] + (g.plus(fl, d) - g.minus(fl, d)) / wid
                tau = D[d][i] + D[i][d]
                if i == d:
                    tau = tau - (2.0 / 3.0) * div
                tau = kf * tau
                visc[i] = visc[i] + (g.plus(tau, d) - g.minus(tau, d)) / wid
        return conv, visc

    def closed_p0(self, T):
        """Thermodynamic pressure of an enclosed system from the equation of
        state integrated over the domain, p0 = m / sum(dV / T) (Eq 2.40)."""
        return self.mass / self.g.integral(1.0 / T)

    def ddt_p0(self, p_new, hist, dt_new=None, dt_old=None):
        """d_t p0 at the level whose pressure is p_new, from the levels before
        it (newest first): BDF2 (Eq 3.5, 3.14); with one earlier level BDF1,
        with none 0 (start-up readings, as for d_t rho). Adaptive steps: the
        spacings dt_new (to the newest earlier level) and dt_old (the one
        before) give BDF2 for unequal steps in level differences, as for
        d_t rho."""
        dt = self.dt if dt_new is None else dt_new
        if len(hist) >= 2:
            if self.p.dt_tol > 0.0:
                w = dt / dt_old
                return ((1.0 + 2.0 * w) / (1.0 + w) * (p_new - hist[0])
                        - w * w / (1.0 + w) * (hist[0] - hist[1])) / dt
            return (3.0 * p_new - 4.0 * hist[0] + hist[1]) / (2.0 * dt)
        if len(hist) == 1:
            return (p_new - hist[0]) / dt
        return 0.0

    def p0_rate(self, st: State):
        """d_t p0 of a semi-enclosed system at one level, Eq 2.38:
        (gamma / V) [qs / Pe integral (div(kappa grad H) + N' div(kappa grad
        Z)) dV - p0 integral div v dV], N' of Eq 2.39 regularised like
        Eq 3.35 (reacting flow only). The first integral is the sum over
        cells of the discrete diffusion terms of the residuals (the H part
        telescopes to the conductive fluxes through the boundary faces);
        the second is the volume flux out through the sides, the given
        normal velocity of each inflow side times its face area (walls and
        periodic sides carry none)."""
        g, p = self.g, self.p
        _, Zp, Hp, Tp = self.padded_fields(st)
        kapp = self.conductivity(Tp)
        _, dif = self._scalar_terms(Hp, kapp, st.F)
        if p.reacting:
            _, difZ = self._scalar_terms(Zp, kapp, st.F)
            dif = dif + n_prime_eps(st.Z, self.fp) * difZ
        heat = float(g.integral(dif))
        flux = 0.0
        for d in range(g.ndim):
            for s in (0, 1):
                if g.bc[d][s] != "inflow":
                    continue
                vn = np.broadcast_to(np.asarray(g.bvalue(d, s, "v", d), dtype=float),
                                     tuple(g.shape[a] for a in range(g.ndim) if a != g.axis(d)))
                if not g.stretched:
                    flux += (1.0 if s == 1 else -1.0) * float(np.sum(vn)) * (g.dV / g.h[d])
                else:
                    # face areas of the side: products of the other widths
                    area = np.take(g.cell_volumes(), 0, axis=g.axis(d)) / g.wid[d][1]
                    flux += (1.0 if s == 1 else -1.0) * float(np.sum(vn * area))
        return p.gamma / g.volume * (p.qs / p.Pe * heat - st.p0 * flux)

    def balance_ddt_p0(self, st: State):
        """d_t p0 at a level with no earlier one (the first step; a start-up
        reading, the paper is silent): the time derivative of Eq 2.40,
        d_t p0 = (p0^2/m) sum(dV d_t T / T^2), with d_t T = qs R_H of the
        non-reacting map T = qs (H - 1) and R_H = R_H|0 + zeta d_t p0 / rho
        (Eq 3.4), solved for d_t p0. (A first-order start, d_t p0 = 0 or a
        one-sided difference, leaves a first-order error in p0.)"""
        p, g = self.p, self.g
        dV = g.cell_volumes() if g.stretched else g.dV
        RH = self.residuals(st, 0.0)["H"]
        w = (st.p0 ** 2 / self.mass) * dV * p.qs / st.T ** 2
        A = np.sum(w * RH)
        B = np.sum(w * p.zeta / st.rho)
        return A / (1.0 - B)

    def residuals(self, st: State, dtp0=0.0):
        """Right-hand sides at one time level.

        R_Z = (1/rho)[-adv Z + div(kappa grad Z)/(Le Pe) + F_Z]      (Eq 3.2, 3.31)
        R_H = (1/rho)[-adv H + div(kappa grad H)/Pe + F_H
                      + (N/Pe) div(kappa grad Z)]                     (Eq 3.4, 3.32)
        R_v = -conv + (Pr/Pe) div tau + (1/Fr^2)(1 - rho) e_y + F_v    (Eq 3.8, 3.30)
        Le and N are the regularised coefficients of Eq 3.35 at the cell.
        The zeta d_t p0 source of Eq 3.4b (inside the 1/rho bracket) is
        taken with the given d_t p0: zero when p0 is constant."""
        g, p, fp = self.g, self.p, self.fp
        vp, Zp, Hp, Tp = self.padded_fields(st)
        kapp = self.conductivity(Tp)
        kap = g.interior(kapp)
        Pe = p.Pe
        chi = self.ib.get("chi")
        R = {}
        advH, difH = self._scalar_terms(Hp, kapp, st.F)
        rH = -advH + difH / Pe
        if p.reacting:
            advZ, difZ = self._scalar_terms(Zp, kapp, st.F)
            le = le_eps(st.Z, fp)
            rZ = -advZ + difZ / (le * Pe)
            rH = rH + n_eps(st.Z, fp) * difZ / Pe
            if chi is not None:
                rZ = rZ - chi * kap * (st.Z - self.ib.get("Z_ib", 0.0)) / (le * Pe * p.Da_ib)
            R["Z"] = rZ / st.rho
        if chi is not None:
            rH = rH - chi * kap * (st.H - self.ib.get("H_ib", 0.0)) / (Pe * p.Da_ib)
        if p.p0_closed:
            rH = rH + p.zeta * dtp0
        R["H"] = rH / st.rho
        conv, visc = self._momentum_terms(vp, kapp, st.F)
        Rv = []
        for i in range(g.ndim):
            r = -conv[i] + (p.Pr / Pe) * visc[i]
            if i == 1 and p.inv_Fr2 != 0.0:
                r = r + p.inv_Fr2 * (1.0 - st.rho)
            if chi is not None:
                vib = self.ib.get("v_ib", [0.0] * g.ndim)[i]
                r = r - chi * (p.Pr / (Pe * p.Da_ib)) * kap * (st.v[i] - vib)
            Rv.append(r)
        R["v"] = Rv
        return R

    # -- projection ----------------------------------------------------------
    def project(self, M, rho_new, drho_dt, stage):
        """Solve for P and project (Eq 3.9-3.11, 3.17-3.19, 3.23-3.25, 3.33).

        Face flux G = avg(M) on interior faces and the prescribed flux on
        boundary faces; b = sum_d delta_1 G + d_t rho - S_m; the outflow flux
        is shifted uniformly so that sum(b) = 0 before the solve (global mass
        closure of section 4.5); P is the zero-mean solution of A P = b
        (P = p dt, Eq 3.8c); F = G - delta_1 P on interior faces;
        v = (M - delta_2 P)/rho_new with P ghosts by quadratic extrapolation
        at non-periodic sides (Eq 3.27)."""
        g = self.g
        Sm = self.ib.get("Sm")
        src = drho_dt if Sm is None else drho_dt - Sm
        G = []
        for d in range(g.ndim):
            Mp = g.pad(M[d])
            fill_ghosts(g, Mp, [(("periodic",),) * 2 if g.periodic(e) else (("extrap",),) * 2
                                for e in range(g.ndim)])
            Gd = self._face_interp(Mp, d)
            self._boundary_faces(Gd, d, M[d], None)
            G.append(Gd)
        # outflow correction: close the global mass balance exactly
        out_sides = [(d, s) for d in range(g.ndim) for s in (0, 1)
                     if not g.periodic(d) and g.bc[d][s] == "outflow"]
        if out_sides:
            div = sum((g.plus(G[d], d) - g.minus(G[d], d)) / g.along(d, g.wid[d][1:-1]) for d in range(g.ndim))
            total = g.integral(div + src)  # (complex under a complex-step tangent)
            area = 0.0
            for d, s in out_sides:
                area += g.volume / g.L[d]
            c = total / area
            for d, s in out_sides:
                f = g.n[d] if s == 1 else 0
                sign = -1.0 if s == 1 else 1.0
                G[d][g.face_index(d, f)] += sign * c
        b = sum((g.plus(G[d], d) - g.minus(G[d], d)) / g.along(d, g.wid[d][1:-1]) for d in range(g.ndim)) + src
        P, lam = self.poisson.solve(b)
        self.stats[stage + "_compat"] = lam
        Pp = g.pad(P)
        fill_ghosts(g, Pp, field_rules(g, "P"))
        F = []
        v = []
        for d in range(g.ndim):
            dP1 = (g.S(Pp, d, g.e(d)) - g.S(Pp, d, None)) / g.along(d, g.dfc[d])
            Fd = G[d] - dP1
            if not g.periodic(d):
                for s in (0, 1):
                    f = 0 if s == 0 else g.n[d]
                    Fd[g.face_index(d, f)] = G[d][g.face_index(d, f)]
            F.append(Fd)
            dP2 = (g.S(Pp, None, g.e(d)) - g.S(Pp, None, g.e(d, -1))) / g.along(d, g.d2[d])
            v.append((M[d] - dP2) / rho_new)
        return P, F, v, b

    # -- time step -------------------------------------------------------------
    def step(self, st: State) -> State:
        """One step n -> n+1 (section 3.1).

        Predictor: AB2 for Z, H and momentum (Eq 3.1, 3.3, 3.10), Euler on the
        first step (Heun start), T* and rho* from the EOS (Eq 3.6), BDF2
        d_t rho (Eq 3.11; BDF1 on the first step, a reading), Poisson and
        projection. Corrector: AM2 (Eq 3.12, 3.13, 3.18) with the predicted
        and level-n residuals, EOS (Eq 3.15), BDF2 d_t rho (Eq 3.19),
        Poisson and projection. The level-(n-1) residuals are the ones cached
        from the previous step's level n (Eq 3.3 prints v^n inside the
        level-(n-1) residual; v^{n-1} is read, consistent with Eq 3.1, 3.7).
        Enclosed systems (p0_closed): p0* and p0^{n+1} from the conserved
        mass (Eq 2.40) before rho* and rho^{n+1} (Eq 3.6, 3.15), and the
        residuals carry zeta d_t p0 at their level (Eq 3.4b, 3.5, 3.14)."""
        g, p, fp = self.g, self.p, self.fp
        dt = self.dt
        closed = p.p0_closed == 1
        ode = p.p0_closed == 2
        first = st.R_prev is None
        if ode:
            # semi-enclosed: p0 integrated from Eq 2.38 like the other
            # unknowns (AB2 predictor, Euler on the first step; trapezoid
            # corrector); its rate is the d_t p0 of each level's residual
            f_n = self.p0_rate(st)
            Rn = self.residuals(st, f_n)
        elif closed and not st.p0_hist:
            Rn = self.residuals(st, self.balance_ddt_p0(st))
        else:
            Rn = self.residuals(st, self.ddt_p0(st.p0, st.p0_hist, st.dt_prev, st.dt_prev2) if closed else 0.0)
        M0 = [st.rho * st.v[i] for i in range(g.ndim)]
        adaptive = p.dt_tol > 0.0
        # ratio of this step to the previous one (adaptive steps)
        w = dt / st.dt_prev if (adaptive and st.dt_prev > 0.0) else 1.0

        def ab2(x, rn, rp):
            if first:
                return x + dt * rn
            if adaptive:
                # Adams-Bashforth 2 for unequal steps: the residual
                # extrapolated linearly through t_{n-1}, t_n and integrated
                # over [t_n, t_n + dt]
                return x + dt * ((1.0 + 0.5 * w) * rn - 0.5 * w * rp)
            return x + dt * (1.5 * rn - 0.5 * rp)

        def am2(x, rs, rn):
            return x + 0.5 * dt * (rs + rn)

        def ddt(rnew):
            if st.rho_prev is None:
                return (rnew - st.rho) / dt
            if adaptive:
                # BDF2 for unequal steps: derivative at t_{n+1} of the
                # quadratic through (t_{n-1}, t_n, t_{n+1}), written with
                # the level differences (the weights of rho^{n+1}, rho^n,
                # rho^{n-1} are (1+2w)/(1+w), -(1+w), w^2/(1+w), over dt)
                return ((1.0 + 2.0 * w) / (1.0 + w) * (rnew - st.rho)
                        - w * w / (1.0 + w) * (st.rho - st.rho_prev)) / dt
            return (3.0 * rnew - 4.0 * st.rho + st.rho_prev) / (2.0 * dt)

        # ---- predictor
        Rp = st.R_prev or {}
        Hs = ab2(st.H, Rn["H"], Rp.get("H"))
        Zs = ab2(st.Z, Rn["Z"], Rp.get("Z")) if p.reacting else None
        Ms = [ab2(M0[i], Rn["v"][i], None if first else Rp["v"][i]) for i in range(g.ndim)]
        Ts = temperature(Zs if Zs is not None else 0.0, Hs, fp)
        if ode:
            if first:
                p0s = st.p0 + dt * f_n
            elif adaptive:
                p0s = st.p0 + dt * ((1.0 + 0.5 * w) * f_n - 0.5 * w * st.p0_rate_prev)
            else:
                p0s = st.p0 + dt * (1.5 * f_n - 0.5 * st.p0_rate_prev)
        else:
            p0s = self.closed_p0(Ts) if closed else p.p0
        rhos = p0s / Ts
        Ps, Fs, vs, bs = self.project(Ms, rhos, ddt(rhos), "pred")
        sts = State(rhos, vs, Zs, Hs, Ts, Ps, Fs, p0=p0s)
        # ---- corrector
        hist_s = (st.p0,) + tuple(st.p0_hist[:1])
        if ode:
            f_s = self.p0_rate(sts)
            Rs = self.residuals(sts, f_s)
        else:
            Rs = self.residuals(sts, self.ddt_p0(p0s, hist_s, dt, st.dt_prev) if closed else 0.0)
        H1 = am2(st.H, Rs["H"], Rn["H"])
        Z1 = am2(st.Z, Rs["Z"], Rn["Z"]) if p.reacting else None
        M1 = [am2(M0[i], Rs["v"][i], Rn["v"][i]) for i in range(g.ndim)]
        T1 = temperature(Z1 if Z1 is not None else 0.0, H1, fp)
        if ode:
            p01 = st.p0 + 0.5 * dt * (f_s + f_n)
        else:
            p01 = self.closed_p0(T1) if closed else p.p0
        rho1 = p01 / T1
        P1, F1, v1, b1 = self.project(M1, rho1, ddt(rho1), "corr")
        out = State(rho1, v1, Z1, H1, T1, P1, F1, rho_prev=st.rho, R_prev=Rn,
                    nstep=st.nstep + 1, p0=p01, p0_hist=(st.p0,) + tuple(st.p0_hist[:1]), dt_prev=dt,
                    p0_rate_prev=f_n if ode else None, dt_prev2=st.dt_prev)
        rms = lambda a: float(np.sqrt(np.mean(np.abs(a) ** 2)))
        self.stats["pc_diff_v"] = [rms(vs[i] - v1[i]) for i in range(g.ndim)]
        self.stats["pc_diff_P"] = rms(Ps - P1)
        self.stats["pc_diff_H"] = rms(Hs - H1)
        self.last_predicted = sts
        if adaptive:
            err = self.pc_error(sts, out)
            self.stats["pc_err"] = err
            self.stats["dt"] = dt
            out.nsame = st.nsame + 1 if (not first and dt == st.dt_prev) else 1
            clean = out.nsame >= 4
            self.stats["pc_err_clean"] = clean
            self.dt = self.next_dt(dt, err, out, clean)
        return out

    def pc_error(self, sts: State, out: State):
        """Local error estimate of a step: the difference between the
        predicted and corrected levels (the estimate behind Tab 2, which
        the paper proposes for adaptive steps): the largest of the RMS of
        |v* - v^{n+1}| (vector norm), the RMS of H* - H^{n+1} and, with
        reaction, the RMS of Z* - Z^{n+1} over S + 1."""
        dv2 = sum((a - b) ** 2 for a, b in zip(sts.v, out.v))
        err = max(math.sqrt(float(np.mean(dv2))), math.sqrt(float(np.mean((sts.H - out.H) ** 2))))
        if self.p.reacting:
            err = max(err, math.sqrt(float(np.mean((sts.Z - out.Z) ** 2))) / (self.p.S + 1.0))
        return err

    def next_dt(self, dt, err, st: State, clean=True):
        """Adaptive step (a reading; the paper only names the estimate).
        The local error of the AB2/AM2 pair is O(dt^3): a decision takes
        the factor 0.9 (dt_tol / err)^{1/3} kept in [0.5, 1.5] (1.5 when
        err = 0) and applies it only outside [0.9, 1.1], so that the step
        stays put while the estimate lies between about 0.55 and 1.0 times
        dt_tol. Only the estimate of the fourth or a later step of exactly
        one size decides: on the collocated grid the cell velocity keeps an
        O(h^2) part proportional to the step (the projection subtracts
        delta_2 P, P = p dt), so levels made by steps of different sizes
        differ by O(h^2 |dt - dt_prev|), which the AB2 extrapolation of the
        next two steps turns into an O(h^2 dt |dt - dt_prev|) term of the
        estimate (decaying by about two orders per step after that); the
        Euler-predicted start behaves alike. The step never exceeds the CFL
        step of the new state: growth stops at it, and when it falls below
        the current step the step drops to 0.9 of it. No step is
        rejected."""
        cap = self.cfl_dt(st)
        new = dt
        if clean:
            fac = 1.5 if err <= 0.0 else min(1.5, max(0.5, 0.9 * (self.p.dt_tol / err) ** (1.0 / 3.0)))
            if fac <= 0.9 or fac >= 1.1:
                new = min(dt * fac, cap)
        if new > cap:
            new = 0.9 * cap
        return new

    def run(self, st: State, nsteps: int) -> State:
        for _ in range(nsteps):
            st = self.step(st)
        return st
