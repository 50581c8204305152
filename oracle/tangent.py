"""Complex-step tangent-linear derivatives of the oracle step.

TEST INFRASTRUCTURE ONLY (see the package header).

For a real-analytic map f, f'(x) d = Im f(x + i h d) / h + O(h^2), with no
subtractive cancellation, so h can be taken tiny (1e-30 here) and the
directional derivative is exact to rounding (complex-step differentiation,
Squire and Trapp 1998). The oracle's step runs on complex fields unchanged
for the non-reacting periodic configuration (only +, -, *, /, powers and
FFTs act on the fields; the flame map's ln cosh takes |x| as x sign(Re x),
analytic near the real axis, and the ghost clamp of Z to [0, S+1] is the
identity on fields inside that range). The time step must be fixed
(``Params.dt > 0``): a CFL step would depend on the perturbed fields
through |v|.
"""
from __future__ import annotations

import numpy as np

from .flame import temperature
from .grid import Grid
from .step import Oracle, Params, State

H_CS = 1e-30


def kinetic_energy(g: Grid, st: State):
    """J = sum over cells of 1/2 rho |v|^2 dV (no complex conjugate: J stays
    analytic in the fields)."""
    return 0.5 * sum(np.sum(st.rho * a * a) for a in st.v) * g.dV


def final_kinetic_energy(g: Grid, p: Params, T0, v0, nsteps: int, ib=None, Z0=None):
    """J after nsteps steps from (T0, v0) (and Z0 in reacting flow); ``ib``:
    the immersed-body arrays (constants of the run)."""
    if not p.dt > 0:
        raise ValueError("complex-step derivatives need a fixed dt")
    o = Oracle(g, p, ib=ib)
    st = o.run(o.initial_state(T0, v0, Z=Z0), nsteps)
    return kinetic_energy(g, st)


def ke_directional(g: Grid, p: Params, T0, v0, dT, nsteps: int, h: float = H_CS, ib=None, Z0=None,
                   dZ=None) -> float:
    """dJ/d(T0, Z0) . (dT, dZ) by one complex-step run (dZ: reacting flow)."""
    Z = None if Z0 is None else np.asarray(Z0) + (0.0 if dZ is None else 1j * h * np.asarray(dZ))
    J = final_kinetic_energy(g, p, np.asarray(T0) + 1j * h * np.asarray(dT), v0, nsteps, ib=ib, Z0=Z)
    return float(J.imag / h)


def with_eos(o: Oracle, st: State) -> State:
    """The state with T and rho re-evaluated from H (Eq 3.42, 2.49): the
    level fields that follow from H, so that a perturbation of H carries
    through them."""
    st.T = temperature(st.Z if o.p.reacting else 0.0, st.H, o.fp)
    st.rho = o.p.p0 / st.T
    return st


def step_tangent(o: Oracle, st: State, dx: dict, h: float = H_CS) -> dict:
    """Tangent of one step along dx = {H, v, F, rho_prev, R_H, R_v} (and
    Z, R_Z in reacting flow; each entry optional) at a state with history
    (st.R_prev set). Returns the tangents of the outputs {H, v, F, rho_prev,
    R_H, R_v} (and Z, R_Z) of the step, where rho_prev and R_* of the output
    are the level-n density and residuals the next step reads."""
    s = st.copy()
    cplx = lambda a: a.astype(np.complex128)
    s.H = cplx(s.H) + 1j * h * dx.get("H", 0.0)
    react = o.p.reacting
    if react:
        s.Z = cplx(s.Z) + 1j * h * dx.get("Z", 0.0)
    s.v = [cplx(a) + 1j * h * (dx["v"][d] if "v" in dx else 0.0) for d, a in enumerate(s.v)]
    s.F = [cplx(a) + 1j * h * (dx["F"][d] if "F" in dx else 0.0) for d, a in enumerate(s.F)]
    if s.rho_prev is not None:
        s.rho_prev = cplx(s.rho_prev) + 1j * h * dx.get("rho_prev", 0.0)
    if s.R_prev is not None:
        s.R_prev = dict(s.R_prev)
        s.R_prev["H"] = cplx(s.R_prev["H"]) + 1j * h * dx.get("R_H", 0.0)
        if react:
            s.R_prev["Z"] = cplx(s.R_prev["Z"]) + 1j * h * dx.get("R_Z", 0.0)
        s.R_prev["v"] = [cplx(a) + 1j * h * (dx["R_v"][d] if "R_v" in dx else 0.0)
                         for d, a in enumerate(s.R_prev["v"])]
    with_eos(o, s)
    out = o.step(s)
    im = lambda a: a.imag / h
    y = dict(H=im(out.H), v=[im(a) for a in out.v], F=[im(a) for a in out.F],
             rho_prev=im(out.rho_prev), R_H=im(out.R_prev["H"]),
             R_v=[im(a) for a in out.R_prev["v"]])
    if react:
        y["Z"] = im(out.Z)
        y["R_Z"] = im(out.R_prev["Z"])
    return y
