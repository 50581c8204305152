"""Helpers shared by the parity tests: build the oracle and the GPU solver
from one seeded workload and compare their fields."""
import math

import numpy as np

from oracle import Grid, Oracle, Params
from workloads import Case

PARAM_KEYS = ("Re", "Pr", "sigma", "inv_Fr2", "reacting", "S", "qs", "eps", "tol", "Le_F", "Le_O",
              "Da_ib", "p0", "dt", "cfl", "p0_closed", "gamma",
              "sutherland_C", "dt_tol")
SIDE_INDEX = {"slip", "noslip", "inflow", "outflow"}


def _params(case: Case, over):
    d = dict(case.params)
    d.update(over)
    return {k: d[k] for k in PARAM_KEYS if k in d}


def oracle_for(case: Case, **over):
    nd = case.ndim
    g = Grid(case.n[:nd], case.L[:nd], bc=case.bc, bnd=case.bnd, faces=case.faces)
    o = Oracle(g, Params(**_params(case, over)), ib=case.ib)
    st = o.initial_state(case.T, case.v, Z=case.Z, H=case.H)
    return o, st


def gpu_for(case: Case, rtol=1e-13, precision="fp64", **over):
    from paper_2603_01727_amd import Solver
    nd = case.ndim
    s = Solver(case.n[:nd], case.L[:nd], bc=case.bc, precision=precision, poisson_rtol=rtol,
               poisson_maxit=400, with_ib=case.ib is not None, faces=case.faces, **_params(case, over))
    for (d, side), data in (case.bnd or {}).items():
        s.set_side(d, side, v=data.get("v"), Z=data.get("Z"), H=data.get("H"), F=data.get("F"),
                   wall=data.get("wall"))
    s.set(T=case.T, H=case.H if case.T is None else None, v=case.v, Z=case.Z, ib=case.ib)
    return s


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = math.sqrt(float(np.sum(b * b)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / (nb if nb > 0 else 1.0)


def compare(st, got):
    """Per-field relative L2 errors between an oracle State and GPU fields
    (numpy arrays as returned by Solver.get(device=False))."""
    err = {"rho": rel_l2(got["rho"], st.rho), "H": rel_l2(got["H"], st.H), "T": rel_l2(got["T"], st.T),
           "P": rel_l2(got["P"], st.P)}
    for d in range(len(st.v)):
        err[f"v{d}"] = rel_l2(got["v"][d], st.v[d])
        err[f"F{d}"] = rel_l2(got["F"][d], st.F[d])
    if st.Z is not None and "Z" in got:
        err["Z"] = rel_l2(got["Z"], st.Z)
    return err
