"""Flame-sheet regularisation (section 3.5, Eq 3.34-3.42) and the T(Z, H) map.

TEST INFRASTRUCTURE ONLY (see the package header).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class FlameParams:
    """S: generalised stoichiometric coefficient; qs = Q/(S+1); eps and tol
    set the regularisation width k = ln((1 - tol)/tol)/(2 eps) (section 3.5);
    Le_F, Le_O: fuel and oxidiser Lewis numbers (Eq 2.47, 3.35)."""
    S: float = 1.0
    qs: float = 1.0
    eps: float = 0.5
    tol: float = 1e-3
    Le_F: float = 1.0
    Le_O: float = 1.0
    reacting: bool = False

    @property
    def k(self):
        return math.log((1.0 - self.tol) / self.tol) / (2.0 * self.eps)


def theta_eps(z_minus_1, fp: FlameParams):
    """Regularised Heaviside (Eq 3.34) about the flame level Z = 1."""
    return 0.5 * (1.0 + np.tanh(fp.k * z_minus_1))


def le_eps(Z, fp: FlameParams):
    """Eq 3.35a: Le_eps = (Le_F - Le_O) theta_eps(Z - 1) + Le_O."""
    return (fp.Le_F - fp.Le_O) * theta_eps(Z - 1.0, fp) + fp.Le_O


def n_eps(Z, fp: FlameParams):
    """Eq 3.35b with N_F = (1 - Le_F)/(S Le_F), N_O = (Le_O - 1)/Le_O (Eq 2.37)."""
    nf = (1.0 - fp.Le_F) / (fp.S * fp.Le_F)
    no = (fp.Le_O - 1.0) / fp.Le_O
    return (nf - no) * theta_eps(Z - 1.0, fp) + no


def n_prime_eps(Z, fp: FlameParams):
    """N' of Eq 2.39 (N'_F = -1/S, N'_O = 1), regularised like Eq 3.35:
    (N'_F - N'_O) theta_eps(Z - 1) + N'_O."""
    return (-1.0 / fp.S - 1.0) * theta_eps(Z - 1.0, fp) + 1.0


def _lncosh(x):
    """ln cosh x written as |x| + log1p(exp(-2|x|)) - ln 2 (no overflow).
    |x| is formed as x times the sign of its real part: the same number for
    real x, and analytic in x near the real axis (away from 0, where ln cosh
    is even and smooth), so a complex-step derivative passes through."""
    ax = x * np.where(np.real(x) < 0.0, -1.0, 1.0)
    return ax + np.log1p(np.exp(-2.0 * ax)) - math.log(2.0)


def f_eps(Z, fp: FlameParams):
    """Closed form of the regularised F (Eq 3.41):
    F_eps = [-(S+1) ln cosh(k (Z-1))/k + (S-1)(Z-1)] / (2 S)."""
    S, k = fp.S, fp.k
    return (-(S + 1.0) * _lncosh(k * (Z - 1.0)) / k + (S - 1.0) * (Z - 1.0)) / (2.0 * S)


def f_tilde(Z, fp: FlameParams):
    """F_eps translated so that the oxidiser boundary value is exact:
    F~(0) = -1 = F(0) (Eq 3.37); section 3.5 asks for a translation of
    F_eps to the boundary values but does not fix it, so the constant is
    c = -1 - F_eps(0)."""
    c = -1.0 - float(f_eps(np.float64(0.0), fp))
    return f_eps(Z, fp) + c


def temperature(Z, H, fp: FlameParams):
    """T = Q/(S+1) (F~(Z) + H) (Eq 3.42); without reaction Z = 0 and
    F(0) = -1 (Eq 3.37), so T = Q/(S+1) (H - 1)."""
    if not fp.reacting:
        return fp.qs * (H - 1.0)
    return fp.qs * (f_tilde(Z, fp) + H)


def enthalpy_from_T(T, Z, fp: FlameParams):
    """Inverse of the map above: H = T/(Q/(S+1)) - F~(Z)."""
    if not fp.reacting:
        return T / fp.qs + 1.0
    return T / fp.qs - f_tilde(Z, fp)
