"""Oracle pins for the regularised flame sheet (section 3.5, Eq 3.34-3.42)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.flame import FlameParams, f_eps, f_tilde, temperature, enthalpy_from_T, theta_eps, le_eps, n_eps

S_C3 = 1.0 / 0.055 - 1.0


def fp(**kw):
    d = dict(S=S_C3, qs=1.0, eps=0.5, tol=1e-3, reacting=True)
    d.update(kw)
    return FlameParams(**d)


def test_theta_hits_tolerance_at_plus_minus_eps():
    """k is chosen so theta_eps(+-eps) = 1 - tol, tol (section 3.5)."""
    p = fp()
    assert abs(theta_eps(np.float64(p.eps), p) - (1 - p.tol)) < 1e-14
    assert abs(theta_eps(np.float64(-p.eps), p) - p.tol) < 1e-14
    assert abs(p.k - 6.906754778648554) < 1e-12


def test_f_eps_vanishes_at_flame():
    assert f_eps(np.float64(1.0), fp()) == 0.0


def test_f_eps_is_integral_of_regularised_derivative():
    """Eq 3.41 equals the quadrature of Eq 3.40 (integrand Eq 3.39)."""
    p = fp()
    for Z in (0.0, 0.4, 0.97, 1.2, 3.0, S_C3 + 1):
        val, _ = quad(lambda z: -(1 / p.S + 1) * theta_eps(z - 1, p) + 1, 1.0, Z,
                      epsabs=1e-13, epsrel=1e-13, limit=200)
        assert abs(f_eps(np.float64(Z), p) - val) < 1e-10


def test_f_eps_tends_to_sheet_limit():
    """As k -> infinity (tol -> 0 at fixed eps), F_eps -> F (Eq 3.37)."""
    p = fp(tol=1e-300)
    for Z in (0.0, 0.5, 2.0, 10.0):
        F = (Z - 1) if Z <= 1 else (1 - Z) / p.S
        # |ln cosh x - |x|| <= ln 2, so |F_eps - F| <= (S+1) ln 2 / (2 S k)
        assert abs(f_eps(np.float64(Z), p) - F) <= (p.S + 1) * math.log(2) / (2 * p.S * p.k) * (1 + 1e-9)
    p2 = fp(eps=1e-4)
    for Z in (0.0, 0.5, 2.0, 10.0):
        F = (Z - 1) if Z <= 1 else (1 - Z) / p2.S
        assert abs(f_eps(np.float64(Z), p2) - F) < 1e-4


def test_translated_levels_and_maximum():
    """F~(0) = -1 exactly, F~(S+1) = -1 to O(e^{-2kS}); argmax at
    Z = 1 + ln S/(2k), where F~' = 0 by Eq 3.39."""
    p = fp()
    assert f_tilde(np.float64(0.0), p) == -1.0
    assert abs(f_tilde(np.float64(S_C3 + 1), p) + 1) < 1e-6
    zmax = 1 + math.log(p.S) / (2 * p.k)
    zs = np.linspace(zmax - 1e-3, zmax + 1e-3, 2001)
    assert abs(zs[np.argmax(f_tilde(zs, p))] - zmax) < 2e-6


def test_c3_calibration_gives_peak_temperature_seven():
    """Q/(S+1) = 6 / (1 + F~(Z_max)) gives T_max = 7 at H = H_inf, with
    T = 1 in the oxidiser (Z = 0)."""
    p0 = fp()
    zmax = 1 + math.log(p0.S) / (2 * p0.k)
    qs = 6.0 / (1.0 + f_tilde(np.float64(zmax), p0))
    p = fp(qs=qs)
    Hinf = 1.0 / qs + 1.0
    assert abs(temperature(np.float64(0.0), Hinf, p) - 1.0) < 1e-14
    assert abs(temperature(np.float64(zmax), Hinf, p) - 7.0) < 1e-12
    z = np.linspace(0, S_C3 + 1, 20001)
    assert np.max(temperature(z, Hinf, p)) <= 7.0 + 1e-12


def test_temperature_inverse_roundtrip():
    p = fp(qs=3.0)
    Z = np.linspace(0, S_C3 + 1, 50)
    T = 1 + np.linspace(0, 5, 50)
    H = enthalpy_from_T(T, Z, p)
    assert np.max(np.abs(temperature(Z, H, p) - T)) < 1e-13
    pn = FlameParams(reacting=False)
    assert np.max(np.abs(temperature(0.0, enthalpy_from_T(T, 0.0, pn), pn) - T)) < 1e-14


def test_lewis_and_n_coefficients_limits():
    """Eq 3.35 with N_F = (1 - Le_F)/(S Le_F), N_O = (Le_O - 1)/Le_O."""
    p = fp(Le_F=0.97, Le_O=1.11)
    assert abs(le_eps(np.float64(-5.0), p) - 1.11) < 1e-12
    assert abs(le_eps(np.float64(10.0), p) - 0.97) < 1e-12
    assert abs(n_eps(np.float64(10.0), p) - (1 - 0.97) / (p.S * 0.97)) < 1e-12
    assert abs(n_eps(np.float64(-5.0), p) - (1.11 - 1) / 1.11) < 1e-12
    pe = fp()
    assert np.all(n_eps(np.linspace(0, 5, 9), pe) == 0.0)


def test_lncosh_sign_form_is_abs_form_and_complex_differentiable():
    """ln cosh takes |x| as x sign(Re x): on real input the same bits as
    the |x| form; under a complex step the derivative of F_eps is the
    regularised dF/dZ = -(1/S + 1) theta_eps(Z - 1) + 1 (Eq 3.39), which a
    wrong sign choice (the derivative of ln cosh is tanh, odd) would flip on
    one side of the flame."""
    from oracle.flame import _lncosh
    x = np.concatenate([np.linspace(-40.0, 40.0, 801), [0.0, -0.0, 1e-300, -1e-300, 700.0, -700.0]])
    ax = np.abs(x)
    ref = ax + np.log1p(np.exp(-2.0 * ax)) - math.log(2.0)
    assert np.array_equal(_lncosh(x), ref)
    p = fp(S=2.0)
    Z = np.array([0.05, 0.5, 0.9, 0.99, 1.01, 1.1, 1.5, 2.9])
    h = 1e-30
    d = f_eps(Z + 1j * h, p).imag / h
    closed = -(1.0 / p.S + 1.0) * theta_eps(Z - 1.0, p) + 1.0
    assert np.max(np.abs(d - closed)) < 1e-13
