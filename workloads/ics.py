"""Initial conditions for the five synthetic workloads.

Workload sizes and distributions follow the configurations the method is
exercised on (periodic Taylor-Green/hot-spot boxes, random-mode variable-density
boxes in 2D and 3D, and a slot-burner flame with an immersed boundary). The
paper's own experiments (Taylor-Green vortex, section 4.2; double Tsuji flame,
section 4.5) are analytic or need data that is not available, so these seeded
fields stand in for them.

Random draws: ``numpy.random.default_rng(seed)``; the order of draws is fixed
and documented in each generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


# Q/(S+1) for S = 1/0.055 - 1, eps = 0.5, tol = 1e-3: 6 / (1 + F~(Z_max)) with
# Z_max = 1 + ln S/(2k), so that the peak regularised temperature is 7.
QS_C3 = 6.09951783620629


@dataclasses.dataclass
class Case:
    """A workload: grid, physical parameters and initial fields.

    ``T`` is temperature at cell centres, ``v`` a list of velocity components,
    ``Z`` the mixture fraction (None for non-reacting cases). ``ib`` holds the
    immersed-boundary arrays (mask, targets, mass source) and ``bnd`` the
    boundary arrays for non-periodic sides, both None for periodic boxes.
    """
    name: str
    ndim: int
    n: tuple
    L: tuple
    bc: tuple                 # per dim: ("periodic","periodic") or side kinds
    params: dict
    T: np.ndarray
    v: list
    Z: Optional[np.ndarray] = None
    ib: Optional[dict] = None
    bnd: Optional[dict] = None
    nsteps: int = 1
    H: Optional[np.ndarray] = None
    faces: Optional[list] = None  # per dim: None (uniform) or the n + 1 face coordinates

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.ndim]))

    @property
    def ncells(self):
        return int(np.prod(self.n[: self.ndim]))


def cell_centres(n, L):
    """Cell-centre coordinates x_i = (i + 1/2) * L / n for each direction,
    returned as broadcastable arrays in (z, y, x) axis order."""
    ndim = len(n)
    out = []
    for d in range(ndim):
        h = L[d] / n[d]
        c = (np.arange(n[d]) + 0.5) * h
        shp = [1] * ndim
        shp[ndim - 1 - d] = n[d]
        out.append(c.reshape(shp))
    return out  # out[d] varies along direction d


def taylor_green(n, L, t=0.0, Re=100.0):
    """Taylor-Green vortex on a periodic square of side L (section 4.2,
    Eq 4.4-4.6 written for side L): wavenumber a = 2*pi/L,
    v1 = sin(a x) cos(a y) e^{-2 a^2 t/Re}, v2 = -cos(a x) sin(a y) e^{-2 a^2 t/Re},
    p = (cos(2 a x) + cos(2 a y))/4 e^{-4 a^2 t/Re}."""
    x, y = cell_centres(n, L)
    a = 2.0 * math.pi / L[0]
    dv = math.exp(-2.0 * a * a * t / Re)
    dp = math.exp(-4.0 * a * a * t / Re)
    v1 = np.sin(a * x) * np.cos(a * y) * dv
    v2 = -np.cos(a * x) * np.sin(a * y) * dv
    p = 0.25 * (np.cos(2 * a * x) + np.cos(2 * a * y)) * dp
    shp = (n[1], n[0])
    return np.broadcast_to(v1, shp).copy(), np.broadcast_to(v2, shp).copy(), \
        np.broadcast_to(p, shp).copy()


def hot_spot_tg(n, seed, amp=4.0, r2scale=0.25, noise_T=1e-3, noise_v=1e-2):
    """Hot spot T = 1 + amp*exp(-r^2/r2scale) centred in a periodic 2*pi box,
    plus U(-noise_T, noise_T) per cell, on a Taylor-Green velocity plus
    N(0, noise_v^2) per component and cell.
    Draw order: T noise (ny, nx), then v noise (2, ny, nx)."""
    L = (2 * math.pi, 2 * math.pi)
    x, y = cell_centres(n, L)
    rng = np.random.default_rng(seed)
    r2 = (x - math.pi) ** 2 + (y - math.pi) ** 2
    T = 1.0 + amp * np.exp(-r2 / r2scale)
    T = T + rng.uniform(-noise_T, noise_T, size=(n[1], n[0]))
    v1 = np.sin(x) * np.cos(y)
    v2 = -np.cos(x) * np.sin(y)
    nz = rng.normal(0.0, noise_v, size=(2, n[1], n[0]))
    return T, [v1 + nz[0], v2 + nz[1]]


def _wavevectors(ndim, kmax):
    """All integer wavevectors k != 0 with |k| <= kmax, in lexicographic order."""
    rng1 = range(-kmax, kmax + 1)
    if ndim == 2:
        ks = [(a, b) for a in rng1 for b in rng1]
    else:
        ks = [(a, b, c) for a in rng1 for b in rng1 for c in rng1]
    ks = [k for k in ks if any(k) and sum(q * q for q in k) <= kmax * kmax]
    return np.array(ks, dtype=np.int64)


def _mode_sum(n, ks, coef):
    """Re sum_m coef_m exp(i theta_m(x)) at the cell centres, theta_m(x) =
    sum_d 2 pi k_md x_d / L_d with x_d = (i_d + 1/2) L_d / n_d, by one
    inverse FFT: exp(i theta) = prod_d exp(i pi k_d / n_d) exp(2 pi i k_d i_d / n_d)."""
    ndim = len(n)
    shp = tuple(reversed(n))
    C = np.zeros(shp, dtype=np.complex128)
    for q in range(len(ks)):
        k = ks[q]
        c = complex(coef[q])
        for d in range(ndim):
            c *= np.exp(1j * math.pi * k[d] / n[d])
        idx = tuple(int(k[ndim - 1 - a]) % n[ndim - 1 - a] for a in range(ndim))
        C[idx] += c
    return np.fft.ifftn(C).real * float(np.prod(shp))


def fourier_temperature(n, L, rng, kmax, amp, m=32):
    """T = 1 + amp * fhat, fhat = (f - min f)/(max f - min f),
    f = sum_m a_m cos(k_m . x + phi_m) over m wavevectors drawn without
    replacement from {k != 0, |k| <= kmax}, a_m ~ U(0,1), phi_m ~ U(0, 2 pi).
    Draw order: indices (m), amplitudes (m), phases (m)."""
    ks = _wavevectors(len(n), kmax)
    idx = rng.choice(len(ks), size=m, replace=False)
    a = rng.random(m)
    ph = 2 * math.pi * rng.random(m)
    f = _mode_sum(n, ks[idx], a * np.exp(1j * ph))
    fh = (f - f.min()) / (f.max() - f.min())
    return 1.0 + amp * fh


def variable_coefficient_problem(n, L, seed, kmax=8, ratio=4.0, m=32):
    """Inputs of a variable-coefficient Poisson solve div(grad P / rho) = b
    shaped like the step's: a density field of random modes with
    max/min = ratio (rho = 1/ratio + (1 - 1/ratio)(1 - fhat), fhat as in
    fourier_temperature) and a right-hand side of random modes (values in
    [0, 1], mean not removed). Draws: the density's modes, then b's."""
    rng = np.random.default_rng(seed)
    fh = fourier_temperature(n, L, rng, kmax, 1.0, m=m) - 1.0
    rho = 1.0 / ratio + (1.0 - 1.0 / ratio) * (1.0 - fh)
    b = fourier_temperature(n, L, rng, kmax, 1.0, m=m) - 1.0
    return rho, b


def solenoidal_velocity(n, L, rng, kmax, rms=0.1, m=32):
    """Divergence-free random velocity, scaled to (mean |v|^2)^(1/2) = rms.

    2D: streamfunction psi = sum a cos(k.x + phi); v = (d psi/dy, -d psi/dx),
    differentiated analytically. Draws: indices, amplitudes, phases.
    3D: v = sum [c_m cos(k.x) + s_m sin(k.x)] with c_m, s_m ~ N(0,1)^3
    projected orthogonal to k. Draws: indices, c (m,3), s (m,3)."""
    ndim = len(n)
    ks = _wavevectors(ndim, kmax)
    idx = rng.choice(len(ks), size=m, replace=False)
    km = ks[idx]
    if ndim == 2:
        a = rng.random(m)
        ph = 2 * math.pi * rng.random(m)
        kx = 2 * math.pi / L[0] * km[:, 0]
        ky = 2 * math.pi / L[1] * km[:, 1]
        e = a * np.exp(1j * ph)
        # -a ky sin(theta + phi) and a kx sin(theta + phi), sin(u) = Re(-i e^{iu})
        v = [_mode_sum(n, km, 1j * ky * e), _mode_sum(n, km, -1j * kx * e)]
    else:
        c = rng.normal(size=(m, 3))
        sn = rng.normal(size=(m, 3))
        coef = np.zeros((3, m), dtype=np.complex128)
        for q in range(m):
            kp = np.array([2 * math.pi / L[d] * km[q][d] for d in range(3)])
            kk = kp / np.linalg.norm(kp)
            cq = c[q] - kk * (kk @ c[q])
            sq = sn[q] - kk * (kk @ sn[q])
            # cq cos(theta) + sq sin(theta) = Re((cq - i sq) e^{i theta})
            coef[:, q] = cq - 1j * sq
        v = [_mode_sum(n, km, coef[d]) for d in range(3)]
    e = math.sqrt(float(np.mean(sum(x * x for x in v))))
    return [x * (rms / e) for x in v]


def c1_case(n=64, seed=1):
    """2D periodic 2*pi box, 64^2: hot spot T = 1 + 4 exp(-r^2/0.25) with
    U(-1e-3, 1e-3) noise, Taylor-Green velocity with N(0, 1e-2^2) noise,
    Re=100, Pr=0.7, CFL 0.2, one step, Poisson to 1e-12."""
    T, v = hot_spot_tg((n, n), seed)
    L = (2 * math.pi, 2 * math.pi)
    return Case("c1_hotspot_tg_64", 2, (n, n, 1), L + (1.0,),
                (("periodic", "periodic"),) * 2,
                dict(Re=100.0, Pr=0.7, cfl=0.2, poisson_rtol=1e-12), T, v,
                nsteps=1)


def c2_case(n=1024, seed=2):
    """2D periodic 2*pi box, 1024^2: T = 1 + 3 fhat (32 modes, |k| <= 8),
    solenoidal velocity |k| <= 8 rms 0.1, Re=500, Pr=0.7, CFL 0.3,
    100 steps, Poisson to 1e-10. Draws: temperature, then velocity."""
    L = (2 * math.pi, 2 * math.pi)
    rng = np.random.default_rng(seed)
    T = fourier_temperature((n, n), L, rng, 8, 3.0)
    v = solenoidal_velocity((n, n), L, rng, 8, 0.1)
    return Case("c2_random_modes_1024", 2, (n, n, 1), L + (1.0,),
                (("periodic", "periodic"),) * 2,
                dict(Re=500.0, Pr=0.7, cfl=0.3, poisson_rtol=1e-10), T, v,
                nsteps=100)


def c4_case(n=256, seed=4):
    """3D periodic 2*pi box, 256^3: T = 1 + 5 fhat (32 modes, |k| <= 6),
    solenoidal velocity |k| <= 6 rms 0.1, Re=400, Pr=0.7, 50 steps,
    Poisson to 1e-10 (CFL 0.3 is the reading for the unstated CFL)."""
    L = (2 * math.pi,) * 3
    rng = np.random.default_rng(seed)
    T = fourier_temperature((n, n, n), L, rng, 6, 5.0)
    v = solenoidal_velocity((n, n, n), L, rng, 6, 0.1)
    return Case("c4_random_modes_256cube", 3, (n, n, n), L,
                (("periodic", "periodic"),) * 3,
                dict(Re=400.0, Pr=0.7, cfl=0.3, poisson_rtol=1e-10), T, v,
                nsteps=50)


def c5_case(n=512, seed=5):
    """2D periodic 2*pi box, 512^2 for the adjoint: T0 = 1 + 3 fhat
    (32 modes, |k| <= 8), solenoidal velocity rms 0.1, Re=300, Pr=0.7,
    200 steps, checkpoint every 20 (CFL 0.3 is the reading)."""
    L = (2 * math.pi, 2 * math.pi)
    rng = np.random.default_rng(seed)
    T = fourier_temperature((n, n), L, rng, 8, 3.0)
    v = solenoidal_velocity((n, n), L, rng, 8, 0.1)
    return Case("c5_adjoint_512", 2, (n, n, 1), L + (1.0,),
                (("periodic", "periodic"),) * 2,
                dict(Re=300.0, Pr=0.7, cfl=0.3, poisson_rtol=1e-10), T, v,
                nsteps=200)


def reacting_periodic_case(n=(64, 64), seed=6, S=2.0, Le_F=0.8, Le_O=1.2):
    """Periodic 2*pi box in 2D or 3D (n = (nx, ny[, nz])) with a reacting
    mixture: T = 1 + 2 fhat and Z = 0.2 + 1.6 fhat' (independent Fourier
    fields, 24 modes, |k| <= 3; Z spans the flame level Z = 1), solenoidal
    velocity rms 0.1, S = 2, qs = 1, eps = 0.5, tol = 1e-3, Lewis numbers
    Le_F = 0.8, Le_O = 1.2, Re = 200, Pr = 0.7. Draws: T, then Z, then v."""
    nd = len(n)
    L = (2 * math.pi,) * nd
    rng = np.random.default_rng(seed)
    T = fourier_temperature(n, L, rng, 3, 2.0, m=24)
    Z = fourier_temperature(n, L, rng, 3, 1.6, m=24) - 0.8
    v = solenoidal_velocity(n, L, rng, 3, 0.1, m=24)
    params = dict(Re=200.0, Pr=0.7, cfl=0.3, reacting=True, S=S, qs=1.0, eps=0.5, tol=1e-3, Le_F=Le_F,
                  Le_O=Le_O)
    return Case(f"reacting_periodic_{'x'.join(map(str, n))}", nd, tuple(n) + (1,) * (3 - nd),
                L + (1.0,) * (3 - nd), (("periodic", "periodic"),) * nd, params, T, v, Z=Z, nsteps=1)


def c3_case(nx=768, ny=1536, seed=3, W=32, wall=4, wall_h=64, inj=4,
            Umax=1.0, coflow=0.1, noise=0.01):
    """Planar slot-jet diffusion flame in a channel (nx x ny cells, dx = 1/W).

    Geometry (in cells): a burner centred at x = nx/2 standing on the bottom
    side: two walls ``wall`` cells thick and ``wall_h`` tall flank a slot of
    W cells; an injector layer ``inj`` cells thick spans the slot floor.
    Slot inflow U(x) = Umax (1 - (2 (x - xc)/W)^2) (1 + noise * xi_col),
    xi_col ~ N(0,1) per slot column (one draw of W values), fixed in time.
    Flame sheet: Z_st = 0.055 so S = 1/Z_st - 1 with fuel at Z = S + 1;
    eps = 0.5, tol = 1e-3; Q/(S+1) = QS_C3 places the peak of the
    regularised temperature at 7 (density ratio 7) with T = 1 in the
    oxidiser; H = H_inf = (S+1)/Q + 1 everywhere. Re = 200, Pr = Sc = 0.7
    (Le_F = Le_O = 1). Sides: slip walls in x, inflow at the bottom (coflow
    outside the burner footprint, wall under it), outflow at the top.
    Immersed boundary: mask of walls and injector, Da_ib = dx^2; targets
    v = 0 in the walls, v = (0, U) with Z = S + 1 in the injector,
    H = H_inf, Z held at its initial profile in the solid; mass source
    S_m = U / (inj dx) in the injector (fuel density 1 at T = 1), so the
    injected rate is sum(U) dx per unit depth. Below the slot the bottom
    side carries Z = S + 1 so the injector's Dirichlet ghost is fuel."""
    rng = np.random.default_rng(seed)
    h = 1.0 / W
    L = (nx * h, ny * h)
    xc = nx // 2
    s0, s1 = xc - W // 2, xc + W // 2          # slot columns [s0, s1)
    w0l, w1l = s0 - wall, s0                    # left wall columns
    w0r, w1r = s1, s1 + wall                    # right wall columns
    xi = rng.normal(size=W)
    shp = (ny, nx)
    chi = np.zeros(shp, dtype=np.uint8)
    chi[0:wall_h, w0l:w1l] = 1
    chi[0:wall_h, w0r:w1r] = 1
    chi[0:inj, s0:s1] = 1
    xcent = (np.arange(nx) + 0.5) * h
    xmid = xc * h
    U = np.zeros(nx)
    sl = slice(s0, s1)
    U[sl] = Umax * (1.0 - (2.0 * (xcent[sl] - xmid) / (W * h)) ** 2) * (1.0 + noise * xi)
    S = 1.0 / 0.055 - 1.0
    qs = QS_C3
    Hinf = 1.0 / qs + 1.0
    zfuel = S + 1.0
    v1 = np.zeros(shp)
    v2 = np.full(shp, coflow)
    v2[0:wall_h, w0l:w1l] = 0.0
    v2[0:wall_h, w0r:w1r] = 0.0
    v2[0:wall_h, s0:s1] = U[sl][None, :]
    yc = (np.arange(ny) + 0.5) * h
    # resolved fuel column: smooth top-hat across the slot edges (tanh over
    # one cell, so the burner walls are oxidiser-cold a few cells out) and
    # at the slot exit (tanh over two cells); the solid keeps this profile
    sx = 0.5 * (np.tanh((xcent - s0 * h) / h) - np.tanh((xcent - s1 * h) / h))
    sy = 0.5 * (1.0 - np.tanh((yc - wall_h * h) / (2.0 * h)))
    Z = zfuel * sy[:, None] * sx[None, :]
    vib1 = np.zeros(shp)
    vib2 = np.zeros(shp)
    vib2[0:inj, s0:s1] = U[sl][None, :]
    zib = Z.copy()
    hib = np.full(shp, Hinf)
    Sm = np.zeros(shp)
    Sm[0:inj, s0:s1] = (U[sl] / (inj * h))[None, :]
    vb2 = np.full(nx, coflow)
    vb2[w0l:w1r] = 0.0
    zb = Z[0, :].copy()                         # the injector floor holds fuel
    foot = np.zeros(nx, dtype=np.uint8)
    foot[w0l:w1r] = 1                           # burner footprint: wall cells of the side
    bnd = {(1, 0): dict(v=[np.zeros(nx), vb2], Z=zb, H=np.full(nx, Hinf), F=vb2.copy(), wall=foot)}
    params = dict(Re=200.0, Pr=0.7, Le_F=1.0, Le_O=1.0, reacting=1, S=S, qs=qs,
                  eps=0.5, tol=1e-3, Da_ib=h * h, p0=1.0, cfl=0.2,
                  poisson_rtol=1e-10)
    ib = dict(chi=chi, v_ib=[vib1, vib2], Z_ib=zib, H_ib=hib, Sm=Sm)
    case = Case(f"c3_slot_flame_{nx}x{ny}", 2, (nx, ny, 1), L + (1.0,),
                (("slip", "slip"), ("inflow", "outflow")), params,
                None, [v1, v2], Z=Z, ib=ib, bnd=bnd, nsteps=500)
    case.H = np.full(shp, Hinf)
    case.injected_rate = float(np.sum(U) * h)
    return case


def taylor_couette_case(n=64, Re=1.0, Da=1e-2, shifted=True, half=2.5):
    """Flow between concentric cylinders of radii 1 and 2 (inner one turning
    with unit surface speed, outer one at rest) in a periodic box
    [-half, half]^2 of n^2 cells, the cylinders immersed by penalisation:
    chi = 1 for r < 1 + s and r > 2 - s, s = sqrt(Da) for the shifted mask
    (the body grown by the Brinkman length), 0 for the cell-exact one. Body
    targets: rigid rotation inside, rest outside. Initial velocity: the exact
    annular profile v_theta = (4 - r^2)/(3 r) in 1 <= r <= 2 and the body
    velocities elsewhere; uniform T = 1 (constant density; the bodies hold
    the excess enthalpy H = 2 of T = 1 at qs = 1)."""
    L = (2.0 * half, 2.0 * half)
    x, y = cell_centres((n, n), L)
    x = x - half
    y = y - half
    X, Y = np.broadcast_arrays(x, y)
    r2 = X * X + Y * Y
    r = np.sqrt(r2)
    s = math.sqrt(Da) if shifted else 0.0
    chi = ((r < 1.0 + s) | (r > 2.0 - s)).astype(np.uint8)
    inner = r < 1.5
    vib = [np.where(inner, -Y, 0.0), np.where(inner, X, 0.0)]
    ann = (r >= 1.0) & (r <= 2.0)
    f = np.where(ann, (4.0 / np.where(ann, r2, 1.0) - 1.0) / 3.0, 0.0)
    v = [np.where(ann, -f * Y, vib[0]), np.where(ann, f * X, vib[1])]
    params = dict(Re=Re, Pr=0.7, Da_ib=Da, cfl=0.2, poisson_rtol=1e-10)
    case = Case(f"taylor_couette_{n}", 2, (n, n, 1), L + (1.0,), (("periodic", "periodic"),) * 2, params,
                np.ones((n, n)), v, ib=dict(chi=chi, v_ib=vib, H_ib=np.full((n, n), 2.0)))
    case.exact_v = [-f * Y, f * X]
    case.annulus = (r >= 1.0 + s) & (r <= 2.0 - s)
    return case


def tanh_stretched_faces(n, m, L=1.0):
    """Face coordinates of an n-cell side of length L clustered towards both
    ends (section 4.4, Eq 4.18): the uniform faces x = k/n mapped by
    x~ = (1 + tanh(a (x - 1/2)) / tanh(a / 2)) / 2, with a > 0 the root of
    max(width) / min(width) = m (the widest cell sits in the middle, the
    narrowest at the walls). m = 1 returns the uniform faces."""
    from scipy.optimize import brentq
    x = np.arange(n + 1) / n
    if m == 1.0:
        return L * x

    def mapped(a):
        return 0.5 + 0.5 * np.tanh(a * (x - 0.5)) / math.tanh(0.5 * a)

    def excess(a):
        w = np.diff(mapped(a))
        return w.max() / w.min() - m

    hi = 1.0
    while excess(hi) < 0.0:
        hi *= 2.0
    a = brentq(excess, 1e-6, hi, xtol=1e-15, rtol=4.0 * np.finfo(float).eps, maxiter=500)
    f = L * mapped(a)
    f[0], f[-1] = 0.0, L
    return f


def sine_stretched_faces(n, amp, L=1.0, shift=0.0):
    """Face coordinates of a smooth periodic stretching of [0, L]: the
    uniform faces x = k/n mapped by x + amp (sin(2 pi (x - shift)) +
    sin(2 pi shift)) / (2 pi), cell widths from (1 - amp) to (1 + amp) times
    L/n, with equal end widths (so the map suits a periodic direction)."""
    x = np.arange(n + 1) / n
    tp = 2.0 * math.pi
    f = x + amp * (np.sin(tp * (x - shift)) + math.sin(tp * shift)) / tp
    f = L * f
    f[0], f[-1] = 0.0, L
    return f


def heated_cavity_case(n=64, Ra=1e2, eps=0.6, Pr=0.71, gamma=1.4, That=600.0, Chat=110.5, cfl=0.15, m=1.0):
    """Differentially heated square cavity of unit side (section 4.4): left
    wall at T_H = 1 + eps, right wall at T_C = 1 - eps (isothermal, Eq
    4.16a-b), adiabatic top and bottom (Eq 4.16c), every wall no-slip;
    non-reacting with Q = S + 1 (qs = 1, T = H - 1). Scales: Pe = Pr Ra^{1/2}
    (Eq 4.10), so Re = Ra^{1/2}; Fr = (2 Pr eps)^{1/2} (Eq 4.11); Sutherland
    conductivity with C = Chat/That (Eq 4.12); enclosed system with gamma.
    Initial state at rest at the mean temperature, T = 1, H = 2 (Eq 4.17),
    p0 = 1 (so the conserved mass is 1). m > 1 clusters the cells of both
    directions towards the walls by the tanh map of Eq 4.18 (largest cell m
    times the smallest). No random draws."""
    nn = (n, n)
    bc = (("noslip", "noslip"), ("noslip", "noslip"))
    params = dict(Re=math.sqrt(Ra), Pr=Pr, inv_Fr2=1.0 / (2.0 * Pr * eps), sutherland_C=Chat / That,
                  p0_closed=True, gamma=gamma, cfl=cfl, poisson_rtol=1e-10)
    side = lambda Tw: dict(H=np.full(n, Tw + 1.0))
    bnd = {(0, 0): side(1.0 + eps), (0, 1): side(1.0 - eps)}
    case = Case(f"heated_cavity_{n}", 2, (n, n, 1), (1.0, 1.0, 1.0), bc, params,
                np.ones(nn), [np.zeros(nn), np.zeros(nn)], bnd=bnd)
    if m != 1.0:
        case.faces = [tanh_stretched_faces(n, m), tanh_stretched_faces(n, m)]
        case.name += f"_tanh{m:g}"
    case.eps = eps
    return case


def double_tsuji_case(n=96, half=6.0, Ub=0.1, Da=1e-4, wF=2.0, TF=1.3, shifted=True):
    """One quadrant [0, half]^2 (n^2 cells) of the double Tsuji burner
    (section 4.5): a cylinder of radius 1 at the origin ejecting fuel
    radially into planar counterflowing oxidiser jets. Symmetry (slip)
    sides on x = 0 and y = 0 (Eq 4.22a-b), inflow v = (x, -y) with Z = 0,
    H = H_inf at the top and outflow on the right (Eq 4.22c). Burner as a
    penalised body: chi = 1 for r < 1 + s, s = sqrt(Da) (shifted) or 0;
    mass source S_m = chi rho_b U_b / r (Eq 4.19) with rho_b = 1 (the fuel
    leaves at T = 1), targets v_ib = U_b x / r (Eq 4.20), Z_ib = S + 1 and
    H_ib = (S+1)/Q + 1 (Eq 4.21). Parameters of section 4.5: Pr = 0.71,
    Re = 100, U_b = 0.1, S = 14.89, Q = 4.17, Le_F = 0.97, Le_O = 1.11,
    Da_ib = 1e-4, eps = 0.5 (tol = 1e-3). Initial state: the potential flow
    of Eq 4.23 and the Z, H profiles of Eq 4.24 outside the body, with the
    flame width w_F and temperature T_F (taken from a reference the paper
    cites, not given: w_F = 2, T_F = 1.3 by default); the body targets
    inside it. No random draws."""
    S, Q = 14.89, 4.17
    qs = Q / (S + 1.0)
    Hinf = (S + 1.0) / Q + 1.0
    h = half / n
    L = (half, half)
    x, y = cell_centres((n, n), L)
    X, Y = np.broadcast_arrays(x, y)
    r2 = X * X + Y * Y
    r = np.sqrt(r2)
    sft = math.sqrt(Da) if shifted else 0.0
    chi = (r < 1.0 + sft).astype(np.uint8)
    body = chi.astype(bool)
    vib = [Ub * X / r, Ub * Y / r]
    # potential flow of Eq 4.23, evaluated outside the body only
    rr2 = np.where(body, 1.0, r2)
    v1 = X * (1.0 - (X * X - 3.0 * Y * Y) / rr2 ** 3 + Ub / rr2)
    v2 = -Y * (1.0 + (3.0 * X * X - Y * Y) / rr2 ** 3 - Ub / rr2)
    v = [np.where(body, vib[0], v1), np.where(body, vib[1], v2)]
    a = Ub / wF ** 2
    Z = np.sqrt((1.0 + a) / ((X / wF) ** 2 + a)) * np.exp(-Y * Y / 2.0)
    H = ((S + 1.0) / Q * (TF - 1.0) - 1.0) * Z + (S + 1.0) / Q + 1.0
    Z = np.where(body, S + 1.0, Z)
    H = np.where(body, Hinf, H)
    Sm = np.where(body, Ub / r, 0.0)
    xc = (np.arange(n) + 0.5) * h
    bnd = {(1, 1): dict(v=[xc.copy(), np.full(n, -half)], Z=np.zeros(n), H=np.full(n, Hinf),
                        F=np.full(n, -half))}
    params = dict(Re=100.0, Pr=0.71, reacting=1, S=S, qs=qs, eps=0.5, tol=1e-3, Le_F=0.97, Le_O=1.11,
                  Da_ib=Da, p0=1.0, cfl=0.2, poisson_rtol=1e-10)
    ib = dict(chi=chi, v_ib=vib, Z_ib=np.full((n, n), S + 1.0), H_ib=np.full((n, n), Hinf), Sm=Sm)
    case = Case(f"double_tsuji_{n}", 2, (n, n, 1), L + (1.0,), (("slip", "outflow"), ("slip", "inflow")),
                params, None, v, Z=Z, ib=ib, bnd=bnd, H=H)
    case.injected_rate = float(np.sum(Sm) * h * h)
    return case


def make_case(name, **kw):
    return dict(c1=c1_case, c2=c2_case, c3=c3_case, c4=c4_case,
                c5=c5_case)[name](**kw)


def fd_directions(shape, k=16, seed=1005):
    """k seeded unit-RMS Gaussian perturbation fields for finite-difference checks."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        d = rng.normal(size=shape)
        out.append(d / math.sqrt(float(np.mean(d * d))))
    return out
