"""The seeded input generators: the Fourier-mode fields summed by inverse
FFT equal the direct sums over the drawn modes (evaluated here mode by mode
at the cell centres), and keep their documented normalisations."""
import math

import numpy as np
import pytest

from workloads.ics import (_wavevectors, cell_centres, fourier_temperature, solenoidal_velocity)


def _theta(n, L, k):
    x = cell_centres(n, L)
    return sum((2 * math.pi / L[d]) * k[d] * x[d] for d in range(len(n)))


@pytest.mark.parametrize("n", [(24, 20), (16, 12, 10)])
def test_fourier_temperature_direct_sum(n):
    L = tuple(2 * math.pi * (1.0 + 0.25 * d) for d in range(len(n)))
    T = fourier_temperature(n, L, np.random.default_rng(3), 6, 3.0)
    rng = np.random.default_rng(3)
    ks = _wavevectors(len(n), 6)
    idx = rng.choice(len(ks), size=32, replace=False)
    a = rng.random(32)
    ph = 2 * math.pi * rng.random(32)
    f = sum(a[q] * np.cos(_theta(n, L, ks[idx[q]]) + ph[q]) for q in range(32))
    ref = 1.0 + 3.0 * (f - f.min()) / (f.max() - f.min())
    assert np.max(np.abs(T - ref)) < 1e-12
    assert abs(T.min() - 1.0) < 1e-14 and abs(T.max() - 4.0) < 1e-14


@pytest.mark.parametrize("n", [(24, 20), (16, 12, 10)])
def test_solenoidal_velocity_direct_sum(n):
    nd = len(n)
    L = tuple(2 * math.pi * (1.0 + 0.25 * d) for d in range(nd))
    v = solenoidal_velocity(n, L, np.random.default_rng(4), 5, 0.1)
    rng = np.random.default_rng(4)
    ks = _wavevectors(nd, 5)
    idx = rng.choice(len(ks), size=32, replace=False)
    ref = [np.zeros(tuple(reversed(n))) for _ in range(nd)]
    if nd == 2:
        a = rng.random(32)
        ph = 2 * math.pi * rng.random(32)
        for q in range(32):
            k = ks[idx[q]]
            s = np.sin(_theta(n, L, k) + ph[q])
            ref[0] -= a[q] * (2 * math.pi / L[1] * k[1]) * s
            ref[1] += a[q] * (2 * math.pi / L[0] * k[0]) * s
    else:
        c = rng.normal(size=(32, 3))
        sn = rng.normal(size=(32, 3))
        for q in range(32):
            k = ks[idx[q]]
            kp = np.array([2 * math.pi / L[d] * k[d] for d in range(3)])
            kk = kp / np.linalg.norm(kp)
            cq = c[q] - kk * (kk @ c[q])
            sq = sn[q] - kk * (kk @ sn[q])
            th = _theta(n, L, k)
            for d in range(3):
                ref[d] += cq[d] * np.cos(th) + sq[d] * np.sin(th)
    e = math.sqrt(float(np.mean(sum(x * x for x in ref))))
    for d in range(nd):
        assert np.max(np.abs(v[d] - ref[d] * (0.1 / e))) < 1e-13
    assert abs(math.sqrt(float(np.mean(sum(x * x for x in v)))) - 0.1) < 1e-14


def test_stretched_face_generators():
    """The tanh faces handed to both sides equal the oracle's own Eq 4.18
    grid (pinned there by Tables 3-4) to rounding; the sine faces span
    [0, L], increase strictly and keep their documented width range."""
    from oracle.grid import tanh_faces
    from workloads import sine_stretched_faces, tanh_stretched_faces
    for m, n in [(2.0, 32), (2.0, 64), (5.0, 32), (21.0, 64), (21.0, 216), (1.0, 16)]:
        f = tanh_stretched_faces(n, m, L=1.5)
        assert np.max(np.abs(f - tanh_faces(n, m, L=1.5))) < 1e-14
        w = np.diff(f)
        assert abs(w.max() / w.min() - m) < 1e-9 and f[0] == 0.0 and f[-1] == 1.5
    n, amp, L = 64, 0.5, 2 * math.pi
    f = sine_stretched_faces(n, amp, L, shift=0.2)
    w = np.diff(f) * n / L
    assert f[0] == 0.0 and f[-1] == L and np.all(w > 0)
    assert 1 - amp - 1e-12 < w.min() and w.max() < 1 + amp + 1e-12
    assert w.max() - w.min() > 1.8 * amp


def test_reacting_periodic_case_ranges():
    """T in [1, 3], Z in [0.2, 1.8] (both ends reached), seeded."""
    from workloads.ics import reacting_periodic_case
    c = reacting_periodic_case((24, 20), seed=3)
    assert c.T.shape == c.Z.shape == (20, 24) and c.ndim == 2 and c.n == (24, 20, 1)
    assert abs(c.T.min() - 1.0) < 1e-12 and abs(c.T.max() - 3.0) < 1e-12
    assert abs(c.Z.min() - 0.2) < 1e-12 and abs(c.Z.max() - 1.8) < 1e-12
    d = reacting_periodic_case((24, 20), seed=3)
    assert np.array_equal(c.Z, d.Z) and np.array_equal(c.v[0], d.v[0])
    e = reacting_periodic_case((8, 6, 4), seed=3)
    assert e.T.shape == (4, 6, 8) and len(e.v) == 3 and e.params["reacting"]
