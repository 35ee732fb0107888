"""Pins of the synthetic Fourier-series sources (closed forms, brute force)."""
import math

import numpy as np

import workload as wl


def test_fourier_source_matches_the_double_sum():
    a = wl.fourier_coeffs(3, modes=5, count=2)
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0, 1, 7), rng.uniform(0, 1, 7)
    got = wl.fourier_source(a, x, y)
    for c in range(2):
        ref = [sum(a[c, i, j] * math.sin(math.pi * (i + 1) * xx) * math.sin(math.pi * (j + 1) * yy)
                   for i in range(5) for j in range(5)) for xx, yy in zip(x, y)]
        assert np.allclose(got[c], ref, rtol=0, atol=1e-14)


def test_fourier_exact_solves_poisson_and_vanishes_on_the_boundary():
    a = wl.fourier_coeffs(4, modes=8, count=1)
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0.1, 0.9, 20), rng.uniform(0.1, 0.9, 20)
    h = 1e-3
    u = lambda xx, yy: wl.fourier_exact(a, xx, yy)[0]
    lap = (u(x + h, y) + u(x - h, y) + u(x, y + h) + u(x, y - h) - 4 * u(x, y)) / h**2
    f = wl.fourier_source(a, x, y)[0]
    assert np.abs(-lap - f).max() <= 1e-4 * np.abs(f).max()
    t = np.linspace(0, 1, 11)
    for bx, by in [(t, 0 * t), (t, 0 * t + 1), (0 * t, t), (0 * t + 1, t)]:
        assert np.abs(u(bx, by)).max() < 1e-13


def test_fourier_features_are_standardised():
    a = wl.fourier_coeffs(5, modes=32, count=64)
    z = wl.fourier_features(a)
    assert z.shape == (64, 1024)
    assert abs(np.mean(z**2) - 1.0) < 0.02
    # row-major: feature k1 * M + k2 holds mode (k1 + 1, k2 + 1)
    assert np.isclose(z[0, 1 * 32 + 2], a[0, 1, 2] * math.sqrt(1 + 4 + 9))


def test_fourier_inputs_have_unit_mean_square():
    a = wl.fourier_coeffs(6, modes=32, count=256)
    z = wl.fourier_inputs(a)
    assert z.shape == (256, 1024)
    assert abs(np.mean(z**2) - 1.0) < 0.03
    assert np.allclose(z[3] / a[3].ravel(), z[3, 0] / a[3, 0, 0])
