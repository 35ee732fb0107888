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


# ---------------------------------------------------------------------------
# Section 5.2.1 manufactured solution and the initialisations of Table 1
# ---------------------------------------------------------------------------
import dataclasses


def _fd_operator(P, x, y, h=1e-4):
    """-div(a grad u*) by central differences of the flux form (second order)."""
    u = lambda xx, yy: wl.exact_u(P, xx, yy)
    a = lambda xx, yy: wl.coefficient(P, xx, yy)[0]
    fx = lambda xx, yy: a(xx, yy) * (u(xx + h / 2, yy) - u(xx - h / 2, yy)) / h
    fy = lambda xx, yy: a(xx, yy) * (u(xx, yy + h / 2) - u(xx, yy - h / 2)) / h
    return -((fx(x + h / 2, y) - fx(x - h / 2, y)) / h + (fy(x, y + h / 2) - fy(x, y - h / 2)) / h)


def test_sin2pi_exp_solution_closed_forms():
    P = dataclasses.replace(wl.CONFIG_SMALL, sol=wl.SOL_SIN2PI_EXP)
    rng = np.random.default_rng(2)
    x, y = rng.uniform(0.05, 0.95, 30), rng.uniform(0.05, 0.95, 30)
    assert np.allclose(wl.exact_u(P, x, y), np.sin(2 * math.pi * x) * np.exp(y), rtol=0, atol=1e-15)
    f = wl.source_f(P, x, y)
    assert np.allclose(f, (4 * math.pi**2 - 1) * np.sin(2 * math.pi * x) * np.exp(y), rtol=1e-14, atol=1e-13)
    assert np.abs(f - _fd_operator(P, x, y)).max() <= 1e-5 * np.abs(f).max()
    V = dataclasses.replace(P, op=wl.OP_VARCOEF, k1=2, k2=3)
    fv = wl.source_f(V, x, y)
    assert np.abs(fv - _fd_operator(V, x, y)).max() <= 1e-5 * np.abs(fv).max()
    # Dirichlet data is u* itself: zero on x = 0, 1, e^y sin(2 pi x) on y = 0, 1
    t = np.linspace(0, 1, 9)
    assert np.abs(wl.boundary_g(P, 0 * t, t)).max() < 1e-15
    assert np.allclose(wl.boundary_g(P, t, 0 * t + 1), math.e * np.sin(2 * math.pi * t), atol=1e-15)


def test_sinsin_solution_unchanged_by_the_refactor():
    P = wl.CONFIG_SMALL
    rng = np.random.default_rng(3)
    x, y = rng.uniform(0, 1, 10), rng.uniform(0, 1, 10)
    u = np.sin(math.pi * x) * np.sin(math.pi * y)
    assert np.array_equal(wl.exact_u(P, x, y), u)
    assert np.allclose(wl.source_f(P, x, y), 2 * math.pi**2 * u, rtol=1e-15, atol=0)


def test_init_half_widths_follow_table_1():
    P = wl.CONFIG_8x8                                    # 64 subdomains x 400 neurons
    assert math.isclose(wl.init_half_width(P, wl.INIT_SUGGESTED), math.sqrt(64 * 400 / 64))   # l = sqrt(n / 64)
    assert wl.init_half_width(P, wl.INIT_MANUAL) == 1.0
    assert math.isclose(wl.init_half_width(P, wl.INIT_HE), math.sqrt(2.0 / 400))


def test_paper_init_bias_rule_and_frame_change():
    P = dataclasses.replace(wl.CONFIG_SMALL, nsub_x=3, nsub_y=2, x1=1.5)   # rectangular subdomains
    W, b, (wg, bg, xi) = wl.hidden_params_init(P, 11, wl.INIT_SUGGESTED, return_global=True)
    l = wl.init_half_width(P, wl.INIT_SUGGESTED)
    assert np.abs(wg).max() <= l and np.abs(wg).max() > 0.95 * l
    # b = -w . xi, xi within r = diam / 2 of its own subdomain
    assert np.allclose(bg, -(wg * xi).sum(-1), rtol=0, atol=1e-13)
    hx, hy = 0.5, 0.5
    r = 0.5 * math.hypot(hx, hy)
    for s in range(P.nsub):
        x0, y0 = (s % 3) * hx, (s // 3) * hy
        dx = np.maximum(np.maximum(x0 - xi[s, :, 0], xi[s, :, 0] - x0 - hx), 0)
        dy = np.maximum(np.maximum(y0 - xi[s, :, 1], xi[s, :, 1] - y0 - hy), 0)
        assert np.hypot(dx, dy).max() <= r + 1e-15
        # the same neuron in both frames: w^ . x^ + b^ = w . x + b with x = x_c + (h / 2) x^
        rng = np.random.default_rng(5 + s)
        xh = rng.uniform(-1, 1, size=(17, 2))
        xg = np.array([x0 + hx / 2, y0 + hy / 2]) + 0.5 * np.array([hx, hy]) * xh
        assert np.allclose(xh @ W[s].T + b[s], xg @ wg[s].T + bg[s], rtol=0, atol=1e-12)
    # deterministic in the seed, different across seeds
    W2, b2 = wl.hidden_params_init(P, 11, wl.INIT_SUGGESTED)
    assert np.array_equal(W, W2) and np.array_equal(b, b2)
    assert not np.array_equal(wl.hidden_params_init(P, 12)[1], b)


def test_neighbourhood_sampler_is_uniform_on_the_rounded_rectangle():
    """Area fractions of the r-neighbourhood of a wx x wy rectangle: the
    rectangle wx wy / A, the side strips 2 r (wx + wy) / A, the corner
    quarter-discs pi r^2 / A, with A = wx wy + 2 r (wx + wy) + pi r^2."""
    wx, wy = 0.5, 0.25
    r = 0.5 * math.hypot(wx, wy)
    p = wl.sample_rect_neighbourhood(np.random.default_rng(7), 200000, wx, wy, r)
    A = wx * wy + 2 * r * (wx + wy) + math.pi * r * r
    inside_x = (p[:, 0] >= 0) & (p[:, 0] <= wx)
    inside_y = (p[:, 1] >= 0) & (p[:, 1] <= wy)
    rect = np.mean(inside_x & inside_y)
    strips = np.mean(inside_x ^ inside_y)
    corners = np.mean(~inside_x & ~inside_y)
    for got, want in ((rect, wx * wy / A), (strips, 2 * r * (wx + wy) / A), (corners, math.pi * r * r / A)):
        assert abs(got - want) < 0.005, (got, want)
    # symmetric about the centre
    assert abs(np.mean(p[:, 0]) - wx / 2) < 0.01 and abs(np.mean(p[:, 1]) - wy / 2) < 0.01


def test_he_and_manual_init_use_the_same_bias_rule():
    P = wl.CONFIG_SMALL
    for scheme in (wl.INIT_HE, wl.INIT_MANUAL):
        W, b, (wg, bg, xi) = wl.hidden_params_init(P, 3, scheme, return_global=True)
        l = wl.init_half_width(P, scheme)
        assert np.abs(wg).max() <= l and np.abs(wg).max() > 0.9 * l
        assert np.allclose(bg, -(wg * xi).sum(-1), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Approximate Gaussian random fields (eq. grf) and rho = tanh(grf) + 1.1
# ---------------------------------------------------------------------------

def test_grf_moments_match_the_distribution():
    """E[grf^2] = terms * E[a^2] * E[sin^2] = alpha^4 / 2 (b uniform), and
    E[|w|^2] = 2 alpha^2: checked over many independent fields."""
    alpha = 16.0
    x = np.array([0.3, 0.7])
    y = np.array([0.2, 0.9])
    vals, w2 = [], []
    for seed in range(400):
        F = wl.grf_params(seed, alpha)
        vals.append(wl.grf_value_and_grad(F, x, y)[0])
        w2.append(np.mean(np.sum(F.freq ** 2, 1)))
    v = np.concatenate(vals)
    assert abs(np.mean(v ** 2) / (alpha ** 4 / 2) - 1) < 0.1
    assert abs(np.mean(w2) / (2 * alpha ** 2) - 1) < 0.02
    F = wl.grf_params(1, alpha)
    assert F.amp.shape == (256,) and F.freq.shape == (256, 2) and np.all((F.phase > 0) & (F.phase < 2 * math.pi))


def test_grf_gradient_and_coefficient_by_finite_differences():
    F = wl.grf_params(5, 16.0)
    rng = np.random.default_rng(9)
    x, y = rng.uniform(0, 1, 25), rng.uniform(0, 1, 25)
    h = 1e-6
    v, vx, vy = wl.grf_value_and_grad(F, x, y)
    fd_x = (wl.grf_value_and_grad(F, x + h, y)[0] - wl.grf_value_and_grad(F, x - h, y)[0]) / (2 * h)
    fd_y = (wl.grf_value_and_grad(F, x, y + h)[0] - wl.grf_value_and_grad(F, x, y - h)[0]) / (2 * h)
    scale = np.abs(np.concatenate([vx, vy])).max()
    assert np.abs(vx - fd_x).max() <= 1e-6 * scale and np.abs(vy - fd_y).max() <= 1e-6 * scale
    a, ax, ay = wl.grf_coefficient(F, x, y)
    assert np.all((a > 0.1 - 1e-15) & (a < 2.1 + 1e-15))
    fa_x = (wl.grf_coefficient(F, x + h, y)[0] - wl.grf_coefficient(F, x - h, y)[0]) / (2 * h)
    assert np.abs(ax - fa_x).max() <= 1e-5 * max(1.0, np.abs(ax).max())
    # the data helpers: f = grf, g = 0 / f = 1, g = 0, coefficient rows like sample_data
    P = dataclasses.replace(wl.CONFIG_SMALL, op=wl.OP_VARCOEF)
    ip, bp = np.stack([x, y], 1), np.stack([y, x], 1)[:4]
    f, g, c = wl.grf_source_data(P, F, ip, bp)
    assert np.array_equal(f, v) and not g.any() and c is None
    f, g, c = wl.grf_coefficient_data(P, F, ip, bp)
    assert np.all(f == 1) and not g.any() and c.shape == (3, 25) and np.array_equal(c[0], a)
