"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module holds problem descriptions and input data only: the subdomain
partition and point counts, the random hidden-layer parameters (which the
method draws once, before anything else), and closed-form manufactured
solutions with their sources.  It contains none of the method's arithmetic
(no features, no least squares, no interface system), so the oracle and the
GPU library can both take their inputs from here without sharing any solver
code.

Problem setting: the elliptic problem L u = f in a rectangle with Dirichlet
data u = g on the boundary (paper, Section 2, eq. pde), with L = -Laplace
(Section 4.2, eq. poisson) or L u = -div(a grad u) (Section 4.2, variable
coefficient problem).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

OP_POISSON = 0
OP_VARCOEF = 1

# Manufactured solutions: u* = sin(pi x) sin(pi y) (zero on the boundary of
# the unit square), or u* = sin(2 pi x) e^y, the exact solution of the 2-D
# Poisson experiment of Section 5.2.1 (nonzero Dirichlet data on y = 0, 1).
SOL_SINSIN = 0
SOL_SIN2PI_EXP = 1


@dataclasses.dataclass(frozen=True)
class Problem:
    """One elliptic problem on a rectangle split into nsub_x x nsub_y subdomains.

    neurons      -- hidden neurons of every local network (n_N in Section 3)
    q_x, q_y     -- interior collocation grid per subdomain (cell-centred)
    m_bdry_edge  -- collocation points per exterior (Dirichlet) edge
    m_ifc_edge   -- interface points per interface edge
    op           -- OP_POISSON or OP_VARCOEF
    R            -- hidden weights and biases are i.i.d. U[-R, R]
    k1, k2       -- wave numbers of the variable coefficient a(x, y)
    sol          -- manufactured solution (SOL_SINSIN or SOL_SIN2PI_EXP)
    """

    nsub_x: int
    nsub_y: int
    neurons: int
    q_x: int
    q_y: int
    m_bdry_edge: int
    m_ifc_edge: int
    op: int = OP_POISSON
    R: float = 1.0
    k1: int = 1
    k2: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    sol: int = SOL_SINSIN

    @property
    def nsub(self) -> int:
        return self.nsub_x * self.nsub_y

    @property
    def n_interface(self) -> int:
        """Number of interface unknowns (one per interface point)."""
        nv = (self.nsub_x - 1) * self.nsub_y
        nh = self.nsub_x * (self.nsub_y - 1)
        return (nv + nh) * self.m_ifc_edge


# The small 2x2 case: 100 tanh neurons per subdomain, U[-2,2], 20x20 interior
# points, 40 points per exterior edge, 20 per interface edge.
CONFIG_SMALL = Problem(nsub_x=2, nsub_y=2, neurons=100, q_x=20, q_y=20,
                       m_bdry_edge=40, m_ifc_edge=20, R=2.0)
# The 8x8 case: 400 neurons per subdomain, U[-4,4], 40x40 interior points,
# 40 points per edge (exterior and interface).
CONFIG_8x8 = Problem(nsub_x=8, nsub_y=8, neurons=400, q_x=40, q_y=40,
                     m_bdry_edge=40, m_ifc_edge=40, R=4.0)


# The 32x32 case: 1000 neurons per subdomain (U[-sqrt(1000)/5, +]), 64x64
# interior points, 64 points per edge (126976 interface unknowns), variable
# coefficient with k1 = 2, k2 = 3.
CONFIG_32x32 = Problem(nsub_x=32, nsub_y=32, neurons=1000, q_x=64, q_y=64, m_bdry_edge=64, m_ifc_edge=64,
                       op=OP_VARCOEF, R=math.sqrt(1000.0) / 5.0, k1=2, k2=3)


def hidden_params(problem: Problem, seed: int):
    """Random hidden layer of every local network.

    Returns W of shape (nsub, n, 2) and b of shape (nsub, n), all i.i.d.
    U[-R, R] (weights act on subdomain-local coordinates in [-1, 1]^2).
    The method fixes these once and never trains them (Section 2.2, ELM).
    """
    rng = np.random.default_rng(seed)
    R = problem.R
    N, n = problem.nsub, problem.neurons
    W = rng.uniform(-R, R, size=(N, n, 2))
    b = rng.uniform(-R, R, size=(N, n))
    return np.ascontiguousarray(W), np.ascontiguousarray(b)


# ---------------------------------------------------------------------------
# The paper's initialisation of the hidden layer (Section 4.1, eq. init) and
# the two it is compared with (Table 1).  The half-width l = c sqrt(n)
# (n = all neurons of the problem) comes from l ~ sqrt(n_N) for a subdomain
# scaled to unit size, times the factor sqrt(N) that undoes the scaling, so
# w and b = -w . xi act on the problem's own coordinates; xi is uniform on
# the closed r-neighbourhood of the subdomain, r = diam(Omega_s) / 2.  The
# local networks see x^ = 2 (x - x_c) / h in [-1, 1]^2, so a global draw
# (w, b) maps exactly to w^ = w * h / 2, b^ = b + w . x_c.
# ---------------------------------------------------------------------------

def _dist_to_rect(px, py, wx, wy):
    """Distance of points to the rectangle [0, wx] x [0, wy]."""
    dx = np.maximum(np.maximum(-px, px - wx), 0.0)
    dy = np.maximum(np.maximum(-py, py - wy), 0.0)
    return np.hypot(dx, dy)


def sample_rect_neighbourhood(rng, count: int, wx: float, wy: float, r: float):
    """count points uniform on the closed r-neighbourhood of [0, wx] x [0, wy]
    (the points at distance <= r from it), by rejection from its bounding
    box.  Returns an array (count, 2)."""
    out = np.empty((0, 2))
    while len(out) < count:
        need = count - len(out)
        m = need + need // 4 + 16
        cand = np.stack([rng.uniform(-r, wx + r, m), rng.uniform(-r, wy + r, m)], 1)
        keep = cand[_dist_to_rect(cand[:, 0], cand[:, 1], wx, wy) <= r]
        out = np.concatenate([out, keep])
    return out[:count]


INIT_SUGGESTED = "suggested"   # l = c sqrt(n), n = all neurons of the problem (eq. init), c = 1/8
INIT_MANUAL = "manual"         # l = 1
INIT_HE = "he"                 # l = sqrt(2 / n_N), n_N = neurons per subdomain


def init_half_width(problem: Problem, scheme: str, c: float = 0.125) -> float:
    """Half-width l of the weight interval [-l, l] of each scheme in Table 1
    (problem coordinates)."""
    if scheme == INIT_SUGGESTED:
        return c * math.sqrt(problem.nsub * problem.neurons)
    if scheme == INIT_MANUAL:
        return 1.0
    if scheme == INIT_HE:
        return math.sqrt(2.0 / problem.neurons)
    raise ValueError(scheme)


def hidden_params_init(problem: Problem, seed: int, scheme: str = INIT_SUGGESTED, c: float = 0.125,
                       return_global: bool = False):
    """Hidden layer drawn as in eq. init: per subdomain and neuron, w ~
    U([-l, l]^2) and b = -w . xi with xi uniform on the closed
    r-neighbourhood of the subdomain, r = diam / 2, all in problem
    coordinates.  The scheme sets l (init_half_width); the bias rule is the
    same for all three.  Returns W (nsub, n, 2), b (nsub, n) for the local
    networks' [-1, 1]^2 coordinates; with return_global also (w, b, xi) in
    problem coordinates."""
    rng = np.random.default_rng(seed)
    N, n = problem.nsub, problem.neurons
    hx = (problem.x1 - problem.x0) / problem.nsub_x
    hy = (problem.y1 - problem.y0) / problem.nsub_y
    r = 0.5 * math.hypot(hx, hy)
    l = init_half_width(problem, scheme, c)
    wg = rng.uniform(-l, l, size=(N, n, 2))
    xi = sample_rect_neighbourhood(rng, N * n, hx, hy, r).reshape(N, n, 2)
    s = np.arange(N)
    lo = np.stack([problem.x0 + (s % problem.nsub_x) * hx, problem.y0 + (s // problem.nsub_x) * hy], 1)
    xi = xi + lo[:, None, :]
    bg = -(wg * xi).sum(-1)
    ctr = lo + 0.5 * np.array([hx, hy])
    W = wg * (0.5 * np.array([hx, hy]))
    b = bg + (wg * ctr[:, None, :]).sum(-1)
    W, b = np.ascontiguousarray(W), np.ascontiguousarray(b)
    if return_global:
        return W, b, (wg, bg, xi)
    return W, b


# ---------------------------------------------------------------------------
# Approximate Gaussian random fields (Section 5.2.1, eq. grf): a sum of 256
# random plane waves, used as a source f with g = 0, or through
# rho = tanh(grf) + 1.1 as the coefficient of -div(rho grad u) = 1, g = 0
# (Section 5.2.2).  Neither problem has a closed-form solution.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class GRF:
    amp: np.ndarray     # (terms,)  a_i ~ N(0, alpha^4 / terms)
    freq: np.ndarray    # (terms, 2) w_i ~ N(0, alpha^2 I)
    phase: np.ndarray   # (terms,)  b_i ~ U(0, 2 pi)


def grf_params(seed: int, alpha: float, terms: int = 256) -> GRF:
    rng = np.random.default_rng(seed)
    amp = rng.normal(0.0, alpha * alpha / math.sqrt(terms), size=terms)
    freq = rng.normal(0.0, alpha, size=(terms, 2))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=terms)
    return GRF(amp, freq, phase)


def grf_value_and_grad(field: GRF, x, y):
    """grf(x, y) = sum_i a_i sin(w_i . x + b_i) and its gradient."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    arg = np.multiply.outer(x, field.freq[:, 0]) + np.multiply.outer(y, field.freq[:, 1]) + field.phase
    v = np.sin(arg) @ field.amp
    c = np.cos(arg) * field.amp
    return v, c @ field.freq[:, 0], c @ field.freq[:, 1]


def grf_source_data(problem: Problem, field: GRF, interior_xy, boundary_xy):
    """f = grf at the interior points, g = 0 (Poisson with the field as source)."""
    f = grf_value_and_grad(field, interior_xy[:, 0], interior_xy[:, 1])[0]
    return f, np.zeros(len(boundary_xy)), None


def grf_coefficient(field: GRF, x, y):
    """rho = tanh(grf) + 1.1 and its gradient (1 - tanh^2) grad grf."""
    v, vx, vy = grf_value_and_grad(field, x, y)
    t = np.tanh(v)
    d = 1.0 - t * t
    return t + 1.1, d * vx, d * vy


def grf_coefficient_data(problem: Problem, field: GRF, interior_xy, boundary_xy):
    """-div(rho grad u) = 1, g = 0: f = 1, and (rho, rho_x, rho_y) at the
    interior points stacked as (3, npts) like sample_data (problem.op must be
    OP_VARCOEF)."""
    a, ax, ay = grf_coefficient(field, interior_xy[:, 0], interior_xy[:, 1])
    return np.ones(len(interior_xy)), np.zeros(len(boundary_xy)), np.stack([a, ax, ay])


# ---------------------------------------------------------------------------
# Manufactured solutions and their data.
# ---------------------------------------------------------------------------

def _u_and_grad(problem: Problem, x, y):
    """u*, du*/dx, du*/dy and -Lap u* of the problem's manufactured solution."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    p = math.pi
    if problem.sol == SOL_SIN2PI_EXP:
        s, c, e = np.sin(2 * p * x), np.cos(2 * p * x), np.exp(y)
        u = s * e
        return u, 2 * p * c * e, u, (4 * p * p - 1.0) * u
    u = np.sin(p * x) * np.sin(p * y)
    ux = p * np.cos(p * x) * np.sin(p * y)
    uy = p * np.sin(p * x) * np.cos(p * y)
    return u, ux, uy, 2.0 * p * p * u


def exact_u(problem: Problem, x, y):
    return _u_and_grad(problem, x, y)[0]


def exact_grad(problem: Problem, x, y):
    """(du*/dx, du*/dy) of the manufactured solution."""
    return _u_and_grad(problem, x, y)[1:3]


def coefficient(problem: Problem, x, y):
    """a, da/dx, da/dy of a = 1 + 0.5 sin(2 pi k1 x) cos(2 pi k2 y); a = 1 for Poisson."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if problem.op == OP_POISSON:
        one = np.ones_like(x)
        return one, np.zeros_like(x), np.zeros_like(x)
    w1 = 2.0 * math.pi * problem.k1
    w2 = 2.0 * math.pi * problem.k2
    a = 1.0 + 0.5 * np.sin(w1 * x) * np.cos(w2 * y)
    ax = 0.5 * w1 * np.cos(w1 * x) * np.cos(w2 * y)
    ay = -0.5 * w2 * np.sin(w1 * x) * np.sin(w2 * y)
    return a, ax, ay


def source_f(problem: Problem, x, y):
    """f = L u* for the manufactured solution u*.

    Poisson: f = -Lap u* (2 pi^2 u* for sin sin, (4 pi^2 - 1) u* for
    sin(2 pi x) e^y).  Variable coefficient: f = -a Lap u* - grad a . grad u*
    (product rule).
    """
    u, ux, uy, mlap = _u_and_grad(problem, x, y)
    if problem.op == OP_POISSON:
        return mlap
    a, ax, ay = coefficient(problem, x, y)
    return a * mlap - (ax * ux + ay * uy)


def boundary_g(problem: Problem, x, y):
    """Dirichlet data g = u* on the boundary."""
    return exact_u(problem, x, y)


def eval_grid(problem: Problem, per_sub: int = 16):
    """Cell-centred per_sub x per_sub evaluation points in every subdomain.

    Returns (x, y) flattened subdomain-major (subdomain s = sy * nsub_x + sx,
    then row-major in y, then x).
    """
    hx = (problem.x1 - problem.x0) / problem.nsub_x
    hy = (problem.y1 - problem.y0) / problem.nsub_y
    t = (np.arange(per_sub) + 0.5) / per_sub
    xs, ys = [], []
    for sy in range(problem.nsub_y):
        for sx in range(problem.nsub_x):
            X, Y = np.meshgrid(problem.x0 + (sx + t) * hx, problem.y0 + (sy + t) * hy)
            xs.append(X.ravel())
            ys.append(Y.ravel())
    return np.concatenate(xs), np.concatenate(ys)


def sample_data(problem: Problem, interior_xy, boundary_xy):
    """Problem data at given points: f at interior points, g at boundary
    points, and (a, da/dx, da/dy) stacked as (3, npts) for the variable
    coefficient operator (None for Poisson)."""
    interior_xy = np.asarray(interior_xy, dtype=np.float64).reshape(-1, 2)
    boundary_xy = np.asarray(boundary_xy, dtype=np.float64).reshape(-1, 2)
    f = source_f(problem, interior_xy[:, 0], interior_xy[:, 1])
    g = boundary_g(problem, boundary_xy[:, 0], boundary_xy[:, 1])
    coef = None
    if problem.op == OP_VARCOEF:
        coef = np.stack(coefficient(problem, interior_xy[:, 0], interior_xy[:, 1]))
    return f, g, coef


# ---------------------------------------------------------------------------
# Random Fourier-series sources on the unit square (the learned-interface
# workload): f = sum_{k1,k2=1..M} alpha_k sin(pi k1 x) sin(pi k2 y) with
# alpha_k ~ N(0, 1/(1 + k1^2 + k2^2)); u = 0 on the boundary; the exact
# Poisson solution is sum alpha_k sin sin / (pi^2 (k1^2 + k2^2)).
# ---------------------------------------------------------------------------

# 16x16 subdomains of the 8x8 case's resolution: 400 neurons, U[-4,4], 40x40
# interior points and 40 points per edge (19200 interface unknowns).
CONFIG_16x16 = Problem(nsub_x=16, nsub_y=16, neurons=400, q_x=40, q_y=40,
                       m_bdry_edge=40, m_ifc_edge=40, R=4.0)


def _modes(M):
    k = np.arange(1, M + 1, dtype=np.float64)
    return k, 1.0 + k[:, None] ** 2 + k[None, :] ** 2


def fourier_coeffs(seed: int, modes: int = 32, count: int = 1):
    """count coefficient arrays alpha of shape (count, modes, modes), indexed [k1-1, k2-1]."""
    _, w = _modes(modes)
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count, modes, modes)) / np.sqrt(w)


def fourier_features(alpha):
    """Network input: alpha row-major, each mode scaled by sqrt(1 + |k|^2) (unit variance)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    M = alpha.shape[-1]
    _, w = _modes(M)
    return (alpha * np.sqrt(w)).reshape(alpha.shape[0], M * M)


def fourier_inputs(alpha):
    """Network input: alpha row-major times one constant that gives the inputs
    unit mean square over the coefficient distribution (sum_k 1/(1+|k|^2) / M^2).
    The per-mode standardisation of fourier_features makes the high modes,
    which hardly move u, as loud as the low ones, and the network then
    generalises far worse from a few thousand samples."""
    alpha = np.asarray(alpha, dtype=np.float64)
    M = alpha.shape[-1]
    _, w = _modes(M)
    c = 1.0 / math.sqrt(float(np.mean(1.0 / w)))
    return (alpha * c).reshape(alpha.shape[0], M * M)


def _sine_table(v, M):
    k, _ = _modes(M)
    return np.sin(math.pi * np.outer(v, k))


def fourier_series_at(alpha, x, y, scale=None):
    """sum_k alpha_k s_k sin(pi k1 x) sin(pi k2 y) at points (x, y) for every
    coefficient array in alpha (count, M, M); returns (count, npts).  Points on
    a tensor grid (any order) are evaluated through the grid."""
    alpha = np.asarray(alpha, dtype=np.float64)
    if scale is not None:
        alpha = alpha * scale
    M = alpha.shape[-1]
    ux, ix = np.unique(np.asarray(x, dtype=np.float64), return_inverse=True)
    uy, iy = np.unique(np.asarray(y, dtype=np.float64), return_inverse=True)
    Sx, Sy = _sine_table(ux, M), _sine_table(uy, M)
    out = np.empty((alpha.shape[0], len(ix)))
    for c in range(alpha.shape[0]):
        grid = (Sx @ alpha[c]) @ Sy.T          # grid[i, j] = f(ux[i], uy[j])
        out[c] = grid[ix, iy]
    return out


def fourier_source(alpha, x, y):
    """Source f of every coefficient array (Poisson: f = -Lap u)."""
    return fourier_series_at(alpha, x, y)


def fourier_exact(alpha, x, y):
    """Exact Poisson solution of every coefficient array."""
    M = np.asarray(alpha).shape[-1]
    _, w = _modes(M)
    return fourier_series_at(alpha, x, y, scale=1.0 / (math.pi ** 2 * (w - 1.0)))


# ---------------------------------------------------------------------------
# Initial weights of the interface-predicting MLP (random numbers only).
# ---------------------------------------------------------------------------

def mlp_dims(in_dim: int, out_dim: int, hidden: int = 512):
    """Layer widths (in, hidden, hidden, out)."""
    return (in_dim, hidden, hidden, out_dim)


def mlp_init(dims, seed: int):
    """Flat float32 parameter vector: for each layer (fan_in -> fan_out) its
    weight matrix (fan_out x fan_in, column-major), then its bias, all
    i.i.d. U[-1/sqrt(fan_in), 1/sqrt(fan_in)]."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        lim = 1.0 / math.sqrt(fi)
        parts.append(rng.uniform(-lim, lim, fo * fi))
        parts.append(rng.uniform(-lim, lim, fo))
    return np.concatenate(parts).astype(np.float32)


# ---------------------------------------------------------------------------
# Ragged batch of independent variable-coefficient problems: subdomain grid
# from {4x4, 8x8, 16x16}, neurons per subdomain from {100, 200, 400, 800},
# k1, k2 from {1, 2, 3}; q = round(2 sqrt(n)) interior points per direction
# (q^2 ~ 4n), q points per edge, weights and biases U[-sqrt(n)/5, sqrt(n)/5].
# ---------------------------------------------------------------------------

def ragged_problems(count: int = 256, seed: int = 3000, grids=(4, 8, 16), neurons=(100, 200, 400, 800)):
    """Problem p is drawn from numpy.random.default_rng([seed, p]); its hidden
    layer seed is seed + p."""
    out = []
    for p in range(count):
        rng = np.random.default_rng([seed, p])
        g = int(grids[rng.integers(len(grids))])
        n = int(neurons[rng.integers(len(neurons))])
        k1, k2 = (int(v) for v in rng.integers(1, 4, size=2))
        q = int(round(2.0 * math.sqrt(n)))
        out.append(Problem(nsub_x=g, nsub_y=g, neurons=n, q_x=q, q_y=q, m_bdry_edge=q, m_ifc_edge=q,
                           op=OP_VARCOEF, R=math.sqrt(n) / 5.0, k1=k1, k2=k2))
    return out
