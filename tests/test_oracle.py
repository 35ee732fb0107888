"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each pin is independent of the oracle's own formulas: finite differences,
closed forms, textbook routines (lstsq, pinv), brute-force global matrices,
and invariants (symmetry, positive definiteness, optimality).
"""
import dataclasses
import math

import numpy as np
import pytest

import workload as wl
from oracle import ddm, literal
from oracle.layout import build_layout, owner_subdomain


def tiny(nx, ny, n=16, q=6, mb=5, mg=4, op=wl.OP_POISSON, R=1.5):
    return wl.Problem(nsub_x=nx, nsub_y=ny, neurons=n, q_x=q, q_y=q, m_bdry_edge=mb,
                      m_ifc_edge=mg, op=op, R=R, k1=1, k2=2)


def setup(P, seed=11):
    lay = build_layout(P)
    W, b = wl.hidden_params(P, seed)
    data = ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient)
    return lay, W, b, data


# ---------------------------------------------------------------------------
# Layout (Section 3: interior, boundary and interface points)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (1, 3), (2, 2), (3, 2), (4, 4)])
def test_layout_structure(nx, ny):
    P = tiny(nx, ny, mb=3, mg=5)
    lay = build_layout(P)
    assert lay.n_interface == P.n_interface
    seen = {}
    for s, sub in enumerate(lay.subs):
        assert sub.sy * nx + sub.sx == s
        assert len(sub.interior) == P.q_x * P.q_y
        # every point of the subdomain lies in its closed box, interior strictly inside
        for pts in (sub.interior, sub.boundary, sub.interface):
            assert np.all(pts[:, 0] >= sub.xa - 1e-15) and np.all(pts[:, 0] <= sub.xa + sub.hx + 1e-15)
            assert np.all(pts[:, 1] >= sub.ya - 1e-15) and np.all(pts[:, 1] <= sub.ya + sub.hy + 1e-15)
        assert np.all(owner_subdomain(P, sub.interior[:, 0], sub.interior[:, 1]) == s)
        n_ext = (sub.sx == 0) + (sub.sx == nx - 1) + (sub.sy == 0) + (sub.sy == ny - 1)
        assert len(sub.boundary) == n_ext * P.m_bdry_edge
        assert len(sub.interface) == (4 - n_ext) * P.m_ifc_edge
        # boundary points lie on the outer boundary
        bx, by = sub.boundary[:, 0], sub.boundary[:, 1]
        on = (np.isclose(bx, 0) | np.isclose(bx, 1) | np.isclose(by, 0) | np.isclose(by, 1))
        assert np.all(on)
        for k, gi in enumerate(sub.gidx):
            seen.setdefault(int(gi), []).append((s, sub.interface[k], sub.normals[k]))
    # each interface unknown is shared by exactly two subdomains, same point, opposite normals
    assert sorted(seen) == list(range(lay.n_interface))
    for gi, lst in seen.items():
        assert len(lst) == 2
        (s0, p0, n0), (s1, p1, n1) = lst
        assert s0 != s1
        assert np.array_equal(p0, p1)
        assert np.array_equal(n0, -n1)
        assert np.array_equal(p0, lay.interface_points[gi])
        # the normal points from s0 toward s1
        c0 = np.array(lay.subs[s0].center)
        c1 = np.array(lay.subs[s1].center)
        assert (c1 - c0) @ n0 > 0
    # all points of a subdomain are distinct (the Proposition's distinct samples)
    for sub in lay.subs:
        allp = np.concatenate([sub.interior, sub.boundary, sub.interface])
        assert len(np.unique(allp, axis=0)) == len(allp)


# ---------------------------------------------------------------------------
# Features and operator rows vs finite differences
# ---------------------------------------------------------------------------

def test_feature_derivatives_match_finite_differences():
    rng = np.random.default_rng(3)
    n = 7
    W = rng.uniform(-3, 3, (n, 2))
    b = rng.uniform(-3, 3, n)
    center, h = (0.3, 0.6), (0.25, 0.5)
    pts = np.stack([rng.uniform(0.2, 0.4, 9), rng.uniform(0.4, 0.8, 9)], 1)

    def phi(p):
        xh = 2 * (p[:, 0:1] - center[0]) / h[0]
        yh = 2 * (p[:, 1:2] - center[1]) / h[1]
        return np.tanh(xh * W[:, 0] + yh * W[:, 1] + b)

    t, px, py, lap = ddm.features(W, b, center, h, pts)
    assert np.allclose(t, phi(pts), rtol=0, atol=1e-15)
    e = 1e-6
    ex = np.array([e, 0.0])
    ey = np.array([0.0, e])
    fx = (phi(pts + ex) - phi(pts - ex)) / (2 * e)
    fy = (phi(pts + ey) - phi(pts - ey)) / (2 * e)
    assert np.allclose(px, fx, rtol=1e-7, atol=1e-7)
    assert np.allclose(py, fy, rtol=1e-7, atol=1e-7)
    e = 1e-4
    ex = np.array([e, 0.0])
    ey = np.array([0.0, e])
    flap = (phi(pts + ex) + phi(pts - ex) + phi(pts + ey) + phi(pts - ey) - 4 * phi(pts)) / e**2
    scale = np.abs(lap).max()
    assert np.abs(lap - flap).max() < 1e-5 * scale


def test_varcoef_operator_rows_match_finite_differences():
    P = tiny(2, 2, op=wl.OP_VARCOEF)
    rng = np.random.default_rng(4)
    n = 5
    W = rng.uniform(-2, 2, (n, 2))
    b = rng.uniform(-2, 2, n)
    center, h = (0.25, 0.75), (0.5, 0.5)
    pts = np.stack([rng.uniform(0.05, 0.45, 6), rng.uniform(0.55, 0.95, 6)], 1)
    coef = wl.coefficient(P, pts[:, 0], pts[:, 1])
    rows = ddm.operator_rows(P, W, b, center, h, pts, coef)

    def phi(p):
        return ddm.features(W, b, center, h, p)[0]

    def a(p):
        return wl.coefficient(P, p[:, 0], p[:, 1])[0][:, None]

    # -div(a grad phi) by nested central differences of the flux a * dphi
    e = 1e-4
    ex = np.array([e, 0.0])
    ey = np.array([0.0, e])
    fxp = a(pts + ex / 2) * (phi(pts + ex) - phi(pts)) / e
    fxm = a(pts - ex / 2) * (phi(pts) - phi(pts - ex)) / e
    fyp = a(pts + ey / 2) * (phi(pts + ey) - phi(pts)) / e
    fym = a(pts - ey / 2) * (phi(pts) - phi(pts - ey)) / e
    fd = -((fxp - fxm) / e + (fyp - fym) / e)
    assert np.abs(rows - fd).max() < 1e-5 * np.abs(rows).max()


@pytest.mark.parametrize("op", [wl.OP_POISSON, wl.OP_VARCOEF])
def test_manufactured_source_matches_finite_differences(op):
    P = tiny(2, 2, op=op)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 0.95, 20)
    y = rng.uniform(0.05, 0.95, 20)
    e = 1e-4

    def u(x, y):
        return wl.exact_u(P, x, y)

    def a(x, y):
        return wl.coefficient(P, x, y)[0]

    fd = -((a(x + e / 2, y) * (u(x + e, y) - u(x, y)) - a(x - e / 2, y) * (u(x, y) - u(x - e, y))) / e**2
           + (a(x, y + e / 2) * (u(x, y + e) - u(x, y)) - a(x, y - e / 2) * (u(x, y) - u(x, y - e))) / e**2)
    f = wl.source_f(P, x, y)
    assert np.abs(f - fd).max() < 1e-5 * np.abs(f).max()
    if op == wl.OP_POISSON:
        assert np.allclose(f, 2 * math.pi**2 * u(x, y), rtol=1e-14, atol=0)
    _, ax, ay = wl.coefficient(P, x, y)
    assert np.allclose(ax, (a(x + e, y) - a(x - e, y)) / (2 * e), atol=1e-6)
    assert np.allclose(ay, (a(x, y + e) - a(x, y - e)) / (2 * e), atol=1e-6)


# ---------------------------------------------------------------------------
# Single domain: the method is plain ELM least squares
# ---------------------------------------------------------------------------

def test_single_domain_is_plain_elm_least_squares():
    """N = 1x1 has no interface; Algorithm 1 reduces to the ELM solution
    trained on the whole domain (Section 4.2, the N = 1x1 rows)."""
    P = tiny(1, 1, n=40, q=12, mb=10)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    assert sol.u_gamma.shape == (0,)
    blk = sol.blocks[0]
    c_ls = np.linalg.lstsq(blk.K, blk.F, rcond=None)[0]
    ex, ey = wl.eval_grid(P, 8)
    uh = ddm.evaluate(P, lay, W, b, sol.c, ex, ey)
    uls = ddm.evaluate(P, lay, W, b, [c_ls], ex, ey)
    assert ddm.rel_l2(uh, uls) < 1e-9


# ---------------------------------------------------------------------------
# Block algebra vs the literal global formula (eq. schur with pinv)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,op", [(1, 2, wl.OP_POISSON), (2, 2, wl.OP_POISSON),
                                      (2, 3, wl.OP_POISSON), (2, 2, wl.OP_VARCOEF)])
def test_schur_matches_literal_pseudo_inverse_form(nx, ny, op):
    P = tiny(nx, ny, op=op)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    K, A, B, F, _ = literal.global_matrices(P, lay, W, b, data)
    S_lit, g_lit = literal.schur_literal(K, A, B, F)
    assert np.linalg.norm(sol.S - S_lit) <= 1e-10 * np.linalg.norm(S_lit)
    assert np.linalg.norm(sol.g - g_lit) <= 1e-10 * np.linalg.norm(g_lit)


@pytest.mark.parametrize("nx,ny", [(2, 1), (2, 2), (3, 2)])
def test_ddm_equals_monolithic_eliminated_least_squares(nx, ny):
    """The DDM returns the least-squares solution of eq. eliminated (eq. LS_system)."""
    P = tiny(nx, ny)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    K, A, B, F, _ = literal.global_matrices(P, lay, W, b, data)
    c_m, u_m = literal.eliminated_lstsq(K, A, B, F)
    assert ddm.rel_l2(sol.u_gamma, u_m) < 1e-8
    assert ddm.rel_l2(K @ np.concatenate(sol.c), K @ c_m) < 1e-8


def test_ddm_is_not_the_least_squares_of_the_original_system():
    """The method solves the eliminated system, a different estimator: its
    original-system residual is no smaller than the original LS optimum."""
    P = tiny(2, 2)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    K, A, B, F, _ = literal.global_matrices(P, lay, W, b, data)
    c_o, u_o = literal.original_lstsq(K, A, B, F)
    J_ddm = literal.original_objective(K, A, B, F, np.concatenate(sol.c), sol.u_gamma)
    J_opt = literal.original_objective(K, A, B, F, c_o, u_o)
    assert J_ddm >= J_opt * (1 - 1e-9)
    assert ddm.rel_l2(sol.u_gamma, u_o) > 1e-8


def test_interface_solution_minimises_the_eliminated_objective():
    P = tiny(3, 2)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    kps = [ddm.KPlus(blk.K) for blk in sol.blocks]
    J0 = ddm.ddm_objective(lay, sol.blocks, kps, sol.u_gamma)
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = rng.standard_normal(len(sol.u_gamma)) * 1e-3
        assert ddm.ddm_objective(lay, sol.blocks, kps, sol.u_gamma + d) >= J0
    # the gradient of J at the solution vanishes: J(u + d) - J(u) = d^T S d
    d = rng.standard_normal(len(sol.u_gamma)) * 1e-2
    dJ = ddm.ddm_objective(lay, sol.blocks, kps, sol.u_gamma + d) - J0
    assert abs(dJ - d @ sol.S @ d) < 1e-6 * abs(dJ)


# ---------------------------------------------------------------------------
# Invariants of S, back-solve, solvers
# ---------------------------------------------------------------------------

def test_schur_matrix_symmetric_positive_definite():
    P = tiny(3, 3, n=24, q=7)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    S = sol.S
    assert np.abs(S - S.T).max() <= 1e-14 * np.abs(S).max()
    ev = np.linalg.eigvalsh(S)
    assert ev[0] > 0
    # every local I - T_s = b^T (I - K K^+) b is a compression of a projector:
    for sub, blk in zip(lay.subs, sol.blocks):
        kp = ddm.KPlus(blk.K)
        bs = ddm.local_B(blk)
        loc = bs.T @ (bs - kp.project(bs))
        e = np.linalg.eigvalsh(0.5 * (loc + loc.T))
        assert e[0] > -1e-12 and e[-1] < 1 + 1e-12


def test_backsolve_satisfies_local_normal_equations():
    P = tiny(2, 3, n=20, q=7)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    for sub, blk, c in zip(lay.subs, sol.blocks, sol.c):
        r = blk.K @ c - blk.F
        if blk.n_ifc:
            r += ddm.local_B(blk) @ sol.u_gamma[sub.gidx]
        nr = np.linalg.norm(blk.K.T @ r)
        assert nr <= 1e-9 * np.linalg.norm(blk.K) * (np.linalg.norm(blk.K) * np.linalg.norm(c) + np.linalg.norm(blk.F))


def test_cg_matches_cholesky():
    P = tiny(3, 3, n=24, q=7)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    u_cg, it = ddm.solve_interface_cg(sol.S, sol.g, tol=1e-14)
    assert it > 0
    assert ddm.rel_l2(u_cg, sol.u_gamma) < 1e-11
    sol9 = ddm.solve(P, W, b, data, lay, interface_solver="cg", cg_tol=1e-9)
    assert np.linalg.norm(sol.S @ sol9.u_gamma - sol.g) < 1e-9 * np.linalg.norm(sol.g)


def test_column_scaling_leaves_solution_unchanged():
    """Scaling feature columns by positive factors rescales c only: u_Gamma and u_h are invariant."""
    P = tiny(2, 2, n=20, q=7)
    lay, W, b, data = setup(P)
    sol = ddm.solve(P, W, b, data, lay)
    rng = np.random.default_rng(9)
    blocks2 = []
    dscale = []
    for blk in sol.blocks:
        d = np.exp(rng.uniform(-3, 3, blk.K.shape[1]))
        dscale.append(d)
        blocks2.append(dataclasses.replace(blk, K=blk.K * d, D=blk.D * d))
    S2, g2, kps2 = ddm.schur_system(P, lay, blocks2)
    u2 = ddm.solve_interface_direct(S2, g2)
    c2 = ddm.backsolve(lay, blocks2, kps2, u2)
    assert ddm.rel_l2(u2, sol.u_gamma) < 1e-11
    for c, cc, d in zip(sol.c, c2, dscale):
        assert ddm.rel_l2(cc * d, c) < 1e-9


# ---------------------------------------------------------------------------
# Method accuracy against the manufactured solution
# ---------------------------------------------------------------------------

def test_small_config_accuracy_vs_exact_solution():
    P = wl.CONFIG_SMALL
    lay, W, b, data = setup(P, seed=1000)
    sol = ddm.solve(P, W, b, data, lay)
    ex, ey = wl.eval_grid(P)
    uh = ddm.evaluate(P, lay, W, b, sol.c, ex, ey)
    err = ddm.rel_l2(uh, wl.exact_u(P, ex, ey))
    assert err < 2e-2
    ip = lay.interface_points
    assert ddm.rel_l2(sol.u_gamma, wl.exact_u(P, ip[:, 0], ip[:, 1])) < 5e-2


def test_accuracy_improves_with_more_neurons():
    errs = []
    for n, q in [(30, 10), (80, 16), (160, 24)]:
        P = wl.Problem(nsub_x=2, nsub_y=2, neurons=n, q_x=q, q_y=q, m_bdry_edge=q, m_ifc_edge=q, R=2.0)
        lay, W, b, data = setup(P, seed=5)
        sol = ddm.solve(P, W, b, data, lay)
        ex, ey = wl.eval_grid(P, 10)
        errs.append(ddm.rel_l2(ddm.evaluate(P, lay, W, b, sol.c, ex, ey), wl.exact_u(P, ex, ey)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_varcoef_accuracy_vs_exact_solution():
    P = wl.Problem(nsub_x=2, nsub_y=2, neurons=160, q_x=24, q_y=24, m_bdry_edge=24, m_ifc_edge=24,
                   op=wl.OP_VARCOEF, R=2.5, k1=1, k2=2)
    lay, W, b, data = setup(P, seed=8)
    sol = ddm.solve(P, W, b, data, lay)
    ex, ey = wl.eval_grid(P, 10)
    assert ddm.rel_l2(ddm.evaluate(P, lay, W, b, sol.c, ex, ey), wl.exact_u(P, ex, ey)) < 1e-2


# ---------------------------------------------------------------------------
# Planted mistakes: each must be caught by one of the pins above
# ---------------------------------------------------------------------------

def test_planted_flux_sign_error_is_caught(monkeypatch):
    """A wrong normal direction breaks flux continuity: the solution no longer
    approximates the manufactured solution."""
    P = wl.Problem(nsub_x=2, nsub_y=2, neurons=80, q_x=16, q_y=16, m_bdry_edge=16, m_ifc_edge=16, R=2.0)
    lay, W, b, data = setup(P, seed=5)
    for sub in lay.subs:
        sub.normals = sub.normals.copy()
        sub.normals[:, 0] *= -1          # planted: x-normal flipped
    sol = ddm.solve(P, W, b, data, lay)
    ex, ey = wl.eval_grid(P, 10)
    assert ddm.rel_l2(ddm.evaluate(P, lay, W, b, sol.c, ex, ey), wl.exact_u(P, ex, ey)) > 1e-2


def test_planted_missing_flux_term_is_caught(monkeypatch):
    """Dropping the M^T M term of S makes it differ from the literal eq. schur."""
    P = tiny(2, 2)
    lay, W, b, data = setup(P)
    K, A, B, F, blocks = literal.global_matrices(P, lay, W, b, data)
    S_lit, _ = literal.schur_literal(K, A, B, F)
    real = ddm.sp.csr_matrix

    def zero_csr(arg, shape):            # planted: every entry of M dropped
        vals, ij = arg
        return real((np.zeros_like(vals), ij), shape=shape)

    monkeypatch.setattr(ddm.sp, "csr_matrix", zero_csr)
    S_bad, _, _ = ddm.schur_system(P, lay, blocks)
    assert np.linalg.norm(S_bad - S_lit) > 1e-3 * np.linalg.norm(S_lit)


def test_solution_gradient_matches_finite_differences_of_the_solution():
    """grad u_h (for the H1 error of Table 2) against central differences of
    u_h itself, at points inside subdomains (away from the box edges, where
    the owning network changes); the value output equals evaluate()."""
    P = tiny(2, 2, n=24)
    lay, W, b, data = setup(P, seed=5)
    sol = ddm.solve(P, W, b, data, lay)
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(0.05, 0.45, 12), rng.uniform(0.55, 0.95, 12)])
    y = np.concatenate([rng.uniform(0.55, 0.95, 12), rng.uniform(0.05, 0.45, 12)])
    u, ux, uy = ddm.evaluate_grad(P, lay, W, b, sol.c, x, y)
    assert np.array_equal(u, ddm.evaluate(P, lay, W, b, sol.c, x, y))
    h = 1e-6
    ev = lambda xx, yy: ddm.evaluate(P, lay, W, b, sol.c, xx, yy)
    fdx = (ev(x + h, y) - ev(x - h, y)) / (2 * h)
    fdy = (ev(x, y + h) - ev(x, y - h)) / (2 * h)
    scale = max(np.abs(ux).max(), np.abs(uy).max())
    assert np.abs(ux - fdx).max() <= 1e-6 * scale and np.abs(uy - fdy).max() <= 1e-6 * scale
