"""Nonoverlapping DDM for ELM, FP64 oracle (test infrastructure only).

Follows the paper step by step:

* Section 3: local one-hidden-layer networks u_s(x) = sum_j c_j^s phi_j^s(x)
  with phi_j^s(x) = tanh(w_j^s . x + b_j^s) (Section 4.1); blocks
  K^s = [L phi(x_i); phi(x_b); phi(x_Gamma)], A^s = d phi / d n_s (x_Gamma),
  B^s = [0; 0; -I], F^s = [f(x_i); g(x_b); 0]  (eq. nonoverlap_discrete).
* Section 3: the Schur complement system (eq. schur)
      B^T (I + K^{+T} A^T A K^+ - K K^+) B u = B^T (I + K^{+T} A^T A K^+ - K K^+) F
  with K = diag(K^s) block diagonal, K^+ = (K^T K)^{-1} K^T.
* Algorithm 1: build the local blocks, solve the interface system (CG in the
  paper, dense Cholesky as the exact judge here), then solve
  K^{sT} K^s c^s = K^{sT} (F^s - B^s u) in every subdomain.

K^+ is applied through a Householder QR of K^s (numpy.linalg.qr): in exact
arithmetic R^{-1} Q^T = (K^T K)^{-1} K^T, and the QR route keeps the error
proportional to cond(K) instead of cond(K)^2.

Coordinates: every local network sees subdomain-local coordinates
xhat = 2 (x - x_c) / h_x, yhat = 2 (y - y_c) / h_y in [-1, 1]^2, so
d/dx = (2/h_x) d/dxhat.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .layout import build_layout, owner_subdomain

OP_POISSON = 0
OP_VARCOEF = 1


# ---------------------------------------------------------------------------
# Features (Section 4.1: phi = sigma(w . x + b), sigma = tanh)
# ---------------------------------------------------------------------------

def features(W, b, center, h, pts):
    """tanh features and their derivatives at pts (physical coordinates).

    Returns phi, phi_x, phi_y, lap_phi, each (npts, n).
    sigma' = 1 - t^2, sigma'' = -2 t (1 - t^2) for t = tanh(z).
    """
    sx, sy = 2.0 / h[0], 2.0 / h[1]
    xh = (pts[:, 0:1] - center[0]) * sx
    yh = (pts[:, 1:2] - center[1]) * sy
    z = xh * W[:, 0][None, :] + yh * W[:, 1][None, :] + b[None, :]
    t = np.tanh(z)
    d1 = 1.0 - t * t
    d2 = -2.0 * t * d1
    wx = W[:, 0][None, :] * sx
    wy = W[:, 1][None, :] * sy
    return t, d1 * wx, d1 * wy, d2 * (wx * wx + wy * wy)


def operator_rows(problem, W, b, center, h, pts, coef):
    """Rows L phi_j at interior points.

    Poisson: L = -Laplace.  Variable coefficient: L u = -div(a grad u)
    = -a Lap u - grad a . grad u, with (a, a_x, a_y) given at the points.
    """
    _, px, py, lap = features(W, b, center, h, pts)
    if problem.op == OP_POISSON:
        return -lap
    a, ax, ay = coef
    return -(a[:, None] * lap) - (ax[:, None] * px + ay[:, None] * py)


@dataclasses.dataclass
class LocalBlocks:
    K: np.ndarray   # (m_s, n)  rows [interior; boundary; interface]
    D: np.ndarray   # (k_s, n)  outward normal derivative at the interface points (rows of A^s)
    F: np.ndarray   # (m_s,)
    n_int: int
    n_bnd: int
    n_ifc: int


def assemble_local(problem, sub, W, b, f_int, g_bnd, coef=None) -> LocalBlocks:
    """K^s, A^s (as D), F^s of eq. nonoverlap_discrete for one subdomain."""
    center, h = sub.center, (sub.hx, sub.hy)
    KI = operator_rows(problem, W, b, center, h, sub.interior, coef)
    Kb = features(W, b, center, h, sub.boundary)[0]
    Kg, gx, gy, _ = features(W, b, center, h, sub.interface)
    D = sub.normals[:, 0:1] * gx + sub.normals[:, 1:2] * gy
    K = np.vstack([KI, Kb, Kg])
    F = np.concatenate([f_int, g_bnd, np.zeros(len(sub.interface))])
    return LocalBlocks(K=K, D=D, F=F, n_int=len(sub.interior), n_bnd=len(sub.boundary),
                       n_ifc=len(sub.interface))


def local_B(blk: LocalBlocks):
    """B^s restricted to the subdomain's own interface unknowns: [0; 0; -I] (m_s x k_s)."""
    m, k = blk.K.shape[0], blk.n_ifc
    Bs = np.zeros((m, k))
    Bs[m - k:, :] = -np.eye(k)
    return Bs


class KPlus:
    """K^+ = (K^T K)^{-1} K^T applied through a Householder QR of K."""

    def __init__(self, K):
        self.Q, self.R = np.linalg.qr(K, mode="reduced")

    def apply(self, X):
        """K^+ X."""
        return sla.solve_triangular(self.R, self.Q.T @ X, lower=False)

    def project(self, X):
        """K K^+ X = Q Q^T X (orthogonal projection onto range K)."""
        return self.Q @ (self.Q.T @ X)


# ---------------------------------------------------------------------------
# Problem data at the oracle's own points
# ---------------------------------------------------------------------------

def problem_data(problem, layout, source_f, boundary_g, coefficient=None):
    """Source at interior points, Dirichlet data at boundary points, coefficients."""
    data = []
    for sub in layout.subs:
        f = source_f(problem, sub.interior[:, 0], sub.interior[:, 1])
        g = boundary_g(problem, sub.boundary[:, 0], sub.boundary[:, 1])
        coef = None
        if problem.op == OP_VARCOEF:
            coef = coefficient(problem, sub.interior[:, 0], sub.interior[:, 1])
        data.append((f, g, coef))
    return data


# ---------------------------------------------------------------------------
# The method
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Solution:
    u_gamma: np.ndarray
    c: list            # per subdomain output-layer coefficients
    S: np.ndarray
    g: np.ndarray
    blocks: list
    cg_iters: int = 0


def schur_system(problem, layout, blocks):
    """S and its right-hand side of eq. schur, from per-subdomain pieces.

    With K = diag(K^s) and B^s = -P_s R_s (P_s picks the interface rows,
    R_s restricts u to the subdomain's interface points),
      B^T (I - K K^+) B  = sum_s R_s^T [b_s^T (I - K_s K_s^+) b_s] R_s,  b_s = [0;0;-I],
      A K^+ B            = sum_s E_s D_s K_s^+ b_s R_s   =: M  (E_s places the
                           flux rows of s into the global flux numbering),
      S = B^T (I - K K^+) B + M^T M,
      rhs = B^T (I - K K^+) F + M^T (A K^+ F).
    """
    nG = layout.n_interface
    S = np.zeros((nG, nG))
    rhs = np.zeros(nG)
    AKF = np.zeros(nG)
    rows, cols, vals = [], [], []
    kps = []
    for sub, blk in zip(layout.subs, blocks):
        kp = KPlus(blk.K)
        kps.append(kp)
        gi = sub.gidx
        if len(gi) == 0:
            continue
        bs = local_B(blk)
        res_b = bs - kp.project(bs)                 # (I - K K^+) b_s
        S[np.ix_(gi, gi)] += bs.T @ res_b
        rhs[gi] += res_b.T @ blk.F                  # b_s^T (I - KK^+) F  (symmetric projector)
        Mloc = blk.D @ kp.apply(bs)                 # D_s K_s^+ b_s   (k_s x k_s)
        r_, c_ = np.meshgrid(gi, gi, indexing="ij")
        rows.append(r_.ravel()); cols.append(c_.ravel()); vals.append(Mloc.ravel())
        AKF[gi] += blk.D @ kp.apply(blk.F)          # A K^+ F, flux rows of s
    if nG:
        M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nG, nG))
        S += (M.T @ M).toarray()
        rhs += M.T @ AKF
    return S, rhs, kps


def solve_interface_direct(S, rhs):
    """Exact judge: dense Cholesky of the SPD Schur matrix (Section 3: S is SPD)."""
    if S.shape[0] == 0:
        return np.zeros(0)
    cf = sla.cho_factor(S, lower=True)
    return sla.cho_solve(cf, rhs)


def solve_interface_cg(S, rhs, tol=1e-9, max_iter=None, x0=None):
    """Conjugate gradients on S u = rhs, stopping at ||r|| / ||rhs|| < tol
    (Section 4: the paper's stopping rule with tol = 1e-9)."""
    n = S.shape[0]
    max_iter = max_iter or 10 * n
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = rhs - S @ x
    p = r.copy()
    rr = r @ r
    nb = np.linalg.norm(rhs)
    it = 0
    while np.sqrt(rr) >= tol * nb and it < max_iter:
        Sp = S @ p
        alpha = rr / (p @ Sp)
        x += alpha * p
        r -= alpha * Sp
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def backsolve(layout, blocks, kps, u):
    """Algorithm 1, last loop: K^{sT} K^s c^s = K^{sT} (F^s - B^s u), i.e. c^s = K_s^+ (F^s - B^s u)."""
    cs = []
    for sub, blk, kp in zip(layout.subs, blocks, kps):
        rhs = blk.F.copy()
        if blk.n_ifc:
            rhs -= local_B(blk) @ u[sub.gidx]
        cs.append(kp.apply(rhs))
    return cs


def solve(problem, W, b, data, layout=None, interface_solver="direct", cg_tol=1e-9):
    """Algorithm 1 end to end.  data[s] = (f at interior pts, g at boundary pts, coef or None)."""
    layout = layout or build_layout(problem)
    blocks = [assemble_local(problem, sub, W[s], b[s], *data[s])
              for s, sub in enumerate(layout.subs)]
    S, rhs, kps = schur_system(problem, layout, blocks)
    iters = 0
    if interface_solver == "direct":
        u = solve_interface_direct(S, rhs)
    else:
        u, iters = solve_interface_cg(S, rhs, tol=cg_tol)
    cs = backsolve(layout, blocks, kps, u)
    return Solution(u_gamma=u, c=cs, S=S, g=rhs, blocks=blocks, cg_iters=iters)


def evaluate(problem, layout, W, b, cs, x, y):
    """u_h at arbitrary points: the local network of the owning subdomain."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    own = owner_subdomain(problem, x, y)
    out = np.zeros(len(x))
    for s, sub in enumerate(layout.subs):
        sel = np.nonzero(own == s)[0]
        if len(sel) == 0:
            continue
        pts = np.stack([x[sel], y[sel]], axis=1)
        out[sel] = features(W[s], b[s], sub.center, (sub.hx, sub.hy), pts)[0] @ cs[s]
    return out


def evaluate_grad(problem, layout, W, b, cs, x, y):
    """u_h and its gradient (u_x, u_y) at arbitrary points, from the owning
    subdomain's network: grad phi_j = sigma'(z_j) (w_j scaled by 2 / h)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    own = owner_subdomain(problem, x, y)
    u, ux, uy = np.zeros(len(x)), np.zeros(len(x)), np.zeros(len(x))
    for s, sub in enumerate(layout.subs):
        sel = np.nonzero(own == s)[0]
        if len(sel) == 0:
            continue
        pts = np.stack([x[sel], y[sel]], axis=1)
        phi, px, py, _ = features(W[s], b[s], sub.center, (sub.hx, sub.hy), pts)
        u[sel], ux[sel], uy[sel] = phi @ cs[s], px @ cs[s], py @ cs[s]
    return u, ux, uy


def ddm_objective(layout, blocks, kps, u):
    """J(u) = ||(I - K K^+)(F - B u)||^2 + ||A K^+ (F - B u)||^2, the least-squares
    objective of eq. eliminated after minimising over c (eq. LS_system)."""
    nG = layout.n_interface
    flux = np.zeros(nG)
    J = 0.0
    for sub, blk, kp in zip(layout.subs, blocks, kps):
        r = blk.F.copy()
        if blk.n_ifc:
            r -= local_B(blk) @ u[sub.gidx]
        res = r - kp.project(r)
        J += res @ res
        if blk.n_ifc:
            flux[sub.gidx] += blk.D @ kp.apply(r)
    return J + flux @ flux


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
