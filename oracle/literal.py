"""Brute-force global forms for tiny problems (oracle pins only).

Builds the global matrices of eq. discrete-simple,
    [K B; A 0] [c; u] = [F; 0],   K = diag(K^s), A = [A^1 ... A^N], B = [B^1; ...; B^N],
densely, and evaluates the paper's formulas literally:

* eq. schur with K^+ taken as the Moore-Penrose pseudo-inverse (numpy.linalg.pinv);
* the least squares of the eliminated system (eq. eliminated),
      [K B; 0 -A K^+ B] [c; u] ~ [F; -A K^+ F],
  solved by numpy.linalg.lstsq -- the "monolithic" problem whose solution the
  DDM must reproduce (eq. LS_system);
* the least squares of the original system eq. nonoverlap_discrete, which is
  a different estimator (the DDM solves the eliminated system instead).

Only sensible for a few subdomains and a few dozen neurons.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .ddm import assemble_local, local_B


def global_matrices(problem, layout, W, b, data):
    blocks = [assemble_local(problem, sub, W[s], b[s], *data[s]) for s, sub in enumerate(layout.subs)]
    K = sla.block_diag(*[blk.K for blk in blocks])
    nG = layout.n_interface
    m_tot = K.shape[0]
    n_off = np.cumsum([0] + [blk.K.shape[1] for blk in blocks])
    m_off = np.cumsum([0] + [blk.K.shape[0] for blk in blocks])
    B = np.zeros((m_tot, nG))
    A = np.zeros((nG, K.shape[1]))
    F = np.concatenate([blk.F for blk in blocks])
    for s, (sub, blk) in enumerate(zip(layout.subs, blocks)):
        if blk.n_ifc == 0:
            continue
        B[m_off[s]:m_off[s + 1], sub.gidx] = local_B(blk)
        A[sub.gidx, n_off[s]:n_off[s + 1]] = blk.D
    return K, A, B, F, blocks


def schur_literal(K, A, B, F):
    """Operator and right-hand side of eq. schur with K^+ = pinv(K)."""
    Kp = np.linalg.pinv(K)
    I = np.eye(K.shape[0])
    Op = I + Kp.T @ A.T @ A @ Kp - K @ Kp
    return B.T @ Op @ B, B.T @ Op @ F


def eliminated_lstsq(K, A, B, F):
    """(c, u) = least-squares solution of eq. eliminated (the DDM's monolithic problem)."""
    Kp = np.linalg.pinv(K)
    top = np.hstack([K, B])
    bot = np.hstack([np.zeros((A.shape[0], K.shape[1])), -A @ Kp @ B])
    M = np.vstack([top, bot])
    rhs = np.concatenate([F, -A @ Kp @ F])
    sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
    n = K.shape[1]
    return sol[:n], sol[n:]


def original_lstsq(K, A, B, F):
    """(c, u) = least-squares solution of eq. nonoverlap_discrete itself."""
    M = np.vstack([np.hstack([K, B]), np.hstack([A, np.zeros((A.shape[0], B.shape[1]))])])
    rhs = np.concatenate([F, np.zeros(A.shape[0])])
    sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
    n = K.shape[1]
    return sol[:n], sol[n:]


def original_objective(K, A, B, F, c, u):
    """||K c + B u - F||^2 + ||A c||^2 (residual of eq. nonoverlap_discrete)."""
    r1 = K @ c + B @ u - F
    r2 = A @ c
    return float(r1 @ r1 + r2 @ r2)
