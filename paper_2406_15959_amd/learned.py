"""Learned interface variable: orchestration of the library calls.

For a fixed geometry and hidden layer, the method's own per-source solves
(elmddm_solve_rhs) generate (source features -> u_Gamma) pairs; the MLP of
the library is trained on them on the GPU and its prediction is used as the
initial guess of the interface CG (elmddm_interface_cg), or accepted
directly when its relative residual ||g - S u|| / ||g|| is at most tau.
Every computation runs in the HIP library; this module only moves
arguments and holds the per-output scale of the targets.
"""
from __future__ import annotations

import numpy as np

from . import binding as B


def generate_pairs(plan, f, nrhs):
    """Exact interface variables u [nrhs][nG] (device, float64) of the sources
    f [nrhs][nsub][q2] (device) through the cached-factor solve."""
    import torch
    u = torch.empty(nrhs * plan.sizes.n_interface, dtype=torch.float64, device=f.device)
    plan.solve_rhs(nrhs, f, None, u)
    return u.view(nrhs, plan.sizes.n_interface)


def train(net, X, U, steps, batch, lr, order, losses=None):
    """Train net on features X [ns][in] (float32, device) and targets U
    [ns][nG] (float64, device) scaled by their root mean square; returns that
    scale (the prediction is scale * network output)."""
    import torch
    scale = float(torch.sqrt(torch.mean(U * U)).item()) or 1.0
    T = (U / scale).to(torch.float32).contiguous()
    net.train(X.shape[0], X, T, order, steps, batch, lr=lr, losses=losses)
    return scale


def predict(net, X, scale, out=None):
    import torch
    n = X.shape[0]
    if out is None:
        out = torch.empty(n * net.dims[-1], dtype=torch.float64, device=X.device)
    for r0 in range(0, n, net.max_batch):
        r1 = min(n, r0 + net.max_batch)
        net.predict(r1 - r0, X[r0:r1].contiguous(), scale, out[r0 * net.dims[-1]:r1 * net.dims[-1]])
    return out.view(n, net.dims[-1])


def residuals(plan, rhs, u):
    """Relative residuals ||g - S u|| / ||g|| of guesses u (no iteration)."""
    n = rhs.shape[0]
    _, _, res = plan.interface_cg(n, rhs.reshape(-1), u.clone().reshape(-1), 1.0, 0, with_residuals=True)
    return res


def solve_with_guess(plan, rhs, guess, tol, maxit, accept_tau=None):
    """CG from the guesses (the paper's interface solver); a guess whose
    relative residual is <= accept_tau is kept as it is.  Returns
    (u, iterations per system, accepted flags)."""
    import torch
    n = rhs.shape[0]
    u = guess.clone().reshape(n, -1)
    accepted = [False] * n
    if accept_tau is not None:
        res = residuals(plan, rhs, guess)
        accepted = [r <= accept_tau for r in res]
    todo = [i for i in range(n) if not accepted[i]]
    its = [0] * n
    st = B.OK
    if todo:
        idx = torch.tensor(todo, device=rhs.device)
        ut = u[idx].contiguous().reshape(-1)
        st, k = plan.interface_cg(len(todo), rhs[idx].contiguous().reshape(-1), ut, tol, maxit)
        u[idx] = ut.view(len(todo), -1)
        for i, kk in zip(todo, k):
            its[i] = kk
    return u, its, accepted, st
