"""The paper's approximate Gaussian random field workloads (Section 5.2.1,
eq. grf, as a source; Section 5.2.2, rho = tanh(grf) + 1.1, as the
coefficient of -div(rho grad u) = 1) through the GPU path.  There is no
closed-form solution: parity with the oracle on the same data."""
import math

import numpy as np
import pytest

import workload as wl
from gpu_helpers import gpu_solve, oracle_solve, to_c_problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _problem(op):
    n = 200
    q = int(round(2 * math.sqrt(n)))
    return wl.Problem(4, 4, n, q, q, q, q, op=op, R=math.sqrt(n) / 5)


@pytest.mark.parametrize("mode,tol", [(0, 1e-8), (1, 1e-6)])
def test_grf_source_matches_oracle(gpu, mode, tol):
    from paper_2406_15959_amd import binding as B
    P = _problem(wl.OP_POISSON)
    F = wl.grf_params(71, alpha=16.0)
    plan = B.Plan(to_c_problem(P))
    plan.set_mode(mode)
    g = gpu_solve(P, 5, plan=plan, data_fn=lambda P_, ip, bp: wl.grf_source_data(P_, F, ip, bp))
    fns = (lambda P_, x, y: wl.grf_value_and_grad(F, x, y)[0], lambda P_, x, y: np.zeros_like(x), wl.coefficient)
    o = oracle_solve(P, 5, fns=fns)
    assert g["info"].status == 0, (g["info"].status, g["info"].bad_pass)
    assert rel(g["u_gamma"], o["u_gamma"]) <= tol
    assert rel(g["uh"], o["uh"]) <= tol


@pytest.mark.parametrize("mode,tol", [(0, 1e-8), (1, 1e-6)])
def test_grf_coefficient_matches_oracle(gpu, mode, tol):
    from paper_2406_15959_amd import binding as B
    P = _problem(wl.OP_VARCOEF)
    F = wl.grf_params(72, alpha=16.0)
    plan = B.Plan(to_c_problem(P))
    plan.set_mode(mode)
    g = gpu_solve(P, 6, plan=plan, data_fn=lambda P_, ip, bp: wl.grf_coefficient_data(P_, F, ip, bp))
    fns = (lambda P_, x, y: np.ones_like(x), lambda P_, x, y: np.zeros_like(x),
           lambda P_, x, y: wl.grf_coefficient(F, x, y))
    o = oracle_solve(P, 6, fns=fns)
    assert g["info"].status == 0, (g["info"].status, g["info"].bad_pass)
    assert rel(g["u_gamma"], o["u_gamma"]) <= tol
    assert rel(g["uh"], o["uh"]) <= tol
