"""Further right-hand sides with cached factors (elmddm_solve_rhs) against
independent oracle solves of the same hidden layer with the new source."""
import numpy as np
import pytest

import workload as wl
from gpu_helpers import gpu_solve, to_c_problem

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-8


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_fourier(P, seed, alpha):
    """Oracle solve with the Fourier source alpha, zero boundary data."""
    from oracle import ddm
    from oracle.layout import build_layout
    lay = build_layout(P)
    W, b = wl.hidden_params(P, seed)
    src = lambda prob, x, y: wl.fourier_source(alpha[None], x, y)[0]
    zero = lambda prob, x, y: np.zeros_like(np.asarray(x, dtype=np.float64))
    data = ddm.problem_data(P, lay, src, zero, wl.coefficient)
    sol = ddm.solve(P, W, b, data, lay)
    ex, ey = wl.eval_grid(P)
    return sol.u_gamma, ddm.evaluate(P, lay, W, b, sol.c, ex, ey)


def run_rhs(P, seed, alphas, reserve):
    import torch
    from paper_2406_15959_amd import binding as B
    dev = torch.device("cuda:0")
    g0 = gpu_solve(P, seed)                       # factors of this hidden layer
    plan = g0["plan"]
    assert g0["info"].status == 0
    s = plan.sizes
    ipts = plan.points(B.POINTS_INTERIOR)
    f = wl.fourier_source(alphas, ipts[:, 0], ipts[:, 1])
    R = len(alphas)
    plan.reserve_rhs(reserve)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    du = torch.zeros(R * s.n_interface, dtype=torch.float64, device=dev)
    dc = torch.zeros(R * s.nsub * s.neurons, dtype=torch.float64, device=dev)
    plan.solve_rhs(R, t(f), None, du, dc)
    torch.cuda.synchronize()
    ex, ey = wl.eval_grid(P)
    xy = t(np.stack([ex, ey], 1))
    dW, db = t(g0["W"]), t(g0["b"])
    out = []
    for r in range(R):
        uh = torch.zeros(len(ex), dtype=torch.float64, device=dev)
        plan.eval(dW, db, dc[r * s.nsub * s.neurons:(r + 1) * s.nsub * s.neurons].contiguous(), xy, uh)
        torch.cuda.synchronize()
        out.append((du[r * s.n_interface:(r + 1) * s.n_interface].cpu().numpy(), uh.cpu().numpy()))
    return out


@pytest.mark.parametrize("P,seed,R,reserve", [
    (wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5), 9, 5, 2),
    (wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0), 21, 3, 8),
    (wl.Problem(1, 1, 90, 12, 12, 11, 4, R=2.0), 8, 2, 1),
])
def test_further_rhs_match_oracle(gpu, P, seed, R, reserve):
    alphas = wl.fourier_coeffs(77 + seed, modes=6, count=R)
    got = run_rhs(P, seed, alphas, reserve)
    for r in range(R):
        ug, uo = oracle_fourier(P, seed, alphas[r])
        if P.n_interface:
            assert rel(got[r][0], ug) <= TOL_FP64, r
        assert rel(got[r][1], uo) <= TOL_FP64, r


def test_further_rhs_8x8_full_size(gpu):
    P = wl.CONFIG_8x8
    alphas = wl.fourier_coeffs(123, modes=32, count=2)
    got = run_rhs(P, 2002, alphas, 2)
    for r in range(2):
        ug, uo = oracle_fourier(P, 2002, alphas[r])
        assert rel(got[r][0], ug) <= TOL_FP64
        assert rel(got[r][1], uo) <= TOL_FP64


def test_further_rhs_need_factors_and_batch_one(gpu):
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.CONFIG_SMALL
    plan = B.Plan(to_c_problem(P))
    plan.reserve_rhs(1)
    s = plan.sizes
    f = torch.zeros(s.nsub * s.n_interior, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(s.n_interface, dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.ElmddmError) as e:
        plan.solve_rhs(1, f, None, u)
    assert e.value.status == B.INVALID_ARG
    pb = B.Plan(to_c_problem(P), batch=2)
    with pytest.raises(B.ElmddmError) as e:
        pb.reserve_rhs(1)
    assert e.value.status == B.UNSUPPORTED
