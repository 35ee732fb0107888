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


def run_rhs(P, seed, alphas, reserve, npass=None):
    import torch
    from paper_2406_15959_amd import binding as B
    dev = torch.device("cuda:0")
    plan = None
    if npass:
        plan = B.Plan(to_c_problem(P))
        plan.set_passes(npass)
    g0 = gpu_solve(P, seed, plan=plan)            # factors of this hidden layer
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


@pytest.mark.parametrize("P,seed,R,reserve,npass", [
    (wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5), 9, 5, 2, None),
    (wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0), 21, 3, 8, None),
    (wl.Problem(1, 1, 90, 12, 12, 11, 4, R=2.0), 8, 2, 1, None),
    (wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0), 22, 3, 2, 4),
])
def test_further_rhs_match_oracle(gpu, P, seed, R, reserve, npass):
    alphas = wl.fourier_coeffs(77 + seed, modes=6, count=R)
    got = run_rhs(P, seed, alphas, reserve, npass)
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


def test_schur_rhs_and_interface_cg_match_oracle_and_direct_solve(gpu):
    """The Schur right-hand side of a new source equals the oracle's g, and
    CG on the kept S (the paper's interface solver) converges to the direct
    solution."""
    import torch
    from oracle import ddm
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0)
    dev = torch.device("cuda:0")
    plan = B.Plan(to_c_problem(P))
    plan.keep_schur(True)
    g0 = gpu_solve(P, 21, plan=plan)
    assert g0["info"].status == 0
    s = plan.sizes
    alphas = wl.fourier_coeffs(5, modes=6, count=3)
    ipts = plan.points(B.POINTS_INTERIOR)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    f = t(wl.fourier_source(alphas, ipts[:, 0], ipts[:, 1]))
    plan.reserve_rhs(2)
    nG = s.n_interface
    rhs = torch.zeros(3 * nG, dtype=torch.float64, device=dev)
    plan.schur_rhs(3, f, None, rhs)
    u_direct = torch.zeros(3 * nG, dtype=torch.float64, device=dev)
    plan.solve_rhs(3, f, None, u_direct)
    u_cg = torch.zeros(3 * nG, dtype=torch.float64, device=dev)
    st, its = plan.interface_cg(3, rhs, u_cg, 1e-13, 5000)
    assert st == B.OK and all(0 < k < 5000 for k in its), its
    lay = build_layout(P)
    W, b = wl.hidden_params(P, 21)
    zero = lambda prob, x, y: np.zeros_like(np.asarray(x, dtype=np.float64))
    for r in range(3):
        src = lambda prob, x, y, r=r: wl.fourier_source(alphas[r:r + 1], x, y)[0]
        sol = ddm.solve(P, W, b, ddm.problem_data(P, lay, src, zero, wl.coefficient), lay)
        got_rhs = rhs[r * nG:(r + 1) * nG].cpu().numpy()
        assert rel(got_rhs, sol.g) <= 1e-9
        ud = u_direct[r * nG:(r + 1) * nG].cpu().numpy()
        uc = u_cg[r * nG:(r + 1) * nG].cpu().numpy()
        assert rel(uc, ud) <= 1e-9
        assert rel(ud, sol.u_gamma) <= TOL_FP64
    # a converged start needs no iteration; maxit 0 leaves the guess untouched
    st, its = plan.interface_cg(1, rhs, u_cg, 1e-6, 100)
    assert st == B.OK and its == [0]
    u0 = torch.zeros(nG, dtype=torch.float64, device=dev)
    st, its = plan.interface_cg(1, rhs, u0, 1e-13, 0)
    assert st == B.NOT_CONVERGED and its == [0] and float(u0.abs().max()) == 0.0
