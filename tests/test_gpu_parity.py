"""End-to-end parity of the HIP path (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

import workload as wl
from gpu_helpers import gpu_solve, oracle_solve, to_c_problem

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-8   # relative L2 of u_Gamma and u_h against the oracle, plain FP64 mode


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_points_match_oracle_layout(gpu):
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B
    for P in [wl.CONFIG_SMALL, wl.Problem(3, 2, 20, 5, 7, 3, 4, R=1.0)]:
        plan = B.Plan(to_c_problem(P))
        lay = build_layout(P)
        assert np.array_equal(plan.points(B.POINTS_INTERIOR), lay.interior_points())
        assert np.array_equal(plan.points(B.POINTS_BOUNDARY), lay.boundary_points())
        assert np.array_equal(plan.points(B.POINTS_INTERFACE), lay.interface_points)
        assert plan.sizes.n_interface == lay.n_interface


@pytest.mark.parametrize("P", [wl.CONFIG_SMALL, wl.Problem(3, 2, 50, 9, 8, 5, 7, op=wl.OP_VARCOEF, R=1.5, k1=2, k2=1)])
def test_assembly_matches_oracle_blocks(gpu, P):
    import torch
    from oracle import ddm
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B
    plan = B.Plan(to_c_problem(P))
    s = plan.sizes
    W, b = wl.hidden_params(P, 3)
    f, g, coef = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    K = torch.zeros(s.nsub * s.neurons * s.max_rows, dtype=torch.float64, device="cuda")
    A = torch.zeros(s.nsub * s.neurons * max(s.max_ifc, 1), dtype=torch.float64, device="cuda")
    F = torch.zeros(s.nsub * s.max_rows, dtype=torch.float64, device="cuda")
    plan.assemble(t(W), t(b), t(f), t(g), t(coef) if coef is not None else None, K, A, F)
    torch.cuda.synchronize()
    Kg = K.cpu().numpy().reshape(s.nsub, s.neurons, s.max_rows)
    Ag = A.cpu().numpy().reshape(s.nsub, s.neurons, max(s.max_ifc, 1))
    Fg = F.cpu().numpy().reshape(s.nsub, s.max_rows)
    lay = build_layout(P)
    data = ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient)
    for si, sub in enumerate(lay.subs):
        blk = ddm.assemble_local(P, sub, W[si], b[si], *data[si])
        m, k = blk.K.shape[0], blk.n_ifc
        assert np.abs(Kg[si, :, :m].T - blk.K).max() <= 1e-13 * np.abs(blk.K).max()
        assert np.abs(Kg[si, :, m:]).max(initial=0) == 0.0
        if k:
            assert np.abs(Ag[si, :, :k].T - blk.D).max() <= 1e-13 * np.abs(blk.D).max()
        assert np.abs(Fg[si, :m] - blk.F).max() <= 1e-14 * np.abs(blk.F).max()


CASES = [
    ("small-2x2", wl.CONFIG_SMALL, 1000),
    ("strip-3x1", wl.Problem(3, 1, 30, 8, 8, 6, 5, R=1.5), 5),
    ("strip-1x2", wl.Problem(1, 2, 40, 9, 7, 6, 9, R=1.5), 6),
    ("ragged-3x2-varcoef", wl.Problem(3, 2, 70, 11, 9, 10, 13, op=wl.OP_VARCOEF, R=2.0, k1=1, k2=3), 7),
    ("single-1x1", wl.Problem(1, 1, 90, 12, 12, 11, 4, R=2.0), 8),
    ("4x3-n130", wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5), 9),
]


@pytest.mark.parametrize("name,P,seed", CASES, ids=[c[0] for c in CASES])
def test_solve_matches_oracle(gpu, name, P, seed):
    g = gpu_solve(P, seed)
    o = oracle_solve(P, seed)
    assert g["info"].status == 0, g["info"].status
    if P.n_interface:
        assert rel(g["u_gamma"], o["u_gamma"]) <= TOL_FP64
    assert rel(g["uh"], o["uh"]) <= TOL_FP64


def test_schur_system_matches_oracle(gpu):
    P = wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0)
    g = gpu_solve(P, 21, keep_schur=True)
    o = oracle_solve(P, 21)
    S, rhs = o["sol"].S, o["sol"].g
    assert np.linalg.norm(g["S"] - S) <= 1e-9 * np.linalg.norm(S)
    assert np.linalg.norm(g["rhs"] - rhs) <= 1e-9 * np.linalg.norm(rhs)


def test_full_8x8_matches_oracle(gpu):
    """The 8x8 workload at full size: 64 subdomains, 400 neurons, 40x40 points."""
    P = wl.CONFIG_8x8
    g = gpu_solve(P, 2000)
    o = oracle_solve(P, 2000)
    assert g["info"].status == 0
    assert rel(g["u_gamma"], o["u_gamma"]) <= TOL_FP64
    assert rel(g["uh"], o["uh"]) <= TOL_FP64
    ex, ey = wl.eval_grid(P)
    assert rel(g["uh"], wl.exact_u(P, ex, ey)) < 1e-4


@pytest.mark.parametrize("mode", [0, 1])
def test_duplicate_neurons_report_not_spd(gpu, mode):
    """Two identical neurons make K^s rank deficient: reported with the subdomain index
    (in both precision modes)."""
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(2, 2, 40, 8, 8, 6, 6, R=2.0)
    plan = B.Plan(to_c_problem(P))
    plan.set_mode(mode)
    s = plan.sizes
    W, b = wl.hidden_params(P, 4)
    W[2, 5] = W[2, 3]
    b[2, 5] = b[2, 3]
    f, g, _ = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    du = torch.zeros(s.n_interface, dtype=torch.float64, device="cuda")
    dc = torch.zeros(s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan.solve(t(W), t(b), t(f), t(g), None, du, dc)
    info = plan.solve_info()
    assert info.status == B.NOT_SPD
    assert info.bad_subdomain == 2


def test_nonfinite_source_is_reported(gpu):
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(2, 2, 40, 8, 8, 6, 6, R=2.0)
    plan = B.Plan(to_c_problem(P))
    s = plan.sizes
    W, b = wl.hidden_params(P, 4)
    f, g, _ = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    f[10] = np.nan
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    du = torch.zeros(s.n_interface, dtype=torch.float64, device="cuda")
    dc = torch.zeros(s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan.solve(t(W), t(b), t(f), t(g), None, du, dc)
    assert plan.solve_info().status == B.NONFINITE


def test_repeated_solves_are_bitwise_reproducible(gpu):
    P = wl.Problem(3, 3, 60, 10, 10, 8, 6, R=2.0)
    from paper_2406_15959_amd import binding as B
    plan = B.Plan(to_c_problem(P))
    a = gpu_solve(P, 5, plan=plan)
    b = gpu_solve(P, 5, plan=plan)
    assert np.array_equal(a["u_gamma"], b["u_gamma"])
    assert np.array_equal(a["c"], b["c"])


def test_batched_instances_match_oracle_and_single_solves(gpu):
    """Three instances in one batched solve (different hidden layers, scaled data):
    each matches its own oracle solve and the unbatched solve bit for bit."""
    import torch
    from oracle import ddm
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(3, 2, 70, 11, 9, 10, 13, op=wl.OP_VARCOEF, R=2.0, k1=1, k2=3)
    seeds, scales = [31, 32, 33], [1.0, -2.5, 0.75]
    nb = len(seeds)
    plan = B.Plan(to_c_problem(P), batch=nb)
    s = plan.sizes
    assert s.batch == nb
    ipts, bpts = plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY)
    f, g, coef = wl.sample_data(P, ipts, bpts)
    Ws, bs = zip(*[wl.hidden_params(P, sd) for sd in seeds])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    dW, db = t(np.stack(Ws)), t(np.stack(bs))
    df = t(np.stack([sc * f for sc in scales]))
    dg = t(np.stack([sc * g for sc in scales]))
    dcoef = t(np.stack([np.stack([coef[i]] * nb) for i in range(3)]))   # [3][batch][...]
    du = torch.zeros(nb * s.n_interface, dtype=torch.float64, device="cuda")
    dc = torch.zeros(nb * s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan.solve(dW, db, df, dg, dcoef, du, dc)
    assert plan.solve_info().status == 0
    U = du.cpu().numpy().reshape(nb, -1)
    Cc = dc.cpu().numpy().reshape(nb, s.nsub, s.neurons)
    lay = build_layout(P)
    ex, ey = wl.eval_grid(P, 12)
    for i, (sd, sc) in enumerate(zip(seeds, scales)):
        data = [(sc * fi, sc * gi, ci) for fi, gi, ci in ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient)]
        o = ddm.solve(P, Ws[i], bs[i], data, lay)
        assert rel(U[i], o.u_gamma) <= TOL_FP64
        uh_g = ddm.evaluate(P, lay, Ws[i], bs[i], list(Cc[i]), ex, ey)
        uh_o = ddm.evaluate(P, lay, Ws[i], bs[i], o.c, ex, ey)
        assert rel(uh_g, uh_o) <= TOL_FP64
    # instance 1 alone, unbatched
    plan1 = B.Plan(to_c_problem(P))
    du1 = torch.zeros(s.n_interface, dtype=torch.float64, device="cuda")
    dc1 = torch.zeros(s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan1.solve(t(Ws[1]), t(bs[1]), t(scales[1] * f), t(scales[1] * g), t(coef), du1, dc1)
    assert plan1.solve_info().status == 0
    assert np.array_equal(du1.cpu().numpy(), U[1])
    assert np.array_equal(dc1.cpu().numpy(), Cc[1].ravel())


def test_batched_failure_names_the_instance(gpu):
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(2, 2, 40, 8, 8, 6, 6, R=2.0)
    plan = B.Plan(to_c_problem(P), batch=2)
    s = plan.sizes
    W, b = wl.hidden_params(P, 4)
    W2, b2 = W.copy(), b.copy()
    W2[3, 7], b2[3, 7] = W2[3, 2], b2[3, 2]   # duplicate neuron in instance 1, subdomain 3
    f, g, _ = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    du = torch.zeros(2 * s.n_interface, dtype=torch.float64, device="cuda")
    dc = torch.zeros(2 * s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan.solve(t(np.stack([W, W2])), t(np.stack([b, b2])), t(np.stack([f, f])), t(np.stack([g, g])), None, du, dc)
    info = plan.solve_info()
    assert info.status == B.NOT_SPD
    assert (info.bad_instance, info.bad_subdomain) == (1, 3)


def test_autotuned_kernels_and_split_envelope_path_match_oracle(gpu):
    """Batch 4 takes the split (panel + trailing GEMM) envelope path; the
    autotuner may pick any of the product kernels; parity must hold."""
    import torch
    from oracle import ddm
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5)
    nb = 4
    plan = B.Plan(to_c_problem(P), batch=nb)
    codes = plan.autotune()
    assert len(codes) == 2 and all(c < 0 or 4 <= c <= 8 for c in codes)
    times = plan.autotune_times()
    assert sorted(times) == [-4, -3, -2, -1, 4, 5, 6, 7, 8] and all(g > 0 and t > 0 for g, t in times.values())
    s = plan.sizes
    f, g, _ = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    seeds = [41, 42, 43, 44]
    Ws, bs = zip(*[wl.hidden_params(P, sd) for sd in seeds])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    du = torch.zeros(nb * s.n_interface, dtype=torch.float64, device="cuda")
    dc = torch.zeros(nb * s.nsub * s.neurons, dtype=torch.float64, device="cuda")
    plan.solve(t(np.stack(Ws)), t(np.stack(bs)), t(np.stack([f] * nb)), t(np.stack([g] * nb)), None, du, dc)
    assert plan.solve_info().status == 0
    U = du.cpu().numpy().reshape(nb, -1)
    lay = build_layout(P)
    data = ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient)
    for i in (0, 3):
        o = ddm.solve(P, Ws[i], bs[i], data, lay)
        assert rel(U[i], o.u_gamma) <= TOL_FP64


@pytest.mark.parametrize("mode,tol", [(0, TOL_FP64), (1, 1e-6)])
def test_four_pass_factorisation_matches_oracle(gpu, mode, tol):
    """Two shifted CholeskyQR passes (forced on a small case) give the same answer."""
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5)
    plan = B.Plan(to_c_problem(P))
    plan.set_passes(4)
    plan.set_mode(mode)
    g = gpu_solve(P, 9, plan=plan)
    o = oracle_solve(P, 9)
    assert g["info"].status == 0
    assert rel(g["u_gamma"], o["u_gamma"]) <= tol
    assert rel(g["uh"], o["uh"]) <= tol
    with pytest.raises(B.ElmddmError):
        plan.set_passes(6)


@pytest.mark.slow
@pytest.mark.parametrize("mode,tol", [(0, TOL_FP64), (1, 1e-6)])
def test_800_neuron_variable_coefficient_problem_matches_oracle(gpu, mode, tol):
    """A ragged-batch shape with badly conditioned blocks (4x4 subdomains,
    800 neurons, column-scaled kappa(K_s) up to ~1e13): four passes by default."""
    from paper_2406_15959_amd import binding as B
    P = [p for p in wl.ragged_problems(64) if p.neurons == 800 and p.nsub_x == 4][0]
    plan = B.Plan(to_c_problem(P))
    plan.set_mode(mode)
    g = gpu_solve(P, 77, plan=plan, eval_per_sub=8)
    o = oracle_solve(P, 77, eval_per_sub=8)
    assert g["info"].status == 0, (g["info"].status, g["info"].bad_pass)
    assert rel(g["u_gamma"], o["u_gamma"]) <= tol
    assert rel(g["uh"], o["uh"]) <= tol


def test_gradient_evaluation_matches_oracle(gpu):
    """elmddm_eval_grad on the oracle's own coefficients (a kernel check,
    1e-12) and the relative H1 seminorm error of a full GPU solve against the
    oracle's (the H1 column of Table 2, 1e-8)."""
    import dataclasses
    import torch
    from oracle import ddm
    P = dataclasses.replace(wl.CONFIG_SMALL, sol=wl.SOL_SIN2PI_EXP)
    g = gpu_solve(P, 7)
    o = oracle_solve(P, 7)
    lay = o["layout"]
    ex, ey = wl.eval_grid(P, 8)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    xy = t(np.stack([ex, ey], 1))
    W, b = t(g["W"]), t(g["b"])
    u, ux, uy = (torch.zeros(len(ex), dtype=torch.float64, device="cuda") for _ in range(3))
    g["plan"].eval_grad(W, b, t(o["sol"].c), xy, u, ux, uy)
    torch.cuda.synchronize()
    ou, oux, ouy = ddm.evaluate_grad(P, lay, g["W"], g["b"], o["sol"].c, ex, ey)
    assert rel(u.cpu().numpy(), ou) <= 1e-12
    assert rel(np.concatenate([ux.cpu().numpy(), uy.cpu().numpy()]), np.concatenate([oux, ouy])) <= 1e-12
    # H1 seminorm of the GPU solve's gradient against the oracle solve's
    g["plan"].eval_grad(W, b, t(g["c"]), xy, None, ux, uy)
    torch.cuda.synchronize()
    gg = np.concatenate([ux.cpu().numpy(), uy.cpu().numpy()])
    assert rel(gg, np.concatenate([oux, ouy])) <= TOL_FP64
