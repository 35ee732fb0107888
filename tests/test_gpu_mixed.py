"""Mixed-precision mode (FP32 matrix-core Gram in the first, shifted
CholeskyQR pass; everything else FP64) against the FP64 oracle.  The bound
for mixed results is relative L2 <= 1e-6 on u_Gamma and u_h."""
import numpy as np
import pytest

import workload as wl
from gpu_helpers import gpu_solve, oracle_solve, to_c_problem

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mixed_plan(P, batch=1):
    from paper_2406_15959_amd import binding as B
    plan = B.Plan(to_c_problem(P), batch=batch)
    plan.set_mode(B.MODE_MIXED)
    return plan


MIXED_CASES = [
    ("small-2x2", wl.CONFIG_SMALL, 1000),
    ("ragged-3x2-varcoef", wl.Problem(3, 2, 70, 11, 9, 10, 13, op=wl.OP_VARCOEF, R=2.0, k1=1, k2=3), 7),
    ("single-1x1", wl.Problem(1, 1, 90, 12, 12, 11, 4, R=2.0), 8),
    ("4x3-n130", wl.Problem(4, 3, 130, 13, 12, 12, 17, R=2.5), 9),
]


@pytest.mark.parametrize("name,P,seed", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_solve_matches_oracle(gpu, name, P, seed):
    g = gpu_solve(P, seed, plan=mixed_plan(P))
    o = oracle_solve(P, seed)
    assert g["info"].status == 0, g["info"].status
    if P.n_interface:
        assert rel(g["u_gamma"], o["u_gamma"]) <= TOL_MIXED
    assert rel(g["uh"], o["uh"]) <= TOL_MIXED


def test_mixed_8x8_matches_oracle_and_fp64_mode(gpu):
    """Full 8x8 workload (kappa(K_s) about 1e10): the FP32 pass only
    preconditions, so the mixed result also agrees with the FP64 mode."""
    P = wl.CONFIG_8x8
    gm = gpu_solve(P, 2001, plan=mixed_plan(P))
    gd = gpu_solve(P, 2001)
    o = oracle_solve(P, 2001)
    assert gm["info"].status == 0 and gd["info"].status == 0
    assert rel(gm["u_gamma"], o["u_gamma"]) <= TOL_MIXED
    assert rel(gm["uh"], o["uh"]) <= TOL_MIXED
    assert rel(gm["uh"], gd["uh"]) <= 1e-8


def test_mode_switch_is_validated_and_reversible(gpu):
    from paper_2406_15959_amd import binding as B
    P = wl.CONFIG_SMALL
    plan = B.Plan(to_c_problem(P))
    with pytest.raises(B.ElmddmError):
        plan.set_mode(7)
    plan.set_mode(B.MODE_MIXED)
    plan.set_mode(B.MODE_FP64)
    g1 = gpu_solve(P, 1000, plan=plan)
    g2 = gpu_solve(P, 1000)
    assert np.array_equal(g1["u_gamma"], g2["u_gamma"])


def test_mixed_8x8_badly_conditioned_instance(gpu):
    """Hidden-layer seed 2009 has a block with column-scaled kappa 4e9: the
    FP32-shifted first pass leaves kappa(Q1) ~ 1e7 and pass-2 pivots near
    3e-12 of the diagonal, legitimate for an unshifted middle pass."""
    P = wl.CONFIG_8x8
    gm = gpu_solve(P, 2009, plan=mixed_plan(P))
    o = oracle_solve(P, 2009)
    assert gm["info"].status == 0, (gm["info"].bad_pass, gm["info"].bad_subdomain)
    assert rel(gm["u_gamma"], o["u_gamma"]) <= TOL_MIXED
    assert rel(gm["uh"], o["uh"]) <= TOL_MIXED
