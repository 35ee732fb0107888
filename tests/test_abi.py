"""The C-ABI library builds, loads and exports every declared symbol (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elmddm.h")


def _lib_path():
    from paper_2406_15959_amd import binding
    if not os.path.exists(binding._LIB_PATH):
        from paper_2406_15959_amd import build
        build.build_library()
    return binding._LIB_PATH


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(elmddm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (elmddm_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    assert len(declared_symbols()) >= 12


def test_binding_covers_the_header():
    from paper_2406_15959_amd import binding
    assert sorted(binding.EXPORTED) == declared_symbols()


def test_library_loads_and_reports_status_strings():
    _lib_path()
    from paper_2406_15959_amd import binding as B
    L = B.lib()
    assert L.elmddm_status_string(B.OK) == b"ok"
    assert b"positive definite" in L.elmddm_status_string(B.NOT_SPD)


@pytest.mark.parametrize("field,value", [("neurons", 0), ("q_x", 0), ("nsub_x", 0), ("m_ifc_edge", 0),
                                         ("op", 7), ("x1", -1.0), ("m_ifc_edge", 65)])
def test_plan_create_rejects_bad_problems_without_a_gpu(field, value):
    """Validation happens on the host before any device call."""
    _lib_path()
    from paper_2406_15959_amd import binding as B
    p = B.make_problem(nsub_x=2, nsub_y=2, neurons=10, q_x=4, q_y=4, m_bdry_edge=3, m_ifc_edge=3)
    setattr(p, field, value)
    with pytest.raises(B.ElmddmError) as e:
        B.Plan(p)
    assert e.value.status in (B.INVALID_ARG, B.UNSUPPORTED)


def test_plan_create_rejects_too_few_interior_points():
    """The Proposition of Section 3 needs m_i >= n_N per subdomain."""
    _lib_path()
    from paper_2406_15959_amd import binding as B
    p = B.make_problem(nsub_x=2, nsub_y=2, neurons=17, q_x=4, q_y=4, m_bdry_edge=3, m_ifc_edge=3)
    with pytest.raises(B.ElmddmError) as e:
        B.Plan(p)
    assert e.value.status == B.INVALID_ARG
    assert b"neurons" in B.lib().elmddm_last_error()


def test_plan_query_sizes_without_a_gpu():
    """The size query builds the layout on the host only."""
    _lib_path()
    from paper_2406_15959_amd import binding as B
    p = B.make_problem(nsub_x=3, nsub_y=2, neurons=30, q_x=8, q_y=8, m_bdry_edge=6, m_ifc_edge=5)
    s1 = B.plan_query(p, 1)
    s3 = B.plan_query(p, 3)
    assert s1.nsub == 6 and s1.neurons == 30 and s1.batch == 1 and s3.batch == 3
    assert s1.n_interface == ((3 - 1) * 2 + 3 * (2 - 1)) * 5
    assert s1.device_bytes > 0 and s3.device_bytes > 2 * s1.device_bytes
    with pytest.raises(B.ElmddmError):
        B.plan_query(p, 0)
    # batch * nsub is bounded by the launch grid (65535 subdomains)
    assert B.plan_query(p, 65535 // 6).batch == 65535 // 6
    with pytest.raises(B.ElmddmError) as e:
        B.plan_query(p, 65535 // 6 + 1)
    assert e.value.status == B.INVALID_ARG


def test_ragged_problem_draws_are_reproducible_and_cover_the_shapes():
    import workload as wl
    a = wl.ragged_problems(64)
    b = wl.ragged_problems(64)
    assert a == b
    assert {P.nsub_x for P in a} == {4, 8, 16} and {P.neurons for P in a} == {100, 200, 400, 800}
    for P in a:
        assert P.q_x ** 2 >= P.neurons and P.op == wl.OP_VARCOEF and 1 <= P.k1 <= 3


def test_the_32x32_case_sizes_to_a_matrix_free_plan():
    """126976 interface unknowns: a dense S would need 3 x 129 GB; the size query
    (matrix-free by default there) stays within one GPU."""
    import workload as wl
    from paper_2406_15959_amd import binding as B
    P = wl.CONFIG_32x32
    s = B.plan_query(B.make_problem(P.x0, P.x1, P.y0, P.y1, P.nsub_x, P.nsub_y, P.neurons, P.q_x, P.q_y,
                                    P.m_bdry_edge, P.m_ifc_edge, P.op), 1)
    assert s.n_interface == 126976
    assert s.device_bytes < 200e9
