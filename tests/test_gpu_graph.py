"""Solves captured into HIP graphs: replays equal eager solves bit for bit
(with eager work between the replays), and a ragged batch of problems of
different shapes in one graph launch matches the oracle problem by problem."""
import numpy as np
import pytest

import workload as wl
from gpu_helpers import to_c_problem

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def inputs_for(P, plan, seed):
    import torch
    from paper_2406_15959_amd import binding as B
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    W, b = wl.hidden_params(P, seed)
    f, g, coef = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    return dict(W=t(W), b=t(b), f=t(f), g=t(g), coef=t(coef) if coef is not None else None)


def test_graph_replays_equal_eager_solves(gpu):
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(3, 2, 60, 10, 10, 8, 6, op=wl.OP_VARCOEF, R=2.0, k1=2, k2=1)
    plan = B.Plan(to_c_problem(P))
    s = plan.sizes
    a = inputs_for(P, plan, 11)
    other = inputs_for(P, plan, 12)
    a["u_gamma"] = torch.zeros(s.n_interface, dtype=torch.float64, device="cuda:0")
    a["c"] = torch.zeros(s.nsub * s.neurons, dtype=torch.float64, device="cuda:0")
    u_e = torch.zeros_like(a["u_gamma"])
    c_e = torch.zeros_like(a["c"])
    plan.solve(a["W"], a["b"], a["f"], a["g"], a["coef"], u_e, c_e)
    torch.cuda.synchronize()
    graph = B.Graph([(plan, a)])
    for rep in range(3):
        a["u_gamma"].zero_()
        a["c"].zero_()
        graph.launch()
        assert graph.info(0).status == 0
        assert torch.equal(a["u_gamma"], u_e) and torch.equal(a["c"], c_e), rep
        # eager work on the same plan between the replays
        plan.solve(other["W"], other["b"], other["f"], other["g"], other["coef"], torch.zeros_like(u_e),
                   torch.zeros_like(c_e))
        torch.cuda.synchronize()



def test_batched_plan_graph_replays_equal_eager_solves(gpu):
    """A batch of 4 instances takes the unfused interface factorisation,
    whose eager solves overlap the trailing updates on a side stream
    (lookahead); a captured solve keeps one stream.  Both orders give the
    same bits, replay after replay."""
    import torch
    from paper_2406_15959_amd import binding as B
    P = wl.Problem(4, 3, 80, 12, 11, 10, 9, R=2.0)
    nb = 4
    plan = B.Plan(to_c_problem(P), batch=nb)
    s = plan.sizes
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    Ws, bs = zip(*[wl.hidden_params(P, 60 + i) for i in range(nb)])
    f, g, _ = wl.sample_data(P, plan.points(B.POINTS_INTERIOR), plan.points(B.POINTS_BOUNDARY))
    a = dict(W=t(np.stack(Ws)), b=t(np.stack(bs)), f=t(np.stack([f] * nb)), g=t(np.stack([g] * nb)), coef=None,
             u_gamma=torch.zeros(nb * s.n_interface, dtype=torch.float64, device="cuda:0"),
             c=torch.zeros(nb * s.nsub * s.neurons, dtype=torch.float64, device="cuda:0"))
    u_e, c_e = torch.zeros_like(a["u_gamma"]), torch.zeros_like(a["c"])
    plan.solve(a["W"], a["b"], a["f"], a["g"], None, u_e, c_e)
    assert plan.solve_info().status == 0
    graph = B.Graph([(plan, a)])
    for rep in range(3):
        a["u_gamma"].zero_()
        a["c"].zero_()
        graph.launch()
        assert graph.info(0).status == 0
        assert torch.equal(a["u_gamma"], u_e) and torch.equal(a["c"], c_e), rep
        plan.solve(a["W"], a["b"], a["f"], a["g"], None, torch.zeros_like(u_e), torch.zeros_like(c_e))
        torch.cuda.synchronize()


@pytest.mark.parametrize("mode,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_ragged_batch_in_one_graph_matches_oracle(gpu, mode, tol):
    import torch
    from oracle import ddm
    from oracle.layout import build_layout
    from paper_2406_15959_amd import binding as B, ragged
    shapes = [wl.Problem(2, 2, 40, 8, 8, 8, 8, op=wl.OP_VARCOEF, R=1.3),
              wl.Problem(3, 3, 60, 10, 10, 10, 10, op=wl.OP_VARCOEF, R=1.5),
              wl.Problem(2, 3, 80, 12, 12, 12, 12, op=wl.OP_VARCOEF, R=1.8)]
    import dataclasses
    probs = [dataclasses.replace(shapes[i % 3], k1=1 + i % 3, k2=1 + (i // 3) % 3) for i in range(8)]
    m = B.MODE_FP64 if mode == "fp64" else B.MODE_MIXED
    # a small budget forces batches of 1-2 and padded chunks
    rb = ragged.RaggedBatch(probs, budget_bytes=3 * B.plan_query(ragged.c_problem(shapes[2]), 1).device_bytes,
                            mode=m)
    assert any(len(ch) < sh["batch"] for sh in rb.shapes for ch in sh["chunks"]) or \
        any(len(sh["chunks"]) > 1 for sh in rb.shapes)
    inputs = [inputs_for(P, rb._shape_of(i)["plan"], 500 + i) for i, P in enumerate(probs)]
    rb.capture(inputs)
    for rep in range(2):
        rb.launch()
        torch.cuda.synchronize()
        for i, P in enumerate(probs):
            u, c, info = rb.result(i)
            assert info.status == 0
            if rep == 1:
                continue
            lay = build_layout(P)
            W, b = wl.hidden_params(P, 500 + i)
            sol = ddm.solve(P, W, b, ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient), lay)
            assert rel(u.cpu().numpy(), sol.u_gamma) <= tol, (i, mode)
            ex, ey = wl.eval_grid(P)
            uo = ddm.evaluate(P, lay, W, b, sol.c, ex, ey)
            plan = rb._shape_of(i)["plan"]
            uh = torch.zeros(len(ex), dtype=torch.float64, device="cuda:0")
            plan.eval(inputs[i]["W"], inputs[i]["b"], c.contiguous(),
                      torch.from_numpy(np.stack([ex, ey], 1)).to("cuda:0"), uh)
            torch.cuda.synchronize()
            assert rel(uh.cpu().numpy(), uo) <= tol, (i, mode)
