"""Ragged batches: many independent problems of different shapes in one
graph launch.

Problems are grouped by shape (subdomain grid, neurons, points, operator);
each shape gets one batched plan, sized to a share of a device-memory
budget, and its problems are solved in chunks of that batch size (a short
last chunk is padded by repeating its last problem).  Every chunk's solve
of every shape is captured, in order, into one HIP graph
(elmddm_graph_capture), so the whole ragged batch is one graph launch and
the chunks of a shape reuse its plan's workspace one after another.
This module only groups problems and moves arguments; every computation
runs in the HIP library.
"""
from __future__ import annotations

from . import binding as B


def shape_key(P):
    return (P.nsub_x, P.nsub_y, P.neurons, P.q_x, P.q_y, P.m_bdry_edge, P.m_ifc_edge, P.op,
            P.x0, P.x1, P.y0, P.y1)


def c_problem(P):
    return B.make_problem(P.x0, P.x1, P.y0, P.y1, P.nsub_x, P.nsub_y, P.neurons, P.q_x, P.q_y,
                          P.m_bdry_edge, P.m_ifc_edge, P.op)


class RaggedBatch:
    def __init__(self, problems, budget_bytes, mode=B.MODE_MIXED, autotune=True):
        self.problems = list(problems)
        groups = {}
        for i, P in enumerate(self.problems):
            groups.setdefault(shape_key(P), []).append(i)
        self.shapes = []
        share = budget_bytes / max(len(groups), 1)
        for key, idx in sorted(groups.items(), key=lambda kv: -len(kv[1])):
            cp = c_problem(self.problems[idx[0]])
            one = B.plan_query(cp, 1).device_bytes
            two = B.plan_query(cp, 2).device_bytes
            per = max(two - one, 1)
            b = int(max(1, min(len(idx), 1 + (share - one) // per)))
            plan = B.Plan(cp, batch=b)
            tuned = plan.autotune() if autotune else None
            plan.set_mode(mode)
            chunks = [idx[k:k + b] for k in range(0, len(idx), b)]
            self.shapes.append(dict(key=key, plan=plan, batch=b, chunks=chunks, tuned=tuned))
        self.graph = None

    def points(self, i, kind):
        """Points of problem i's shape (the plan's layout)."""
        return self._shape_of(i)["plan"].points(kind)

    def _shape_of(self, i):
        k = shape_key(self.problems[i])
        for sh in self.shapes:
            if sh["key"] == k:
                return sh
        raise KeyError(i)

    def capture(self, inputs):
        """inputs[i] = dict(W, b, f, g, coef) of problem i as device tensors
        (coef None for Poisson).  Allocates the stacked chunk inputs and the
        outputs, and captures every solve into one graph."""
        import torch
        solves = []
        self.out = [None] * len(self.problems)
        for sh in self.shapes:
            plan, b = sh["plan"], sh["batch"]
            s = plan.sizes
            for chunk in sh["chunks"]:
                padded = chunk + [chunk[-1]] * (b - len(chunk))
                st = lambda k: torch.stack([inputs[i][k].reshape(-1) for i in padded]).contiguous()
                a = dict(W=st("W"), b=st("b"), f=st("f"))
                a["g"] = st("g") if s.n_boundary else None
                if inputs[padded[0]].get("coef") is not None:
                    # [3][batch][nsub * q2]
                    a["coef"] = torch.stack([inputs[i]["coef"].reshape(3, -1) for i in padded], 1).contiguous()
                else:
                    a["coef"] = None
                dev = a["W"].device
                a["u_gamma"] = torch.zeros(b * max(s.n_interface, 1), dtype=torch.float64, device=dev)
                a["c"] = torch.zeros(b * s.nsub * s.neurons, dtype=torch.float64, device=dev)
                solves.append((plan, a))
                for slot, i in enumerate(chunk):
                    self.out[i] = (a, slot, len(solves) - 1, s)
        self.graph = B.Graph(solves)
        return self.graph

    def launch(self):
        self.graph.launch()

    def result(self, i):
        """(u_gamma, c, info) of problem i after a launch (device views)."""
        a, slot, solve, s = self.out[i]
        nG = s.n_interface
        u = a["u_gamma"][slot * nG:(slot + 1) * nG]
        c = a["c"][slot * s.nsub * s.neurons:(slot + 1) * s.nsub * s.neurons]
        return u, c, self.graph.info(solve)
