"""Helpers shared by the GPU tests: run the HIP library on a workload problem
and run the oracle on the same inputs."""
import numpy as np

import workload as wl


def to_c_problem(P):
    from paper_2406_15959_amd import binding as B
    return B.make_problem(P.x0, P.x1, P.y0, P.y1, P.nsub_x, P.nsub_y, P.neurons, P.q_x, P.q_y,
                          P.m_bdry_edge, P.m_ifc_edge, P.op)


def gpu_solve(P, seed, plan=None, keep_schur=False, eval_per_sub=16, params=None, data_fn=None):
    """Solve on the GPU through the C ABI.  Returns a dict of numpy arrays.
    params: (W, b) of the hidden layer, else drawn with hidden_params(P, seed);
    data_fn(P, interior_xy, boundary_xy) -> (f, g, coef), else sample_data."""
    import torch
    from paper_2406_15959_amd import binding as B
    dev = torch.device("cuda:0")
    plan = plan or B.Plan(to_c_problem(P))
    if keep_schur:
        plan.keep_schur(True)
    s = plan.sizes
    W, b = params if params is not None else wl.hidden_params(P, seed)
    ipts = plan.points(B.POINTS_INTERIOR)
    bpts = plan.points(B.POINTS_BOUNDARY)
    f, g, coef = (data_fn or wl.sample_data)(P, ipts, bpts)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    dW, db, df = t(W), t(b), t(f)
    dg = t(g) if len(g) else None
    dcoef = t(coef) if coef is not None else None
    du = torch.zeros(max(s.n_interface, 1), dtype=torch.float64, device=dev)
    dc = torch.zeros(s.nsub * s.neurons, dtype=torch.float64, device=dev)
    plan.solve(dW, db, df, dg, dcoef, du if s.n_interface else None, dc)
    info = plan.solve_info()
    ex, ey = wl.eval_grid(P, eval_per_sub)
    xy = t(np.stack([ex, ey], 1))
    uh = torch.zeros(len(ex), dtype=torch.float64, device=dev)
    plan.eval(dW, db, dc, xy, uh)
    out = dict(info=info, u_gamma=du[:s.n_interface].cpu().numpy(), c=dc.cpu().numpy().reshape(s.nsub, -1),
               uh=uh.cpu().numpy(), W=W, b=b, plan=plan, points=(ipts, bpts, plan.points(B.POINTS_INTERFACE)))
    if keep_schur and s.n_interface:
        S = torch.zeros(s.n_interface * s.n_interface, dtype=torch.float64, device=dev)
        rhs = torch.zeros(s.n_interface, dtype=torch.float64, device=dev)
        plan.get_schur(S, rhs)
        torch.cuda.synchronize()
        out["S"] = S.cpu().numpy().reshape(s.n_interface, s.n_interface).T
        out["rhs"] = rhs.cpu().numpy()
    return out


def oracle_solve(P, seed, eval_per_sub=16, params=None, fns=None):
    """fns: (source_f, boundary_g, coefficient) functions of (P, x, y), else
    the manufactured solution's."""
    from oracle import ddm
    from oracle.layout import build_layout
    lay = build_layout(P)
    W, b = params if params is not None else wl.hidden_params(P, seed)
    data = ddm.problem_data(P, lay, *(fns or (wl.source_f, wl.boundary_g, wl.coefficient)))
    sol = ddm.solve(P, W, b, data, lay)
    ex, ey = wl.eval_grid(P, eval_per_sub)
    uh = ddm.evaluate(P, lay, W, b, sol.c, ex, ey)
    return dict(sol=sol, layout=lay, uh=uh, u_gamma=sol.u_gamma, W=W, b=b)
