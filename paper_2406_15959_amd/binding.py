"""Thin ctypes binding of libelmddm (argument marshalling only).

Every computation runs in the HIP library; this module only converts
torch device tensors into pointers and the current torch stream into a
hipStream_t.  It fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libelmddm.so")

OK = 0
INVALID_ARG = 1
OOM = 2
NOT_SPD = 3
SCHUR_NOT_SPD = 4
NOT_CONVERGED = 5
NONFINITE = 6
HIP_ERROR = 7
UNSUPPORTED = 8

OP_POISSON = 0
OP_VARCOEF = 1
POINTS_INTERIOR = 0
POINTS_BOUNDARY = 1
POINTS_INTERFACE = 2
MODE_FP64 = 0
MODE_MIXED = 1
PLAN_MATRIX_FREE = 1
PLAN_DENSE = 2

EXPORTED = [
    "elmddm_plan_create", "elmddm_plan_create_batch", "elmddm_plan_destroy", "elmddm_plan_sizes", "elmddm_points",
    "elmddm_solve", "elmddm_solve_info", "elmddm_eval", "elmddm_eval_grad", "elmddm_assemble",
    "elmddm_plan_keep_schur", "elmddm_get_schur", "elmddm_set_timing", "elmddm_stage_times", "elmddm_pass_times",
    "elmddm_autotune", "elmddm_autotune_times", "elmddm_plan_set_kernels", "elmddm_plan_set_mode", "elmddm_plan_set_passes", "elmddm_plan_reserve_rhs", "elmddm_solve_rhs",
    "elmddm_schur_rhs", "elmddm_interface_cg",
    "elmddm_mlp_create", "elmddm_mlp_destroy", "elmddm_mlp_num_params", "elmddm_mlp_set_params",
    "elmddm_mlp_get_params", "elmddm_mlp_forward", "elmddm_mlp_loss_grad", "elmddm_mlp_adam_step",
    "elmddm_mlp_train", "elmddm_mlp_predict",
    "elmddm_plan_query", "elmddm_plan_create_ex", "elmddm_plan_is_matrix_free", "elmddm_plan_set_cg",
    "elmddm_plan_cg_stats", "elmddm_plan_set_cg_precond", "elmddm_graph_capture", "elmddm_graph_launch", "elmddm_graph_info",
    "elmddm_graph_destroy",
    "elmddm_status_string", "elmddm_last_error",
]

NUM_STAGES = 8
STAGE_NAMES = ["assembly", "gram_syrk", "local_cholesky", "local_trsm", "schur_assembly",
               "interface_cholesky", "interface_backsub", "local_backsolve"]


class Problem(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("nsub_x", ctypes.c_int32), ("nsub_y", ctypes.c_int32),
                ("neurons", ctypes.c_int32), ("q_x", ctypes.c_int32), ("q_y", ctypes.c_int32),
                ("m_bdry_edge", ctypes.c_int32), ("m_ifc_edge", ctypes.c_int32), ("op", ctypes.c_int32)]


class Sizes(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32), ("batch", ctypes.c_int32), ("neurons", ctypes.c_int32), ("n_interior", ctypes.c_int32),
                ("n_interface", ctypes.c_int32), ("n_boundary", ctypes.c_int64),
                ("max_rows", ctypes.c_int32), ("max_ifc", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("bad_subdomain", ctypes.c_int32),
                ("bad_pass", ctypes.c_int32), ("bad_instance", ctypes.c_int32)]


class SolveArgs(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p), ("b", ctypes.c_void_p), ("f", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("u_gamma", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class ElmddmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"elmddm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libelmddm.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with python -m paper_2406_15959_amd.build")
        L = ctypes.CDLL(_LIB_PATH)
        vp, dp, i32, i64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.elmddm_plan_create.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(vp)]
        L.elmddm_plan_create_batch.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(vp)]
        L.elmddm_plan_destroy.argtypes = [vp]
        L.elmddm_plan_sizes.argtypes = [vp, ctypes.POINTER(Sizes)]
        L.elmddm_points.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i64]
        L.elmddm_solve.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
        L.elmddm_solve_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.elmddm_eval.argtypes = [vp, dp, dp, dp, dp, i64, dp, vp]
        L.elmddm_eval_grad.argtypes = [vp, dp, dp, dp, dp, i64, dp, dp, dp, vp]
        L.elmddm_assemble.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp, vp]
        L.elmddm_plan_keep_schur.argtypes = [vp, i32]
        L.elmddm_get_schur.argtypes = [vp, dp, dp, vp]
        L.elmddm_set_timing.argtypes = [vp, i32]
        L.elmddm_autotune.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.elmddm_plan_set_mode.argtypes = [vp, i32]
        L.elmddm_plan_set_passes.argtypes = [vp, i32]
        L.elmddm_plan_set_kernels.argtypes = [vp, i32, i32]
        L.elmddm_autotune_times.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]
        L.elmddm_plan_reserve_rhs.argtypes = [vp, i32]
        L.elmddm_solve_rhs.argtypes = [vp, i32, dp, dp, dp, dp, vp]
        L.elmddm_schur_rhs.argtypes = [vp, i32, dp, dp, dp, vp]
        L.elmddm_interface_cg.argtypes = [vp, i32, dp, dp, ctypes.c_double, i32, ctypes.POINTER(i32),
                                          ctypes.POINTER(ctypes.c_double), vp]
        L.elmddm_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
        L.elmddm_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
        L.elmddm_plan_query.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(Sizes)]
        L.elmddm_plan_create_ex.argtypes = [ctypes.POINTER(Problem), i32, ctypes.c_uint32, ctypes.POINTER(vp)]
        L.elmddm_plan_is_matrix_free.argtypes = [vp]
        L.elmddm_plan_set_cg.argtypes = [vp, ctypes.c_double, i32]
        L.elmddm_plan_set_cg_precond.argtypes = [vp, i32]
        L.elmddm_plan_cg_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        L.elmddm_graph_capture.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SolveArgs), i32, ctypes.POINTER(vp)]
        L.elmddm_graph_launch.argtypes = [vp, vp]
        L.elmddm_graph_info.argtypes = [vp, i32, ctypes.POINTER(Info)]
        L.elmddm_graph_destroy.argtypes = [vp]
        f32 = ctypes.c_float
        L.elmddm_mlp_create.argtypes = [i32, i32, i32, i32, ctypes.POINTER(vp)]
        L.elmddm_mlp_destroy.argtypes = [vp]
        L.elmddm_mlp_num_params.argtypes = [vp, ctypes.POINTER(i64)]
        L.elmddm_mlp_set_params.argtypes = [vp, dp, vp]
        L.elmddm_mlp_get_params.argtypes = [vp, dp, vp]
        L.elmddm_mlp_forward.argtypes = [vp, i32, dp, dp, vp]
        L.elmddm_mlp_loss_grad.argtypes = [vp, i32, dp, dp, dp, dp, vp]
        L.elmddm_mlp_adam_step.argtypes = [vp, f32, f32, f32, f32, vp]
        L.elmddm_mlp_train.argtypes = [vp, i32, dp, dp, dp, i32, i32, f32, f32, f32, f32, dp, vp]
        L.elmddm_mlp_predict.argtypes = [vp, i32, dp, ctypes.c_double, dp, vp]
        L.elmddm_status_string.argtypes = [i32]
        L.elmddm_status_string.restype = ctypes.c_char_p
        L.elmddm_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("elmddm_status_string", "elmddm_last_error"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        L = lib()
        raise ElmddmError(st, f"{L.elmddm_status_string(st).decode()}: {L.elmddm_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), \
        "expected a contiguous float64 CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _ptr_t(t, dtype):
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous(), \
        f"expected a contiguous {dtype} CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_problem(x0=0.0, x1=1.0, y0=0.0, y1=1.0, nsub_x=1, nsub_y=1, neurons=1, q_x=1, q_y=1,
                 m_bdry_edge=1, m_ifc_edge=1, op=OP_POISSON) -> Problem:
    return Problem(x0, x1, y0, y1, nsub_x, nsub_y, neurons, q_x, q_y, m_bdry_edge, m_ifc_edge, op)


class Plan:
    """Owns an elmddm_plan (host layout + device workspace)."""

    def __init__(self, problem: Problem, batch: int = 1, flags: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().elmddm_plan_create_ex(ctypes.byref(problem), batch, flags, ctypes.byref(self._h)))
        s = Sizes()
        _check(lib().elmddm_plan_sizes(self._h, ctypes.byref(s)))
        self.sizes = s
        self.problem = problem

    def close(self):
        if self._h:
            lib().elmddm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def points(self, kind) -> np.ndarray:
        s = self.sizes
        count = {POINTS_INTERIOR: s.nsub * s.n_interior, POINTS_BOUNDARY: s.n_boundary,
                 POINTS_INTERFACE: s.n_interface}[kind]
        out = np.zeros((max(count, 1), 2), dtype=np.float64)
        _check(lib().elmddm_points(self._h, kind, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   max(count, 1)))
        return out[:count]

    def solve(self, W, b, f, g, coef, u_gamma, c):
        _check(lib().elmddm_solve(self._h, _ptr(W), _ptr(b), _ptr(f), _ptr(g), _ptr(coef),
                                  _ptr(u_gamma), _ptr(c), _stream()))

    def solve_info(self) -> Info:
        info = Info()
        _check(lib().elmddm_solve_info(self._h, ctypes.byref(info)))
        return info

    def eval(self, W, b, c, xy, u):
        _check(lib().elmddm_eval(self._h, _ptr(W), _ptr(b), _ptr(c), _ptr(xy), xy.shape[0], _ptr(u),
                                 _stream()))

    def eval_grad(self, W, b, c, xy, u, dudx, dudy):
        """u_h (u may be None) and its gradient at the points xy."""
        _check(lib().elmddm_eval_grad(self._h, _ptr(W), _ptr(b), _ptr(c), _ptr(xy), xy.shape[0],
                                      _ptr(u) if u is not None else None, _ptr(dudx), _ptr(dudy), _stream()))

    def assemble(self, W, b, f, g, coef, K, A, F):
        _check(lib().elmddm_assemble(self._h, _ptr(W), _ptr(b), _ptr(f), _ptr(g), _ptr(coef),
                                     _ptr(K), _ptr(A), _ptr(F), _stream()))

    def reserve_rhs(self, max_rhs):
        _check(lib().elmddm_plan_reserve_rhs(self._h, max_rhs))

    def solve_rhs(self, nrhs, f, g, u_gamma, c=None):
        """nrhs further right-hand sides with the factors of the last solve."""
        _check(lib().elmddm_solve_rhs(self._h, nrhs, _ptr(f), _ptr(g), _ptr(u_gamma), _ptr(c), _stream()))

    def schur_rhs(self, nrhs, f, g, rhs):
        _check(lib().elmddm_schur_rhs(self._h, nrhs, _ptr(f), _ptr(g), _ptr(rhs), _stream()))

    def interface_cg(self, nrhs, rhs, u, tol, maxit, check=True, with_residuals=False):
        """CG on the kept S from the guesses in u; returns (status, iteration counts[, relative residuals])."""
        its = (ctypes.c_int32 * max(nrhs, 1))()
        res = (ctypes.c_double * max(nrhs, 1))()
        st = lib().elmddm_interface_cg(self._h, nrhs, _ptr(rhs), _ptr(u), tol, maxit, its, res, _stream())
        if check and st not in (OK, NOT_CONVERGED):
            _check(st)
        if with_residuals:
            return st, list(its)[:nrhs], list(res)[:nrhs]
        return st, list(its)[:nrhs]

    def set_mode(self, mode):
        """MODE_FP64 or MODE_MIXED for later solves."""
        _check(lib().elmddm_plan_set_mode(self._h, mode))

    def keep_schur(self, keep=True):
        _check(lib().elmddm_plan_keep_schur(self._h, 1 if keep else 0))

    def autotune(self):
        """Pick the fastest kernels for this plan's large products; returns their codes."""
        ch = (ctypes.c_int32 * 2)()
        _check(lib().elmddm_autotune(self._h, _stream(), ch))
        return list(ch)

    def autotune_times(self):
        """{code: (gram ms, trsm ms)} of the last autotune."""
        c = (ctypes.c_int32 * 9)()
        g = (ctypes.c_double * 9)()
        t = (ctypes.c_double * 9)()
        _check(lib().elmddm_autotune_times(self._h, c, g, t))
        return {c[i]: (g[i], t[i]) for i in range(9)}

    def set_timing(self, enable=True):
        _check(lib().elmddm_set_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """(milliseconds per stage summed over timed solves, number of timed solves)."""
        ms = (ctypes.c_double * NUM_STAGES)()
        n = ctypes.c_int32()
        _check(lib().elmddm_stage_times(self._h, ms, ctypes.byref(n)))
        return list(ms), n.value

    def pass_times(self):
        """([[gram, cholesky, trsm] ms for passes 1..5] summed over timed solves, number of solves)."""
        ms = (ctypes.c_double * 15)()
        n = ctypes.c_int32()
        _check(lib().elmddm_pass_times(self._h, ms, ctypes.byref(n)))
        return [list(ms[3 * p:3 * p + 3]) for p in range(5)], n.value

    @property
    def matrix_free(self):
        return bool(lib().elmddm_plan_is_matrix_free(self._h))

    def set_cg(self, tol, maxit):
        _check(lib().elmddm_plan_set_cg(self._h, tol, maxit))

    def set_cg_precond(self, kind):
        """1: block-Jacobi on the interface edges (default), 0: plain CG."""
        _check(lib().elmddm_plan_set_cg_precond(self._h, kind))

    def cg_stats(self):
        """(iterations, relative residuals) of the last CG per instance (matrix-free plans)."""
        b = self.sizes.batch
        it = (ctypes.c_int32 * b)()
        rr = (ctypes.c_double * b)()
        _check(lib().elmddm_plan_cg_stats(self._h, it, rr))
        return list(it), list(rr)

    def set_kernels(self, gram_code, trsm_code):
        _check(lib().elmddm_plan_set_kernels(self._h, gram_code, trsm_code))

    def set_passes(self, npass):
        _check(lib().elmddm_plan_set_passes(self._h, npass))

    def get_schur(self, S, rhs):
        _check(lib().elmddm_get_schur(self._h, _ptr(S), _ptr(rhs), _stream()))


class MLP:
    """Interface-variable MLP (FP32) owned by the HIP library."""

    def __init__(self, in_dim, hidden, out_dim, max_batch):
        self._h = ctypes.c_void_p()
        self.max_batch = max_batch
        _check(lib().elmddm_mlp_create(in_dim, hidden, out_dim, max_batch, ctypes.byref(self._h)))
        n = ctypes.c_int64()
        _check(lib().elmddm_mlp_num_params(self._h, ctypes.byref(n)))
        self.num_params = n.value
        self.dims = (in_dim, hidden, hidden, out_dim)

    def close(self):
        if self._h:
            lib().elmddm_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import torch
        _check(lib().elmddm_mlp_set_params(self._h, _ptr_t(params, torch.float32), _stream()))

    def get_params(self, out):
        import torch
        _check(lib().elmddm_mlp_get_params(self._h, _ptr_t(out, torch.float32), _stream()))

    def forward(self, batch, x, y):
        import torch
        _check(lib().elmddm_mlp_forward(self._h, batch, _ptr_t(x, torch.float32), _ptr_t(y, torch.float32),
                                        _stream()))

    def loss_grad(self, batch, x, t, loss, grad=None):
        import torch
        f = torch.float32
        _check(lib().elmddm_mlp_loss_grad(self._h, batch, _ptr_t(x, f), _ptr_t(t, f), _ptr_t(loss, f),
                                          _ptr_t(grad, f), _stream()))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().elmddm_mlp_adam_step(self._h, lr, beta1, beta2, eps, _stream()))

    def train(self, nsamples, X, T, order, steps, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              losses=None):
        import torch
        f = torch.float32
        _check(lib().elmddm_mlp_train(self._h, nsamples, _ptr_t(X, f), _ptr_t(T, f), _ptr_t(order, torch.int32),
                                      steps, batch, lr, beta1, beta2, eps, _ptr_t(losses, f), _stream()))

    def predict(self, batch, x, scale, out):
        import torch
        _check(lib().elmddm_mlp_predict(self._h, batch, _ptr_t(x, torch.float32), scale,
                                        _ptr_t(out, torch.float64), _stream()))


def plan_query(problem: Problem, batch: int = 1) -> Sizes:
    """Sizes of a plan (device bytes included) without allocating it."""
    s = Sizes()
    _check(lib().elmddm_plan_query(ctypes.byref(problem), batch, ctypes.byref(s)))
    return s


class Graph:
    """Solves of several plans captured into one HIP graph (one launch)."""

    def __init__(self, solves):
        """solves: list of (Plan, dict(W=, b=, f=, g=, coef=, u_gamma=, c=)) with device tensors
        (g, coef may be None).  The tensors are kept alive with the graph."""
        n = len(solves)
        plans = (ctypes.c_void_p * n)(*[p._h.value for p, _ in solves])
        args = (SolveArgs * n)()
        self._keep = []
        for i, (_, a) in enumerate(solves):
            ptrs = {}
            for k in ("W", "b", "f", "g", "coef", "u_gamma", "c"):
                t = a.get(k)
                ptrs[k] = _ptr(t).value if t is not None else None
                self._keep.append(t)
            args[i] = SolveArgs(**ptrs)
        self._plans = [p for p, _ in solves]
        self._h = ctypes.c_void_p()
        _check(lib().elmddm_graph_capture(plans, args, n, ctypes.byref(self._h)))
        self.n = n

    def launch(self):
        _check(lib().elmddm_graph_launch(self._h, _stream()))

    def info(self, i) -> Info:
        inf = Info()
        _check(lib().elmddm_graph_info(self._h, i, ctypes.byref(inf)))
        return inf

    def close(self):
        if self._h:
            lib().elmddm_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
