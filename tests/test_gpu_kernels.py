"""Kernel-level parity of the batched FP64 MFMA GEMM and the blocked Cholesky
against numpy (float64), through the test-hooks library."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2406_15959_amd")


@pytest.fixture(scope="module")
def hooks(gpu):
    path = os.path.join(PKG, "libelmddm_testhooks.so")
    if not os.path.exists(path):
        pytest.fail("libelmddm_testhooks.so is not built (python -m paper_2406_15959_amd.build)")
    L = ctypes.CDLL(path)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double
    L.elmddm_test_gemm.argtypes = [i32, i32, i32, i32, i32, i32, i32, d, vp, i32, i64, vp, i32, i64,
                                   d, vp, i32, i64, i32, vp]
    L.elmddm_test_mfma_layout.argtypes = [vp, vp, vp, vp]
    L.elmddm_test_gram_strip.argtypes = [i32, i32, vp, i32, i64, vp, i32, i64, i32, vp]
    L.elmddm_test_trsm_strip.argtypes = [i32, i32, vp, i32, i64, vp, i32, i64, vp, i64, i32, vp]
    L.elmddm_test_potrf.argtypes = [vp, i32, i64, i32, i32, vp, i64, vp, i32, i64, vp, vp, i32, vp]
    L.elmddm_test_mfma_layout_f32.argtypes = [vp, vp, vp, vp]
    L.elmddm_test_gram_f32.argtypes = [i32, i32, vp, i32, i64, vp, i32, i64, i32, vp]
    L.elmddm_test_gram.argtypes = [i32, i32, i32, vp, i32, i64, vp, i32, i64, i32, vp]
    L.elmddm_test_set_gemm_variant.argtypes = [i32, i32]
    return L


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_mfma_f64_lane_layout(hooks):
    """The GEMM kernel assumes: lane l holds A[l%16][l/16], B[l/16][l%16], and
    accumulator element r of lane l is D[4r + l/16][l%16]."""
    import torch
    rng = np.random.default_rng(0)
    A = rng.integers(-4, 5, (16, 4)).astype(np.float64)
    B = rng.integers(-4, 5, (4, 16)).astype(np.float64)
    lanes = np.arange(64)
    a = A[lanes % 16, lanes // 16]
    b = B[lanes // 16, lanes % 16]
    out = torch.zeros(256, dtype=torch.float64, device="cuda:0")
    da, db = _dev(a), _dev(b)          # keep the device buffers alive across the launch
    st = hooks.elmddm_test_mfma_layout(_p(da), _p(db), _p(out), _stream())
    assert st == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(64, 4)
    D = A @ B
    expect = np.array([[D[4 * r + l // 16, l % 16] for r in range(4)] for l in range(64)])
    assert np.array_equal(got, expect), got


def test_mfma_f32_lane_layout(hooks):
    """The FP32 Gram assumes: lane l holds A[l%16][l/16], B[l/16][l%16], and
    accumulator element r of lane l is D[4 (l/16) + r][l%16]."""
    import torch
    rng = np.random.default_rng(1)
    A = rng.integers(-4, 5, (16, 4)).astype(np.float32)
    B = rng.integers(-4, 5, (4, 16)).astype(np.float32)
    lanes = np.arange(64)
    da, db = _dev(A[lanes % 16, lanes // 16]), _dev(B[lanes // 16, lanes % 16])
    out = torch.zeros(256, dtype=torch.float32, device="cuda:0")
    assert hooks.elmddm_test_mfma_layout_f32(_p(da), _p(db), _p(out), _stream()) == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(64, 4)
    D = A @ B
    expect = np.array([[D[4 * (l // 16) + r, l % 16] for r in range(4)] for l in range(64)])
    assert np.array_equal(got, expect), got


@pytest.mark.parametrize("n,rows,batch", [(400, 1856, 2), (100, 520, 3), (37, 70, 2)])
def test_gram_f32_within_float32_bound(hooks, n, rows, batch):
    """FP32 operands and accumulation: every lower entry within the classical
    bound (rows + 2) u32 (|X|^T |X|) of the exact Gram, and visibly not FP64."""
    import torch
    rng = np.random.default_rng(n + 3 * rows)
    ldx, ldg = rows + 8, n + 5
    X = rng.standard_normal((batch, n + 1, ldx))
    dX = _dev(X)
    dG = torch.zeros(batch * (n + 1) * ldg, dtype=torch.float64, device="cuda:0")
    st = hooks.elmddm_test_gram_f32(n, rows, _p(dX), ldx, (n + 1) * ldx, _p(dG), ldg, (n + 1) * ldg, batch,
                                    _stream())
    assert st == 0
    torch.cuda.synchronize()
    G = dG.cpu().numpy().reshape(batch, n + 1, ldg)
    mask = np.tril(np.ones((n, n), bool))
    worst = 0.0
    for z in range(batch):
        Xz = X[z, :n, :rows].T
        ref = Xz.T @ Xz
        bound = (rows + 2) * 2.0**-24 * (np.abs(Xz).T @ np.abs(Xz))
        err = np.abs(G[z, :n, :n].T - ref)
        assert np.all(np.where(mask, err <= bound, True))
        worst = max(worst, np.where(mask, err / np.abs(ref).max(), 0).max())
    assert worst > 1e-12


def ref_gemm(ta, tb, kmode, lower, M, N, K, alpha, A, B, beta, C):
    """Column-major reference: C = alpha op(A) op(B) + beta C (restricted as the kernel documents)."""
    opA = A[:K, :M].T if ta else A[:M, :K]      # arrays given as (rows, cols) in math orientation
    opB = B[:N, :K].T if tb else B[:K, :N]
    return alpha * opA @ opB + beta * C[:M, :N]


def structured_B(B, tb, kmode, K, N):
    """Zero the entries of op(B) that kmode declares zero (the kernel skips them)."""
    k = np.arange(K)[:, None]
    j = np.arange(N)[None, :]
    keep = np.ones((K, N), bool)
    if kmode == 1:
        keep = k >= j
    if kmode == 2:
        keep = k <= j
    return B * (keep.T if tb else keep)


# Kernel variants: K depth 16 (double-buffered LDS) or 32, tile order plain or
# XCD-grouped; every case runs on each.  Odd M gives beta != 0, which takes
# the instance that reads C before the K loop.
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("ta,tb,kmode,lower,M,N,K,batch", [
    (0, 0, 0, 0, 70, 33, 129, 2), (0, 1, 0, 0, 64, 64, 64, 1), (1, 0, 0, 0, 100, 90, 37, 3),
    (1, 1, 0, 0, 17, 130, 16, 1), (1, 0, 0, 1, 150, 150, 300, 2), (0, 1, 0, 1, 131, 130, 64, 2),
    (0, 0, 1, 0, 40, 200, 200, 2), (0, 1, 2, 0, 300, 150, 150, 2), (0, 1, 0, 0, 1, 64, 64, 3),
    (0, 0, 1, 0, 41, 150, 150, 2), (0, 1, 2, 0, 301, 150, 150, 2), (1, 0, 0, 1, 97, 97, 45, 2),
])
def test_gemm_matches_numpy(hooks, variant, ta, tb, kmode, lower, M, N, K, batch):
    hooks.elmddm_test_set_gemm_variant(0, variant)
    hooks.elmddm_test_set_gemm_variant(1, variant)
    try:
        _check_gemm(hooks, ta, tb, kmode, lower, M, N, K, batch)
    finally:
        hooks.elmddm_test_set_gemm_variant(0, 1)   # the library's defaults
        hooks.elmddm_test_set_gemm_variant(1, 0)


def _check_gemm(hooks, ta, tb, kmode, lower, M, N, K, batch):
    import torch
    rng = np.random.default_rng(M * 7 + N + K)
    # math-orientation arrays, stored column-major => pass transposes as C-contiguous
    Ash = (K, M) if ta else (M, K)
    Bsh = (N, K) if tb else (K, N)
    A = rng.standard_normal((batch,) + Ash)
    B = structured_B(rng.standard_normal((batch,) + Bsh), tb, kmode, K, N)
    C = rng.standard_normal((batch, M, N))
    alpha, beta = -0.75, (0.5 if M % 2 else 0.0)
    dA = _dev(np.swapaxes(A, 1, 2))   # column-major storage
    dB = _dev(np.swapaxes(B, 1, 2))
    dC = _dev(np.swapaxes(C, 1, 2))
    st = hooks.elmddm_test_gemm(ta, tb, kmode, lower, M, N, K, alpha, _p(dA), Ash[0], Ash[0] * Ash[1],
                                _p(dB), Bsh[0], Bsh[0] * Bsh[1], beta, _p(dC), M, M * N, batch, _stream())
    assert st == 0
    torch.cuda.synchronize()
    got = np.swapaxes(dC.cpu().numpy(), 1, 2)
    for z in range(batch):
        ref = ref_gemm(ta, tb, kmode, lower, M, N, K, alpha, A[z], B[z], beta, C[z])
        g = got[z]
        if lower:
            # only tiles on or below the diagonal are written; compare the lower triangle
            mask = np.arange(M)[:, None] >= np.arange(N)[None, :]
            g = np.where(mask, g, 0.0)
            ref = np.where(mask, ref, 0.0)
        err = np.abs(g - ref).max() / max(np.abs(ref).max(), 1.0)
        assert err < 1e-13, (z, err)


@pytest.mark.parametrize("n,extra,batch", [(64, 0, 1), (150, 1, 3), (200, 0, 2), (37, 1, 2), (400, 1, 2),
                                           (256, 0, 2), (320, 1, 1), (130, 1, 2)])
def test_blocked_cholesky_and_inverse(hooks, n, extra, batch):
    import torch
    rng = np.random.default_rng(n + batch)
    Mrows = n + extra
    ld = n + 1 + 16
    A = np.zeros((batch, n + 1, ld))   # [col][row] storage per matrix
    Ls, invs, hs = [], [], []
    for z in range(batch):
        X = rng.standard_normal((3 * n, n + 1))
        X[:, :n] *= np.exp(rng.uniform(-4, 4, n))     # badly scaled columns
        G = X.T @ X
        L = np.linalg.cholesky(G[:n, :n])
        Ls.append(L)
        invs.append(np.linalg.inv(L))
        hs.append(np.linalg.solve(L, G[:n, n]))
        A[z, :, :n + 1] = G.T          # column-major
    nblk = (n + 63) // 64
    dA = _dev(A)
    dD = torch.zeros(batch * nblk * 64 * 64, dtype=torch.float64, device="cuda:0")
    dLi = torch.zeros(batch * n * ld, dtype=torch.float64, device="cuda:0")
    dT = torch.zeros(batch * 64 * n, dtype=torch.float64, device="cuda:0")
    info = torch.tensor([0, 2**31 - 1, 0, 0], dtype=torch.int32, device="cuda:0")
    st = hooks.elmddm_test_potrf(_p(dA), ld, (n + 1) * ld, Mrows, n, _p(dD), nblk * 4096, _p(dLi), ld, n * ld,
                                 _p(dT), _p(info), batch, _stream())
    assert st == 0
    torch.cuda.synchronize()
    assert info[0].item() == 0
    out = dA.cpu().numpy()
    Li = dLi.cpu().numpy().reshape(batch, n, ld)
    for z in range(batch):
        Lg = np.tril(out[z, :n, :n].T)
        assert np.abs(Lg - Ls[z]).max() <= 1e-12 * np.abs(Ls[z]).max()
        Lig = Li[z, :, :n].T
        assert np.abs(np.triu(Lig, 1)).max() == 0.0
        rel = np.linalg.norm(Lig @ Ls[z] - np.eye(n)) / np.sqrt(n)
        assert rel < 1e-12 * np.linalg.cond(Ls[z])
        if extra:
            h = out[z, :n, n]
            assert np.linalg.norm(h - hs[z]) <= 1e-10 * np.linalg.norm(hs[z])


def test_cholesky_reports_indefinite_matrix(hooks):
    import torch
    n, ld = 80, 96
    rng = np.random.default_rng(1)
    X = rng.standard_normal((200, n))
    G = X.T @ X
    G[70, 70] = -1.0
    A = np.zeros((1, n + 1, ld))
    A[0, :n, :n] = G.T
    dA = _dev(A)
    dD = torch.zeros(2 * 4096, dtype=torch.float64, device="cuda:0")
    dT = torch.zeros(64 * n, dtype=torch.float64, device="cuda:0")
    info = torch.tensor([0, 2**31 - 1, 0, 0], dtype=torch.int32, device="cuda:0")
    st = hooks.elmddm_test_potrf(_p(dA), ld, (n + 1) * ld, n, n, _p(dD), 2 * 4096, None, ld, 0, _p(dT),
                                 _p(info), 1, _stream())
    assert st == 0
    torch.cuda.synchronize()
    assert info[0].item() == 3 and info[1].item() == 0


@pytest.mark.parametrize("n,rows,batch", [(400, 1856, 2), (100, 480, 3), (30, 70, 2), (200, 900, 1), (1000, 300, 1)])
def test_gram_strip_lower_triangle(hooks, n, rows, batch):
    import torch
    assert 4 <= hooks.elmddm_test_strip_width(n) <= 8
    rng = np.random.default_rng(n + rows)
    ldx, ldg = rows + 8, n + 5
    X = rng.standard_normal((batch, n + 1, ldx))      # [col][row]
    dX = _dev(X)
    dG = torch.zeros(batch * (n + 1) * ldg, dtype=torch.float64, device="cuda:0")
    st = hooks.elmddm_test_gram_strip(n, rows, _p(dX), ldx, (n + 1) * ldx, _p(dG), ldg, (n + 1) * ldg, batch, _stream())
    assert st == 0
    torch.cuda.synchronize()
    G = dG.cpu().numpy().reshape(batch, n + 1, ldg)
    for z in range(batch):
        Xz = X[z, :n, :rows].T
        ref = Xz.T @ Xz
        got = G[z, :n, :n].T                         # back to row-major math orientation
        mask = np.tril(np.ones((n, n), bool))
        assert np.abs(np.where(mask, got - ref, 0)).max() <= 1e-13 * np.abs(ref).max()


GRAM_CODES = [-1, -2, -3, -4, 4, 5, 6, 7, 8]


@pytest.mark.parametrize("code", GRAM_CODES)
@pytest.mark.parametrize("n,rows,batch", [(400, 1920, 3), (130, 71, 2), (257, 300, 1), (16, 5, 2), (1, 9, 2)])
def test_gram_candidates_lower_triangle_and_bounds(hooks, code, n, rows, batch):
    """Every Gram candidate of the autotuner gives the lower triangle of X^T X
    and writes nothing outside the n x n block of each matrix (sentinel
    padding in the leading dimension, the extra column and between
    batch entries stays)."""
    import torch
    rng = np.random.default_rng(1000 * n + rows + code)
    ldx, ldg = rows + 3, n + 7
    X = rng.standard_normal((batch, n + 1, ldx))
    dX = _dev(X)
    sentinel = 12345.0
    dG = torch.full((batch * (n + 1) * ldg,), sentinel, dtype=torch.float64, device="cuda:0")
    st = hooks.elmddm_test_gram(code, n, rows, _p(dX), ldx, (n + 1) * ldx, _p(dG), ldg, (n + 1) * ldg, batch,
                                _stream())
    assert st == 0
    torch.cuda.synchronize()
    G = dG.cpu().numpy().reshape(batch, n + 1, ldg)
    mask = np.tril(np.ones((n, n), bool))
    for z in range(batch):
        Xz = X[z, :n, :rows].T
        ref = Xz.T @ Xz
        got = G[z, :n, :n].T
        assert np.abs(np.where(mask, got - ref, 0)).max() <= 1e-13 * np.abs(ref).max()
        assert np.all(G[z, :n, n:] == sentinel) and np.all(G[z, n, :] == sentinel)


@pytest.mark.parametrize("rows,n,batch", [(2016, 400, 2), (480, 100, 3), (70, 30, 2), (333, 200, 1)])
def test_trsm_strip_matches_product_with_triangular_inverse(hooks, rows, n, batch):
    import torch
    rng = np.random.default_rng(rows + n)
    ldx, ldl = rows + 4, n + 3
    X = rng.standard_normal((batch, n + 1, ldx))
    Li = np.zeros((batch, n, ldl))
    for z in range(batch):
        Li[z, :, :n] = np.tril(rng.standard_normal((n, n))).T    # col-major lower
    dX, dL = _dev(X), _dev(Li)
    dY = torch.zeros_like(dX)
    st = hooks.elmddm_test_trsm_strip(rows, n, _p(dX), ldx, (n + 1) * ldx, _p(dL), ldl, n * ldl, _p(dY), (n + 1) * ldx, batch, _stream())
    assert st == 0
    torch.cuda.synchronize()
    Y = dY.cpu().numpy()
    for z in range(batch):
        Lz = Li[z, :, :n].T
        ref = X[z, :n, :rows].T @ Lz.T
        got = Y[z, :n, :rows].T
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
