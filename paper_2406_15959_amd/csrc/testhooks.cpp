// Test-only entry points into the internal kernels (built as a separate
// library, libelmddm_testhooks.so, used by the kernel-level parity tests).
#include <hip/hip_runtime.h>

#include "internal.h"

using namespace elmddm;

typedef double v4d __attribute__((ext_vector_type(4)));

// One V_MFMA_F64_16X16X4 with per-lane operands a[lane], b[lane]; writes the
// raw accumulator: out[lane * 4 + r].
__global__ void mfma_probe_kernel(const double* a, const double* b, double* out)
{
    const int l = threadIdx.x;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[l], b[l], acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = acc[r];
}

typedef float v4f __attribute__((ext_vector_type(4)));

// One V_MFMA_F32_16X16X4 with per-lane operands; raw accumulator out[lane * 4 + r].
__global__ void mfma_probe_f32_kernel(const float* a, const float* b, float* out)
{
    const int l = threadIdx.x;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[l * 4 + r] = acc[r];
}

extern "C" {

// a, b: 64 floats each (device); out: 256 floats (device).  One wave.
int elmddm_test_mfma_layout_f32(const float* a, const float* b, float* out, void* stream)
{
    hipLaunchKernelGGL(mfma_probe_f32_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, a, b, out);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

// Lower triangle of X^T X (n x n) with FP32 operands and accumulation.
int elmddm_test_gram_f32(int n, int rows, const double* X, int ldx, long long sX, double* G, int ldg,
                         long long sG, int batch, void* stream)
{
    gram_product_f32((hipStream_t)stream, n, rows, X, ldx, sX, G, ldg, sG, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

// a, b: 64 doubles each (device); out: 256 doubles (device).  One wave.
int elmddm_test_mfma_layout(const double* a, const double* b, double* out, void* stream)
{
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, a, b, out);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

int elmddm_test_gemm(int ta, int tb, int kmode, int lower, int M, int N, int K, double alpha,
                     const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                     double beta, double* C, int ldc, long long sC, int batch, void* stream)
{
    gemm_f64((hipStream_t)stream, ta != 0, tb != 0, kmode, lower != 0, M, N, K, alpha, A, lda, sA,
             B, ldb, sB, beta, C, ldc, sC, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

void elmddm_test_set_gemm_variant(int which, int v) { set_gemm_variant(which, v); }

int elmddm_test_strip_width(int n) { return strip_width(n); }

// Plain column-major C = A B with the strip kernel of width T (4..8).
int elmddm_test_strip_gemm(int T, int M, int N, int K, const double* A, int lda, const double* B,
                           int ldb, double* C, int ldc, void* stream)
{
    strip_gemm_nn((hipStream_t)stream, T, M, N, K, A, lda, B, ldb, C, ldc);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

int elmddm_test_gram_strip(int n, int rows, const double* X, int ldx, long long sX, double* G, int ldg,
                           long long sG, int batch, void* stream)
{
    gram_strip((hipStream_t)stream, strip_width(n), n, rows, X, ldx, sX, G, ldg, sG, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

int elmddm_test_trsm_strip(int rows, int n, const double* X, int ldx, long long sX, const double* Li,
                           int ldl, long long sL, double* Y, long long sY, int batch, void* stream)
{
    trsm_strip((hipStream_t)stream, strip_width(n), rows, n, X, ldx, sX, Li, ldl, sL, Y, sY, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

// info: device int32[4] (status, bad_subdomain, bad_pass, pad), initialised by the caller.
int elmddm_test_potrf(double* A, int lda, long long sA, int Mrows, int n, double* Dinv,
                      long long sD, double* Linv, int ldl, long long sL, double* Tbuf, int* info,
                      int batch, void* stream)
{
    blocked_potrf((hipStream_t)stream, A, lda, sA, Mrows, n, Dinv, sD, Linv, ldl, sL, Tbuf,
                  reinterpret_cast<DevInfo*>(info), 1, batch, nullptr, 0);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

}  // extern "C"
