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

// Gram product through the autotuner's dispatch: code as in elmddm_autotune.
int elmddm_test_gram(int code, int n, int rows, const double* X, int ldx, long long sX, double* G, int ldg,
                     long long sG, int batch, void* stream)
{
    gram_product((hipStream_t)stream, code, n, rows, X, ldx, sX, G, ldg, sG, batch);
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

// Sustained rate of the FP64 matrix instructions from registers alone (no
// memory traffic in the loop): the ceiling that any kernel built on the
// instruction can reach on this device, next to the published peak.
// SHAPE 0: V_MFMA_F64_16X16X4, 8 independent accumulators per wave.
// SHAPE 1: V_MFMA_F64_4X4X4_4B, a 4 x 4 outer product of operand registers
// (16 accumulators per wave).
template <int SHAPE>
__global__ __launch_bounds__(256) void mfma_rate_kernel(double* out, int iters)
{
    double s = 0.0;
    if (SHAPE == 0) {
        v4d acc[8];
        for (int j = 0; j < 8; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
        const double a = threadIdx.x * 1e-3, b = 1.0 + blockIdx.x * 1e-6;
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    } else {
        double acc[16], a[4], b[4];
        for (int j = 0; j < 16; ++j) acc[j] = 0.0;
        for (int j = 0; j < 4; ++j) {
            a[j] = threadIdx.x * 1e-3 + j;
            b[j] = 1.0 + blockIdx.x * 1e-6 + j;
        }
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[4 * p + q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[p], b[q], acc[4 * p + q], 0, 0, 0);
        for (int j = 0; j < 16; ++j) s += acc[j];
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Runs the loop above with waves_per_simd waves on every SIMD of the device
// (workgroups of four waves, one per SIMD) and returns the rate in TFLOP/s
// (*tflops) measured with events on stream.  Returns 0, or 7 on a HIP error.
extern "C" int elmddm_test_mfma_f64_rate(int shape, int waves_per_simd, int iters, double* tflops, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 7;
    const int blocks = cus * waves_per_simd;
    double* out = nullptr;
    if (hipMalloc(&out, sizeof(double) * blocks * 256) != hipSuccess) return 7;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 7;
    auto launch = [&] {
        if (shape == 0) hipLaunchKernelGGL(mfma_rate_kernel<0>, dim3(blocks), dim3(256), 0, st, out, iters);
        else hipLaunchKernelGGL(mfma_rate_kernel<1>, dim3(blocks), dim3(256), 0, st, out, iters);
    };
    launch();
    (void)hipEventRecord(e0, st);
    launch();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double flops_per_inst = shape == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 4 * 4 * 4 * 4;
    const double insts = (double)blocks * 4 * iters * (shape == 0 ? 8 : 16);
    *tflops = insts * flops_per_inst / (ms * 1e-3) / 1e12;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const bool ok = hipGetLastError() == hipSuccess;
    (void)hipFree(out);
    return ok ? 0 : 7;
}
