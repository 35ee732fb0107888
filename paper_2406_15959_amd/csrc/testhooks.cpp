// Test-only entry points into the internal kernels (built as a separate
// library, libelmddm_testhooks.so, used by the kernel-level parity tests).
#include <hip/hip_runtime.h>

#include "internal.h"

using namespace elmddm;

extern "C" {

int elmddm_test_gemm(int ta, int tb, int kmode, int lower, int M, int N, int K, double alpha,
                     const double* A, int lda, long long sA, const double* B, int ldb, long long sB,
                     double beta, double* C, int ldc, long long sC, int batch, void* stream)
{
    gemm_f64((hipStream_t)stream, ta != 0, tb != 0, kmode, lower != 0, M, N, K, alpha, A, lda, sA,
             B, ldb, sB, beta, C, ldc, sC, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

// info: device int32[4] (status, bad_subdomain, bad_pass, pad), initialised by the caller.
int elmddm_test_potrf(double* A, int lda, long long sA, int Mrows, int n, double* Dinv,
                      long long sD, double* Linv, int ldl, long long sL, double* Tbuf, int* info,
                      int batch, void* stream)
{
    blocked_potrf((hipStream_t)stream, A, lda, sA, Mrows, n, Dinv, sD, Linv, ldl, sL, Tbuf,
                  reinterpret_cast<DevInfo*>(info), 1, batch);
    return hipGetLastError() == hipSuccess ? 0 : 7;
}

}  // extern "C"
