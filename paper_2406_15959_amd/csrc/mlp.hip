// Interface-variable MLP on the matrix cores (FP32): forward, backward and
// Adam kernels and the C ABI around them.
//
// Not a part of the paper's method: for a fixed geometry and hidden layer
// the interface variable u_Gamma of the Schur system (Section 3, eq. schur)
// is a function of the source; a network x -> GELU(W1 x + b1) ->
// GELU(W2 h1 + b2) -> W3 h2 + b3 (exact GELU z Phi(z)) learns it from pairs
// that the method generates, and its prediction serves as an initial guess
// for the interface solve.  Loss: mean squared error over batch and output
// entries; optimiser: Adam with bias correction (Kingma and Ba, 2015).
//
// Storage: FP32, column-major.  Activations are (features x batch), i.e.
// one contiguous column per sample; weight matrices (fan_out x fan_in).
// Flat parameter vector: W1, b1, W2, b2, W3, b3.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/elmddm.h"
#include "internal.h"

namespace elmddm {

typedef float v4f __attribute__((ext_vector_type(4)));

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

__device__ __forceinline__ float gelu_f(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C (M x N) = op(A) op(B) with the epilogue EPI; 64 x 64 workgroup tile, four
// waves (2 x 2) of 2 x 2 V_MFMA_F32_16X16X4 tiles, K staged 32 at a time in
// LDS (rows padded so a wave's four k rows fall in different banks).
//   op(A)(i, k) = TA ? A[i lda + k] : A[k lda + i]
//   op(B)(k, j) = TB ? B[k ldb + j] : B[j ldb + k]
// Accumulator element r of lane l is D[4 (l/16) + r][l % 16].
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, const float* __restrict__ A,
                                                    int lda, const float* __restrict__ B, int ldb,
                                                    float* __restrict__ C, int ldc,
                                                    const float* __restrict__ bias,
                                                    const float* __restrict__ Zin,
                                                    float* __restrict__ Aout)
{
    constexpr int BK = 32;
    __shared__ float As[BK][64 + 16];
    __shared__ float Bs[BK][64 + 16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    float ra[8], rb[8];
    auto load = [&](int k0) {
        if (!TA) {
            const int kk = k0 + tid / 8, mm = m0 + (tid % 8) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) ra[e] = (kk < K && mm + e < M) ? A[(long long)kk * lda + mm + e] : 0.f;
        } else {
            const int mm = m0 + tid / 4, kk = k0 + (tid % 4) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) ra[e] = (mm < M && kk + e < K) ? A[(long long)mm * lda + kk + e] : 0.f;
        }
        if (!TB) {
            const int nn = n0 + tid / 4, kk = k0 + (tid % 4) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[e] = (nn < N && kk + e < K) ? B[(long long)nn * ldb + kk + e] : 0.f;
        } else {
            const int kk = k0 + tid / 8, nn = n0 + (tid % 8) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[e] = (kk < K && nn + e < N) ? B[(long long)kk * ldb + nn + e] : 0.f;
        }
    };
    auto store = [&]() {
        if (!TA) {
            const int k = tid / 8, m = (tid % 8) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) As[k][m + e] = ra[e];
        } else {
            const int m = tid / 4, k = (tid % 4) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) As[k + e][m] = ra[e];
        }
        if (!TB) {
            const int nn = tid / 4, k = (tid % 4) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) Bs[k + e][nn] = rb[e];
        } else {
            const int k = tid / 8, nn = (tid % 8) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) Bs[k][nn + e] = rb[e];
        }
    };
    v4f acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = (v4f){0.f, 0.f, 0.f, 0.f};
    const int nk = (K + BK - 1) / BK;
    const int lr = lane & 15, lq = lane >> 4;
    if (nk > 0) {
        load(0);
        store();
        __syncthreads();
        for (int it = 0; it < nk; ++it) {
            if (it + 1 < nk) load((it + 1) * BK);
            float av[BK / 4][2], bv[BK / 4][2];
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks) {
                const int k = ks * 4 + lq;
                av[ks][0] = As[k][wm * 32 + lr];
                av[ks][1] = As[k][wm * 32 + 16 + lr];
                bv[ks][0] = Bs[k][wn * 32 + lr];
                bv[ks][1] = Bs[k][wn * 32 + 16 + lr];
            }
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v)
                        acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][u], bv[ks][v], acc[u][v], 0, 0, 0);
            __syncthreads();
            if (it + 1 < nk) {
                store();
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + u * 16 + 4 * lq + r;
                const int col = n0 + wn * 32 + v * 16 + lr;
                if (row >= M || col >= N) continue;
                const long long ci = (long long)col * ldc + row;
                float val = acc[u][v][r];
                if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) val += bias[row];
                if (EPI == EPI_GELU_BWD) val *= gelu_grad_f(Zin[ci]);
                C[ci] = val;
                if (EPI == EPI_BIAS_GELU) Aout[ci] = gelu_f(val);
            }
}

template <bool TA, bool TB, int EPI>
static void sgemm(hipStream_t st, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                  float* C, int ldc, const float* bias = nullptr, const float* Zin = nullptr,
                  float* Aout = nullptr)
{
    dim3 grid((M + 63) / 64, (N + 63) / 64);
    hipLaunchKernelGGL((sgemm_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                       bias, Zin, Aout);
}

// db[o] = sum_b dZ[b ld + o]
__global__ void bias_grad_kernel(int O, int B, const float* dZ, int ld, float* db)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    float acc = 0.f;
    for (int b = 0; b < B; ++b) acc += dZ[(long long)b * ld + o];
    db[o] = acc;
}

// dY = 2 (Y - T) / count; per-block partial sums of (Y - T)^2.
__global__ __launch_bounds__(256) void mse_kernel(long long count, const float* Y, const float* T, float* dY,
                                                  float two_over, float* partial)
{
    __shared__ float red[256];
    float acc = 0.f;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < count; i += (long long)gridDim.x * 256) {
        const float d = Y[i] - T[i];
        dY[i] = two_over * d;
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_partials_kernel(int nparts, const float* partial, float scale,
                                                           float* out)
{
    __shared__ float red[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// One Adam step over the flat parameter vector; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_kernel(long long n, float* theta, const float* g, float* m, float* v, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Xb[b][d] = X[idx[b]][d] (zero for an index outside [0, ns))
__global__ void gather_rows_kernel(int D, int B, int ns, const float* X, const int32_t* idx, float* Xb)
{
    const int b = blockIdx.y;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    const int i = idx[b];
    Xb[(long long)b * D + d] = (i >= 0 && i < ns) ? X[(long long)i * D + d] : 0.f;
}

__global__ void scale_out_kernel(long long n, const float* y, double scale, double* out)
{
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) out[i] = scale * (double)y[i];
}

}  // namespace elmddm

using namespace elmddm;

struct elmddm_mlp {
    int D = 0, H = 0, O = 0, maxB = 0;
    long long nparam = 0;
    long long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Y = nullptr;
    float *dY = nullptr, *dA = nullptr, *dB = nullptr, *Xb = nullptr, *Tb = nullptr, *partial = nullptr;
    int step = 0;
    std::vector<void*> allocs;

    template <class T>
    bool alloc(T** p, size_t count)
    {
        if (hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
        allocs.push_back(*p);
        return true;
    }
    ~elmddm_mlp()
    {
        for (void* q : allocs) (void)hipFree(q);
    }

    // forward pass on a batch x (D x Bn): fills Z1, A1, Z2, A2, Y
    void forward(hipStream_t st, int Bn, const float* x)
    {
        sgemm<false, false, EPI_BIAS_GELU>(st, H, Bn, D, theta + oW1, H, x, D, Z1, H, theta + ob1, nullptr, A1);
        sgemm<false, false, EPI_BIAS_GELU>(st, H, Bn, H, theta + oW2, H, A1, H, Z2, H, theta + ob2, nullptr, A2);
        sgemm<false, false, EPI_BIAS>(st, O, Bn, H, theta + oW3, O, A2, H, Y, O, theta + ob3);
    }

    // gradient of the mean squared error against t (O x Bn) into grad; loss into *loss
    void backward(hipStream_t st, int Bn, const float* x, const float* t, float* loss)
    {
        const long long cnt = (long long)O * Bn;
        const int nparts = (int)std::min<long long>(1024, (cnt + 255) / 256);
        hipLaunchKernelGGL(mse_kernel, dim3(nparts), dim3(256), 0, st, cnt, Y, t, dY, 2.0f / (float)cnt, partial);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, nparts, partial, 1.0f / (float)cnt, loss);
        // layer 3
        sgemm<false, true, EPI_STORE>(st, O, H, Bn, dY, O, A2, H, grad + oW3, O);
        hipLaunchKernelGGL(bias_grad_kernel, dim3((O + 255) / 256), dim3(256), 0, st, O, Bn, dY, O, grad + ob3);
        sgemm<true, false, EPI_GELU_BWD>(st, H, Bn, O, theta + oW3, O, dY, O, dA, H, nullptr, Z2);
        // layer 2 (dA holds dZ2)
        sgemm<false, true, EPI_STORE>(st, H, H, Bn, dA, H, A1, H, grad + oW2, H);
        hipLaunchKernelGGL(bias_grad_kernel, dim3((H + 255) / 256), dim3(256), 0, st, H, Bn, dA, H, grad + ob2);
        sgemm<true, false, EPI_GELU_BWD>(st, H, Bn, H, theta + oW2, H, dA, H, dB, H, nullptr, Z1);
        // layer 1 (dB holds dZ1)
        sgemm<false, true, EPI_STORE>(st, H, D, Bn, dB, H, x, D, grad + oW1, H);
        hipLaunchKernelGGL(bias_grad_kernel, dim3((H + 255) / 256), dim3(256), 0, st, H, Bn, dB, H, grad + ob1);
    }

    void adam(hipStream_t st, float lr, float b1, float b2, float eps)
    {
        ++step;
        const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
        hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((nparam + 255) / 256)), dim3(256), 0, st, nparam, theta,
                           grad, m, v, lr, b1, b2, eps, c1, c2);
    }
};

namespace {
elmddm_status err(elmddm_status s, const char* msg) { return (elmddm_status)record_error(s, msg); }
elmddm_status launched(const char* where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return err(ELMDDM_HIP_ERROR, (std::string(where) + ": " + hipGetErrorString(e)).c_str());
    return ELMDDM_OK;
}
}  // namespace

extern "C" {

elmddm_status elmddm_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t max_batch,
                                elmddm_mlp** out)
{
    if (!out) return err(ELMDDM_INVALID_ARG, "NULL output pointer");
    *out = nullptr;
    if (in_dim < 1 || hidden < 1 || out_dim < 1 || max_batch < 1 || in_dim > (1 << 20) ||
        hidden > (1 << 14) || out_dim > (1 << 22) || max_batch > (1 << 16))
        return err(ELMDDM_INVALID_ARG, "MLP sizes out of range");
    elmddm_mlp* P = new elmddm_mlp();
    P->D = in_dim;
    P->H = hidden;
    P->O = out_dim;
    P->maxB = max_batch;
    const long long D = in_dim, H = hidden, O = out_dim, B = max_batch;
    P->oW1 = 0;
    P->ob1 = H * D;
    P->oW2 = P->ob1 + H;
    P->ob2 = P->oW2 + H * H;
    P->oW3 = P->ob2 + H;
    P->ob3 = P->oW3 + O * H;
    P->nparam = P->ob3 + O;
    bool ok = P->alloc(&P->theta, P->nparam) && P->alloc(&P->grad, P->nparam) && P->alloc(&P->m, P->nparam) &&
              P->alloc(&P->v, P->nparam) && P->alloc(&P->Z1, H * B) && P->alloc(&P->A1, H * B) &&
              P->alloc(&P->Z2, H * B) && P->alloc(&P->A2, H * B) && P->alloc(&P->Y, O * B) &&
              P->alloc(&P->dY, O * B) && P->alloc(&P->dA, H * B) && P->alloc(&P->dB, H * B) &&
              P->alloc(&P->Xb, D * B) && P->alloc(&P->Tb, O * B) && P->alloc(&P->partial, 1025);
    if (!ok) {
        delete P;
        return err(ELMDDM_OOM, "hipMalloc failed for the MLP");
    }
    *out = P;
    return ELMDDM_OK;
}

elmddm_status elmddm_mlp_destroy(elmddm_mlp* P)
{
    delete P;
    return ELMDDM_OK;
}

elmddm_status elmddm_mlp_num_params(const elmddm_mlp* P, int64_t* count)
{
    if (!P || !count) return err(ELMDDM_INVALID_ARG, "NULL argument");
    *count = P->nparam;
    return ELMDDM_OK;
}

elmddm_status elmddm_mlp_set_params(elmddm_mlp* P, const float* params, void* stream)
{
    if (!P || !params) return err(ELMDDM_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)P->nparam * sizeof(float);
    if (hipMemcpyAsync(P->theta, params, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(P->m, 0, bytes, st) != hipSuccess || hipMemsetAsync(P->v, 0, bytes, st) != hipSuccess)
        return launched("mlp_set_params");
    P->step = 0;
    return ELMDDM_OK;
}

elmddm_status elmddm_mlp_get_params(const elmddm_mlp* P, float* params, void* stream)
{
    if (!P || !params) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (hipMemcpyAsync(params, P->theta, (size_t)P->nparam * sizeof(float), hipMemcpyDeviceToDevice,
                       (hipStream_t)stream) != hipSuccess)
        return launched("mlp_get_params");
    return ELMDDM_OK;
}

elmddm_status elmddm_mlp_forward(elmddm_mlp* P, int32_t batch, const float* x, float* y, void* stream)
{
    if (!P || !x || !y) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (batch < 1 || batch > P->maxB) return err(ELMDDM_INVALID_ARG, "batch out of range");
    hipStream_t st = (hipStream_t)stream;
    P->forward(st, batch, x);
    if (hipMemcpyAsync(y, P->Y, (size_t)P->O * batch * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return launched("mlp_forward copy");
    return launched("mlp_forward");
}

elmddm_status elmddm_mlp_loss_grad(elmddm_mlp* P, int32_t batch, const float* x, const float* t, float* loss,
                                   float* grad, void* stream)
{
    if (!P || !x || !t || !loss) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (batch < 1 || batch > P->maxB) return err(ELMDDM_INVALID_ARG, "batch out of range");
    hipStream_t st = (hipStream_t)stream;
    P->forward(st, batch, x);
    P->backward(st, batch, x, t, loss);
    if (grad && hipMemcpyAsync(grad, P->grad, (size_t)P->nparam * sizeof(float), hipMemcpyDeviceToDevice, st) !=
                    hipSuccess)
        return launched("mlp_loss_grad copy");
    return launched("mlp_loss_grad");
}

elmddm_status elmddm_mlp_adam_step(elmddm_mlp* P, float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!P) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return err(ELMDDM_INVALID_ARG, "bad Adam hyper-parameters");
    P->adam((hipStream_t)stream, lr, beta1, beta2, eps);
    return launched("mlp_adam_step");
}

elmddm_status elmddm_mlp_train(elmddm_mlp* P, int32_t nsamples, const float* X, const float* T,
                               const int32_t* order, int32_t steps, int32_t batch, float lr, float beta1,
                               float beta2, float eps, float* losses, void* stream)
{
    if (!P || !X || !T || !order) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (batch < 1 || batch > P->maxB || nsamples < 1 || steps < 0)
        return err(ELMDDM_INVALID_ARG, "bad batch, sample count or step count");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return err(ELMDDM_INVALID_ARG, "bad Adam hyper-parameters");
    hipStream_t st = (hipStream_t)stream;
    for (int k = 0; k < steps; ++k) {
        const int32_t* idx = order + (long long)k * batch;
        hipLaunchKernelGGL(gather_rows_kernel, dim3((P->D + 255) / 256, batch), dim3(256), 0, st, P->D, batch,
                           nsamples, X, idx, P->Xb);
        hipLaunchKernelGGL(gather_rows_kernel, dim3((P->O + 255) / 256, batch), dim3(256), 0, st, P->O, batch,
                           nsamples, T, idx, P->Tb);
        P->forward(st, batch, P->Xb);
        P->backward(st, batch, P->Xb, P->Tb, losses ? losses + k : P->partial + 1024);
        // cosine decay from lr to 0 over the run
        const float lrk = 0.5f * lr * (1.f + std::cos(3.14159265358979f * (float)k / (float)std::max(steps, 1)));
        P->adam(st, lrk, beta1, beta2, eps);
    }
    return launched("mlp_train");
}

elmddm_status elmddm_mlp_predict(elmddm_mlp* P, int32_t batch, const float* x, double scale, double* out,
                                 void* stream)
{
    if (!P || !x || !out) return err(ELMDDM_INVALID_ARG, "NULL argument");
    if (batch < 1 || batch > P->maxB) return err(ELMDDM_INVALID_ARG, "batch out of range");
    hipStream_t st = (hipStream_t)stream;
    P->forward(st, batch, x);
    const long long n = (long long)P->O * batch;
    hipLaunchKernelGGL(scale_out_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, P->Y, scale, out);
    return launched("mlp_predict");
}

}  // extern "C"
