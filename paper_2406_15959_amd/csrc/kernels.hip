// HIP kernels for gfx950 (MI355X): feature assembly, batched FP64 MFMA GEMM,
// blocked Cholesky pieces, interface Schur assembly, triangular solves and
// evaluation.  Column-major storage throughout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace elmddm {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Feature assembly (paper, Section 3, eq. nonoverlap_discrete; Section 4.1):
// one row per collocation point, one column per neuron plus the rhs column.
//   interior row : L phi_j = -Lap phi_j            (Poisson)
//                  L phi_j = -a Lap phi_j - grad a . grad phi_j  (variable coefficient)
//   boundary row : phi_j,  rhs g
//   interface row: phi_j,  rhs 0
//   flux row     : grad phi_j . n_s  (outward normal), rhs 0
// with phi_j = tanh(z), z = w_x xhat + w_y yhat + b, tanh' = 1 - t^2,
// tanh'' = -2 t (1 - t^2), and d/dx = s_x d/dxhat.
// A wave covers 64 consecutive rows of one column, so stores are coalesced.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void assemble_kernel(
    int ldx, int n, RowTable rows, SubGeom geom, int op, const double* __restrict__ W,
    const double* __restrict__ bias, const double* __restrict__ f, const double* __restrict__ g,
    const double* __restrict__ coef, long long coef_stride, double* __restrict__ X, long long sX,
    bool compact, double* __restrict__ Fout, int ldF, double* __restrict__ Kout, int ldK,
    long long sK, double* __restrict__ Dout, int ldD, long long sD)
{
    const int s = blockIdx.z;
    const int r = blockIdx.x * 64 + (threadIdx.x & 63);
    const int cg = threadIdx.x >> 6;
    if (r >= ldx) return;
    const long long ri = (long long)s * ldx + r;
    const int kind = rows.kind[ri];
    const int src = rows.src[ri];
    const double xh = (rows.x[ri] - geom.cx[s]) * geom.sx;
    const double yh = (rows.y[ri] - geom.cy[s]) * geom.sy;
    const double nxv = rows.nx[ri], nyv = rows.ny[ri];
    double a = 1.0, ax = 0.0, ay = 0.0;
    if (op == 1 && kind == ROW_INTERIOR) {
        a = coef[src];
        ax = coef[coef_stride + src];
        ay = coef[2 * coef_stride + src];
    }
    const int crow = compact ? rows.cmap[ri] : -1;
    const int c0 = blockIdx.y * 64;
    for (int cc = cg; cc < 64; cc += 4) {
        const int col = c0 + cc;
        if (col > n) break;
        double v = 0.0;
        if (col == n) {
            if (kind == ROW_INTERIOR) v = f[src];
            else if (kind == ROW_BOUNDARY) v = g[src];
        } else if (kind != ROW_ZERO) {
            const long long wi = (long long)s * n + col;
            const double w0 = W[2 * wi], w1 = W[2 * wi + 1];
            const double wx = w0 * geom.sx;
            const double wy = w1 * geom.sy;
            const double z = w0 * xh + w1 * yh + bias[wi];
            const double t = tanh(z);
            const double d1 = 1.0 - t * t;
            if (kind == ROW_INTERIOR) {
                const double lap = (-2.0 * t * d1) * (wx * wx + wy * wy);
                v = (op == 0) ? -lap : (-(a * lap) - (ax * (d1 * wx) + ay * (d1 * wy)));
            } else if (kind == ROW_FLUX) {
                v = d1 * (nxv * wx + nyv * wy);
            } else {
                v = t;
            }
        }
        if (!compact) {
            X[s * sX + (long long)col * ldx + r] = v;
        } else if (crow >= 0) {
            if (col == n) Fout[(long long)s * ldF + crow] = v;
            else Kout[s * sK + (long long)col * ldK + crow] = v;
        } else if (crow <= -2 && col < n) {
            Dout[s * sD + (long long)col * ldD + (-2 - crow)] = v;
        }
    }
}

void assemble(hipStream_t st, int N, int ldx, int n, const RowTable& rows, const SubGeom& geom,
              int op, const double* W, const double* b, const double* f, const double* g,
              const double* coef, int q2, double* X, double* Fout, int ldF, double* Kout, int ldK,
              double* Dout, int ldD)
{
    dim3 grid((ldx + 63) / 64, (n + 1 + 63) / 64, N);
    const bool compact = (Kout != nullptr);
    hipLaunchKernelGGL(assemble_kernel, grid, dim3(256), 0, st, ldx, n, rows, geom, op, W, b, f, g,
                       coef, (long long)N * q2, X, (long long)ldx * (n + 1), compact, Fout, ldF,
                       Kout, ldK, (long long)ldK * n, Dout, ldD, (long long)ldD * n);
}

// ---------------------------------------------------------------------------
// Batched FP64 GEMM on the matrix cores: C = alpha op(A) op(B) + beta C.
// Workgroup tile 64x64, K staged 16 at a time through LDS, four waves in a
// 2x2 arrangement, each wave a 32x32 block of 2x2 V_MFMA_F64_16X16X4 tiles.
// MFMA operand layout (16x16x4, f64): lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the accumulator's element r of lane l is D[4*r + l/16][l%16].
// The next K stage is fetched into registers while the current one computes.
// ---------------------------------------------------------------------------
#define GB_M 64
#define GB_N 64
#define GB_K 16

template <bool TA, bool TB, int KMODE, bool LOWER>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double* A, int lda, long long sA, const double* B,
    int ldb, long long sB, double beta, double* C, int ldc, long long sC)
{
    const int tm = blockIdx.x, tn = blockIdx.y;
    if (LOWER && tm < tn) return;
    const long long z = blockIdx.z;
    A += z * sA;
    B += z * sB;
    C += z * sC;
    const int m0 = tm * GB_M, n0 = tn * GB_N;
    int kbeg = 0, kend = K;
    if (KMODE == 1) kbeg = n0 < K ? n0 : K;
    if (KMODE == 2) kend = (n0 + GB_N) < K ? (n0 + GB_N) : K;

    __shared__ double As[GB_K][GB_M];
    __shared__ double Bs[GB_K][GB_N];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    v4d acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

    double ra[4], rb[4];
    // Thread -> tile element mapping for global loads.
    // "contiguous-in-row" pattern: k = tid/16, 4 consecutive m (or n) from (tid%16)*4.
    // "contiguous-in-k" pattern:   m (or n) = tid/4, 4 consecutive k from (tid%4)*4.
    auto load = [&](int k0) {
        if (!TA) {
            const int k = tid >> 4, m = (tid & 15) * 4;
            const int kk = k0 + k;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int mm = m0 + m + e;
                ra[e] = (kk < kend && mm < M) ? A[(long long)kk * lda + mm] : 0.0;
            }
        } else {
            const int m = tid >> 2, k = (tid & 3) * 4;
            const int mm = m0 + m;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kk = k0 + k + e;
                ra[e] = (kk < kend && mm < M) ? A[(long long)mm * lda + kk] : 0.0;
            }
        }
        if (!TB) {
            const int nn_ = tid >> 2, k = (tid & 3) * 4;
            const int nn = n0 + nn_;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kk = k0 + k + e;
                rb[e] = (kk < kend && nn < N) ? B[(long long)nn * ldb + kk] : 0.0;
            }
        } else {
            const int k = tid >> 4, nn_ = (tid & 15) * 4;
            const int kk = k0 + k;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int nn = n0 + nn_ + e;
                rb[e] = (kk < kend && nn < N) ? B[(long long)kk * ldb + nn] : 0.0;
            }
        }
    };
    auto store = [&]() {
        if (!TA) {
            const int k = tid >> 4, m = (tid & 15) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[k][m + e] = ra[e];
        } else {
            const int m = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[k + e][m] = ra[e];
        }
        if (!TB) {
            const int nn_ = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[k + e][nn_] = rb[e];
        } else {
            const int k = tid >> 4, nn_ = (tid & 15) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[k][nn_ + e] = rb[e];
        }
    };

    const int nk = (kend > kbeg) ? (kend - kbeg + GB_K - 1) / GB_K : 0;
    if (nk > 0) {
        load(kbeg);
        store();
        __syncthreads();
        const int lr = lane & 15, lk = lane >> 4;
        for (int it = 0; it < nk; ++it) {
            if (it + 1 < nk) load(kbeg + (it + 1) * GB_K);
#pragma unroll
            for (int ks = 0; ks < GB_K / 4; ++ks) {
                const int k = ks * 4 + lk;
                const double a0 = As[k][wm * 32 + lr];
                const double a1 = As[k][wm * 32 + 16 + lr];
                const double b0 = Bs[k][wn * 32 + lr];
                const double b1 = Bs[k][wn * 32 + 16 + lr];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
            __syncthreads();
            if (it + 1 < nk) {
                store();
                __syncthreads();
            }
        }
    }
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + bi * 16 + r * 4 + lq;
                const int col = n0 + wn * 32 + bj * 16 + lr;
                if (row < M && col < N) {
                    const long long ci = (long long)col * ldc + row;
                    double v = alpha * acc[bi][bj][r];
                    if (beta != 0.0) v += beta * C[ci];
                    C[ci] = v;
                }
            }
}

template <bool TA, bool TB, int KMODE, bool LOWER>
static void gemm_launch(hipStream_t st, int M, int N, int K, double alpha, const double* A, int lda,
                        long long sA, const double* B, int ldb, long long sB, double beta,
                        double* C, int ldc, long long sC, int batch)
{
    dim3 grid((M + GB_M - 1) / GB_M, (N + GB_N - 1) / GB_N, batch);
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, KMODE, LOWER>), grid, dim3(256), 0, st, M, N, K,
                       alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
}

void gemm_f64(hipStream_t st, bool ta, bool tb, int kmode, bool lower, int M, int N, int K,
              double alpha, const double* A, int lda, long long sA, const double* B, int ldb,
              long long sB, double beta, double* C, int ldc, long long sC, int batch)
{
    if (M <= 0 || N <= 0 || batch <= 0) return;
#define GEMM_CASE(TA_, TB_, KM_, LO_)                                                            \
    if (ta == TA_ && tb == TB_ && kmode == KM_ && lower == LO_) {                                 \
        gemm_launch<TA_, TB_, KM_, LO_>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, \
                                        sC, batch);                                              \
        return;                                                                                  \
    }
    GEMM_CASE(false, false, 0, false)
    GEMM_CASE(false, true, 0, false)
    GEMM_CASE(true, false, 0, false)
    GEMM_CASE(true, true, 0, false)
    GEMM_CASE(true, false, 0, true)
    GEMM_CASE(false, true, 0, true)
    GEMM_CASE(false, false, 1, false)
    GEMM_CASE(false, true, 2, false)
#undef GEMM_CASE
}

// ---------------------------------------------------------------------------
// Cholesky pieces.
// ---------------------------------------------------------------------------
__global__ void scale_diag_kernel(double* A, int lda, long long sA, int n, double factor)
{
    A += blockIdx.y * sA;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[(long long)i * lda + i] *= factor;
}

void scale_diag(hipStream_t st, double* A, int lda, long long sA, int n, double factor, int batch)
{
    dim3 grid((n + 255) / 256, batch);
    hipLaunchKernelGGL(scale_diag_kernel, grid, dim3(256), 0, st, A, lda, sA, n, factor);
}

// Value of v in lane k, broadcast to the whole wave (k uniform).
__device__ __forceinline__ double lane_bcast(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// 16x16 tile product on the matrix cores: acc += A * B, where the wave's lane
// l supplies A[l%16][4s + l/16] and B[4s + l/16][l%16] for s = 0..3 through
// the accessors; acc element r of lane l is C[4r + l/16][l%16].
template <class FA, class FB>
__device__ __forceinline__ v4d mfma16(v4d acc, FA fa, FB fb)
{
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(s4), fb(s4), acc, 0, 0, 0);
    return acc;
}

// Cholesky of the jb x jb (jb <= 64) diagonal block at (j, j) and the inverse
// of its factor, by one workgroup of four waves with the block in LDS (rows
// and columns beyond jb are identity).  The block is processed as four
// 16-wide column panels: wave 0 factors the 16 x 16 diagonal tile in
// registers (lane i holds row i; pivots and columns move between lanes by
// lane reads) together with its inverse; the panel below is multiplied by that
// inverse and the trailing tiles are updated with 16x16x4 FP64 MFMA tiles
// spread over the waves.  The full inverse X = L^{-1} is then assembled from
// the diagonal-tile inverses by diagonals:
//     X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj   (16 x 16 tiles, i > j).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* A, int lda, long long sA, int j,
                                                         int jb, double* Dinv, long long sD,
                                                         double* Linv, int ldl, long long sL,
                                                         DevInfo* info, int pass,
                                                         const double* dsave, long long sS,
                                                         double tau, double* rhs)
{
    __shared__ double T[64][65];
    __shared__ double Xs[64][65];
    __shared__ double tmp[4][16][17];
    __shared__ double fl[64];
    __shared__ int bad_any;
    const int z = blockIdx.x;
    A += z * sA;
    Dinv += z * sD;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    if (tid == 0) bad_any = 0;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int c = idx >> 6, r = idx & 63;   // column-major walk: coalesced loads
        double v = (r == c) ? 1.0 : 0.0;
        if (r < jb && c < jb && r >= c) v = A[(long long)(j + c) * lda + (j + r)];
        T[r][c] = v;
        Xs[r][c] = 0.0;
    }
    if (tid < 64) fl[tid] = (dsave && tid < jb) ? tau * dsave[z * sS + j + tid] : 0.0;
    __syncthreads();

    for (int sb = 0; sb < 4; ++sb) {
        const int s0 = 16 * sb;
        if (w == 0) {
            // factor the 16 x 16 diagonal tile: lane i (< 16) holds row i
            const int i = lane;
            double r[16], x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) r[c] = (i < 16 && c <= i) ? T[s0 + i][s0 + c] : 0.0;
            const double myfl = i < 16 ? fl[s0 + i] : 0.0;
            int bad = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                double d = lane_bcast(r[k], k);
                const double f = lane_bcast(myfl, k);
                if (!(d > f) || !isfinite(d)) {
                    bad = 1;
                    d = 1.0;
                }
                const double p = sqrt(d);
                const double rp = 1.0 / p;
                r[k] = (i == k) ? p : ((i > k) ? r[k] * rp : r[k]);
#pragma unroll
                for (int c = k + 1; c < 16; ++c) {
                    const double lck = lane_bcast(r[k], c);
                    if (i > k) r[c] -= r[k] * lck;
                }
            }
            // inverse of the tile: lane i holds row i of X
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = (c == i) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double rkk = 1.0 / lane_bcast(r[k], k);
#pragma unroll
                for (int c = 0; c <= k; ++c) {
                    if (i == k) x[c] *= rkk;
                    const double xk = lane_bcast(x[c], k);
                    if (i > k) x[c] -= r[k] * xk;
                }
            }
            if (i < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    if (c <= i) {
                        T[s0 + i][s0 + c] = r[c];
                        Xs[s0 + i][s0 + c] = x[c];
                    }
                }
            }
            if (bad && lane == 0) bad_any = 1;
        }
        __syncthreads();
        if (sb == 3) break;
        // panel: rows below, T[rt][s0 tile] = T[rt][s0 tile] * X_ss^T
        const int nrt = 3 - sb;
        if (w < nrt) {
            const int rt = s0 + 16 * (w + 1);
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            acc = mfma16(acc, [&](int s4) { return T[rt + lr][s0 + 4 * s4 + lq]; },
                         [&](int s4) { return Xs[s0 + lr][s0 + 4 * s4 + lq]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) T[rt + 4 * r + lq][s0 + lr] = acc[r];
        }
        __syncthreads();
        // trailing: T[ti][tj] -= P_ti P_tj^T for tiles below the panel, ti >= tj
        int pairs[6][2];
        int np = 0;
        for (int a = 1; a <= nrt; ++a)
            for (int b = 1; b <= a; ++b) {
                pairs[np][0] = s0 + 16 * a;
                pairs[np][1] = s0 + 16 * b;
                ++np;
            }
        for (int pi = w; pi < np; pi += 4) {
            const int ti = pairs[pi][0], tj = pairs[pi][1];
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            acc = mfma16(acc, [&](int s4) { return T[ti + lr][s0 + 4 * s4 + lq]; },
                         [&](int s4) { return T[tj + lr][s0 + 4 * s4 + lq]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) T[ti + 4 * r + lq][tj + lr] -= acc[r];
        }
        __syncthreads();
    }

    // full inverse by diagonals of 16 x 16 tiles
    for (int d = 1; d < 4; ++d) {
        const int bi = d + w, bj = w;   // waves 0 .. 3-d handle tile (bi, bj)
        const bool act = (w < 4 - d);
        if (act) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            for (int kb = bj; kb < bi; ++kb)
                acc = mfma16(acc, [&](int s4) { return T[16 * bi + lr][16 * kb + 4 * s4 + lq]; },
                             [&](int s4) { return Xs[16 * kb + 4 * s4 + lq][16 * bj + lr]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) tmp[w][4 * r + lq][lr] = acc[r];
        }
        __syncthreads();
        if (act) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            acc = mfma16(acc, [&](int s4) { return Xs[16 * bi + lr][16 * bi + 4 * s4 + lq]; },
                         [&](int s4) { return tmp[w][4 * s4 + lq][lr]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) Xs[16 * bi + 4 * r + lq][16 * bj + lr] = -acc[r];
        }
        __syncthreads();
    }

    if (rhs) {
        // forward substitution for this block: y_J = L_JJ^{-1} r_J
        if (tid < 64) fl[tid] = tid < jb ? rhs[j + tid] : 0.0;   // fl is free by now
        __syncthreads();
        if (tid < jb) {
            double acc = 0.0;
            for (int c = 0; c <= tid; ++c) acc += Xs[tid][c] * fl[c];
            rhs[j + tid] = acc;
        }
    }
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int c = idx >> 6, r = idx & 63;
        const bool in = (r < jb) && (c < jb);
        const double xv = (in && c <= r) ? Xs[r][c] : 0.0;
        Dinv[c * 64 + r] = xv;
        if (in && c <= r) A[(long long)(j + c) * lda + (j + r)] = T[r][c];
        if (Linv && in) Linv[z * sL + (long long)(j + c) * ldl + (j + r)] = xv;
    }
    __syncthreads();
    if (tid == 0 && bad_any && info) {
        if (pass <= 3) {
            atomicMin(&info->bad_subdomain, z);
            atomicMax(&info->bad_pass, pass);
            atomicCAS(&info->status, 0, 3);   // ELMDDM_NOT_SPD
        } else {
            atomicCAS(&info->status, 0, 4);   // ELMDDM_SCHUR_NOT_SPD
        }
    }
}

void potrf_diag(hipStream_t st, double* A, int lda, long long sA, int j, int jb, double* Dinv,
                long long sD, double* Linv, int ldl, long long sL, DevInfo* info, int pass,
                int batch, const double* dsave, long long sS, double tau, double* rhs)
{
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(batch), dim3(256), 0, st, A, lda, sA, j, jb, Dinv,
                       sD, Linv, ldl, sL, info, pass, dsave, sS, tau, rhs);
}

// r_I -= L_{I,J} y_J for the rows I = [r0, r1) below a factored panel J = [j, j + jb).
__global__ void rhs_update_kernel(const double* L, int ld, int j, int jb, int r0, int r1, double* r)
{
    __shared__ double yj[64];
    if (threadIdx.x < 64) yj[threadIdx.x] = threadIdx.x < jb ? r[j + threadIdx.x] : 0.0;
    __syncthreads();
    const int row = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= r1) return;
    double acc = 0.0;
    for (int c = 0; c < jb; ++c) acc += L[(long long)(j + c) * ld + row] * yj[c];
    r[row] -= acc;
}

void rhs_update(hipStream_t st, const double* L, int ld, int j, int jb, int r0, int r1, double* r)
{
    if (r1 <= r0) return;
    hipLaunchKernelGGL(rhs_update_kernel, dim3((r1 - r0 + 255) / 256), dim3(256), 0, st, L, ld, j, jb,
                       r0, r1, r);
}

__global__ void save_diag_kernel(const double* A, int lda, long long sA, int n, double* d,
                                 long long sS)
{
    const long long z = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[z * sS + i] = A[z * sA + (long long)i * lda + i];
}

void save_diag(hipStream_t st, const double* A, int lda, long long sA, int n, double* d,
               long long sS, int batch)
{
    dim3 grid((n + 255) / 256, batch);
    hipLaunchKernelGGL(save_diag_kernel, grid, dim3(256), 0, st, A, lda, sA, n, d, sS);
}

__global__ void copy_row_kernel(const double* src, int lsrc, long long sS, double* dst, int ldd,
                                long long sD, int count)
{
    const long long z = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[z * sD + (long long)i * ldd] = src[z * sS + (long long)i * lsrc];
}

void copy_row(hipStream_t st, const double* src, int lsrc, long long sS, double* dst, int ldd,
              long long sD, int count, int batch)
{
    dim3 grid((count + 255) / 256, batch);
    hipLaunchKernelGGL(copy_row_kernel, grid, dim3(256), 0, st, src, lsrc, sS, dst, ldd, sD, count);
}

// ---------------------------------------------------------------------------
// Interface Schur complement assembly (eq. schur in per-subdomain form).
// Per subdomain the product P_s holds T_s = Y^T Y (rows/cols < kpad),
// q_s = Y^T h (column kpad), C_s = Z^T Y (rows from cbase) and a_s = Z^T h.
// M, the flux rows of A K^+ P, is stored as dense mg x mg blocks M_{g,E}
// (rows: flux points of edge g, columns: unknowns of edge E).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void schur_mblocks_kernel(const int32_t* desc, const double* P,
                                                            int ldp, long long sP, int cbase,
                                                            int mg, double* Mbuf)
{
    const int blk = blockIdx.x;
    const int32_t* d = desc + 8 * blk;
    double* out = Mbuf + (long long)blk * mg * mg;
    for (int idx = threadIdx.x; idx < mg * mg; idx += blockDim.x) {
        const int r = idx % mg, c = idx / mg;
        double v = 0.0;
        for (int t = 0; t < 2; ++t) {
            const int s = d[3 * t];
            if (s < 0) continue;
            const int ro = d[3 * t + 1], co = d[3 * t + 2];
            v += P[s * sP + (long long)(co + c) * ldp + (cbase + ro + r)];
        }
        out[idx] = v;
    }
}

void schur_mblocks(hipStream_t st, int nblk, const int32_t* desc, const double* P, int ldp,
                   long long sP, int cbase, int mg, double* Mbuf)
{
    if (nblk <= 0) return;
    hipLaunchKernelGGL(schur_mblocks_kernel, dim3(nblk), dim3(256), 0, st, desc, P, ldp, sP, cbase,
                       mg, Mbuf);
}

__global__ void schur_avec_kernel(const int32_t* desc, const double* P, int ldp, long long sP,
                                  int cbase, int acol, int mg, double* abuf)
{
    const int e = blockIdx.x;
    const int32_t* d = desc + 4 * e;
    for (int r = threadIdx.x; r < mg; r += blockDim.x) {
        double v = 0.0;
        for (int t = 0; t < 2; ++t) {
            const int s = d[2 * t];
            if (s < 0) continue;
            v += P[s * sP + (long long)acol * ldp + (cbase + d[2 * t + 1] + r)];
        }
        abuf[(long long)e * mg + r] = v;
    }
}

void schur_avec(hipStream_t st, int nE, const int32_t* desc, const double* P, int ldp, long long sP,
                int cbase, int acol, int mg, double* abuf)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(schur_avec_kernel, dim3(nE), dim3(64), 0, st, desc, P, ldp, sP, cbase, acol,
                       mg, abuf);
}

// One workgroup per mg x mg block (E1, E2) of S:
//   S_{E1,E2} = sum_s [delta_{E1E2} I - T_s(E1, E2)] + sum_g M_{g,E1}^T M_{g,E2}.
// Terms are listed per block in a fixed order, so the sum is deterministic.
__global__ __launch_bounds__(256) void schur_sblocks_kernel(int nE, int mg, const int32_t* tptr,
                                                            const int32_t* tdesc,
                                                            const int32_t* mptr,
                                                            const int32_t* mdesc, const double* P,
                                                            int ldp, long long sP,
                                                            const double* Mbuf, double* S, int lds,
                                                            const int32_t* perm)
{
    __shared__ double M1[64 * 64];
    __shared__ double M2[64 * 64];
    const int E1 = blockIdx.x, E2 = blockIdx.y;
    const int blk = E1 + E2 * nE;
    const int mm = mg * mg;
    const int tid = threadIdx.x;
    double acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.0;
    for (int it = tptr[blk]; it < tptr[blk + 1]; ++it) {
        const int32_t* d = tdesc + 4 * it;
        const int s = d[0], o1 = d[1], o2 = d[2], dg = d[3];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t;
            if (idx < mm) {
                const int r = idx % mg, c = idx / mg;
                double v = -P[s * sP + (long long)(o2 + c) * ldp + (o1 + r)];
                if (dg && r == c) v += 1.0;
                acc[t] += v;
            }
        }
    }
    for (int it = mptr[blk]; it < mptr[blk + 1]; ++it) {
        const double* A1 = Mbuf + (long long)mdesc[2 * it] * mm;
        const double* A2 = Mbuf + (long long)mdesc[2 * it + 1] * mm;
        __syncthreads();
        for (int idx = tid; idx < mm; idx += 256) {
            M1[idx] = A1[idx];
            M2[idx] = A2[idx];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t;
            if (idx < mm) {
                const int r = idx % mg, c = idx / mg;
                double v = 0.0;
                for (int p = 0; p < mg; ++p) v += M1[r * mg + p] * M2[c * mg + p];
                acc[t] += v;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        if (idx < mm) {
            const int r = idx % mg, c = idx / mg;
            S[(long long)(perm[E2] * mg + c) * lds + (perm[E1] * mg + r)] = acc[t];
        }
    }
}

void schur_sblocks(hipStream_t st, int nE, int mg, const int32_t* tptr, const int32_t* tdesc,
                   const int32_t* mptr, const int32_t* mdesc, const double* P, int ldp,
                   long long sP, const double* Mbuf, double* S, int lds, const int32_t* perm)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(schur_sblocks_kernel, dim3(nE, nE), dim3(256), 0, st, nE, mg, tptr, tdesc,
                       mptr, mdesc, P, ldp, sP, Mbuf, S, lds, perm);
}

// rhs_E = sum_s q_s(E) - sum_g M_{g,E}^T a_g.
__global__ void schur_rhs_kernel(int mg, const int32_t* qdesc, const int32_t* gptr,
                                 const int32_t* gdesc, const double* P, int ldp, long long sP,
                                 int qcol, const double* Mbuf, const double* abuf, double* rhs,
                                 int inc, const int32_t* perm)
{
    const int E = blockIdx.x;
    const int mm = mg * mg;
    const int32_t* q = qdesc + 4 * E;
    for (int r = threadIdx.x; r < mg; r += blockDim.x) {
        double v = 0.0;
        for (int t = 0; t < 2; ++t) {
            const int s = q[2 * t];
            if (s < 0) continue;
            v += P[s * sP + (long long)qcol * ldp + (q[2 * t + 1] + r)];
        }
        for (int it = gptr[E]; it < gptr[E + 1]; ++it) {
            const double* Mb = Mbuf + (long long)gdesc[2 * it] * mm;
            const double* ag = abuf + (long long)gdesc[2 * it + 1] * mg;
            double acc = 0.0;
            for (int p = 0; p < mg; ++p) acc += Mb[r * mg + p] * ag[p];
            v -= acc;
        }
        rhs[(long long)(perm[E] * mg + r) * inc] = v;
    }
}

void schur_rhs(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr,
               const int32_t* gdesc, const double* P, int ldp, long long sP, int qcol,
               const double* Mbuf, const double* abuf, double* rhs, int inc, const int32_t* perm)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(schur_rhs_kernel, dim3(nE), dim3(64), 0, st, mg, qdesc, gptr, gdesc, P, ldp,
                       sP, qcol, Mbuf, abuf, rhs, inc, perm);
}

// ---------------------------------------------------------------------------
// One block step of the backward solve L^T u = y (L lower, blocked by 64):
// u_J = Dinv_J^T y_J, then y_K -= L_{J,K}^T u_J for every K < J.  Every
// workgroup recomputes u_J from the unchanged y_J, so the launch needs no
// inter-workgroup ordering.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trsv_lt_step_kernel(const double* L, int ld, int j0, int jb,
                                                           int kbeg, const double* Dinv, double* y,
                                                           double* u)
{
    __shared__ double yj[64], uj[64];
    const int tid = threadIdx.x;
    if (tid < 64) yj[tid] = tid < jb ? y[j0 + tid] : 0.0;
    __syncthreads();
    if (tid < 64) {
        double s = 0.0;
        for (int i = tid; i < jb; ++i) s += Dinv[tid * 64 + i] * yj[i];
        uj[tid] = s;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < jb) u[j0 + tid] = uj[tid];
    // one wave per column K < j0: lanes run over the 64 rows of block row J
    const int lane = tid & 63;
    const int wave = blockIdx.x * 4 + (tid >> 6);
    const int nwave = gridDim.x * 4;
    const double ul = lane < jb ? uj[lane] : 0.0;
    for (int kcol = kbeg + wave; kcol < j0; kcol += nwave) {
        double v = lane < jb ? L[(long long)kcol * ld + j0 + lane] * ul : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) y[kcol] -= v;
    }
}

void trsv_lower_t_step(hipStream_t st, const double* L, int ld, int j0, int jb, int kbeg,
                       const double* Dinv, double* y, double* u)
{
    int nb = (j0 - kbeg + 15) / 16;   // about 4 columns per wave
    nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
    hipLaunchKernelGGL(trsv_lt_step_kernel, dim3(nb), dim3(256), 0, st, L, ld, j0, jb, kbeg, Dinv, y,
                       u);
}

// ---------------------------------------------------------------------------
// Local back-solve (Algorithm 1, last loop): c = R^{-1} (h + Q_Gamma^T u_s)
// with R^{-1} = Linv1^T Linv2^T Linv3^T from the three CholeskyQR passes.
// One wave per output entry, lanes along the contiguous column: coalesced.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// v[s][col] = h_s[col] + sum_i Q_Gamma[i][col] u[gidx_s[i]]
__global__ __launch_bounds__(256) void bs_rhs_kernel(int n, int kpad, const double* X, int ldx,
                                                     long long sX, int mI, int hrow,
                                                     const int32_t* gidx, const double* u,
                                                     double* v)
{
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= n) return;
    const double* xc = X + s * sX + (long long)col * ldx;
    double acc = 0.0;
    for (int i = lane; i < kpad; i += 64) {
        const int gi = gidx[s * kpad + i];
        if (gi >= 0) acc += xc[mI + i] * u[gi];
    }
    acc = wave_sum(acc);
    if (lane == 0) v[(long long)s * n + col] = acc + xc[hrow];
}

// out[s][i] = sum_{k >= i} Li[s][k + i*ldg] in[s][k]   (Linv^T times a vector)
__global__ __launch_bounds__(256) void trmv_t_kernel(int n, const double* Li, int ldg, long long sG,
                                                     const double* in, double* out)
{
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double* colp = Li + s * sG + (long long)i * ldg;
    const double* vin = in + (long long)s * n;
    double acc = 0.0;
    for (int k = i + lane; k < n; k += 64) acc += colp[k] * vin[k];
    acc = wave_sum(acc);
    if (lane == 0) out[(long long)s * n + i] = acc;
}

void local_backsolve(hipStream_t st, int N, int n, int kpad, const double* X, int ldx, long long sX,
                     int mI, int hrow, const int32_t* gidx, const double* u, const double* Linv1,
                     const double* Linv2, const double* Linv3, int ldg, long long sG, double* c,
                     double* tmp1, double* tmp2)
{
    dim3 grid((n + 3) / 4, N);
    hipLaunchKernelGGL(bs_rhs_kernel, grid, dim3(256), 0, st, n, kpad, X, ldx, sX, mI, hrow, gidx, u,
                       tmp1);
    hipLaunchKernelGGL(trmv_t_kernel, grid, dim3(256), 0, st, n, Linv3, ldg, sG, tmp1, tmp2);
    hipLaunchKernelGGL(trmv_t_kernel, grid, dim3(256), 0, st, n, Linv2, ldg, sG, tmp2, tmp1);
    hipLaunchKernelGGL(trmv_t_kernel, grid, dim3(256), 0, st, n, Linv1, ldg, sG, tmp1, c);
}

// u[E*mg + r] = up[perm[E]*mg + r]
__global__ void unpermute_kernel(int nE, int mg, const int32_t* perm, const double* up, double* u)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nE * mg) return;
    const int E = idx / mg, r = idx % mg;
    u[idx] = up[(long long)perm[E] * mg + r];
}

void unpermute(hipStream_t st, int nE, int mg, const int32_t* perm, const double* up, double* u)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(unpermute_kernel, dim3((nE * mg + 255) / 256), dim3(256), 0, st, nE, mg, perm,
                       up, u);
}

// Dense S in the original interface order from the permuted copy (ld lds).
__global__ void unpermute_matrix_kernel(int nE, int mg, const int32_t* perm, const double* Sp, int lds,
                                        double* S)
{
    const long long n = (long long)nE * mg;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int row = (int)(idx % n), col = (int)(idx / n);
    const int pr = perm[row / mg] * mg + row % mg, pc = perm[col / mg] * mg + col % mg;
    S[idx] = Sp[(long long)pc * lds + pr];
}

void unpermute_matrix(hipStream_t st, int nE, int mg, const int32_t* perm, const double* Sp, int lds,
                      double* S)
{
    const long long n = (long long)nE * mg;
    if (n <= 0) return;
    hipLaunchKernelGGL(unpermute_matrix_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st,
                       nE, mg, perm, Sp, lds, S);
}

// ---------------------------------------------------------------------------
// u_h at arbitrary points by the network of the owning box.
// ---------------------------------------------------------------------------
__global__ void eval_kernel(int npts, const double* xy, int nx, int ny, double x0, double x1,
                            double y0, double y1, int n, const double* W, const double* b,
                            const double* c, double* u)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const double x = xy[2 * p], y = xy[2 * p + 1];
    const double hx = (x1 - x0) / nx, hy = (y1 - y0) / ny;
    int sx = (int)floor((x - x0) * nx / (x1 - x0));
    int sy = (int)floor((y - y0) * ny / (y1 - y0));
    sx = sx < 0 ? 0 : (sx > nx - 1 ? nx - 1 : sx);
    sy = sy < 0 ? 0 : (sy > ny - 1 ? ny - 1 : sy);
    const int s = sy * nx + sx;
    const double xc = (x0 + sx * hx) + 0.5 * hx;
    const double yc = (y0 + sy * hy) + 0.5 * hy;
    const double xh = (x - xc) * (2.0 / hx);
    const double yh = (y - yc) * (2.0 / hy);
    const double* Ws = W + (long long)s * n * 2;
    const double* bs = b + (long long)s * n;
    const double* cs = c + (long long)s * n;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += cs[j] * tanh(Ws[2 * j] * xh + Ws[2 * j + 1] * yh + bs[j]);
    u[p] = acc;
}

void eval_points(hipStream_t st, int npts, const double* xy, int nx, int ny, double x0, double x1,
                 double y0, double y1, int n, const double* W, const double* b, const double* c,
                 double* u)
{
    if (npts <= 0) return;
    hipLaunchKernelGGL(eval_kernel, dim3((npts + 255) / 256), dim3(256), 0, st, npts, xy, nx, ny,
                       x0, x1, y0, y1, n, W, b, c, u);
}

__global__ void init_info_kernel(DevInfo* info)
{
    info->status = 0;
    info->bad_subdomain = 0x7fffffff;
    info->bad_pass = 0;
    info->pad = 0;
}

void init_info(hipStream_t st, DevInfo* info)
{
    hipLaunchKernelGGL(init_info_kernel, dim3(1), dim3(1), 0, st, info);
}

__global__ void check_finite_kernel(const double* v, long long count, DevInfo* info)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && !isfinite(v[i])) atomicCAS(&info->status, 0, 6);  // ELMDDM_NONFINITE
}

void check_finite(hipStream_t st, const double* v, long long count, DevInfo* info)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       v, count, info);
}

}  // namespace elmddm
