// HIP kernels for gfx950 (MI355X): feature assembly, batched FP64 MFMA GEMM,
// blocked Cholesky pieces, interface Schur assembly, triangular solves and
// evaluation.  Column-major storage throughout.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "internal.h"

namespace elmddm {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// tanh in FP64 through the identity tanh|z| = -expm1(-2|z|) / (2 + expm1(-2|z|)),
// sign restored: one expm1 and one division, accurate to full relative
// precision for small |z| as well (measured on the device: within 3.7e-16
// relative of the library tanh over [-20, 20], about three times faster).
__device__ __forceinline__ double tanh_feat(double z)
{
    const double e = expm1(-2.0 * fabs(z));
    return copysign(-e / (2.0 + e), z);
}


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
    long long sK, double* __restrict__ Dout, int ldD, long long sD, int ngeo, int q2, long long nbnd)
{
    const int s = blockIdx.z;            // subdomain of the whole batch
    const int sg = s % ngeo;             // its geometry
    const long long inst = s / ngeo;     // its problem instance
    const int r = blockIdx.x * 64 + (threadIdx.x & 63);
    const int cg = threadIdx.x >> 6;
    const int c0 = blockIdx.y * 64;
    // hidden-layer parameters of this block's 64 columns, read once into LDS
    // (a load per column inside the loop below would wait on memory each time)
    __shared__ double wsh[3][64];
    if (threadIdx.x < 64) {
        const int col = c0 + threadIdx.x;
        if (col < n) {
            const long long wi = (long long)s * n + col;
            wsh[0][threadIdx.x] = W[2 * wi];
            wsh[1][threadIdx.x] = W[2 * wi + 1];
            wsh[2][threadIdx.x] = bias[wi];
        }
    }
    __syncthreads();
    if (r >= ldx) return;
    const long long ri = (long long)sg * ldx + r;
    const int kind = rows.kind[ri];
    // data index: interior rows -> s * q2 + i, boundary rows -> instance * nbnd + global index
    const long long src = kind == ROW_INTERIOR ? rows.src[ri] + inst * ngeo * (long long)q2
                                               : rows.src[ri] + inst * nbnd;
    const double xh = (rows.x[ri] - geom.cx[sg]) * geom.sx;
    const double yh = (rows.y[ri] - geom.cy[sg]) * geom.sy;
    const double nxv = rows.nx[ri], nyv = rows.ny[ri];
    double a = 1.0, ax = 0.0, ay = 0.0;
    if (op == 1 && kind == ROW_INTERIOR) {
        a = coef[src];
        ax = coef[coef_stride + src];
        ay = coef[2 * coef_stride + src];
    }
    const int crow = compact ? rows.cmap[ri] : -1;
    for (int cc = cg; cc < 64; cc += 4) {
        const int col = c0 + cc;
        if (col > n) break;
        double v = 0.0;
        if (col == n) {
            if (kind == ROW_INTERIOR) v = f[src];
            else if (kind == ROW_BOUNDARY) v = g[src];
        } else if (kind != ROW_ZERO) {
            const double w0 = wsh[0][cc], w1 = wsh[1][cc];
            const double wx = w0 * geom.sx;
            const double wy = w1 * geom.sy;
            const double z = w0 * xh + w1 * yh + wsh[2][cc];
            const double t = tanh_feat(z);
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

void assemble(hipStream_t st, int N, int ngeo, long long nbnd, int ldx, int n, const RowTable& rows,
              const SubGeom& geom, int op, const double* W, const double* b, const double* f,
              const double* g, const double* coef, int q2, double* X, double* Fout, int ldF,
              double* Kout, int ldK, double* Dout, int ldD)
{
    dim3 grid((ldx + 63) / 64, (n + 1 + 63) / 64, N);
    const bool compact = (Kout != nullptr);
    hipLaunchKernelGGL(assemble_kernel, grid, dim3(256), 0, st, ldx, n, rows, geom, op, W, b, f, g,
                       coef, (long long)N * q2, X, (long long)ldx * (n + 1), compact, Fout, ldF,
                       Kout, ldK, (long long)ldK * n, Dout, ldD, (long long)ldD * n, ngeo, q2, nbnd);
}

// ---------------------------------------------------------------------------
// Batched GEMM on the matrix cores: C = alpha op(A) op(B) + beta C, FP64
// operands and result, computed in FP64 (CT = float rounds the staged
// operands to FP32 and accumulates in FP32; the mixed-precision Gram has a
// kernel of its own, gram_f32_kernel).
// Workgroup tile 64x64, K staged 16 (double-buffered) or 32 at a time
// through LDS, four waves in a 2x2 arrangement, each wave a 32x32 block of
// 2x2 V_MFMA_F64_16X16X4 tiles.
// MFMA operand layout (16x16x4, f64): lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the accumulator's element r of lane l is D[4*r + l/16][l%16].
// Global loads move GB_K / 4 consecutive doubles per thread (16-byte vector
// loads when aligned and in bounds); a K stage is fetched into registers two
// stages (K depth 16) or one stage (K depth 32) before it is stored to LDS,
// while the stages in between compute.  Workgroups are renumbered so that each
// XCD (the hardware deals workgroups to the 8 XCDs in turn) receives a
// contiguous run of tiles, i.e. whole matrices of the batch, and their
// operands stay in that XCD's L2.
// ---------------------------------------------------------------------------
#define GB_M 64
#define GB_N 64

__device__ __forceinline__ bool aligned16(const double* p)
{
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Compute type CT: double (V_MFMA_F64_16X16X4) or float (V_MFMA_F32_16X16X4,
// FP32 accumulation; operands rounded to FP32 when they are staged in LDS,
// result widened to FP64 on store).  The FP32 accumulator's element r of lane
// l is D[4*(l/16) + r][l%16].  LDS rows are padded so that the four k rows a
// wave reads at once fall in different banks (for FP64: the two 16-lane
// groups of each half-wave).
template <class CT, bool TA, bool TB, int KMODE, bool LOWER, int GB_K, bool XCD, bool CPRE = false>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(
    int M, int N, int K, double alpha, const double* A, int lda, long long sA, const double* B,
    int ldb, long long sB, double beta, double* C, int ldc, long long sC)
{
    constexpr bool F64 = sizeof(CT) == 8;
    constexpr int PAD = 16;
    typedef CT acc_t __attribute__((ext_vector_type(4)));
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned total = gx * gy * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = (!XCD || (total & 7u)) ? p : (p & 7u) * (total >> 3) + (p >> 3);
    int tm, tn;
    long long z;
    if (LOWER && M == N) {
        // triangular launch: gx = g (g + 1) / 2 lower tiles per matrix, column by column
        z = q / gx;
        int t = q % gx;
        const int g = (GB_M + M - 1) / GB_M;
        tn = 0;
        while (t >= g - tn) {
            t -= g - tn;
            ++tn;
        }
        tm = tn + t;
    } else {
        tm = q % gx;
        tn = (q / gx) % gy;
        z = q / (gx * gy);
        if (LOWER && tm < tn) return;
    }
    A += z * sA;
    B += z * sB;
    C += z * sC;
    const int m0 = tm * GB_M, n0 = tn * GB_N;
    int kbeg = 0, kend = K;
    if (KMODE == 1) kbeg = n0 < K ? n0 : K;
    if (KMODE == 2) kend = (n0 + GB_N) < K ? (n0 + GB_N) : K;

    // An operand that is loaded along k (A with TA, B without TB) is staged
    // k-contiguous per row: stores are contiguous and the MFMA reads of the 16
    // rows x 2 k of a half-wave fall in distinct banks (row stride GB_K + 2
    // doubles or GB_K + 4 floats); the other layout is k-major with padded rows.
    constexpr bool AK = TA, BK = !TB;
    constexpr int SK = GB_K + (F64 ? 2 : 4);
    constexpr int SM = GB_M + PAD;
    // K depth 16: two LDS buffers, the next stage is stored into the other
    // one while this one is read, one barrier per stage.  K depth 32: one
    // buffer (two of them would halve the workgroups per CU).
    constexpr int NBUF = GB_K == 16 ? 2 : 1;
    __shared__ __attribute__((aligned(16))) CT As_[NBUF][AK ? GB_M * SK : GB_K * SM];
    __shared__ __attribute__((aligned(16))) CT Bs_[NBUF][BK ? GB_N * SK : GB_K * SM];
    auto As = [&](int b, int k, int m) -> CT& { return AK ? As_[b][m * SK + k] : As_[b][k * SM + m]; };
    auto Bs = [&](int b, int k, int nn) -> CT& { return BK ? Bs_[b][nn * SK + k] : Bs_[b][k * SM + nn]; };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = (acc_t){0, 0, 0, 0};

    // Per thread and stage: V = GB_K / 4 consecutive doubles of A and of B.
    // "along-row": k = tid / (64 / V), V consecutive m (or n) from (tid % (64/V)) * V.
    // "along-k":   m (or n) = tid / 4, V consecutive k from (tid % 4) * V.
    constexpr int V = GB_K / 4;
    constexpr int RS = 64 / V;   // threads per k row in the along-row pattern
    // K depth 16: two register sets, so that a stage is fetched two stages
    // before it is stored to LDS (the LDS size, not the registers, bounds the
    // occupancy of this variant); K depth 32: one set.
    double ra[V], rb[V], ra2[V], rb2[V];
    auto loadv = [&](double (&r)[V], const double* p, bool all, auto ok) {
        if (all && aligned16(p)) {
            const double2* q2 = reinterpret_cast<const double2*>(p);
#pragma unroll
            for (int e = 0; e < V / 2; ++e) {
                const double2 v = q2[e];
                r[2 * e] = v.x;
                r[2 * e + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r[e] = ok(e) ? p[e] : 0.0;
        }
    };
    auto load = [&](double (&xa)[V], double (&xb)[V], int k0) {
        if (!TA) {
            const int kk = k0 + tid / RS, mm = m0 + (tid % RS) * V;
            const double* pa = A + (long long)kk * lda + mm;
            loadv(xa, pa, kk < kend && mm + V - 1 < M, [&](int e) { return kk < kend && mm + e < M; });
        } else {
            const int mm = m0 + (tid >> 2), kk = k0 + (tid & 3) * V;
            const double* pa = A + (long long)mm * lda + kk;
            loadv(xa, pa, mm < M && kk + V - 1 < kend, [&](int e) { return mm < M && kk + e < kend; });
        }
        if (!TB) {
            const int nn = n0 + (tid >> 2), kk = k0 + (tid & 3) * V;
            const double* pb = B + (long long)nn * ldb + kk;
            loadv(xb, pb, nn < N && kk + V - 1 < kend, [&](int e) { return nn < N && kk + e < kend; });
        } else {
            const int kk = k0 + tid / RS, nn = n0 + (tid % RS) * V;
            const double* pb = B + (long long)kk * ldb + nn;
            loadv(xb, pb, kk < kend && nn + V - 1 < N, [&](int e) { return kk < kend && nn + e < N; });
        }
    };
    auto store = [&](int b, const double (&xa)[V], const double (&xb)[V]) {
        if (!TA) {
            const int k = tid / RS, m = (tid % RS) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) As(b, k, m + e) = (CT)xa[e];
        } else {
            const int m = tid >> 2, k = (tid & 3) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) As(b, k + e, m) = (CT)xa[e];
        }
        if (!TB) {
            const int nn = tid >> 2, k = (tid & 3) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) Bs(b, k + e, nn) = (CT)xb[e];
        } else {
            const int k = tid / RS, nn = (tid % RS) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) Bs(b, k, nn + e) = (CT)xb[e];
        }
    };

    // 16 x 16 blocks of this wave that carry work: bit 2u + v for block (u, v).
    // Blocks outside M x N, and in lower mode blocks strictly above the
    // diagonal, are skipped; with KMODE 1/2 a block also drops out of the K
    // stages where op(B) is zero for its columns.  (One code path with a
    // scalar test per instruction measured 10% faster than a switch over the
    // 15 masks with a branch-free sequence each.)
    const int lr = lane & 15, lk = lane >> 4;
    int wmask = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int R0 = m0 + wm * 32 + u * 16, C0 = n0 + wn * 32 + v * 16;
            if (R0 < M && C0 < N && (!LOWER || R0 + 15 >= C0)) wmask |= 1 << (2 * u + v);
        }
    auto mma = [](CT a, CT b, acc_t c) {
        if constexpr (F64) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    };
    // One K stage from LDS buffer b for the 16 x 16 blocks in mask mk (a
    // wave-uniform value, so the tests are scalar branches).  The instruction
    // multiplies op(B)^T op(A)^T: its result is the transposed C block, so
    // that a lane's accumulator runs along a column of C (see the store below).
    auto stage = [&](int mk, int b) {
#pragma unroll
        for (int ks = 0; ks < GB_K / 4; ++ks) {
            const int k = ks * 4 + lk;
            const CT a0 = As(b, k, wm * 32 + lr), a1 = As(b, k, wm * 32 + 16 + lr);
            const CT b0 = Bs(b, k, wn * 32 + lr), b1 = Bs(b, k, wn * 32 + 16 + lr);
            if (mk & 1) acc[0][0] = mma(b0, a0, acc[0][0]);
            if (mk & 2) acc[0][1] = mma(b1, a0, acc[0][1]);
            if (mk & 4) acc[1][0] = mma(b0, a1, acc[1][0]);
            if (mk & 8) acc[1][1] = mma(b1, a1, acc[1][1]);
        }
    };
    // acc[bi][bj] holds the transposed 16 x 16 block: C row = lane % 16, so
    // the 16 lanes of a quarter-wave read and write one contiguous 128-byte
    // column segment of C.  With CPRE (chosen by the launcher when beta != 0)
    // the C values are fetched before the K loop, so that their latency hides
    // behind it (short-K updates); the beta = 0 instances keep the registers.
    const int lq = lane >> 4;
    auto crow = [&](int bi) { return m0 + wm * 32 + bi * 16 + lr; };
    auto ccol = [&](int bj, int r) { return n0 + wn * 32 + bj * 16 + (F64 ? r * 4 + lq : lq * 4 + r); };
    double cpre[2][2][4];
    if constexpr (CPRE) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = crow(bi), col = ccol(bj, r);
                    cpre[bi][bj][r] = ((wmask & (1 << (2 * bi + bj))) && row < M && col < N)
                                          ? C[(long long)col * ldc + row]
                                          : 0.0;
                }
    }
    const int nk = (kend > kbeg) ? (kend - kbeg + GB_K - 1) / GB_K : 0;
    auto live = [&](int k0) {   // blocks with work in the K stage starting at k0
        int mk = wmask;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int C0 = n0 + wn * 32 + v * 16;
            const bool dead = (KMODE == 2 && k0 >= C0 + 16) || (KMODE == 1 && k0 + GB_K <= C0);
            if (dead) mk &= ~((1 << v) | (1 << (2 + v)));
        }
        return mk;
    };
    if constexpr (NBUF == 2) {
        // Stage it is computed from LDS buffer it % 2.  Register set it % 2
        // receives stage it + 2 at the start of step it (it held stage it,
        // stored in step it - 1), and the other set, holding stage it + 1
        // since step it - 1, is stored into buffer (it + 1) % 2 after the
        // compute (that buffer was last read in step it - 1, which every wave
        // finished before the barrier that ended it).
        auto step = [&](int it, auto par) {
            constexpr bool odd = decltype(par)::value != 0;
            const int k0 = kbeg + it * GB_K;
            if (it + 2 < nk) {
                if constexpr (odd) load(ra2, rb2, k0 + 2 * GB_K);
                else load(ra, rb, k0 + 2 * GB_K);
            }
            const int mk = live(k0);
            if (mk) stage(mk, odd ? 1 : 0);
            if (it + 1 < nk) {
                if constexpr (odd) store(0, ra, rb);
                else store(1, ra2, rb2);
            }
            __syncthreads();
        };
        if (nk > 0) {
            load(ra, rb, kbeg);
            store(0, ra, rb);
            if (nk > 1) load(ra2, rb2, kbeg + GB_K);
            __syncthreads();
            for (int it = 0; it < nk; it += 2) {
                step(it, std::integral_constant<int, 0>{});
                if (it + 1 < nk) step(it + 1, std::integral_constant<int, 1>{});
            }
        }
    } else if (nk > 0) {
        load(ra, rb, kbeg);
        store(0, ra, rb);
        __syncthreads();
        for (int it = 0; it < nk; ++it) {
            const int k0 = kbeg + it * GB_K;
            if (it + 1 < nk) load(ra, rb, k0 + GB_K);
            const int mk = live(k0);
            if (mk) stage(mk, 0);
            __syncthreads();
            if (it + 1 < nk) {
                store(0, ra, rb);
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!(wmask & (1 << (2 * bi + bj)))) continue;
                const int row = crow(bi), col = ccol(bj, r);
                if (row < M && col < N) {
                    const long long ci = (long long)col * ldc + row;
                    double v = alpha * (double)acc[bi][bj][r];
                    if constexpr (CPRE) v += beta * cpre[bi][bj][r];
                    else if (beta != 0.0) v += beta * C[ci];
                    C[ci] = v;
                }
            }
}

// Kernel variant (K depth 16 or 32, XCD-aware tile order on/off); index =
// (bk32 ? 2 : 0) + (xcd ? 1 : 0).  Selected per call class by gemm_variant.
static int g_gemm_variant[2] = {1, 0};   // [0]: large batched products, [1]: small ones

void set_gemm_variant(int which, int v)
{
    if (which >= 0 && which < 2 && v >= 0 && v < 4) g_gemm_variant[which] = v;
}

template <bool TA, bool TB, int KMODE, bool LOWER, int BK, bool XCD, class CT = double>
static void gemm_launch(hipStream_t st, int M, int N, int K, double alpha, const double* A, int lda,
                        long long sA, const double* B, int ldb, long long sB, double beta,
                        double* C, int ldc, long long sC, int batch)
{
    dim3 grid((M + GB_M - 1) / GB_M, (N + GB_N - 1) / GB_N, batch);
    if (LOWER && M == N) grid = dim3(grid.x * (grid.x + 1) / 2, 1, batch);   // lower tiles only
    if (beta != 0.0)
        hipLaunchKernelGGL((gemm_mfma_kernel<CT, TA, TB, KMODE, LOWER, BK, XCD, true>), grid, dim3(256), 0, st,
                           M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
    else
        hipLaunchKernelGGL((gemm_mfma_kernel<CT, TA, TB, KMODE, LOWER, BK, XCD>), grid, dim3(256), 0, st, M,
                           N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
}

template <bool TA, bool TB, int KMODE, bool LOWER>
static void gemm_dispatch(int variant, hipStream_t st, int M, int N, int K, double alpha,
                          const double* A, int lda, long long sA, const double* B, int ldb,
                          long long sB, double beta, double* C, int ldc, long long sC, int batch)
{
    switch (variant) {
        case 0: gemm_launch<TA, TB, KMODE, LOWER, 16, false>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        case 1: gemm_launch<TA, TB, KMODE, LOWER, 16, true>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        case 2: gemm_launch<TA, TB, KMODE, LOWER, 32, false>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        default: gemm_launch<TA, TB, KMODE, LOWER, 32, true>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
    }
}

void gemm_f64(hipStream_t st, bool ta, bool tb, int kmode, bool lower, int M, int N, int K,
              double alpha, const double* A, int lda, long long sA, const double* B, int ldb,
              long long sB, double beta, double* C, int ldc, long long sC, int batch)
{
    if (M <= 0 || N <= 0 || batch <= 0) return;
    const long long work = (long long)M * N * (K > 0 ? K : 1) * batch;
    const int variant = g_gemm_variant[work >= (1LL << 30) ? 0 : 1];
#define GEMM_CASE(TA_, TB_, KM_, LO_)                                                               \
    if (ta == TA_ && tb == TB_ && kmode == KM_ && lower == LO_) {                                    \
        gemm_dispatch<TA_, TB_, KM_, LO_>(variant, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, \
                                          C, ldc, sC, batch);                                       \
        return;                                                                                     \
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
// Strip-tiled batched FP64 GEMM for the large products (Gram matrices and the
// triangular solves of the local factorisations).  The workgroup tile is
// (16 T) x (16 T) with T waves; wave w owns the 16 x 16T strip of rows
// [16w, 16w + 16) as T accumulators of V_MFMA_F64_16X16X4.  T is chosen so
// that 16 T divides the (16-rounded) neuron count: n = 400 gives T = 5 and no
// padded columns.  In lower mode the diagonal tiles skip the strictly upper
// 16 x 16 blocks, so a symmetric product costs only its lower triangle.
// ---------------------------------------------------------------------------
template <int T, bool TA, bool TB, int KMODE, bool LOWER>
__global__ __launch_bounds__(64 * T) void gemm_strip_kernel(
    int M, int N, int K, double alpha, const double* A, int lda, long long sA, const double* B,
    int ldb, long long sB, double beta, double* C, int ldc, long long sC)
{
    constexpr int BT = 16 * T;
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned total = gx * gy * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = (total & 7u) ? p : (p & 7u) * (total >> 3) + (p >> 3);
    const int tm = q % gx, tn = (q / gx) % gy;
    const long long z = q / (gx * gy);
    if (LOWER && tm < tn) return;
    A += z * sA;
    B += z * sB;
    C += z * sC;
    const int m0 = tm * BT, n0 = tn * BT;
    int kbeg = 0, kend = K;
    if (KMODE == 1) kbeg = n0 < K ? n0 : K;
    if (KMODE == 2) kend = (n0 + BT) < K ? (n0 + BT) : K;

    // rows padded so that the two 16-lane groups of a half-wave read
    // disjoint LDS banks
    constexpr int SPAD = (BT % 32 == 0) ? 16 : 0;
    __shared__ double As[16][BT + SPAD];
    __shared__ double Bs[16][BT + SPAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // live 16-column blocks of this wave's strip: j in [jlo, jhi).  jhi drops
    // blocks beyond N or (lower mode, diagonal tile) above the diagonal; with
    // KMODE 2 the blocks whose columns precede the K stage die (jlo).
    int jhi = (m0 + 16 * w < M) ? min(T, (N - n0 + 15) / 16) : 0;
    if (LOWER && tm == tn) jhi = min(jhi, w + 1);

    v4d acc[T];
#pragma unroll
    for (int j = 0; j < T; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
    double ra[4], rb[4];
    constexpr int RS = 4 * T;   // threads per k row in the along-row pattern
    auto load = [&](int k0) {
        if (!TA) {
            const int kk = k0 + tid / RS, mm = m0 + (tid % RS) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ra[e] = (kk < kend && mm + e < M) ? A[(long long)kk * lda + mm + e] : 0.0;
        } else {
            const int mm = m0 + (tid >> 2), kk = k0 + (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                ra[e] = (mm < M && kk + e < kend) ? A[(long long)mm * lda + kk + e] : 0.0;
        }
        if (!TB) {
            const int nn = n0 + (tid >> 2), kk = k0 + (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                rb[e] = (nn < N && kk + e < kend) ? B[(long long)nn * ldb + kk + e] : 0.0;
        } else {
            const int kk = k0 + tid / RS, nn = n0 + (tid % RS) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                rb[e] = (kk < kend && nn + e < N) ? B[(long long)kk * ldb + nn + e] : 0.0;
        }
    };
    auto store = [&]() {
        if (!TA) {
            const int k = tid / RS, m = (tid % RS) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[k][m + e] = ra[e];
        } else {
            const int m = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) As[k + e][m] = ra[e];
        }
        if (!TB) {
            const int nn = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[k + e][nn] = rb[e];
        } else {
            const int k = tid / RS, nn = (tid % RS) * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[k][nn + e] = rb[e];
        }
    };
    const int nk = (kend > kbeg) ? (kend - kbeg + 15) / 16 : 0;
    if (nk > 0) {
        load(kbeg);
        store();
        __syncthreads();
        // one stage for the blocks [JLO, JHI): all operands into registers
        // first, then the MFMAs back to back (no branches between them)
        auto body = [&](auto lo_c, auto hi_c) {
            constexpr int JLO = decltype(lo_c)::value < T ? decltype(lo_c)::value : T;
            constexpr int JHI = decltype(hi_c)::value < T ? decltype(hi_c)::value : T;
            if constexpr (JHI > JLO) {
                double av[4], bv[4][T];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = ks * 4 + lk;
                    av[ks] = As[k][16 * w + lr];
#pragma unroll
                    for (int j = JLO; j < JHI; ++j) bv[ks][j] = Bs[k][16 * j + lr];
                }
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int j = JLO; j < JHI; ++j)
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks][j], acc[j], 0, 0, 0);
            }
        };
        auto body_any = [&](int lo, int hi) {
            double av[4], bv[4][T];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k = ks * 4 + lk;
                av[ks] = As[k][16 * w + lr];
#pragma unroll
                for (int j = 0; j < T; ++j) bv[ks][j] = Bs[k][16 * j + lr];
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int j = 0; j < T; ++j)
                    if (j >= lo && j < hi)
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks][j], acc[j], 0, 0, 0);
        };
        for (int it = 0; it < nk; ++it) {
            const int k0 = kbeg + it * 16;
            if (it + 1 < nk) load(k0 + 16);
            int jlo = 0;
            if (KMODE == 2 && k0 >= n0) jlo = min(T, (k0 - n0) / 16);
            if (jlo >= jhi) {
                // nothing to do for this wave in this stage
            } else if (jhi == T) {
                switch (jlo) {
                    case 0: body(std::integral_constant<int, 0>{}, std::integral_constant<int, T>{}); break;
                    case 1: body(std::integral_constant<int, 1>{}, std::integral_constant<int, T>{}); break;
                    case 2: body(std::integral_constant<int, 2>{}, std::integral_constant<int, T>{}); break;
                    case 3: body(std::integral_constant<int, 3>{}, std::integral_constant<int, T>{}); break;
                    case 4: body(std::integral_constant<int, 4>{}, std::integral_constant<int, T>{}); break;
                    case 5: body(std::integral_constant<int, 5>{}, std::integral_constant<int, T>{}); break;
                    case 6: body(std::integral_constant<int, 6>{}, std::integral_constant<int, T>{}); break;
                    default: body(std::integral_constant<int, 7>{}, std::integral_constant<int, T>{}); break;
                }
            } else if (jlo == 0) {
                switch (jhi) {
                    case 1: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{}); break;
                    case 2: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 2>{}); break;
                    case 3: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{}); break;
                    case 4: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{}); break;
                    case 5: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 5>{}); break;
                    case 6: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 6>{}); break;
                    default: body(std::integral_constant<int, 0>{}, std::integral_constant<int, 7>{}); break;
                }
            } else {
                body_any(jlo, jhi);
            }
            __syncthreads();
            if (it + 1 < nk) {
                store();
                __syncthreads();
            }
        }
    }
    const int lq = lane >> 4;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        if (j >= jhi) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + 16 * w + 4 * r + lq;
            const int col = n0 + 16 * j + lr;
            if (row < M && col < N) {
                const long long ci = (long long)col * ldc + row;
                double v = alpha * acc[j][r];
                if (beta != 0.0) v += beta * C[ci];
                C[ci] = v;
            }
        }
    }
}

int strip_width(int n)
{
    const int nb = (n + 15) / 16;
    int best = 4, waste = 1 << 30;
    for (int t = 4; t <= 8; ++t) {
        const int wst = (nb + t - 1) / t * t - nb;
        if (wst < waste || (wst == waste && t > best)) {
            best = t;
            waste = wst;
        }
    }
    return best;
}

template <int T, bool TA, bool TB, int KMODE, bool LOWER>
static void strip_launch(hipStream_t st, int M, int N, int K, double alpha, const double* A, int lda,
                         long long sA, const double* B, int ldb, long long sB, double beta,
                         double* C, int ldc, long long sC, int batch)
{
    dim3 grid((M + 16 * T - 1) / (16 * T), (N + 16 * T - 1) / (16 * T), batch);
    hipLaunchKernelGGL((gemm_strip_kernel<T, TA, TB, KMODE, LOWER>), grid, dim3(64 * T), 0, st, M, N,
                       K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
}

template <bool TA, bool TB, int KMODE, bool LOWER>
static void strip_dispatch(int T, hipStream_t st, int M, int N, int K, double alpha, const double* A,
                           int lda, long long sA, const double* B, int ldb, long long sB,
                           double beta, double* C, int ldc, long long sC, int batch)
{
    switch (T) {
        case 4: strip_launch<4, TA, TB, KMODE, LOWER>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        case 5: strip_launch<5, TA, TB, KMODE, LOWER>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        case 6: strip_launch<6, TA, TB, KMODE, LOWER>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        case 7: strip_launch<7, TA, TB, KMODE, LOWER>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
        default: strip_launch<8, TA, TB, KMODE, LOWER>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch); break;
    }
}

void gram_strip(hipStream_t st, int T, int n, int rows, const double* X, int ldx, long long sX,
                double* G, int ldg, long long sG, int batch)
{
    if (n <= 0 || batch <= 0) return;
    strip_dispatch<true, false, 0, true>(T, st, n, n, rows, 1.0, X, ldx, sX, X, ldx, sX, 0.0, G, ldg,
                                         sG, batch);
}

void trsm_strip(hipStream_t st, int T, int rows, int n, const double* X, int ldx, long long sX,
                const double* Linv, int ldl, long long sL, double* Y, long long sY, int batch)
{
    if (rows <= 0 || n <= 0 || batch <= 0) return;
    strip_dispatch<false, true, 2, false>(T, st, rows, n, n, 1.0, X, ldx, sX, Linv, ldl, sL, 0.0, Y,
                                          ldx, sY, batch);
}

void gram_product(hipStream_t st, int code, int n, int rows, const double* X, int ldx, long long sX,
                  double* G, int ldg, long long sG, int batch)
{
    if (n <= 0 || batch <= 0) return;
    if (code >= 4) {
        gram_strip(st, code, n, rows, X, ldx, sX, G, ldg, sG, batch);
        return;
    }
    gemm_dispatch<true, false, 0, true>(-1 - code, st, n, n, rows, 1.0, X, ldx, sX, X, ldx, sX, 0.0, G,
                                        ldg, sG, batch);
}

// Gram product with FP32 operands and FP32 accumulation (lower triangle,
// widened to FP64): the first, shifted pass of the mixed-precision mode.
// Workgroup tile 128 x 128 (lower tiles only, XCD-grouped order), eight waves
// in 2 (rows) x 4 (columns), each a 64 x 32 block of 4 x 2 V_MFMA_F32_16X16X4
// tiles (32 accumulator floats per lane).  FP64 operands are loaded 4 k at a
// time per thread (row tid / 4), rounded to FP32 into a double-buffered LDS
// stage of K depth 16 (row stride 20 floats).  The FP32 accumulators take
// half the registers of FP64 ones, which is what makes the larger tile (half
// the operand bytes per flop of a 64 x 64 tile) affordable; measured at the
// 8x8 Gram shape, batch 64: 16.5 ms against 18.5 ms for the 64 x 64 kernel.
__global__ __launch_bounds__(512) void gram_f32_kernel(int M, int K, const double* X, int ldx, long long sX,
                                                       double* G, int ldg, long long sG)
{
    constexpr int TM = 128, BKK = 16, SK = BKK + 4, V = BKK / 4;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const unsigned gx = gridDim.x;
    const unsigned total = gx * gridDim.y * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned q = (total & 7u) ? p : (p & 7u) * (total >> 3) + (p >> 3);
    const long long z = q / gx;
    int t = q % gx;
    const int g = (TM + M - 1) / TM;
    int tn = 0;
    while (t >= g - tn) {   // lower tiles, column by column
        t -= g - tn;
        ++tn;
    }
    const int tm = tn + t;
    X += z * sX;
    G += z * sG;
    const int m0 = tm * TM, n0 = tn * TM;
    __shared__ __attribute__((aligned(16))) float As_[2][TM * SK];
    __shared__ __attribute__((aligned(16))) float Bs_[2][TM * SK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 15, lk = lane >> 4;
    v4f acc[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = (v4f){0.f, 0.f, 0.f, 0.f};
    double ra[V], rb[V];
    auto ld = [&](double (&r)[V], int mm, int kk) {
        const double* pp = X + (long long)mm * ldx + kk;
        if (mm < M && kk + V - 1 < K && aligned16(pp)) {
#pragma unroll
            for (int e = 0; e < V / 2; ++e) {
                const double2 vv = reinterpret_cast<const double2*>(pp)[e];
                r[2 * e] = vv.x;
                r[2 * e + 1] = vv.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r[e] = (mm < M && kk + e < K) ? pp[e] : 0.0;
        }
    };
    auto load = [&](int k0) {
        const int kk = k0 + (tid & 3) * V;
        ld(ra, m0 + (tid >> 2), kk);
        ld(rb, n0 + (tid >> 2), kk);
    };
    auto store = [&](int b) {
        const int m = tid >> 2, k = (tid & 3) * V;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            As_[b][m * SK + k + e] = (float)ra[e];
            Bs_[b][m * SK + k + e] = (float)rb[e];
        }
    };
    // 16 x 16 blocks of this wave inside the matrix and on or below the diagonal
    int wmask = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int R0 = m0 + wm * 64 + u * 16, C0 = n0 + wn * 32 + v * 16;
            if (R0 < M && C0 < M && R0 + 15 >= C0) wmask |= 1 << (2 * u + v);
        }
    const int nk = (K + BKK - 1) / BKK;
    if (nk > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
        const int cb = it & 1;
        if (it + 1 < nk) load((it + 1) * BKK);
        if (wmask) {
#pragma unroll
            for (int ks = 0; ks < BKK / 4; ++ks) {
                const int k = ks * 4 + lk;
                float a[4], b[2];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = As_[cb][(wm * 64 + u * 16 + lr) * SK + k];
#pragma unroll
                for (int v = 0; v < 2; ++v) b[v] = Bs_[cb][(wn * 32 + v * 16 + lr) * SK + k];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v)
                        if (wmask & (1 << (2 * u + v)))
                            acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[v], acc[u][v], 0, 0, 0);
            }
        }
        // buffer cb ^ 1 was last read in the previous stage, which every wave
        // finished before the barrier that ended it
        if (it + 1 < nk) store(cb ^ 1);
        __syncthreads();
    }
    // FP32 accumulator element r of lane l is D[4 (l / 16) + r][l % 16]
    const int lq = lane >> 4;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            if (!(wmask & (1 << (2 * u + v)))) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + u * 16 + 4 * lq + r;
                const int col = n0 + wn * 32 + v * 16 + lr;
                if (row < M && col < M) G[(long long)col * ldg + row] = (double)acc[u][v][r];
            }
        }
}

void gram_product_f32(hipStream_t st, int n, int rows, const double* X, int ldx, long long sX,
                      double* G, int ldg, long long sG, int batch)
{
    if (n <= 0 || batch <= 0) return;
    const int g = (n + 127) / 128;
    hipLaunchKernelGGL(gram_f32_kernel, dim3(g * (g + 1) / 2, 1, batch), dim3(512), 0, st, n, rows, X, ldx,
                       sX, G, ldg, sG);
}

void trsm_product(hipStream_t st, int code, int rows, int n, const double* X, int ldx, long long sX,
                  const double* Linv, int ldl, long long sL, double* Y, long long sY, int batch)
{
    if (code >= 4) {
        trsm_strip(st, code, rows, n, X, ldx, sX, Linv, ldl, sL, Y, sY, batch);
        return;
    }
    if (rows <= 0 || n <= 0 || batch <= 0) return;
    gemm_dispatch<false, true, 2, false>(-1 - code, st, rows, n, n, 1.0, X, ldx, sX, Linv, ldl, sL, 0.0,
                                         Y, ldx, sY, batch);
}

void strip_gemm_nn(hipStream_t st, int T, int M, int N, int K, const double* A, int lda,
                   const double* B, int ldb, double* C, int ldc)
{
    strip_dispatch<false, false, 0, false>(T, st, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0, 1);
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
                                                         double tau, double* rhs, long long sR)
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
#pragma unroll
    for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
        const int idx = tid + 256 * it;
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
            // Factor the 16 x 16 diagonal tile and invert it with the whole wave:
            // lane l holds row i = l % 16, columns c = 4t + l / 16 (t = 0..3).
            // Step k publishes column k (resp. row k of the inverse) in LDS;
            // LDS operations of one wave complete in program order, so a
            // scheduling fence between publishing and reading is enough.
            const int i = lane & 15, q = lane >> 4;
            double r[4], x[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * t + q;
                r[t] = (c <= i) ? T[s0 + i][s0 + c] : 0.0;
                x[t] = (c == i) ? 1.0 : 0.0;
            }
            double* colb = &tmp[0][0][0];      // 16 entries: column k
            double* rowb = &tmp[0][1][0];      // 16 entries: row k of the inverse
            double rpiv[16];                   // 1 / L_kk
            int bad = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (q == (k & 3)) colb[i] = r[k >> 2];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                double d = colb[k];
                const double f = fl[s0 + k];
                if (!(d > f) || !isfinite(d)) {
                    bad = 1;
                    d = 1.0;
                }
                // 1/sqrt(d): hardware estimate refined by two Newton steps
                double rp = __builtin_amdgcn_rsq(d);
                rp = rp * (1.5 - 0.5 * d * rp * rp);
                rp = rp * (1.5 - 0.5 * d * rp * rp);
                const double p = d * rp;
                rpiv[k] = rp;
                const double lik = (i > k) ? colb[i] * rp : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = 4 * t + q;
                    if (c == k) r[t] = (i == k) ? p : lik;
                    else if (c > k && c <= i) r[t] -= lik * (colb[c] * rp);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            // publish L, then X = L^{-1} row by row
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * t + q;
                if (c <= i) T[s0 + i][s0 + c] = r[t];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double rkk = rpiv[k];
                if (i == k) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        x[t] *= rkk;
                        rowb[4 * t + q] = x[t];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const double lik = (i > k) ? T[s0 + i][s0 + k] : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = 4 * t + q;
                    if (c <= k) x[t] -= lik * rowb[c];
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * t + q;
                if (c <= i) Xs[s0 + i][s0 + c] = x[t];
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
        rhs += z * sR;
        if (tid < 64) fl[tid] = tid < jb ? rhs[j + tid] : 0.0;   // fl is free by now
        __syncthreads();
        if (tid < jb) {
            double acc = 0.0;
            for (int c = 0; c <= tid; ++c) acc += Xs[tid][c] * fl[c];
            rhs[j + tid] = acc;
        }
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
        const int idx = tid + 256 * it;
        const int c = idx >> 6, r = idx & 63;
        const bool in = (r < jb) && (c < jb);
        const double xv = (in && c <= r) ? Xs[r][c] : 0.0;
        Dinv[c * 64 + r] = xv;
        if (in && c <= r) A[(long long)(j + c) * lda + (j + r)] = T[r][c];
        if (Linv && in) Linv[z * sL + (long long)(j + c) * ldl + (j + r)] = xv;
    }
    __syncthreads();
    if (tid == 0 && bad_any && info) {
        if (pass >= 1) {   // a local CholeskyQR pass; pass < 1: the interface matrix
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
                int batch, const double* dsave, long long sS, double tau, double* rhs, long long sR)
{
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(batch), dim3(256), 0, st, A, lda, sA, j, jb, Dinv,
                       sD, Linv, ldl, sL, info, pass, dsave, sS, tau, rhs, sR);
}

// One step of the envelope Cholesky after the diagonal block J = [j, j + jb)
// has been factored (Dinv = L_JJ^{-1}): for the 64-row tiles I >= I' of the
// band [j + jb, r1), one workgroup per tile pair forms the panel tiles
// L_I = A_IJ Dinv^T and L_I' (on the matrix cores, from LDS), applies the
// trailing update A_II' -= L_I L_I'^T in place and, on diagonal pairs, stores
// L_I into the factor Lo and applies the forward-substitution update
// y_I -= L_I y_J.  L goes to a separate matrix because other workgroups of the
// same launch still read the unsolved panel A_IJ.
__global__ __launch_bounds__(256) void envelope_step_kernel(double* A, int lda, long long sA,
                                                            double* Lo, int ldo, long long sLo,
                                                            int j, int jb, const double* Dinv,
                                                            long long sD, int r1, double* rhs,
                                                            long long sR)
{
    {
        const long long zb = blockIdx.y;
        A += zb * sA;
        Lo += zb * sLo;
        Dinv += zb * sD;
        if (rhs) rhs += zb * sR;
    }
    __shared__ double Dv[64][65];
    __shared__ double S1[64][65];
    __shared__ double S2[64][65];
    __shared__ double yj[64];
    const int p = blockIdx.x;
    int a = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= p) ++a;
    while (a * (a + 1) / 2 > p) --a;
    const int b = p - a * (a + 1) / 2;
    const int base = j + jb;
    const int I = base + 64 * a, Ib = base + 64 * b;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
        const int idx = tid + 256 * it;
        const int c = idx >> 6, r = idx & 63;
        Dv[r][c] = (r < jb && c < jb) ? Dinv[c * 64 + r] : 0.0;
        S1[r][c] = (I + r < r1 && c < jb) ? A[(long long)(j + c) * lda + I + r] : 0.0;
        S2[r][c] = (a != b && Ib + r < r1 && c < jb) ? A[(long long)(j + c) * lda + Ib + r] : 0.0;
    }
    if (tid < 64) yj[tid] = (rhs && tid < jb) ? rhs[j + tid] : 0.0;
    __syncthreads();
    // panel tiles: L = P Dinv^T, each wave a 32 x 32 quarter (2 x 2 MFMA tiles)
    auto panel = [&](double (*Sx)[65]) {
        v4d acc[2][2];
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) acc[u][v] = (v4d){0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int kk = k0 + lq;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        Sx[wm * 32 + u * 16 + lr][kk], Dv[wn * 32 + v * 16 + lr][kk], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) Sx[wm * 32 + u * 16 + 4 * r + lq][wn * 32 + v * 16 + lr] = acc[u][v][r];
        __syncthreads();
    };
    panel(S1);
    if (a != b) panel(S2);
    double (*Lb)[65] = (a != b) ? S2 : S1;
    // trailing tile C = A[I, Ib] - L_I L_Ib^T
    v4d acc[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) acc[u][v] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int kk = k0 + lq;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    S1[wm * 32 + u * 16 + lr][kk], Lb[wn * 32 + v * 16 + lr][kk], acc[u][v], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = I + wm * 32 + u * 16 + 4 * r + lq;
                const int col = Ib + wn * 32 + v * 16 + lr;
                if (row < r1 && col < r1) A[(long long)col * lda + row] -= acc[u][v][r];
            }
    if (a == b) {
#pragma unroll
        for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
            const int idx = tid + 256 * it;
            const int c = idx >> 6, r = idx & 63;
            if (I + r < r1 && c < jb) Lo[(long long)(j + c) * ldo + I + r] = S1[r][c];
        }
        if (rhs && tid < 64 && I + tid < r1) {
            double acc1 = 0.0;
            for (int c = 0; c < jb; ++c) acc1 += S1[tid][c] * yj[c];
            rhs[I + tid] -= acc1;
        }
    }
}

void envelope_step(hipStream_t st, double* A, int lda, long long sA, double* Lo, int ldo,
                   long long sLo, int j, int jb, const double* Dinv, long long sD, int r1,
                   double* rhs, long long sR, int batch)
{
    const int rows = r1 - j - jb;
    if (rows <= 0) return;
    const int nt = (rows + 63) / 64;
    hipLaunchKernelGGL(envelope_step_kernel, dim3(nt * (nt + 1) / 2, batch), dim3(256), 0, st, A, lda,
                       sA, Lo, ldo, sLo, j, jb, Dinv, sD, r1, rhs, sR);
}

// Panel of one envelope Cholesky step without the trailing update: for each
// 64-row tile I of [j + jb, r1), L_I = A_IJ Dinv^T is written to Lo and the
// forward-substitution update y_I -= L_I y_J is applied.  Used with a
// separate trailing-update GEMM when many matrices are factored together.
__global__ __launch_bounds__(256) void envelope_panel_kernel(const double* A, int lda, long long sA,
                                                             double* Lo, int ldo, long long sLo,
                                                             int j, int jb, const double* Dinv,
                                                             long long sD, int r1, double* rhs,
                                                             long long sR)
{
    __shared__ double Dv[64][65];
    __shared__ double S1[64][65];
    __shared__ double yj[64];
    const long long zb = blockIdx.y;
    A += zb * sA;
    Lo += zb * sLo;
    Dinv += zb * sD;
    if (rhs) rhs += zb * sR;
    const int I = j + jb + 64 * blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
        const int idx = tid + 256 * it;
        const int c = idx >> 6, r = idx & 63;
        Dv[r][c] = (r < jb && c < jb) ? Dinv[c * 64 + r] : 0.0;
        S1[r][c] = (I + r < r1 && c < jb) ? A[(long long)(j + c) * lda + I + r] : 0.0;
    }
    if (tid < 64) yj[tid] = (rhs && tid < jb) ? rhs[j + tid] : 0.0;
    __syncthreads();
    v4d acc[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) acc[u][v] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int kk = k0 + lq;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    S1[wm * 32 + u * 16 + lr][kk], Dv[wn * 32 + v * 16 + lr][kk], acc[u][v], 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) S1[wm * 32 + u * 16 + 4 * r + lq][wn * 32 + v * 16 + lr] = acc[u][v][r];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 16; ++it) {   // 64 x 64 tile, 256 threads
        const int idx = tid + 256 * it;
        const int c = idx >> 6, r = idx & 63;
        if (I + r < r1 && c < jb) Lo[(long long)(j + c) * ldo + I + r] = S1[r][c];
    }
    if (rhs && tid < 64 && I + tid < r1) {
        double a1 = 0.0;
        for (int c = 0; c < jb; ++c) a1 += S1[tid][c] * yj[c];
        rhs[I + tid] -= a1;
    }
}

void envelope_panel(hipStream_t st, const double* A, int lda, long long sA, double* Lo, int ldo,
                    long long sLo, int j, int jb, const double* Dinv, long long sD, int r1,
                    double* rhs, long long sR, int batch)
{
    const int rows = r1 - j - jb;
    if (rows <= 0) return;
    hipLaunchKernelGGL(envelope_panel_kernel, dim3((rows + 63) / 64, batch), dim3(256), 0, st, A, lda,
                       sA, Lo, ldo, sLo, j, jb, Dinv, sD, r1, rhs, sR);
}

// Backward substitution L^T u = y over one block row of up to 256 rows
// [j0, j0 + br), in two launches.  trsv_lt_diag_kernel (one workgroup per
// system) solves the block's four 64-row sub-blocks in turn, using their
// diagonal inverses and the L tiles inside the block, and writes u_block;
// trsv_lt_offdiag_kernel then updates y_K -= L_{block,K}^T u_block for the
// columns K in [kbeg, j0) (one wave per column, lanes along the rows).
__global__ __launch_bounds__(256) void trsv_lt_diag_kernel(const double* L, int ld, long long sL, int j0, int br,
                                                           const double* Dinv, long long sD, const double* y,
                                                           double* u, long long sY)
{
    {
        const long long zb = blockIdx.y;
        L += zb * sL;
        Dinv += zb * sD;
        y += zb * sY;
        u += zb * sY;
    }
    __shared__ double yb[256], ub[256];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    yb[tid] = tid < br ? y[j0 + tid] : 0.0;
    ub[tid] = 0.0;
    __syncthreads();
    const int nsub = (br + 63) / 64;
    for (int sb = nsub - 1; sb >= 0; --sb) {
        const int s0 = 64 * sb, sl = (br - s0) < 64 ? (br - s0) : 64;
        // y_sb -= sum over later sub-blocks of L[later, sb]^T u_later: one wave
        // per column of the sub-block, lanes along the (contiguous) rows
        if (s0 + 64 < br) {
            for (int t = wave; t < sl; t += 4) {
                const double* colp = L + (long long)(j0 + s0 + t) * ld + j0;
                double v = 0.0;
                for (int r = s0 + 64 + lane; r < br; r += 64) v += colp[r] * ub[r];
                v = wave_sum(v);
                if (lane == 0) yb[s0 + t] -= v;
            }
            __syncthreads();
        }
        // u_sb = D y_sb with D the stored inverse factor of the diagonal
        // sub-block (row t holds D[t][i] at t * 64 + i, i >= t): one wave per
        // row, lanes along the row (coalesced)
        const double* D = Dinv + (long long)((j0 + s0) / 64) * 64 * 64;
        for (int t = wave; t < sl; t += 4) {
            double v = (lane >= t && lane < sl) ? D[t * 64 + lane] * yb[s0 + lane] : 0.0;
            v = wave_sum(v);
            if (lane == 0) ub[s0 + t] = v;
        }
        __syncthreads();
    }
    if (tid < br) u[j0 + tid] = ub[tid];
}

__global__ __launch_bounds__(256) void trsv_lt_offdiag_kernel(const double* L, int ld, long long sL, int j0,
                                                              int br, int kbeg, double* y, const double* u,
                                                              long long sY)
{
    {
        const long long zb = blockIdx.y;
        L += zb * sL;
        y += zb * sY;
        u += zb * sY;
    }
    __shared__ double ub[256];
    const int tid = threadIdx.x;
    ub[tid] = tid < br ? u[j0 + tid] : 0.0;
    __syncthreads();
    const int lane = tid & 63;
    const int wave = blockIdx.x * 4 + (tid >> 6);
    const int nwave = gridDim.x * 4;
    for (int kcol = kbeg + wave; kcol < j0; kcol += nwave) {
        const double* colp = L + (long long)kcol * ld + j0;
        double v = 0.0;
        for (int r = lane; r < br; r += 64) v += colp[r] * ub[r];
        v = wave_sum(v);
        if (lane == 0) y[kcol] -= v;
    }
}

void trsv_lower_t_block(hipStream_t st, const double* L, int ld, long long sL, int j0, int br,
                        int kbeg, const double* Dinv, long long sD, double* y, double* u,
                        long long sY, int batch)
{
    hipLaunchKernelGGL(trsv_lt_diag_kernel, dim3(1, batch), dim3(256), 0, st, L, ld, sL, j0, br, Dinv, sD, y, u,
                       sY);
    if (j0 <= kbeg) return;
    int nb = (j0 - kbeg + 7) / 8;   // about two columns per wave
    nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
    hipLaunchKernelGGL(trsv_lt_offdiag_kernel, dim3(nb, batch), dim3(256), 0, st, L, ld, sL, j0, br, kbeg, y, u,
                       sY);
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
                                                            int mg, double* Mbuf, int ngeo)
{
    const int blk = blockIdx.x;
    const long long inst = blockIdx.y;
    P += inst * ngeo * sP;
    const int32_t* d = desc + 8 * blk;
    double* out = Mbuf + ((long long)gridDim.x * inst + blk) * mg * mg;
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
                   long long sP, int cbase, int mg, double* Mbuf, int ngeo, int ninst)
{
    if (nblk <= 0) return;
    hipLaunchKernelGGL(schur_mblocks_kernel, dim3(nblk, ninst), dim3(256), 0, st, desc, P, ldp, sP,
                       cbase, mg, Mbuf, ngeo);
}

__global__ void schur_avec_kernel(const int32_t* desc, const double* P, int ldp, long long sP,
                                  int cbase, int acol, int mg, double* abuf, int ngeo)
{
    const int e = blockIdx.x;
    const long long inst = blockIdx.y;
    P += inst * ngeo * sP;
    abuf += inst * gridDim.x * (long long)mg;
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
                int cbase, int acol, int mg, double* abuf, int ngeo, int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(schur_avec_kernel, dim3(nE, ninst), dim3(64), 0, st, desc, P, ldp, sP, cbase,
                       acol, mg, abuf, ngeo);
}

// One workgroup per mg x mg block (E1, E2) of S:
//   S_{E1,E2} = sum_s [delta_{E1E2} I - T_s(E1, E2)] + sum_g M_{g,E1}^T M_{g,E2}.
// Terms are listed per block in a fixed order, so the sum is deterministic.
__global__ __launch_bounds__(256) void schur_sblocks_kernel(int nE, int mg, const int32_t* blocks,
                                                            const int32_t* tptr,
                                                            const int32_t* tdesc,
                                                            const int32_t* mptr,
                                                            const int32_t* mdesc, const double* P,
                                                            int ldp, long long sP,
                                                            const double* Mbuf, double* S, int lds,
                                                            const int32_t* perm, int ngeo,
                                                            long long sM, long long sS)
{
    // M blocks staged column-major with a padded column stride (mg + 1
    // doubles), so that the 16 lanes of a fragment read (consecutive columns,
    // same k) do not fold onto a few LDS banks; 2 mg (mg + 1) doubles of
    // dynamic LDS (26 KB at mg = 40), so that several workgroups share a CU
    extern __shared__ double schur_lds[];
    double* M1 = schur_lds;
    double* M2 = schur_lds + mg * (mg + 1);
    const int blk = blocks[blockIdx.x];   // a block that receives T or M contributions
    const int E1 = blk % nE, E2 = blk / nE;
    {
        const long long inst = blockIdx.y;
        P += inst * ngeo * sP;
        Mbuf += inst * sM;
        S += inst * sS;
    }
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
    // M^T M contributions on the matrix cores: D = sum over pairs of A1^T A2
    // (A = M_{g,E} blocks, column-major), the mg x mg output split into
    // 16 x 16 tiles dealt to the four waves (tile tau = wave + 4u), k in
    // steps of 4; lane l supplies A1[k][i], A2[k][j] with i or j = 16 t + l % 16
    // and k = 4 ks + l / 16 (entries beyond mg are zero)
    const int npair = mptr[blk + 1] - mptr[blk];
    if (npair > 0) {
        const int ms = mg + 1, nt = (mg + 15) / 16, nks = (mg + 3) / 4;
        const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lq = lane >> 4;
        v4d macc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) macc[u] = (v4d){0.0, 0.0, 0.0, 0.0};
        for (int it = mptr[blk]; it < mptr[blk + 1]; ++it) {
            const double* A1 = Mbuf + (long long)mdesc[2 * it] * mm;
            const double* A2 = Mbuf + (long long)mdesc[2 * it + 1] * mm;
            __syncthreads();
            for (int idx = tid; idx < mm; idx += 256) {
                const int q = (idx / mg) * ms + idx % mg;
                M1[q] = A1[idx];
                M2[q] = A2[idx];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tau = wave + 4 * u;
                if (tau >= nt * nt) continue;
                const int i = 16 * (tau % nt) + lr, j = 16 * (tau / nt) + lr;
                for (int ks = 0; ks < nks; ++ks) {
                    const int k = 4 * ks + lq;
                    const double a = (i < mg && k < mg) ? M1[i * ms + k] : 0.0;
                    const double b = (j < mg && k < mg) ? M2[j * ms + k] : 0.0;
                    macc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, macc[u], 0, 0, 0);
                }
            }
        }
        // through LDS (column-major, stride ms) back to the element layout of acc
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int tau = wave + 4 * u;
            if (tau >= nt * nt) continue;
            const int j = 16 * (tau / nt) + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * (tau % nt) + 4 * r + lq;
                if (i < mg && j < mg) M1[j * ms + i] = macc[u][r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t;
            if (idx < mm) acc[t] += M1[(idx / mg) * ms + idx % mg];
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

// The blocks of S that no subdomain touches are zero: written by a plain fill
// kernel (no LDS, so many workgroups run at once) instead of by the product
// kernel above.
__global__ __launch_bounds__(256) void schur_zero_kernel(int nE, int mg, const int32_t* blocks, double* S, int lds,
                                                         const int32_t* perm, long long sS)
{
    const int blk = blocks[blockIdx.x];
    const int E1 = blk % nE, E2 = blk / nE;
    S += (long long)blockIdx.y * sS;
    const int mm = mg * mg;
    for (int idx = threadIdx.x; idx < mm; idx += 256) {
        const int r = idx % mg, c = idx / mg;
        S[(long long)(perm[E2] * mg + c) * lds + (perm[E1] * mg + r)] = 0.0;
    }
}

void schur_sblocks(hipStream_t st, int nE, int mg, const int32_t* nzb, int nnz, const int32_t* zb, int nz,
                   const int32_t* tptr, const int32_t* tdesc, const int32_t* mptr, const int32_t* mdesc,
                   const double* P, int ldp, long long sP, const double* Mbuf, double* S, int lds,
                   const int32_t* perm, int ngeo, long long sM, long long sS, int ninst)
{
    if (nE <= 0 || ninst <= 0) return;
    if (nnz > 0)
        hipLaunchKernelGGL(schur_sblocks_kernel, dim3(nnz, ninst), dim3(256), 2 * mg * (mg + 1) * sizeof(double), st,
                           nE, mg, nzb, tptr, tdesc, mptr, mdesc, P, ldp, sP, Mbuf, S, lds, perm, ngeo, sM, sS);
    if (nz > 0)
        hipLaunchKernelGGL(schur_zero_kernel, dim3(nz, ninst), dim3(256), 0, st, nE, mg, zb, S, lds, perm, sS);
}

// rhs_E = sum_s q_s(E) - sum_g M_{g,E}^T a_g.
__global__ void schur_rhs_kernel(int mg, const int32_t* qdesc, const int32_t* gptr,
                                 const int32_t* gdesc, const double* P, int ldp, long long sP,
                                 int qcol, const double* Mbuf, const double* abuf, double* rhs,
                                 int inc, const int32_t* perm, int ngeo, long long sM,
                                 long long sA, long long sR)
{
    const int E = blockIdx.x;
    {
        const long long inst = blockIdx.y;
        P += inst * ngeo * sP;
        Mbuf += inst * sM;
        abuf += inst * sA;
        rhs += inst * sR;
    }
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
               const double* Mbuf, const double* abuf, double* rhs, int inc, const int32_t* perm,
               int ngeo, long long sM, long long sA, long long sR, int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(schur_rhs_kernel, dim3(nE, ninst), dim3(64), 0, st, mg, qdesc, gptr, gdesc, P,
                       ldp, sP, qcol, Mbuf, abuf, rhs, inc, perm, ngeo, sM, sA, sR);
}

// ---------------------------------------------------------------------------
// Local back-solve (Algorithm 1, last loop): c = R^{-1} (h + Q_Gamma^T u_s)
// with R^{-1} = Linv1^T Linv2^T Linv3^T from the three CholeskyQR passes.
// One wave per output entry, lanes along the contiguous column: coalesced.
// ---------------------------------------------------------------------------
// v[s][col] = h_s[col] + sum_i Q_Gamma[i][col] u[gidx_s[i]]
__global__ __launch_bounds__(256) void bs_rhs_kernel(int n, int kpad, const double* X, int ldx,
                                                     long long sX, int mI, int hrow,
                                                     const int32_t* gidx, const double* u,
                                                     double* v, int ngeo, long long nG)
{
    const int s = blockIdx.y;
    const int sg = s % ngeo;
    u += (s / ngeo) * nG;
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= n) return;
    const double* xc = X + s * sX + (long long)col * ldx;
    double acc = 0.0;
    for (int i = lane; i < kpad; i += 64) {
        const int gi = gidx[sg * kpad + i];
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

void local_backsolve(hipStream_t st, int N, int ngeo, long long nG, int n, int kpad, const double* X,
                     int ldx, long long sX, int mI, int hrow, const int32_t* gidx, const double* u,
                     double* const* Linv, int npass, int ldg, long long sG, double* c, double* tmp1,
                     double* tmp2)
{
    dim3 grid((n + 3) / 4, N);
    hipLaunchKernelGGL(bs_rhs_kernel, grid, dim3(256), 0, st, n, kpad, X, ldx, sX, mI, hrow, gidx, u,
                       tmp1, ngeo, nG);
    double* cur = tmp1;
    double* nxt = tmp2;
    for (int q = npass - 1; q >= 0; --q) {
        double* out = q == 0 ? c : nxt;
        hipLaunchKernelGGL(trmv_t_kernel, grid, dim3(256), 0, st, n, Linv[q], ldg, sG, cur, out);
        std::swap(cur, nxt);
    }
}

// u[E*mg + r] = up[perm[E]*mg + r]
__global__ void unpermute_kernel(int nE, int mg, const int32_t* perm, const double* up, double* u)
{
    const long long n = (long long)nE * mg;
    const long long inst = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int E = idx / mg, r = idx % mg;
    u[inst * n + idx] = up[inst * n + (long long)perm[E] * mg + r];
}

void unpermute(hipStream_t st, int nE, int mg, const int32_t* perm, const double* up, double* u,
               int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(unpermute_kernel, dim3((nE * mg + 255) / 256, ninst), dim3(256), 0, st, nE, mg,
                       perm, up, u);
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
    for (int j = 0; j < n; ++j) acc += cs[j] * tanh_feat(Ws[2 * j] * xh + Ws[2 * j + 1] * yh + bs[j]);
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

// u_h and its gradient: d/dx sum_j c_j tanh(z_j) = sum_j c_j (1 - t_j^2) w_j,x (2 / h_x),
// likewise in y (the local networks see xhat = 2 (x - x_c) / h_x).  u may be NULL.
__global__ void eval_grad_kernel(int npts, const double* xy, int nx, int ny, double x0, double x1, double y0,
                                 double y1, int n, const double* W, const double* b, const double* c, double* u,
                                 double* ux, double* uy)
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
    double a0 = 0.0, ax = 0.0, ay = 0.0;
    for (int j = 0; j < n; ++j) {
        const double t = tanh_feat(Ws[2 * j] * xh + Ws[2 * j + 1] * yh + bs[j]);
        const double d = cs[j] * (1.0 - t * t);
        a0 += cs[j] * t;
        ax += d * Ws[2 * j];
        ay += d * Ws[2 * j + 1];
    }
    if (u) u[p] = a0;
    ux[p] = ax * (2.0 / hx);
    uy[p] = ay * (2.0 / hy);
}

void eval_points_grad(hipStream_t st, int npts, const double* xy, int nx, int ny, double x0, double x1,
                      double y0, double y1, int n, const double* W, const double* b, const double* c,
                      double* u, double* ux, double* uy)
{
    if (npts <= 0) return;
    hipLaunchKernelGGL(eval_grad_kernel, dim3((npts + 255) / 256), dim3(256), 0, st, npts, xy, nx, ny, x0, x1,
                       y0, y1, n, W, b, c, u, ux, uy);
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

// ---------------------------------------------------------------------------
// Solves for further right-hand sides with the factors of an earlier solve
// (same hidden layer, new source f and boundary data g): only the F column
// of eq. nonoverlap_discrete changes, so h = Q^T F, the Schur rhs, the two
// triangular solves on S and the back-solve are repeated.
// ---------------------------------------------------------------------------
namespace elmddm {

// Fr[s][r][row] = F column of subdomain s for rhs r (rows [0, rows)).
__global__ __launch_bounds__(256) void rhs_assemble_kernel(RowTable rows, int ldx, int nrows, int ldf,
                                                           const double* f, const double* g, int N,
                                                           int nrhs, long long nf, long long nbnd,
                                                           double* Fr)
{
    const int row = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int r = blockIdx.z;
    if (row >= nrows) return;
    const long long ri = (long long)s * ldx + row;
    const int kind = rows.kind[ri];
    double v = 0.0;
    if (kind == ROW_INTERIOR) v = f[r * nf + rows.src[ri]];
    else if (kind == ROW_BOUNDARY && g) v = g[r * nbnd + rows.src[ri]];
    Fr[((long long)s * nrhs + r) * ldf + row] = v;
}

void rhs_assemble(hipStream_t st, const RowTable& rows, int ldx, int nrows, int ldf, const double* f,
                  const double* g, int N, int nrhs, long long nf, long long nbnd, double* Fr)
{
    dim3 grid((nrows + 255) / 256, N, nrhs);
    hipLaunchKernelGGL(rhs_assemble_kernel, grid, dim3(256), 0, st, rows, ldx, nrows, ldf, f, g, N, nrhs,
                       nf, nbnd, Fr);
}

// Forward substitution L y = g over one block row of up to 256 rows
// [j0, j0 + br) of the envelope factor (diagonal 64-blocks through their
// inverses Dinv, off-diagonal tiles in L): every workgroup solves the block
// (four 64-row sub-blocks, right-looking inside the block), workgroup 0
// stores it, and each workgroup then subtracts L[r, block] y_block from its
// share of the rows r in [j0 + br, r1) (one thread per row, coalesced along
// the columns of L).  Batch index z: y += z sY, L += z sL, Dinv += z sD.
__global__ __launch_bounds__(256) void trsv_l_block_kernel(const double* L, int ld, long long sL, int j0,
                                                           int br, int r1, const double* Dinv,
                                                           long long sD, double* y, long long sY)
{
    {
        const long long zb = blockIdx.y;
        L += zb * sL;
        Dinv += zb * sD;
        y += zb * sY;
    }
    __shared__ double yb[256], ub[256];
    const int tid = threadIdx.x;
    yb[tid] = tid < br ? y[j0 + tid] : 0.0;
    ub[tid] = 0.0;
    __syncthreads();
    const int nsub = (br + 63) / 64;
    for (int sb = 0; sb < nsub; ++sb) {
        const int s0 = 64 * sb, sl = (br - s0) < 64 ? (br - s0) : 64;
        if (tid < sl) {
            const double* D = Dinv + (long long)((j0 + s0) / 64) * 64 * 64;
            double acc = 0.0;
            for (int k = 0; k <= tid; ++k) acc += D[k * 64 + tid] * yb[s0 + k];
            ub[s0 + tid] = acc;
        }
        __syncthreads();
        if (tid >= s0 + 64 && tid < br) {
            double acc = 0.0;
            for (int t = 0; t < sl; ++t) acc += L[(long long)(j0 + s0 + t) * ld + j0 + tid] * ub[s0 + t];
            yb[tid] -= acc;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && tid < br) y[j0 + tid] = ub[tid];
    for (int r = j0 + br + blockIdx.x * 256 + tid; r < r1; r += gridDim.x * 256) {
        double acc = 0.0;
        for (int c = 0; c < br; ++c) acc += L[(long long)(j0 + c) * ld + r] * ub[c];
        y[r] -= acc;
    }
}

void trsv_lower_block(hipStream_t st, const double* L, int ld, long long sL, int j0, int br, int r1,
                      const double* Dinv, long long sD, double* y, long long sY, int batch)
{
    const int rows = r1 - j0 - br;
    int nb = (rows + 255) / 256;
    nb = nb < 1 ? 1 : nb;
    hipLaunchKernelGGL(trsv_l_block_kernel, dim3(nb, batch), dim3(256), 0, st, L, ld, sL, j0, br, r1,
                       Dinv, sD, y, sY);
}

// V[s][r][col] = H[s][r][col] + sum_i Q_Gamma,s[i][col] u_r[gidx_s[i]]: the
// right-hand side of the local back-solve for nrhs interface vectors.
__global__ __launch_bounds__(256) void bs_rhs_multi_kernel(int n, int kpad, const double* X, int ldx,
                                                           long long sX, int mI, const int32_t* gidx,
                                                           const double* u, long long nG,
                                                           const double* H, double* V, int nrhs)
{
    const int s = blockIdx.y;
    const int r = blockIdx.z;
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= n) return;
    const double* xc = X + s * sX + (long long)col * ldx + mI;
    const double* ur = u + r * nG;
    double acc = 0.0;
    for (int i = lane; i < kpad; i += 64) {
        const int gi = gidx[s * kpad + i];
        if (gi >= 0) acc += xc[i] * ur[gi];
    }
    acc = wave_sum(acc);
    const long long o = ((long long)s * nrhs + r) * n + col;
    if (lane == 0) V[o] = acc + H[o];
}

void backsolve_rhs_multi(hipStream_t st, int N, int n, int kpad, const double* X, int ldx, long long sX,
                         int mI, const int32_t* gidx, const double* u, long long nG, const double* H,
                         double* V, int nrhs)
{
    dim3 grid((n + 3) / 4, N, nrhs);
    hipLaunchKernelGGL(bs_rhs_multi_kernel, grid, dim3(256), 0, st, n, kpad, X, ldx, sX, mI, gidx, u, nG,
                       H, V, nrhs);
}

}  // namespace elmddm

// ---------------------------------------------------------------------------
// Conjugate gradients on the interface system S u = g (the paper's interface
// solver, Section 3), on the kept dense S in the envelope order, for nrhs
// right-hand sides at once.
// ---------------------------------------------------------------------------
namespace elmddm {

// up[r][perm[E] mg + i] = u[r][E mg + i]
__global__ void permute_kernel(int nE, int mg, const int32_t* perm, const double* u, double* up)
{
    const long long n = (long long)nE * mg;
    const long long r = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int E = idx / mg, i = idx % mg;
    up[r * n + (long long)perm[E] * mg + i] = u[r * n + idx];
}

void permute(hipStream_t st, int nE, int mg, const int32_t* perm, const double* u, double* up, int nrhs)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(permute_kernel, dim3((nE * mg + 255) / 256, nrhs), dim3(256), 0, st, nE, mg, perm, u, up);
}

// y_r = S x_r for symmetric S (full storage, column-major, ld lds) whose
// column i is zero outside rows [rb[i/64], re[i/64]): y_r[i] is the dot
// product of column i with x_r.  One wave per column, lanes along the rows;
// up to 8 right-hand sides per pass over the column.
__global__ __launch_bounds__(256) void band_symv_kernel(int n, const double* S, int lds, const int32_t* rb,
                                                        const int32_t* re, const double* x, double* y,
                                                        int nrhs)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int r0 = rb[i / 64], r1 = re[i / 64];
    const double* col = S + (long long)i * lds;
    for (int q0 = 0; q0 < nrhs; q0 += 8) {
        const int nq = nrhs - q0 < 8 ? nrhs - q0 : 8;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int r = r0 + lane; r < r1; r += 64) {
            const double s = col[r];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nq) acc[q] += s * x[(long long)(q0 + q) * n + r];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < nq) {
                const double v = wave_sum(acc[q]);
                if (lane == 0) y[(long long)(q0 + q) * n + i] = v;
            }
    }
}

void band_symv(hipStream_t st, int n, const double* S, int lds, const int32_t* rb, const int32_t* re,
               const double* x, double* y, int nrhs)
{
    hipLaunchKernelGGL(band_symv_kernel, dim3((n + 3) / 4), dim3(256), 0, st, n, S, lds, rb, re, x, y, nrhs);
}

__device__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    return t;
}

// state[r] = {rr, bb, done, iterations}
__global__ __launch_bounds__(1024) void cg_init_kernel(int n, const double* b, const double* Sx, double* r,
                                                       double* p, double* state, double tol)
{
    __shared__ double red[16];
    const long long o = (long long)blockIdx.x * n;
    double rr = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double ri = b[o + i] - Sx[o + i];
        r[o + i] = ri;
        p[o + i] = ri;
        rr += ri * ri;
        bb += b[o + i] * b[o + i];
    }
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        double* s = state + 4 * blockIdx.x;
        s[0] = rr;
        s[1] = bb;
        s[2] = (rr <= tol * tol * bb) ? 1.0 : 0.0;
        s[3] = 0.0;
    }
}

// One CG step for right-hand side blockIdx.x, given q = S p.
__global__ __launch_bounds__(1024) void cg_step_kernel(int n, double* x, double* r, double* p, const double* q,
                                                       double* state, double tol)
{
    __shared__ double red[16];
    double* s = state + 4 * blockIdx.x;
    if (s[2] != 0.0) return;   // converged (uniform over the block)
    const long long o = (long long)blockIdx.x * n;
    double pq = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) pq += p[o + i] * q[o + i];
    pq = block_sum(pq, red);
    const double rr = s[0];
    const double alpha = pq > 0.0 ? rr / pq : 0.0;
    double rr2 = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[o + i] += alpha * p[o + i];
        const double ri = r[o + i] - alpha * q[o + i];
        r[o + i] = ri;
        rr2 += ri * ri;
    }
    rr2 = block_sum(rr2, red);
    const bool done = rr2 <= tol * tol * s[1] || !(pq > 0.0);
    const double beta = rr > 0.0 ? rr2 / rr : 0.0;
    if (!done)
        for (int i = threadIdx.x; i < n; i += blockDim.x) p[o + i] = r[o + i] + beta * p[o + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        s[0] = rr2;
        s[2] = done ? (pq > 0.0 ? 1.0 : 2.0) : 0.0;
        s[3] += 1.0;
    }
}

void cg_init(hipStream_t st, int n, const double* b, const double* Sx, double* r, double* p, double* state,
             double tol, int nrhs)
{
    hipLaunchKernelGGL(cg_init_kernel, dim3(nrhs), dim3(1024), 0, st, n, b, Sx, r, p, state, tol);
}

void cg_step(hipStream_t st, int n, double* x, double* r, double* p, const double* q, double* state, double tol,
             int nrhs)
{
    hipLaunchKernelGGL(cg_step_kernel, dim3(nrhs), dim3(1024), 0, st, n, x, r, p, q, state, tol);
}

}  // namespace elmddm

// ---------------------------------------------------------------------------
// Matrix-free interface operator (Section 3, eq. schur, applied without
// forming S):  S v = sum_s R_s^T (I - T_s) R_s v + M^T M v, with T_s the
// Y^T Y block of the Schur products P_s and M given by its nonzero blocks
// M_{g,E} (flux edge g x value edge E), stored column-major mg x mg
// (element (p, r) at r * mg + p) and, for M^T, transposed.
// ---------------------------------------------------------------------------
namespace elmddm {

// t_s = v_s - T_s v_s with v_s = v[gidx_s] (zero for unused slots); one
// workgroup per subdomain of the batch, v_s staged in LDS, one wave per row
// block of T_s (lanes along the contiguous column index).
__global__ __launch_bounds__(256) void mf_tpart_kernel(int kpad, const double* P, int ldp, long long sP,
                                                       const int32_t* gidx, const double* v, long long nG,
                                                       double* t, long long sT, int ngeo, bool shared)
{
    extern __shared__ double vs[];
    const int s = blockIdx.x;
    const int sg = s % ngeo;
    const long long inst = s / ngeo;
    v += inst * nG;
    // one operator per instance, or one shared by all right-hand sides
    const double* Ps = P + (shared ? sg : s) * sP;
    for (int i = threadIdx.x; i < kpad; i += blockDim.x) {
        const int gi = gidx[(long long)sg * kpad + i];
        vs[i] = gi >= 0 ? v[gi] : 0.0;
    }
    __syncthreads();
    // T is symmetric: (T v)[r] = sum_j T[j][r] v[j], column r of T contiguous
    const int lane = threadIdx.x & 63;
    for (int r = threadIdx.x >> 6; r < kpad; r += blockDim.x >> 6) {
        const double* col = Ps + (long long)r * ldp;
        double acc = 0.0;
        for (int j = lane; j < kpad; j += 64) acc += col[j] * vs[j];
        acc = wave_sum(acc);
        if (lane == 0) t[s * sT + r] = vs[r] - acc;
    }
}

void mf_tpart(hipStream_t st, int NT, int ngeo, int kpad, const double* P, int ldp, long long sP,
              const int32_t* gidx, const double* v, long long nG, double* t, long long sT, bool shared)
{
    if (kpad <= 0) return;
    hipLaunchKernelGGL(mf_tpart_kernel, dim3(NT), dim3(256), kpad * sizeof(double), st, kpad, P, ldp, sP, gidx,
                       v, nG, t, sT, ngeo, shared);
}


}  // namespace elmddm

namespace elmddm {

// MbT[b][p * mg + r] = Mb[b][r * mg + p]: the M blocks transposed, so that
// M^T w reads them with consecutive lanes on consecutive addresses.
__global__ __launch_bounds__(256) void transpose_blocks_kernel(int mg, const double* Mb, double* MbT)
{
    __shared__ double tile[64][65];
    const long long b = blockIdx.x;
    const int mm = mg * mg;
    const double* src = Mb + b * mm;
    double* dst = MbT + b * mm;
    for (int i = threadIdx.x; i < mm; i += 256) tile[i / mg][i % mg] = src[i];
    __syncthreads();
    for (int i = threadIdx.x; i < mm; i += 256) dst[i] = tile[i % mg][i / mg];
}

void transpose_blocks(hipStream_t st, long long nblocks, int mg, const double* Mb, double* MbT)
{
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(transpose_blocks_kernel, dim3((unsigned)nblocks), dim3(256), 0, st, mg, Mb, MbT);
}

// w_g = -sum_{E in adj(g)} M_{g,E} v_E: four waves per flux edge share its
// blocks, lane p accumulates row p, the waves' partial sums meet in LDS.
__global__ __launch_bounds__(256) void mf_mv4_kernel(int mg, const int32_t* mstart, const int32_t* mE,
                                                     const double* Mbuf, long long sM, const double* v,
                                                     long long nG, double* w, long long sW)
{
    __shared__ double part[4][64];
    const int g = blockIdx.x;
    const long long inst = blockIdx.y;
    Mbuf += inst * sM;
    v += inst * nG;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int mm = mg * mg;
    double acc = 0.0;
    if (lane < mg)
        for (int it = mstart[g] + wv; it < mstart[g + 1]; it += 4) {
            const double* Mb = Mbuf + (long long)it * mm;
            const double* vE = v + (long long)mE[it] * mg;
            for (int r = 0; r < mg; ++r) acc += Mb[(long long)r * mg + lane] * vE[r];
        }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < mg)
        w[inst * sW + (long long)g * mg + lane] = -(part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
}

// y_E = sum over the owners o of E of t_o[slot + r] - sum_{(b, g) in gl(E)} M_b^T w_g
// (w holds -M v, so this is (I - T) v + M^T M v for the edge): four waves per
// value edge share its blocks (transposed copies: coalesced), LDS reduction.
__global__ __launch_bounds__(256) void mf_mtv4_kernel(int mg, const int32_t* qdesc, const int32_t* gptr,
                                                      const int32_t* gdesc, const double* t, int kpad,
                                                      const double* MbT, long long sM, const double* w,
                                                      long long sW, double* y, long long nG, int ngeo,
                                                      bool shared_t)
{
    __shared__ double part[4][64];
    const int E = blockIdx.x;
    const long long inst = blockIdx.y;
    MbT += inst * sM;
    w += inst * sW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int mm = mg * mg;
    double acc = 0.0;
    if (lane < mg)
        for (int it = gptr[E] + wv; it < gptr[E + 1]; it += 4) {
            const double* Mb = MbT + (long long)gdesc[2 * it] * mm;
            const double* wg = w + (long long)gdesc[2 * it + 1] * mg;
            for (int p = 0; p < mg; ++p) acc += Mb[(long long)p * mg + lane] * wg[p];
        }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && lane < mg) {
        double v = -(part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
        const int32_t* q = qdesc + 4 * E;
        for (int k = 0; k < 2; ++k) {
            const int s = q[2 * k];
            if (s < 0) continue;
            v += t[(inst * ngeo + s) * (long long)kpad + q[2 * k + 1] + lane];
        }
        y[inst * nG + (long long)E * mg + lane] = v;
    }
    (void)shared_t;
}

void mf_mv4(hipStream_t st, int nE, int mg, const int32_t* mstart, const int32_t* mE, const double* Mbuf,
            long long sM, const double* v, long long nG, double* w, long long sW, int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(mf_mv4_kernel, dim3(nE, ninst), dim3(256), 0, st, mg, mstart, mE, Mbuf, sM, v, nG, w, sW);
}

void mf_mtv4(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr, const int32_t* gdesc,
             const double* t, int kpad, const double* MbT, long long sM, const double* w, long long sW, double* y,
             long long nG, int ngeo, int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(mf_mtv4_kernel, dim3(nE, ninst), dim3(256), 0, st, mg, qdesc, gptr, gdesc, t, kpad, MbT, sM,
                       w, sW, y, nG, ngeo, false);
}

}  // namespace elmddm

// ---------------------------------------------------------------------------
// Block-Jacobi preconditioner of the interface system: the diagonal edge
// blocks S_EE = sum_{owners s} (I - T_s[E, E]) + sum_{g: E in adj(g)}
// M_{g,E}^T M_{g,E} (mg x mg), factored by the 64 x 64 diagonal Cholesky
// kernel, applied as z_E = L_E^{-T} L_E^{-1} r_E.  PCG recurrences with the
// state {rz, bb, done, iterations, rr} per system.
// ---------------------------------------------------------------------------
namespace elmddm {

__global__ __launch_bounds__(256) void mf_diag_blocks_kernel(int mg, const int32_t* qdesc, const int32_t* gptr,
                                                             const int32_t* gdesc, const double* P, int ldp,
                                                             long long sP, const double* Mbuf, long long sM,
                                                             double* D, int ngeo, int nE)
{
    __shared__ double Mb[64][65];
    const int E = blockIdx.x;
    const long long inst = blockIdx.y;
    P += inst * ngeo * sP;
    Mbuf += inst * sM;
    double* De = D + (inst * nE + E) * 4096LL;
    const int mm = mg * mg;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    // owners: I - T_s on the edge's slots
    const int32_t* q4 = qdesc + 4 * E;
    for (int k = 0; k < 2; ++k) {
        const int s = q4[2 * k];
        if (s < 0) continue;
        const int slot = q4[2 * k + 1];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int idx = threadIdx.x + 256 * q;
            const int r = idx & 63, c = idx >> 6;
            if (r < mg && c < mg)
                acc[q] += (r == c ? 1.0 : 0.0) - P[s * sP + (long long)(slot + c) * ldp + slot + r];
        }
    }
    // M^T M on the edge: D[r][c] += sum_p M[p][r] M[p][c]
    for (int it = gptr[E]; it < gptr[E + 1]; ++it) {
        const double* M = Mbuf + (long long)gdesc[2 * it] * mm;
        __syncthreads();
        for (int i = threadIdx.x; i < mm; i += 256) Mb[i / mg][i % mg] = M[i];   // Mb[r][p] = M(p, r)
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int idx = threadIdx.x + 256 * q;
            const int r = idx & 63, c = idx >> 6;
            if (r < mg && c < mg) {
                double v = 0.0;
                for (int p = 0; p < mg; ++p) v += Mb[r][p] * Mb[c][p];
                acc[q] += v;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int idx = threadIdx.x + 256 * q;
        const int r = idx & 63, c = idx >> 6;
        De[idx] = (r < mg && c < mg) ? acc[q] : (r == c ? 1.0 : 0.0);
    }
}

void mf_diag_blocks(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr, const int32_t* gdesc,
                    const double* P, int ldp, long long sP, const double* Mbuf, long long sM, double* D, int ngeo,
                    int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(mf_diag_blocks_kernel, dim3(nE, ninst), dim3(256), 0, st, mg, qdesc, gptr, gdesc, P, ldp, sP,
                       Mbuf, sM, D, ngeo, nE);
}

// z_E = L^{-T} (L^{-1} r_E) with L^{-1} = Dinv (64 x 64 column-major, lower)
__global__ __launch_bounds__(64) void mf_bjacobi_kernel(int mg, int nE, const double* Dinv, long long sD,
                                                        const double* r, double* z, long long nG)
{
    __shared__ double Li[64][65];
    __shared__ double y[64];
    const int E = blockIdx.x;
    const long long inst = blockIdx.y;
    const double* Di = Dinv + inst * sD + (long long)E * 4096;
    const int i = threadIdx.x;
    for (int k = 0; k < 64; ++k) Li[i][k] = Di[k * 64 + i];   // Li[i][k] = L^{-1}(i, k)
    const double* rE = r + inst * nG + (long long)E * mg;
    __syncthreads();
    double acc = 0.0;
    if (i < mg)
        for (int k = 0; k <= i; ++k) acc += Li[i][k] * rE[k];
    y[i] = acc;
    __syncthreads();
    if (i < mg) {
        double v = 0.0;
        for (int k = i; k < mg; ++k) v += Li[k][i] * y[k];
        z[inst * nG + (long long)E * mg + i] = v;
    }
}

void mf_bjacobi(hipStream_t st, int nE, int mg, const double* Dinv, long long sD, const double* r, double* z,
                long long nG, int ninst)
{
    if (nE <= 0) return;
    hipLaunchKernelGGL(mf_bjacobi_kernel, dim3(nE, ninst), dim3(64), 0, st, mg, nE, Dinv, sD, r, z, nG);
}

// r = b - q (q = S x); rr = r.r, bb = b.b
__global__ __launch_bounds__(1024) void pcg_init1_kernel(int n, const double* b, const double* q, double* r,
                                                         double* state)
{
    __shared__ double red[16];
    const long long o = (long long)blockIdx.x * n;
    double rr = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double ri = b[o + i] - q[o + i];
        r[o + i] = ri;
        rr += ri * ri;
        bb += b[o + i] * b[o + i];
    }
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        double* s = state + 8 * blockIdx.x;
        s[1] = bb;
        s[4] = rr;
        s[3] = 0.0;
    }
}

// p = z; rz = r.z; done if rr <= tol^2 bb
__global__ __launch_bounds__(1024) void pcg_init2_kernel(int n, const double* r, const double* z, double* p,
                                                         double* state, double tol)
{
    __shared__ double red[16];
    const long long o = (long long)blockIdx.x * n;
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        p[o + i] = z[o + i];
        rz += r[o + i] * z[o + i];
    }
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        double* s = state + 8 * blockIdx.x;
        s[0] = rz;
        s[2] = (s[4] <= tol * tol * s[1]) ? 1.0 : 0.0;
    }
}

// alpha = rz / p.q; x += alpha p; r -= alpha q; rr = r.r; done if rr <= tol^2 bb
__global__ __launch_bounds__(1024) void pcg_step1_kernel(int n, double* x, double* r, const double* p,
                                                         const double* q, double* state, double tol)
{
    __shared__ double red[16];
    double* s = state + 8 * blockIdx.x;
    if (s[2] != 0.0) return;
    const long long o = (long long)blockIdx.x * n;
    double pq = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) pq += p[o + i] * q[o + i];
    pq = block_sum(pq, red);
    const double alpha = pq > 0.0 ? s[0] / pq : 0.0;
    double rr = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[o + i] += alpha * p[o + i];
        const double ri = r[o + i] - alpha * q[o + i];
        r[o + i] = ri;
        rr += ri * ri;
    }
    rr = block_sum(rr, red);
    __syncthreads();
    if (threadIdx.x == 0) {
        s[4] = rr;
        s[3] += 1.0;
        if (!(pq > 0.0)) s[2] = 2.0;
        else if (rr <= tol * tol * s[1]) s[2] = 1.0;
    }
}

// rz' = r.z; beta = rz'/rz; p = z + beta p
__global__ __launch_bounds__(1024) void pcg_step2_kernel(int n, const double* r, const double* z, double* p,
                                                         double* state)
{
    __shared__ double red[16];
    double* s = state + 8 * blockIdx.x;
    if (s[2] != 0.0) return;
    const long long o = (long long)blockIdx.x * n;
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) rz += r[o + i] * z[o + i];
    rz = block_sum(rz, red);
    const double beta = s[0] > 0.0 ? rz / s[0] : 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[o + i] = z[o + i] + beta * p[o + i];
    __syncthreads();
    if (threadIdx.x == 0) s[0] = rz;
}

void pcg_init1(hipStream_t st, int n, const double* b, const double* q, double* r, double* state, int nrhs)
{
    hipLaunchKernelGGL(pcg_init1_kernel, dim3(nrhs), dim3(1024), 0, st, n, b, q, r, state);
}
void pcg_init2(hipStream_t st, int n, const double* r, const double* z, double* p, double* state, double tol, int nrhs)
{
    hipLaunchKernelGGL(pcg_init2_kernel, dim3(nrhs), dim3(1024), 0, st, n, r, z, p, state, tol);
}
void pcg_step1(hipStream_t st, int n, double* x, double* r, const double* p, const double* q, double* state,
               double tol, int nrhs)
{
    hipLaunchKernelGGL(pcg_step1_kernel, dim3(nrhs), dim3(1024), 0, st, n, x, r, p, q, state, tol);
}
void pcg_step2(hipStream_t st, int n, const double* r, const double* z, double* p, double* state, int nrhs)
{
    hipLaunchKernelGGL(pcg_step2_kernel, dim3(nrhs), dim3(1024), 0, st, n, r, z, p, state);
}

}  // namespace elmddm
