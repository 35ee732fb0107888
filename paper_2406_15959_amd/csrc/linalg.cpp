// Blocked factorisation drivers built from the batched kernels.
#include <algorithm>

#include "internal.h"

namespace elmddm {

// Blocked right-looking Cholesky of a batch of (Mrows x n) lower trapezoids
// (Mrows = n or n + 1; an extra last row r is turned into r L^{-T}).  Writes
// the inverses of the 64 x 64 diagonal blocks to Dinv and, if Linv is given,
// the full inverse factor L^{-1} (strictly upper part left untouched).
void blocked_potrf(hipStream_t st, double* A, int lda, long long sA, int Mrows, int n, double* Dinv,
                   long long sD, double* Linv, int ldl, long long sL, double* Tbuf, DevInfo* info,
                   int pass, int batch, double* dsave, long long sS, double tau)
{
    if (tau < 0.0) tau = 64.0 * n * 0x1p-53;
    if (dsave) save_diag(st, A, lda, sA, n, dsave, sS, batch);
    // Block columns are taken in pairs [j, j2) and [j2, j3): the panel of the
    // first updates only the second block column, and one rank-(jb + jb2)
    // update with both panels then brings the trailing matrix [j3, Mrows) x
    // [j3, n) up to date: the trailing matrix is read and written once per
    // 128 columns instead of once per 64.
    auto factor_block = [&](int j, int jb) {   // diagonal block, then its panel rows [j + jb, Mrows)
        double* Dj = Dinv + (long long)(j / NB) * NB * NB;
        potrf_diag(st, A, lda, sA, j, jb, Dj, sD, Linv, ldl, sL, info, pass, batch, dsave, sS, tau,
                   nullptr, 0);
        const int Mb = Mrows - j - jb;
        if (Mb > 0) {
            double* panel = A + (long long)j * lda + (j + jb);
            gemm_f64(st, false, true, 0, false, Mb, jb, jb, 1.0, panel, lda, sA, Dj, NB, sD, 0.0,
                     panel, lda, sA, batch);
        }
    };
    for (int j = 0; j < n; j += 2 * NB) {
        const int jb = std::min(NB, n - j);
        factor_block(j, jb);
        const int j2 = j + jb;
        const int jb2 = std::min(NB, n - j2);
        if (jb2 <= 0) break;
        // block column j2, rows [j2, Mrows): A -= L[., j:j2] L[j2:j2+jb2, j:j2]^T
        const double* L1 = A + (long long)j * lda + j2;
        gemm_f64(st, false, true, 0, false, Mrows - j2, jb2, jb, -1.0, L1, lda, sA, L1, lda, sA, 1.0,
                 A + (long long)j2 * lda + j2, lda, sA, batch);
        factor_block(j2, jb2);
        const int j3 = j2 + jb2;
        if (j3 < n) {
            const double* L12 = A + (long long)j * lda + j3;   // rows [j3, Mrows) of block columns j, j2
            gemm_f64(st, false, true, 0, true, Mrows - j3, n - j3, jb + jb2, -1.0, L12, lda, sA, L12, lda,
                     sA, 1.0, A + (long long)j3 * lda + j3, lda, sA, batch);
        }
    }
    if (!Linv) return;
    // L^{-1}, block row by block row: Linv[I, 0:i] = -Dinv_I (L[I, 0:i] Linv[0:i, 0:i]).
    for (int i = NB; i < n; i += NB) {
        const int ib = std::min(NB, n - i);
        gemm_f64(st, false, false, 1, false, ib, i, i, 1.0, A + i, lda, sA, Linv, ldl, sL, 0.0, Tbuf,
                 NB, (long long)NB * n, batch);
        gemm_f64(st, false, false, 0, false, ib, i, ib, -1.0, Dinv + (long long)(i / NB) * NB * NB,
                 NB, sD, Tbuf, NB, (long long)NB * n, 0.0, Linv + i, ldl, sL, batch);
    }
}

void envelope_potrf(hipStream_t st, double* A, int lda, long long sA, double* Lo, int ldo,
                    long long sLo, int n, const int* rend, double* Dinv, long long sD, DevInfo* info,
                    int pass, double* dsave, double* rhs, long long sR, int batch, bool fused,
                    hipStream_t st2, hipEvent_t ev_fork, hipEvent_t ev_join)
{
    const double tau = 64.0 * n * 0x1p-53;
    const bool look = !fused && st2 && ev_fork && ev_join;
    bool pending = false;   // a trailing update of the previous step is running on st2
    if (dsave) save_diag(st, A, lda, sA, n, dsave, n, batch);
    for (int j = 0, p = 0; j < n; j += NB, ++p) {
        const int jb = std::min(NB, n - j);
        double* Dj = Dinv + (long long)p * NB * NB;
        const int r1 = std::min(n, rend[p]);
        // Block column p is final here: the previous step updated it on st,
        // and every earlier side-stream update was joined before that.
        potrf_diag(st, A, lda, sA, j, jb, Dj, sD, nullptr, 0, 0, info, pass, batch, dsave, n, tau, rhs,
                   sR);
        if (fused) {
            // one launch: latency-optimal for a few matrices (panel tiles recomputed per pair)
            envelope_step(st, A, lda, sA, Lo, ldo, sLo, j, jb, Dj, sD, r1, rhs, sR, batch);
            continue;
        }
        // panel, then the trailing GEMM: throughput-optimal for many matrices
        envelope_panel(st, A, lda, sA, Lo, ldo, sLo, j, jb, Dj, sD, r1, rhs, sR, batch);
        const int Mb = r1 - j - jb;
        const double* Lp = Lo + (long long)j * ldo + j + jb;
        double* Tr = A + (long long)(j + jb) * lda + (j + jb);
        if (!look) {
            if (Mb > 0)
                gemm_f64(st, false, true, 0, true, Mb, Mb, jb, -1.0, Lp, ldo, sLo, Lp, ldo, sLo, 1.0, Tr, lda, sA,
                         batch);
            continue;
        }
        // The previous step's side-stream update also wrote the next block
        // column: wait for it before touching that column.
        if (pending) {
            (void)hipStreamWaitEvent(st, ev_join, 0);
            pending = false;
        }
        if (Mb <= 0) continue;
        const int na = std::min(NB, Mb);
        // next block column (all its rows), on st: the next step needs it first
        gemm_f64(st, false, true, 0, false, Mb, na, jb, -1.0, Lp, ldo, sLo, Lp, ldo, sLo, 1.0, Tr, lda, sA, batch);
        const int Mr = Mb - na;
        if (Mr > 0) {
            // the rest of the trailing matrix (lower part), on st2
            (void)hipEventRecord(ev_fork, st);
            (void)hipStreamWaitEvent(st2, ev_fork, 0);
            gemm_f64(st2, false, true, 0, true, Mr, Mr, jb, -1.0, Lp + na, ldo, sLo, Lp + na, ldo, sLo, 1.0,
                     Tr + (long long)na * lda + na, lda, sA, batch);
            (void)hipEventRecord(ev_join, st2);
            pending = true;
        }
    }
    if (pending) (void)hipStreamWaitEvent(st, ev_join, 0);
}

}  // namespace elmddm
