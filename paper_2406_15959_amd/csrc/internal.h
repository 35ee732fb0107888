// Internal interfaces between the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace elmddm {

// Set the message returned by elmddm_last_error() on this thread; returns status.
int record_error(int status, const char* msg);

// Row kinds of the per-subdomain row table (one entry per row of X).
enum RowKind : int32_t {
    ROW_ZERO = 0,       // padding row: all zero
    ROW_INTERIOR = 1,   // operator row L phi at an interior point, rhs = f
    ROW_BOUNDARY = 2,   // value row phi at a Dirichlet point, rhs = g
    ROW_IFC_VALUE = 3,  // value row phi at an interface point, rhs = 0
    ROW_FLUX = 4        // outward normal derivative at an interface point, rhs = 0
};

struct RowTable {
    const double* x;      // [N][ldx] physical coordinates
    const double* y;
    const double* nx;     // outward normal (flux rows)
    const double* ny;
    const int32_t* kind;  // RowKind
    const int32_t* src;   // index into f (interior: s*q2 + i) or g (boundary)
    const int32_t* cmap;  // compact row: >= 0 row of K^s, <= -2 row (-2 - cmap) of A^s, -1 none
};

struct SubGeom {
    const double* cx;     // [N] box centre
    const double* cy;
    double sx, sy;        // chain-rule factors 2/h_x, 2/h_y
};

// Device status record written by kernels.
struct DevInfo {
    int32_t status;
    int32_t bad_subdomain;
    int32_t bad_pass;
    int32_t pad;
};

// ---- launchers (kernels.hip) ----

// C = alpha * op(A) * op(B) + beta * C for a batch of column-major matrices.
// op(A) is M x K (ta: A stored K x M), op(B) is K x N (tb: B stored N x K).
// kmode 0: full K range; 1: op(B)(k, j) == 0 for k < j (skip k below the tile's first column);
// 2: op(B)(k, j) == 0 for k > j (stop at the tile's last column).
// lower: only output tiles on or below the diagonal (M, N share the tile grid).
void gemm_f64(hipStream_t st, bool ta, bool tb, int kmode, bool lower, int M, int N, int K,
              double alpha, const double* A, int lda, long long sA, const double* B, int ldb,
              long long sB, double beta, double* C, int ldc, long long sC, int batch);
// Kernel variant for large (which = 0, >= 2^30 multiply-adds) or small (1) products:
// bit 1 = K depth 32 instead of 16, bit 0 = XCD-aware tile order.
void set_gemm_variant(int which, int v);

// Strip-tiled MFMA products (tile 16 T x 16 T, T waves); strip_width picks T for n.
int strip_width(int n);
// Kernel choice for the large local products: code < 0 selects the 64 x 64
// kernel variant (-1 - code), code >= 4 the strip kernel of that width.
void gram_product(hipStream_t st, int code, int n, int rows, const double* X, int ldx, long long sX,
                  double* G, int ldg, long long sG, int batch);
void trsm_product(hipStream_t st, int code, int rows, int n, const double* X, int ldx, long long sX,
                  const double* Linv, int ldl, long long sL, double* Y, long long sY, int batch);
// G = X^T X (lower triangle) over `rows` rows and n columns of every X in the batch.
// Gram product in FP32 (operands rounded to FP32, FP32 accumulation on the
// matrix cores), lower triangle written as FP64.
void gram_product_f32(hipStream_t st, int n, int rows, const double* X, int ldx, long long sX,
                      double* G, int ldg, long long sG, int batch);
void gram_strip(hipStream_t st, int T, int n, int rows, const double* X, int ldx, long long sX,
                double* G, int ldg, long long sG, int batch);
// Y = X Linv^T for Linv lower triangular (n x n); X, Y: rows x n, leading dimension ldx.
void trsm_strip(hipStream_t st, int T, int rows, int n, const double* X, int ldx, long long sX,
                const double* Linv, int ldl, long long sL, double* Y, long long sY, int batch);
void strip_gemm_nn(hipStream_t st, int T, int M, int N, int K, const double* A, int lda,
                   const double* B, int ldb, double* C, int ldc);

// Writes X (plan layout, ldx rows x (n+1) columns per subdomain) or, if Kout != nullptr,
// the compact K^s [n][ldK], A^s [n][ldD] and F^s [ldF] per subdomain.
// N counts the subdomains of the whole batch; subdomain s has geometry s % ngeo and
// belongs to instance s / ngeo (whose boundary data start at instance * nbnd).
void assemble(hipStream_t st, int N, int ngeo, long long nbnd, int ldx, int n, const RowTable& rows,
              const SubGeom& geom, int op, const double* W, const double* b, const double* f,
              const double* g, const double* coef, int q2, double* X, double* Fout, int ldF,
              double* Kout, int ldK, double* Dout, int ldD);

void scale_diag(hipStream_t st, double* A, int lda, long long sA, int n, double factor, int batch);

// Factor the jb x jb diagonal block at (j, j) in place (lower), write its inverse to
// Dinv (ld 64, stride sD) and, if Linv != nullptr, into Linv at (j, j).  A pivot
// that is not above tau * dsave[j + k] (the matrix's original diagonal entry;
// 0 if dsave is null) or not finite marks the matrix as not positive definite.
void potrf_diag(hipStream_t st, double* A, int lda, long long sA, int j, int jb, double* Dinv,
                long long sD, double* Linv, int ldl, long long sL, DevInfo* info, int pass,
                int batch, const double* dsave, long long sS, double tau, double* rhs,
                long long sR);
// Panel, trailing update and forward-substitution update of one envelope
// Cholesky step (see envelope_potrf); L tiles below the diagonal go to Lo.
void envelope_step(hipStream_t st, double* A, int lda, long long sA, double* Lo, int ldo,
                   long long sLo, int j, int jb, const double* Dinv, long long sD, int r1,
                   double* rhs, long long sR, int batch);
// Panel and forward-substitution update only (L tiles to Lo); pair with a trailing GEMM.
void envelope_panel(hipStream_t st, const double* A, int lda, long long sA, double* Lo, int ldo,
                    long long sLo, int j, int jb, const double* Dinv, long long sD, int r1,
                    double* rhs, long long sR, int batch);
// Backward substitution over a block row of br <= 256 rows (four 64-row sub-blocks).
void trsv_lower_t_block(hipStream_t st, const double* L, int ld, long long sL, int j0, int br,
                        int kbeg, const double* Dinv, long long sD, double* y, double* u,
                        long long sY, int batch);
void save_diag(hipStream_t st, const double* A, int lda, long long sA, int n, double* d,
               long long sS, int batch);

void copy_row(hipStream_t st, const double* src, int lds_, long long sS, double* dst, int ldd,
              long long sD, int count, int batch);

// The Schur-assembly kernels run over ninst problem instances; P holds ngeo
// subdomains per instance.
void schur_mblocks(hipStream_t st, int nblk, const int32_t* desc, const double* P, int ldp,
                   long long sP, int cbase, int mg, double* Mbuf, int ngeo, int ninst);
void schur_avec(hipStream_t st, int nE, const int32_t* desc, const double* P, int ldp, long long sP,
                int cbase, int acol, int mg, double* abuf, int ngeo, int ninst);
// S blocks and rhs are written at the permuted edge positions perm[E].
// nzb [nnz]: blocks E1 + E2 nE with T or M contributions (formed with
// LDS-staged products); zb [nz]: the other blocks (written as zeros).
void schur_sblocks(hipStream_t st, int nE, int mg, const int32_t* nzb, int nnz, const int32_t* zb, int nz,
                   const int32_t* tptr, const int32_t* tdesc, const int32_t* mptr, const int32_t* mdesc,
                   const double* P, int ldp, long long sP, const double* Mbuf, double* S, int lds_,
                   const int32_t* perm, int ngeo, long long sM, long long sS, int ninst);
void schur_rhs(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr,
               const int32_t* gdesc, const double* P, int ldp, long long sP, int qcol,
               const double* Mbuf, const double* abuf, double* rhs, int inc, const int32_t* perm,
               int ngeo, long long sM, long long sA, long long sR, int ninst);
void unpermute(hipStream_t st, int nE, int mg, const int32_t* perm, const double* up, double* u,
               int ninst);
void unpermute_matrix(hipStream_t st, int nE, int mg, const int32_t* perm, const double* Sp, int lds,
                      double* S);

void local_backsolve(hipStream_t st, int N, int ngeo, long long nG, int n, int kpad, const double* X,
                     int ldx, long long sX, int mI, int hrow, const int32_t* gidx, const double* u,
                     double* const* Linv, int npass, int ldg, long long sG, double* c, double* tmp1,
                     double* tmp2);

void eval_points(hipStream_t st, int npts, const double* xy, int nx, int ny, double x0, double x1,
                 double y0, double y1, int n, const double* W, const double* b, const double* c,
                 double* u);
void eval_points_grad(hipStream_t st, int npts, const double* xy, int nx, int ny, double x0, double x1,
                      double y0, double y1, int n, const double* W, const double* b, const double* c,
                      double* u, double* ux, double* uy);

constexpr int NB = 64;  // block size of the blocked Cholesky

// Blocked right-looking Cholesky of a batch of (Mrows x n) lower trapezoids
// (Mrows = n or n + 1; an extra last row r becomes r L^{-T}).  Writes the
// inverses of the 64 x 64 diagonal blocks to Dinv (stride sD per matrix) and,
// if Linv != nullptr, the inverse factor L^{-1} (strictly upper part untouched).
// Breakdown: a pivot at or below 64 n u times its original diagonal entry
// (saved into dsave, stride sS per matrix) is reported through info.
void blocked_potrf(hipStream_t st, double* A, int lda, long long sA, int Mrows, int n, double* Dinv,
                   long long sD, double* Linv, int ldl, long long sL, double* Tbuf, DevInfo* info,
                   int pass, int batch, double* dsave, long long sS,
                   double tau = -1.0);

// Cholesky of one n x n SPD matrix whose nonzeros lie inside a column
// envelope: rend[p] = one past the last row that may be nonzero in the
// columns of 64-wide panel p (nondecreasing).  Fill-in stays inside the
// envelope, so panel and trailing updates are restricted to it.  rhs (n) is
// overwritten by L^{-1} rhs (forward substitution fused with the panels).
// The strictly lower 64 x 64 tiles of L are written to Lo (ld ldo); the
// diagonal tiles stay in A and their inverses in Dinv.
// With a side stream and two events (unfused path only), each step updates
// just the next block column on st and runs the rest of its trailing update
// on st2, overlapped with the next diagonal factorisation and panel
// (lookahead); st waits for st2 before it returns.
void envelope_potrf(hipStream_t st, double* A, int lda, long long sA, double* Lo, int ldo,
                    long long sLo, int n, const int* rend, double* Dinv, long long sD, DevInfo* info,
                    int pass, double* dsave, double* rhs, long long sR, int batch, bool fused,
                    hipStream_t st2 = nullptr, hipEvent_t ev_fork = nullptr, hipEvent_t ev_join = nullptr);

void init_info(hipStream_t st, DevInfo* info);
void check_finite(hipStream_t st, const double* v, long long count, DevInfo* info);

// Further right-hand sides with cached factors.
void rhs_assemble(hipStream_t st, const RowTable& rows, int ldx, int nrows, int ldf, const double* f,
                  const double* g, int N, int nrhs, long long nf, long long nbnd, double* Fr);
void trsv_lower_block(hipStream_t st, const double* L, int ld, long long sL, int j0, int br, int r1,
                      const double* Dinv, long long sD, double* y, long long sY, int batch);
void backsolve_rhs_multi(hipStream_t st, int N, int n, int kpad, const double* X, int ldx, long long sX,
                         int mI, const int32_t* gidx, const double* u, long long nG, const double* H,
                         double* V, int nrhs);

// Conjugate gradients on the kept interface matrix.
void permute(hipStream_t st, int nE, int mg, const int32_t* perm, const double* u, double* up, int nrhs);
void band_symv(hipStream_t st, int n, const double* S, int lds, const int32_t* rb, const int32_t* re,
               const double* x, double* y, int nrhs);
void cg_init(hipStream_t st, int n, const double* b, const double* Sx, double* r, double* p, double* state,
             double tol, int nrhs);
void cg_step(hipStream_t st, int n, double* x, double* r, double* p, const double* q, double* state, double tol,
             int nrhs);

// Matrix-free interface operator pieces.
void mf_tpart(hipStream_t st, int NT, int ngeo, int kpad, const double* P, int ldp, long long sP,
              const int32_t* gidx, const double* v, long long nG, double* t, long long sT, bool shared);

void transpose_blocks(hipStream_t st, long long nblocks, int mg, const double* Mb, double* MbT);
void mf_mv4(hipStream_t st, int nE, int mg, const int32_t* mstart, const int32_t* mE, const double* Mbuf,
            long long sM, const double* v, long long nG, double* w, long long sW, int ninst);
void mf_mtv4(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr, const int32_t* gdesc,
             const double* t, int kpad, const double* MbT, long long sM, const double* w, long long sW, double* y,
             long long nG, int ngeo, int ninst);

// Block-Jacobi preconditioned CG on the interface system.
void mf_diag_blocks(hipStream_t st, int nE, int mg, const int32_t* qdesc, const int32_t* gptr, const int32_t* gdesc,
                    const double* P, int ldp, long long sP, const double* Mbuf, long long sM, double* D, int ngeo,
                    int ninst);
void mf_bjacobi(hipStream_t st, int nE, int mg, const double* Dinv, long long sD, const double* r, double* z,
                long long nG, int ninst);
void pcg_init1(hipStream_t st, int n, const double* b, const double* q, double* r, double* state, int nrhs);
void pcg_init2(hipStream_t st, int n, const double* r, const double* z, double* p, double* state, double tol, int nrhs);
void pcg_step1(hipStream_t st, int n, double* x, double* r, const double* p, const double* q, double* state,
               double tol, int nrhs);
void pcg_step2(hipStream_t st, int n, const double* r, const double* z, double* p, double* state, int nrhs);

}  // namespace elmddm
