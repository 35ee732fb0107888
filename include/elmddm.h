/*
 * elmddm -- nonoverlapping domain decomposition for extreme learning machines
 * (one-hidden-layer tanh networks, one per subdomain) on a single AMD MI355X
 * (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The method (paper, Section 3 and Algorithm 1): for
 *     L u = f in the rectangle [x0,x1] x [y0,y1],   u = g on its boundary
 * (Section 2, eq. pde; L = -Laplace or L u = -div(a grad u), Section 4.2), the
 * rectangle is split into nsub_x x nsub_y equal boxes.  Each box s carries a
 * network u_s(x) = sum_j c_j tanh(w_j . xhat + b_j) with fixed random hidden
 * parameters (w_j, b_j) acting on box-local coordinates
 * xhat = 2 (x - x_center)/h_x, yhat = 2 (y - y_center)/h_y  in [-1, 1]^2.
 * The local least-squares blocks K^s, A^s, B^s, F^s (eq. nonoverlap_discrete)
 * are coupled through one auxiliary unknown u_Gamma per interface point; the
 * library eliminates the output-layer coefficients c, solves the interface
 * Schur complement system (eq. schur) for u_Gamma, and back-solves every
 * K^{sT} K^s c^s = K^{sT} (F^s - B^s u_Gamma).
 *
 * Point layout (the paper leaves it open; this is the library's reading):
 *  - interior points: cell-centred q_x x q_y grid per box, row-major (y outer);
 *  - every box edge carries points at the midpoints (k + 1/2)/m of m equal
 *    pieces: m_bdry_edge Dirichlet points on an outer edge, m_ifc_edge
 *    interface points on an edge shared by two boxes; box corners carry none,
 *    so every interface point has exactly two owners and one flux row;
 *  - boxes are numbered s = sy * nsub_x + sx; per box the edges are visited
 *    bottom, right, top, left;
 *  - interface numbering: all vertical interface edges (edge row outer,
 *    x inner), then all horizontal ones; points along an edge by increasing
 *    coordinate.
 *
 * Memory: every device pointer is caller-owned device memory on the current
 * HIP device, float64 unless stated.  A plan owns its own device workspace,
 * allocated by elmddm_plan_create and released by elmddm_plan_destroy; no
 * solve call allocates.  Every device call is enqueued on the caller's HIP
 * stream (hipStream_t passed as void*, NULL = default stream) and returns
 * after enqueueing; results are valid after the stream is synchronised.  A
 * plan may be used by one stream at a time.
 *
 * Errors: functions return an elmddm_status.  Argument errors are detected
 * on the host before anything is enqueued.  Numerical failures found on the
 * device (a local Gram block or the Schur matrix not positive definite: a
 * Cholesky pivot at or below 64 n u times its original diagonal entry,
 * non-finite values) are recorded in the plan and returned by
 * elmddm_solve_info after synchronisation.  elmddm_last_error() gives a
 * human-readable message for the last failing call on the calling thread.
 */
#ifndef ELMDDM_H
#define ELMDDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum elmddm_status {
    ELMDDM_OK = 0,
    ELMDDM_INVALID_ARG = 1,
    ELMDDM_OOM = 2,
    ELMDDM_NOT_SPD = 3,        /* a local Gram matrix lost positive definiteness */
    ELMDDM_SCHUR_NOT_SPD = 4,  /* the interface Schur matrix lost positive definiteness */
    ELMDDM_NOT_CONVERGED = 5,
    ELMDDM_NONFINITE = 6,
    ELMDDM_HIP_ERROR = 7,
    ELMDDM_UNSUPPORTED = 8
} elmddm_status;

enum { ELMDDM_OP_POISSON = 0, ELMDDM_OP_VARCOEF = 1 };

/* Plan flags (elmddm_plan_create_ex). */
enum { ELMDDM_PLAN_MATRIX_FREE = 1, ELMDDM_PLAN_DENSE = 2 };

/* Precision modes (see elmddm_plan_set_mode). */
enum { ELMDDM_MODE_FP64 = 0, ELMDDM_MODE_MIXED = 1 };

enum {
    ELMDDM_POINTS_INTERIOR = 0,   /* nsub * q_x * q_y points, box-major          */
    ELMDDM_POINTS_BOUNDARY = 1,   /* all Dirichlet points, box-major, local order */
    ELMDDM_POINTS_INTERFACE = 2   /* n_interface points, global interface order   */
};

/* Problem statement (Section 2, eq. pde, and Section 3): domain, operator,
 * partition, neurons and collocation points per subdomain. */
typedef struct elmddm_problem {
    double x0, x1, y0, y1;   /* the rectangle                                   */
    int32_t nsub_x, nsub_y;  /* subdomain grid                                  */
    int32_t neurons;         /* hidden neurons per local network (n_N), >= 1    */
    int32_t q_x, q_y;        /* interior collocation grid per subdomain         */
    int32_t m_bdry_edge;     /* Dirichlet points per outer edge, >= 1           */
    int32_t m_ifc_edge;      /* interface points per interface edge, >= 1      */
    int32_t op;              /* ELMDDM_OP_POISSON or ELMDDM_OP_VARCOEF          */
} elmddm_problem;

/* Sizes derived from a problem (filled by elmddm_plan_sizes). */
typedef struct elmddm_sizes {
    int32_t nsub;            /* number of subdomains N                          */
    int32_t batch;           /* problem instances per solve                     */
    int32_t neurons;         /* n_N                                             */
    int32_t n_interior;      /* interior points per subdomain (q_x * q_y)       */
    int32_t n_interface;     /* interface unknowns nG                           */
    int64_t n_boundary;      /* Dirichlet points over all subdomains            */
    int32_t max_rows;        /* largest local row count m_s                     */
    int32_t max_ifc;         /* largest local interface count k_s               */
    uint64_t device_bytes;   /* device memory owned by the plan                 */
} elmddm_sizes;

/* Per-solve diagnostics (filled by elmddm_solve_info). */
typedef struct elmddm_info {
    int32_t status;          /* elmddm_status of the last solve                 */
    int32_t bad_subdomain;   /* first subdomain whose local factorisation failed, else -1 */
    int32_t bad_pass;        /* CholeskyQR pass (1..5) of that failure, else 0  */
    int32_t bad_instance;    /* problem instance of that failure, else -1       */
} elmddm_info;

typedef struct elmddm_plan elmddm_plan;

/* Validate the problem, build the point layout and interface maps on the host
 * and allocate the plan's device workspace on the current device.
 * Requires q_x * q_y >= neurons (the Proposition of Section 3 needs at least
 * as many interior points as neurons per subdomain); otherwise INVALID_ARG.
 * On failure *plan is set to NULL. */
elmddm_status elmddm_plan_create(const elmddm_problem* problem, elmddm_plan** plan);

/* As elmddm_plan_create, for `batch` independent instances of the same
 * problem geometry solved together: every per-instance argument of
 * elmddm_solve gains a leading [batch] dimension (W [batch][nsub][neurons][2],
 * b, f, g, coef [3][batch][nsub][q_x*q_y], u_gamma [batch][n_interface],
 * c [batch][nsub][neurons]).  All stages run over the whole batch in the same
 * launches.  elmddm_plan_create is elmddm_plan_create_batch with batch = 1.
 * elmddm_assemble writes all batch * nsub subdomains; elmddm_get_schur
 * returns instance 0.  batch * nsub may be at most 65535 (INVALID_ARG
 * beyond): the subdomains of a batch are a grid dimension of the launches. */
elmddm_status elmddm_plan_create_batch(const elmddm_problem* problem, int32_t batch,
                                       elmddm_plan** plan);

/* As elmddm_plan_create_batch, with the interface-solver choice:
 *  ELMDDM_PLAN_DENSE: S is formed and factored (envelope Cholesky, exact);
 *  ELMDDM_PLAN_MATRIX_FREE: S is never formed; the interface system is solved
 *    by CG (the paper's interface solver, Section 3) with S v applied from
 *    the per-subdomain blocks T_s = Y_s^T Y_s and the nonzero blocks of M
 *    (memory O(sum_s k_s^2) instead of O(nG^2)).  elmddm_solve then runs CG
 *    to ||g - S u|| <= tol ||g|| (elmddm_plan_set_cg; default tol 1e-12,
 *    100000 iterations) and synchronises the stream while it polls the
 *    convergence flags every 32 iterations; NOT_CONVERGED is reported by
 *    elmddm_solve_info.  Matrix-free plans cannot be captured into graphs and
 *    keep no S.
 *  0: dense unless the three nG x nG arrays of the dense path would exceed
 *    64 GB (the 32 x 32 case with 64 points per edge needs 387 GB). */
elmddm_status elmddm_plan_create_ex(const elmddm_problem* problem, int32_t batch, uint32_t flags,
                                    elmddm_plan** plan);

/* 1 if the plan solves the interface system matrix-free, else 0. */
int32_t elmddm_plan_is_matrix_free(const elmddm_plan* plan);

/* CG stopping rule of matrix-free plans: ||g - S u|| <= tol ||g|| (0 < tol < 1),
 * at most maxit iterations. */
elmddm_status elmddm_plan_set_cg(elmddm_plan* plan, double tol, int32_t maxit);

/* Preconditioner of that CG: 1 (default) block-Jacobi on the interface edges
 * (each mg x mg diagonal block S_EE = sum over the edge's two owners of
 * I - T_s[E, E] plus sum_g M_{g,E}^T M_{g,E}, Cholesky-factored in the
 * solve), 0 none (the paper's plain CG). */
elmddm_status elmddm_plan_set_cg_precond(elmddm_plan* plan, int32_t kind);

/* Iterations and final relative residuals (recurrence) of the last CG run on a
 * matrix-free plan, per instance (host arrays of batch entries). */
elmddm_status elmddm_plan_cg_stats(const elmddm_plan* plan, int32_t* iters, double* relres);

/* Sizes (including device_bytes) that elmddm_plan_create_batch would give,
 * computed on the host without allocating anything. */
elmddm_status elmddm_plan_query(const elmddm_problem* problem, int32_t batch, elmddm_sizes* sizes);

/* Release the plan and its device memory.  NULL is accepted. */
elmddm_status elmddm_plan_destroy(elmddm_plan* plan);

elmddm_status elmddm_plan_sizes(const elmddm_plan* plan, elmddm_sizes* sizes);

/* Host copy of the plan's points of one kind (see ELMDDM_POINTS_*), as
 * interleaved (x, y) pairs in the documented order.  capacity is the number
 * of points xy can hold; fails with INVALID_ARG if too small.  Callers use
 * these points to sample f, g and the coefficient a. */
elmddm_status elmddm_points(const elmddm_plan* plan, int32_t kind, double* xy, int64_t capacity);

/* Algorithm 1 (Section 3) end to end on the device:
 *   W     [nsub][neurons][2]  hidden weights (w_x, w_y) on box-local coordinates
 *   b     [nsub][neurons]     hidden biases
 *   f     [nsub][q_x*q_y]     source at the interior points (ELMDDM_POINTS_INTERIOR order)
 *   g     [n_boundary]        Dirichlet data at the boundary points (ELMDDM_POINTS_BOUNDARY order)
 *   coef  [3][nsub][q_x*q_y]  a, da/dx, da/dy at the interior points (VARCOEF only; else NULL)
 *   u_gamma [n_interface]     output: interface variable
 *   c     [nsub][neurons]     output: output-layer coefficients of every local network
 * Local least squares: shifted CholeskyQR (3 or 4 passes, see
 * elmddm_plan_set_passes) in float64 (Gram by
 * MFMA, Cholesky, triangular solves); interface system: dense float64
 * Cholesky.  Enqueued on stream; check elmddm_solve_info afterwards. */
elmddm_status elmddm_solve(elmddm_plan* plan, const double* W, const double* b, const double* f,
                           const double* g, const double* coef, double* u_gamma, double* c,
                           void* stream);

/* Synchronise the stream of the last solve and report its device-side status. */
elmddm_status elmddm_solve_info(elmddm_plan* plan, elmddm_info* info);

/* Network solution u_h at npts arbitrary points xy [npts][2] (device): each
 * point is evaluated by the local network of the box that holds it (boxes
 * half-open, the last one closed).  Writes u [npts] (device). */
elmddm_status elmddm_eval(elmddm_plan* plan, const double* W, const double* b, const double* c,
                          const double* xy, int64_t npts, double* u, void* stream);

/* u_h and its gradient at npts points (device arrays, same owner rule as
 * elmddm_eval): writes u [npts] (if not NULL), dudx [npts] and dudy [npts],
 * the derivatives of the owning local network (for the relative H1 errors
 * reported in Section 5.2.1, Table 2).  INVALID_ARG on NULL W, b, c, or on
 * NULL xy, dudx or dudy with npts > 0. */
elmddm_status elmddm_eval_grad(elmddm_plan* plan, const double* W, const double* b, const double* c,
                               const double* xy, int64_t npts, double* u, double* dudx, double* dudy,
                               void* stream);

/* The feature-assembly stage alone (the rows of eq. nonoverlap_discrete):
 * writes, per subdomain s, K^s in column-major [nsub][neurons][max_rows]
 * (rows: interior, boundary, interface; rows beyond m_s are zero), the flux
 * rows A^s column-major [nsub][neurons][max_ifc] (outward normal
 * derivatives at the interface points; rows beyond k_s zero) and
 * F^s [nsub][max_rows].  For checking the assembly; not needed to solve. */
elmddm_status elmddm_assemble(elmddm_plan* plan, const double* W, const double* b, const double* f,
                              const double* g, const double* coef, double* K, double* A, double* F,
                              void* stream);

/* Copy the interface Schur matrix S [n_interface][n_interface] (column-major)
 * and its right-hand side [n_interface] of eq. schur, as assembled by the
 * last elmddm_solve, into caller device buffers.  Valid only if the plan was
 * told to keep them with elmddm_plan_keep_schur(plan, 1) before that solve. */
elmddm_status elmddm_plan_keep_schur(elmddm_plan* plan, int32_t keep);
elmddm_status elmddm_get_schur(elmddm_plan* plan, double* S, double* rhs, void* stream);

/* Further right-hand sides with cached factors (plans with batch 1).  After
 * an elmddm_solve, the plan's workspace holds every factor that depends on
 * the hidden layer (the CholeskyQR factors of each K^s, the Schur matrix's
 * envelope Cholesky factor); a new source f and boundary data g only change
 * the F column of eq. nonoverlap_discrete.  elmddm_solve_rhs repeats, for
 * nrhs such columns at once, h = Q^T F, the Schur right-hand side g of
 * eq. schur, the two triangular solves with the factor of S and the local
 * back-solve, and gives the same result as elmddm_solve with that data.
 *   f [nrhs][nsub][q_x*q_y]  sources at the interior points
 *   g [nrhs][n_boundary]     Dirichlet data (NULL: zero boundary data)
 *   u_gamma [nrhs][n_interface]  output
 *   c [nrhs][nsub][neurons]  output (NULL: skip the local back-solve)
 * elmddm_plan_reserve_rhs allocates the workspace for up to max_rhs columns
 * per pass (1..4096; larger nrhs are processed in passes of max_rhs).
 * Fails with INVALID_ARG if no solve has been enqueued since the plan was
 * created or autotuned, UNSUPPORTED for plans with batch > 1. */
elmddm_status elmddm_plan_reserve_rhs(elmddm_plan* plan, int32_t max_rhs);
elmddm_status elmddm_solve_rhs(elmddm_plan* plan, int32_t nrhs, const double* f, const double* g,
                               double* u_gamma, double* c, void* stream);

/* The right-hand side g of eq. schur (interface order) for nrhs further
 * sources with the factors of the last solve (same conditions and layouts
 * as elmddm_solve_rhs): rhs [nrhs][n_interface], device. */
elmddm_status elmddm_schur_rhs(elmddm_plan* plan, int32_t nrhs, const double* f, const double* g,
                               double* rhs, void* stream);

/* Conjugate gradients on the interface system S u = rhs (Section 3; the
 * paper's interface solver), with S the Schur matrix of the last solve, kept
 * by elmddm_plan_keep_schur(plan, 1) before that solve.  u [nrhs][n_interface]
 * (device) holds the initial guesses on entry and the iterates on return.
 * Each system stops when ||rhs - S u|| <= tol ||rhs|| (checked every
 * iteration; the host polls every 16 iterations) or after maxit iterations.
 * iters (host int32 [nrhs], or NULL) receives the iteration counts, relres
 * (host double [nrhs], or NULL) the final relative residuals
 * ||rhs - S u|| / ||rhs|| as tracked by the recurrence (maxit = 0: the
 * residual of the initial guess, computed directly).
 * Synchronises the stream; returns NOT_CONVERGED if any system did not reach
 * tol.  Needs elmddm_plan_reserve_rhs (passes of up to max_rhs systems). */
elmddm_status elmddm_interface_cg(elmddm_plan* plan, int32_t nrhs, const double* rhs, double* u, double tol,
                                  int32_t maxit, int32_t* iters, double* relres, void* stream);

/* Number of CholeskyQR passes of the local least squares (3 to 5; passes
 * 1 .. npass - 2 carry the diagonal shift, the last one also yields h).  One
 * shifted pass handles column-scaled condition numbers of K^s up to about
 * 1e12, two up to about 1e14, three up to about 1e16.  Default: 5 for neurons
 * >= 900, 4 for neurons >= 600, else 3 (the tanh feature blocks of the
 * configured scales reach 1e12..1e13 at 800 and ~1e15 at 1000 neurons).
 * Allocates further inverse factors on first use. */
elmddm_status elmddm_plan_set_passes(elmddm_plan* plan, int32_t npass);

/* Precision mode of later solves on this plan.
 *  ELMDDM_MODE_FP64 (default): every product in float64.
 *  ELMDDM_MODE_MIXED: the Gram matrices of the first CholeskyQR pass are
 *    formed on the matrix cores from float32-rounded features with float32
 *    accumulation, and that pass's diagonal shift is raised from the float64
 *    bound to s = 16 sqrt(m n) u32 (u32 = 2^-24) times diag(G) so that it
 *    covers the float32 rounding of the Gram entries.  The first pass only
 *    conditions the features (its factor is used as a triangular right
 *    preconditioner, applied in float64); passes 2 and 3, the Cholesky
 *    factorisations, the Schur complement and the interface solve stay
 *    float64, so the result agrees with the float64 mode to float64
 *    accuracy whenever the shifted pass leaves the preconditioned features
 *    with condition number below about 1e7.
 * Returns INVALID_ARG for an unknown mode. */
elmddm_status elmddm_plan_set_mode(elmddm_plan* plan, int32_t mode);

/* Time the candidate kernels for the two large local products (the Gram
 * matrices of the CholeskyQR passes and the triangular solves) on this plan's
 * shapes and keep the fastest for later solves: the 64 x 64 tile kernel in
 * four variants (K depth 16 with two LDS buffers or 32 with one, XCD-aware
 * tile order on/off) and the strip kernel with 16T-wide tiles, T = 4..8.
 * Overwrites the plan's workspace (call before a solve, not between a solve
 * and elmddm_get_schur); runs synchronously on stream.  Candidates are tried
 * in the fixed order -4, -2, -3, -1, 8, 7, 6, 5, 4 and a later one is kept
 * only if it is at least 2% faster, so near-ties do not flip between runs.
 * choice (NULL or int32[2]) receives the codes of the kernels kept: < 0 is
 * the 64 x 64 kernel variant (-1 - code: bit 1 K depth 32, bit 0 XCD-aware
 * tile order), >= 4 the strip width T. */
elmddm_status elmddm_autotune(elmddm_plan* plan, void* stream, int32_t* choice);

/* Choose the kernels of the two large local products by code (as reported
 * by elmddm_autotune) instead of tuning. */
elmddm_status elmddm_plan_set_kernels(elmddm_plan* plan, int32_t gram_code, int32_t trsm_code);

/* Candidate timings of the last elmddm_autotune (zeros before one): codes
 * [9] receives the kernel codes, gram_ms [9] and trsm_ms [9] the time of
 * one Gram product and one triangular solve over the whole batch with each
 * (host arrays). */
elmddm_status elmddm_autotune_times(const elmddm_plan* plan, int32_t* codes, double* gram_ms, double* trsm_ms);

/* Per-stage device timing of solves (HIP events recorded on the solve's
 * stream around each stage).  When enabled, every elmddm_solve adds the
 * elapsed time of each stage to running totals; elmddm_stage_times
 * synchronises the last solve's stream and reads the totals (milliseconds)
 * and the number of solves they cover.  Stages:
 *   0 feature assembly            1 Gram products (exactly the 3 MFMA Gram launches)
 *   2 local Cholesky + inverses   3 triangular solves (3 MFMA GEMM launches)
 *   4 Schur complement assembly   5 interface Cholesky
 *   6 interface back-substitution 7 local back-solve
 * Enabling resets the totals. */
#define ELMDDM_NUM_STAGES 8
elmddm_status elmddm_set_timing(elmddm_plan* plan, int32_t enable);
elmddm_status elmddm_stage_times(elmddm_plan* plan, double* ms, int32_t* solves);

/* The local-factorisation stages split by CholeskyQR pass (same timing
 * switch and totals as elmddm_stage_times): ms[3 p + 0] Gram product,
 * ms[3 p + 1] Cholesky + inverses, ms[3 p + 2] triangular solve of pass
 * p + 1 (p = 0 .. 4; zeros beyond the plan's pass count), in milliseconds
 * summed over the timed solves.  ms holds 15 doubles. */
elmddm_status elmddm_pass_times(elmddm_plan* plan, double* ms, int32_t* solves);

/* ------------------------------------------------------------------------
 * Learned interface variable (not part of the paper's method).  For a fixed
 * geometry and hidden layer, u_Gamma of eq. schur depends only on the source;
 * a small MLP
 *     y = W3 GELU(W2 GELU(W1 x + b1) + b2) + b3,   GELU(z) = z Phi(z) (exact),
 * trained on (source features -> u_Gamma) pairs produced by the method
 * itself, predicts u_Gamma as an initial guess for the interface solve.
 * FP32 weights and activations on the matrix cores.
 *
 * Layout: x [batch][in_dim], y and targets [batch][out_dim] (float32, device,
 * one contiguous row per sample).  Flat parameter vector (float32, device,
 * elmddm_mlp_num_params entries): W1 (hidden x in_dim, column-major), b1,
 * W2 (hidden x hidden), b2, W3 (out_dim x hidden), b3.  The library draws
 * no random numbers: initial weights come in through elmddm_mlp_set_params,
 * the sample order of training through `order`.
 * ------------------------------------------------------------------------ */
typedef struct elmddm_mlp elmddm_mlp;

/* Allocate a network and its workspace for batches of up to max_batch
 * samples (device memory, released by elmddm_mlp_destroy). */
elmddm_status elmddm_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t max_batch,
                                elmddm_mlp** mlp);
elmddm_status elmddm_mlp_destroy(elmddm_mlp* mlp);
elmddm_status elmddm_mlp_num_params(const elmddm_mlp* mlp, int64_t* count);

/* Copy parameters in (and reset the Adam state) / out; device buffers. */
elmddm_status elmddm_mlp_set_params(elmddm_mlp* mlp, const float* params, void* stream);
elmddm_status elmddm_mlp_get_params(const elmddm_mlp* mlp, float* params, void* stream);

/* Network output y for a batch x. */
elmddm_status elmddm_mlp_forward(elmddm_mlp* mlp, int32_t batch, const float* x, float* y, void* stream);

/* Mean squared error L = sum (y - t)^2 / (batch out_dim) into *loss (device
 * float) and its gradient with respect to the flat parameters (kept for
 * elmddm_mlp_adam_step; also copied to grad if not NULL). */
elmddm_status elmddm_mlp_loss_grad(elmddm_mlp* mlp, int32_t batch, const float* x, const float* t,
                                   float* loss, float* grad, void* stream);

/* One Adam step (bias-corrected moments) with the gradient of the last
 * elmddm_mlp_loss_grad. */
elmddm_status elmddm_mlp_adam_step(elmddm_mlp* mlp, float lr, float beta1, float beta2, float eps,
                                   void* stream);

/* `steps` training steps on the samples X [nsamples][in_dim], targets T
 * [nsamples][out_dim]: step k uses the samples order[k*batch .. k*batch+batch)
 * (int32, device; an index outside [0, nsamples) reads a zero sample),
 * then one Adam step with learning rate
 * lr (1 + cos(pi k / steps)) / 2.  losses (device float [steps], or NULL)
 * receives each step's loss before its update. */
elmddm_status elmddm_mlp_train(elmddm_mlp* mlp, int32_t nsamples, const float* X, const float* T,
                               const int32_t* order, int32_t steps, int32_t batch, float lr, float beta1,
                               float beta2, float eps, float* losses, void* stream);

/* Prediction in float64: out [batch][out_dim] = scale * y. */
elmddm_status elmddm_mlp_predict(elmddm_mlp* mlp, int32_t batch, const float* x, double scale, double* out,
                                 void* stream);

/* ------------------------------------------------------------------------
 * Ragged batches in one graph launch.  Problems of different shapes (grid,
 * neurons, points, operator) go to different plans (each a batch of
 * same-shape instances); elmddm_graph_capture records the solves
 * elmddm_solve(plans[i], args[i]) for i = 0..nsolves-1, in this order, into
 * one HIP graph.  A plan may appear several times (e.g. one chunk of its
 * shape after another): its solves run one after the other and reuse its
 * workspace.  elmddm_graph_launch replays every solve with one graph launch
 * on the caller's stream; the input and output buffers named in args must
 * stay valid for as long as the graph is launched.  Capture enqueues nothing
 * (it records on a private stream) and needs stage timing off on every plan.
 * After a launch each plan's workspace holds the factors of its last solve in
 * the graph.  elmddm_graph_info synchronises the launch stream and reports
 * solve i as elmddm_solve_info would.
 * ------------------------------------------------------------------------ */
typedef struct elmddm_solve_args {
    const double* W;
    const double* b;
    const double* f;
    const double* g;
    const double* coef;
    double* u_gamma;
    double* c;
} elmddm_solve_args;

typedef struct elmddm_graph elmddm_graph;

elmddm_status elmddm_graph_capture(elmddm_plan* const* plans, const elmddm_solve_args* args, int32_t nsolves,
                                   elmddm_graph** graph);
elmddm_status elmddm_graph_launch(elmddm_graph* graph, void* stream);
elmddm_status elmddm_graph_info(elmddm_graph* graph, int32_t solve, elmddm_info* info);
elmddm_status elmddm_graph_destroy(elmddm_graph* graph);

const char* elmddm_status_string(elmddm_status status);
const char* elmddm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ELMDDM_H */
