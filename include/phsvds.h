/*
 * phsvds.h -- C ABI of the MI355X PHSVDS library (libphsvds.so).
 *
 * PHSVDS computes the k smallest (or largest) singular triplets
 * (sigma_i, u_i, v_i) of a large sparse A in R^{m x n}, m >= n, full column
 * rank (problem statement, Section 1, eq. (1)), by a two-stage method:
 * stage 1 is a block GD+k eigensolver on C = A^T A stopped at the best
 * accuracy C allows (Section 3.1, Algorithm 1); stage 2 is GD+k with a
 * refined projection on B = [0 A^T; A 0] seeded by stage 1 (Section 3.2,
 * Algorithm 2).
 *
 * Conventions for every entry point:
 *   - "device" pointers are HIP device memory owned by the caller; the
 *     library only reads inputs and writes outputs through them.
 *   - All device work is enqueued on `stream` (a hipStream_t, NULL = the
 *     null stream).  Host outputs are valid when the call returns.
 *   - Block vectors passed to the SpMM calls are ROW-major (entry (i, j) of
 *     an N x b block at index i*b + j).  Dense outputs U, V of phsvds_svds are
 *     COLUMN-major (entry (i, j) at index i + j*ld with ld = rows).
 *   - CSR inputs are zero-based, rows sorted by column, no duplicates,
 *     rowptr[0] = 0, nnz < 2^31.
 *   - Return value: PHSVDS_OK, PHSVDS_NOT_CONVERGED, or a negative error
 *     code; phsvds_last_error() gives a message for the calling thread.
 *     No C++ exception crosses this boundary.
 */
#ifndef PHSVDS_H
#define PHSVDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHSVDS_OK 0
#define PHSVDS_NOT_CONVERGED 1 /* outputs hold the best approximations */
#define PHSVDS_EINVAL (-1)     /* invalid argument */
#define PHSVDS_EBREAKDOWN (-2) /* unrecoverable numerical breakdown */
#define PHSVDS_EHIP (-3)       /* HIP runtime error */
#define PHSVDS_ENOMEM (-4)     /* workspace too small */
#define PHSVDS_EUSER (-5)      /* the caller's preconditioner returned nonzero */

/* Sparse A in CSR, float64 values (device pointers, caller-owned, read-only). */
typedef struct {
  int64_t m, n, nnz;
  const int64_t *rowptr; /* m+1 */
  const int32_t *colind; /* nnz */
  const double *val;     /* nnz */
} phsvds_csr;

/* Preconditioner of the correction step t = Prec(r) (Algorithm 2 step 13;
 * Section 4).  NONE: t = r.  JACOBI: t = (diag(C) - theta)^-1 r in stage 1
 * (Olsen form), its B-form [M A^T g; A M f] in stage 2 (Section 4).
 * GNN: the learned message-passing network given by `gnn_weights`
 * (layout below, phsvds_gnn_nweights floats), stage 1 only, with Jacobi as
 * the fallback when the leading residual stops halving within
 * fallback_window iterations.  USER: the caller's preconditioner M of
 * C = A^T A (Section 4 admits any; Section 3.3 lets the user supply
 * operators as functions), called through `user_apply`:
 *   T = M R, R and T device n x b column-major (ld n), float64 if fp64,
 *   float32 otherwise (a float32 first stage); theta: host array of the b
 *   eigenvalue estimates of C the columns belong to (M may approximate
 *   (C - theta I)^-1 or ignore theta); stream: the solver's stream, on which
 *   the call must enqueue its work (it may also synchronise).  Stage 1 uses
 *   T = M R directly; stage 2 applies the B-form [M A^T g; A M f] (two
 *   calls per correction, theta = the squared target estimate), also inside
 *   the JDQMR inner solve.  A nonzero return ends the solve with
 *   PHSVDS_EUSER; the library owns R and T only for the duration of the
 *   call. */
enum {
  PHSVDS_PREC_NONE = 0,
  PHSVDS_PREC_JACOBI = 1,
  PHSVDS_PREC_GNN = 2,
  PHSVDS_PREC_USER = 3,
  PHSVDS_PREC_USER_A = 4
};

typedef int (*phsvds_user_apply)(void *ctx, const void *R, void *T, int64_t n, int b,
                                 const double *theta, int fp64, void *stream);

/* USER_A: a preconditioner M ~ A (Section 4: an incomplete LU of a square A,
 * say) given by its solves, from which the library forms M^-1 M^-T for C in
 * stage 1 and [0 M^-1; M^-T 0], i.e. [f; g] -> [M^-1 g; M^-T f], for B in
 * stage 2 (no product with A):
 *   trans = 0: Y = M^-1 X, X device m x b, Y device n x b;
 *   trans = 1: Y = M^-T X, X device n x b, Y device m x b;
 * column-major blocks (ld = their row count), float64 if fp64, float32 in a
 * float32 first stage; stream as for user_apply.  A nonzero return ends the
 * solve with PHSVDS_EUSER. */
typedef int (*phsvds_user_solve)(void *ctx, const void *X, void *Y, int b, int trans, int fp64,
                                 void *stream);

typedef struct {
  int kind;
  const float *gnn_weights; /* device, phsvds_gnn_nweights() floats, or NULL */
  int gnn_width;            /* hidden width of the network (e.g. 32) */
  int fallback_window;      /* GNN safeguard window in iterations (0: 25; -1: never) */
  phsvds_user_apply user_apply; /* USER: the caller's M of C (see above), or NULL
                                   (stage 1 then runs without one) */
  void *user_ctx;               /* USER, USER_A: passed back as the first argument */
  phsvds_user_solve user_solve; /* USER_A: the solves with M ~ A (see above) */
  /* USER: a preconditioner of B itself (Section 4 admits one "directly for
   * B"), or NULL for the B-form of user_apply: T = M_B R with R and T device
   * N x b column-major float64 (N = m + n, rows 0..n-1 the v part), theta
   * the b singular value estimates; used by the second stage instead of the
   * B-form, also inside JDQMR.  user_apply and user_apply_B may not both be
   * NULL. */
  phsvds_user_apply user_apply_B;
} phsvds_precond;

typedef struct {
  int which;       /* 0: smallest (default), 1: largest (Section 1, Section 3.1) */
  int block;       /* block size b of the GD+k iteration (default 1) */
  int max_basis;   /* p_max; 0: max(35, 2k + 2b) (Section 5 uses 35) */
  int min_restart; /* p_min; 0: max(21, ceil(0.6 p_max)), capped at p_max - 2b */
  int stage1_fp32; /* 1: stage 1 in float32 with float32 accumulation */
  int fp64_continue; /* with stage1_fp32: continue stage 1 in float64 before B */
  int stage2;      /* 0: automatic (Section 3.1 rule), 1: force, -1: never */
  int max_restarts;   /* per stage (default 10000, Section 5) */
  int64_t max_matvecs; /* budget of products with A (stage 1, transition and
                          stage 2 together; 0: unlimited): the solve stops
                          with PHSVDS_NOT_CONVERGED once it is spent */
  uint64_t seed;      /* counter-based stream for random vectors */
  const double *init_block; /* device n x b column-major initial block, or NULL
                               for [ones/sqrt(n), random] (Section 5) */
  double anorm;        /* ||A|| if known (> 0), else the running estimate */
  double floor_factor; /* multiple of eps*||C|| that ends stage 1 (default 10) */
  int gnn_width;       /* width of the learned preconditioner the workspace must
                          hold (0: none); must match phsvds_precond.gnn_width */
  int verbose;         /* 1: a progress line on stderr every 1000 iterations
                          and at each lock; 0 (default): silent */
  int stage2_method;   /* second stage (Section 3.2): 0 GD+k with the refined
                          projection, the residual block as correction;
                          1 (default) JDQMR: the same outer iteration, expanded
                          by the target's correction equation
                          P (B - s I) P t = -r (P orthogonal to the locked
                          vectors and the refined vector, s the target shift)
                          solved by symmetric QMR with dynamic inner stopping */
  int max_inner;       /* JDQMR inner step cap (0: 50) */
  const double *init_V; /* device n x k0 column-major, or NULL.  Without
                           shifts: the first stage starts from these k0
                           vectors (1 <= k0 <= p_min; overrides init_block).
                           With shifts: saved first-stage output (Algorithm 2
                           step 1 inputs); the first stage is skipped, the
                           left vectors are u_i = A v_i / ||A v_i|| (random for
                           ||A v_i|| <= 10 eps ||A||, Section 3.3) and every
                           one of the k pairs goes through the second stage
                           with shifts[i] as its target; needs k <= k0 and the
                           smallest end */
  int k0;               /* columns of init_V */
  const double *shifts; /* host, k0 singular value estimates, or NULL */
  int dynamic;          /* 1: choose between C and B at run time (Section 4.1,
                           Algorithm 3): short GD+k runs alternate between
                           C (Algorithm 1's iteration) and B (harmonic Ritz
                           vectors for the target 0, the estimates being too
                           rough to serve as shifts), each from the other's
                           latest approximations, and the measured mean
                           per-iteration residual reduction decides; run
                           lengths start at init_iter and double while the
                           same approach wins, halve (j -> floor(j/2)) when it
                           changes; switching stops once a pair converged in
                           the first two runs or two later, or after
                           max_switch switches.  C then finishes as the
                           two-stage method from the approximations, B as
                           GD+k on B (harmonic) without an iteration limit.
                           Needs the smallest end, float64 (stage1_fp32 = 0),
                           stage2_method 0, k <= p_min, no init_V and a
                           preconditioner other than GNN */
  int init_iter;        /* dynamic: length of the first runs (0: 50) */
  int max_switch;       /* dynamic: switch limit (0: 8) */
  /* The caller's operator in place of C = A^T A in the first stage (Section
   * 3.3 accepts a function for C): Y = C X, or with c_inverse Y = C^-1 X
   * (shift-invert, Section 4: the largest eigenvalues mu of C^-1 give
   * sigma = mu^-1/2), on row-major n x b device blocks (b the padded block
   * width), float64, work on `stream`; NULL: C X = A^T (A X).  The
   * transition, the second stage and the final check still use A.  With
   * c_inverse the first stage locks on ||C^-1 x - mu x|| < tol sqrt(mu) /
   * ||A||, the image of its test on C, with ||A|| = anorm or twelve power
   * steps on A^T A; it needs the smallest end and no preconditioner.  With
   * either, stage1_fp32 and dynamic must be 0.  A nonzero return ends the
   * solve with PHSVDS_EUSER. */
  int (*c_apply)(void *ctx, const void *X, void *Y, int b, int fp64, void *stream);
  void *c_ctx;
  int c_inverse;
} phsvds_opts;

typedef struct {
  int64_t mv_stage1, mv_rr, mv_stage2, mv_final; /* products with A (Section 5 "MV") */
  int64_t mv_prec;    /* A products inside preconditioners */
  int64_t mv_floor;   /* |A| products for the float32 accuracy floor */
  int64_t iters1, iters2, restarts1, restarts2;
  int64_t stage2_pairs, fp32_locked;
  int64_t fallbacks;  /* learned preconditioner replaced by Jacobi (safeguard) */
  int64_t refreshes;  /* W = C V rebuilt after a failed explicit-residual check */
  int64_t rollbacks;  /* basis expansions undone after a failed deferred check */
  int64_t inner2;     /* JDQMR inner steps (each one product with B, in mv_stage2) */
  double t_setup, t_stage1, t_stage2, t_total; /* seconds (host wall clock) */
  double anorm_est;
  double res_stage1[64]; /* residual ||r_C|| of each pair on leaving stage 1 */
  /* dynamic mode: the approach chosen (1 C, 2 B; 0 when not dynamic), how
   * (1: a run locked all k pairs, 0: the faster one), and up to 16 runs:
   * the approach (1 C, 2 B), the iteration limit, the pairs locked and the
   * measured rate (mean one-step reduction factor of the residual) */
  int64_t dyn_choice, dyn_found, dyn_runs;
  int64_t dyn_on[16], dyn_iters[16], dyn_locked[16];
  double dyn_rate[16];
  int64_t dep_cols; /* new basis columns that Gram-Schmidt found dependent on the
                       basis and replaced by seeded random vectors */
} phsvds_stats;

/* The caller's operator in place of a CSR A (Section 3.3 accepts a matrix
 * function for the products with A and A^T):
 *   trans = 0: Y = A X, X device n x b, Y device m x b;
 *   trans = 1: Y = A^T X, X device m x b, Y device n x b;
 * row-major blocks (element (i, j) at X[i * b + j]) with b the block width
 * padded to a power of two (extra columns are products like the others),
 * float64 (fp64 is always 1: the first stage cannot run in float32 with an
 * operator).  Work goes on `stream` (the call may also synchronise); the
 * library owns X and Y only for the duration of the call.  A nonzero
 * return ends the solve with PHSVDS_EUSER. */
typedef int (*phsvds_op_apply)(void *ctx, const void *X, void *Y, int b, int trans, int fp64,
                               void *stream);
typedef struct {
  int64_t m, n; /* m >= n */
  phsvds_op_apply apply;
  void *ctx;    /* passed back as the first argument */
} phsvds_operator;

/* Defaults of every field (paper parameters of Section 5). */
void phsvds_default_opts(phsvds_opts *opts);

/* Library version string; never NULL. */
const char *phsvds_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char *phsvds_last_error(void);

/* Y = A X (or Y = |A| |X| if `absval`), X n x b, Y m x b, row-major blocks,
 * b in {1, 2, 4, 8, 16, 32}.  "Matrix times block of vectors" of Section 3.3. */
int phsvds_spmm_f64(const phsvds_csr *A, int b, const double *X, double *Y, int absval,
                    void *stream);
/* Same with float32 values/vectors (the float32 value array `val32` has the
 * sparsity of A; A->val is not read). */
int phsvds_spmm_f32(const phsvds_csr *A, const float *val32, int b, const float *X, float *Y,
                    int absval, void *stream);

/* Y = op(A) X with op(A) = A (trans = 0) or A^T (trans = 1): the "matrix
 * times block of vectors" with A and A^T of Section 3.3.  Row-major blocks:
 * X is (trans ? m : n) x b, Y is (trans ? n : m) x b, b in {1, 2, 4, 8, 16,
 * 32}.  fp32 = 0: X, Y float64 and A->val is used; fp32 = 1: X, Y float32,
 * with val32 (float32 values in A's sparsity) for trans = 0 and A->val
 * (converted on the device) for trans = 1.  A transposed product builds the
 * CSR of A^T on the device in `ws` on every call (phsvds_spmm_ws_bytes
 * bytes; 0 and ws may be NULL for trans = 0), so its rows are summed in
 * column order and results are deterministic; that build checks A and
 * returns PHSVDS_EINVAL for row pointers that do not start at 0, decrease
 * or do not end at nnz, columns outside [0, n), or unsorted or repeated
 * columns in a row.  Too small a workspace is PHSVDS_ENOMEM. */
size_t phsvds_spmm_ws_bytes(const phsvds_csr *A, int trans, int fp32);
int phsvds_spmm(const phsvds_csr *A, const float *val32, int trans, int fp32, int b,
                const void *X, void *Y, void *ws, size_t ws_bytes, void *stream);

/* phsvds_spmm without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels, with the
 * transpose built in a scratch array the library holds on each GPU for the
 * life of the process (64 MiB per GPU, enough for a transposed product of
 * about 2M nonzeros; the need is phsvds_spmm_ws_bytes).  Calls no hipMalloc,
 * hipFree or other allocating routine and records no profiling events.  A
 * product needing more scratch returns PHSVDS_ENOMEM before touching the
 * device.  Every call on one GPU shares that GPU's scratch and leaves its
 * contents behind: calls that overlap on one GPU (other streams or host
 * threads) race and must be serialised by the caller.  A transposed call
 * synchronises the stream (the build reads back a validity flag and a row
 * count). */
int phsvds_spmm_noalloc(const phsvds_csr *A, const float *val32, int trans, int fp32, int b,
                        const void *X, void *Y, void *stream);

/* Rayleigh-Ritz eigenproblem of the search space, H s = theta s with
 * H = V^T C V (Algorithm 1, the projection step of each iteration):
 * H device p x p column-major (ld ldh >= p, symmetric part used, not
 * modified), 1 <= p <= 64, 1 <= nvec <= p.  Writes the nvec eigenpairs at the
 * wanted end (smallest ascending, or largest descending if `largest`) to
 * theta[0..nvec) and columns 0..nvec-1 of S (device, ld lds >= p), and the
 * eigenvalue at the other end to theta[p-1]; other entries are untouched. */
int phsvds_rr_eig(const double *H, int ldh, int p, int nvec, int largest, double *theta,
                  double *S, int lds, void *stream);

/* Small singular value decomposition of the refined projection (Section
 * 3.2; Algorithm 2 step 9: the smallest right singular vector of the R
 * factor of W - sigma V): M device rows x cols column-major (ld ldm >=
 * rows, not modified), 1 <= cols <= 64, cols <= rows <= 128.  One-sided
 * (Hestenes) Jacobi; writes the cols singular values in ascending order to
 * sv[0..cols) and the matching right singular vectors to the columns of Y
 * (device cols x cols, ld ldy >= cols).  Small singular values have high
 * relative accuracy when M is a well-conditioned matrix times a diagonal
 * scaling of its columns.  PHSVDS_EINVAL for sizes out of range. */
int phsvds_small_svd(const double *M, int ldm, int rows, int cols, double *sv, double *Y, int ldy,
                     void *stream);

/* Tall-skinny products of the block iteration (Algorithm 1: the
 * Rayleigh-Ritz border V^T W, the Gram-Schmidt coefficients [X_lock V]^T T
 * and the CholQR Gram matrices are X^T Y; the basis updates and restarts are
 * X S).  Long operands (rows >= 65536, ny <= 16) run on the matrix cores.
 *   tsgemm_tn: G = X^T Y, X device rows x nx, Y device rows x ny; layout
 *     bit 0 set: Y column-major with ld ldy >= rows, else row-major with row
 *     stride ldy >= ny; bit 1 set: X row-major with row stride ldx >= nx,
 *     else column-major with ld ldx >= rows; other bits are PHSVDS_EINVAL.
 *     (The Gram matrix X^T X of one row-major block of 8 columns, X == Y,
 *     rows >= 65536, takes a kernel of its own.)  G device nx x ny float64
 *     column-major (ld ldg >= nx).  1 <= nx <= 128, 1 <= ny <= 32.  fp32:
 *     X, Y float32, products accumulated in float32 within a block of rows
 *     and the blocks added in float64, in a fixed order (deterministic).
 *     ws: phsvds_tsgemm_ws_bytes() bytes of device scratch for the partials.
 *   tsgemm_nn: Y = alpha X S + beta Y, X rows x nx column-major, S device
 *     nx x ny float64 column-major (ld lds >= nx), Y rows x ny column-major
 *     (ld ldy >= rows), X and Y float32 if fp32; 1 <= nx <= 160,
 *     1 <= ny <= 64. */
size_t phsvds_tsgemm_ws_bytes(void);
int phsvds_tsgemm_tn(int fp32, int64_t rows, int nx, int ny, const void *X, int64_t ldx,
                     const void *Y, int64_t ldy, int layout, double *G, int ldg, void *ws,
                     size_t ws_bytes, void *stream);
int phsvds_tsgemm_nn(int fp32, int64_t rows, int nx, int ny, double alpha, const void *X,
                     int64_t ldx, const double *S, int lds, double beta, void *Y, int64_t ldy,
                     void *stream);

/* CSR of A^T (n x m) built on the device: t_rowptr (n+1), t_colind (nnz),
 * t_val (nnz); rows of A^T come out sorted by column.  `ws` must hold
 * phsvds_transpose_ws_bytes(A) bytes.  The sort of a row of A^T with L
 * entries costs O(L^2) comparisons in one workgroup when L > 32.  A is
 * checked as for phsvds_spmm (PHSVDS_EINVAL on a malformed CSR). */
size_t phsvds_transpose_ws_bytes(const phsvds_csr *A);
int phsvds_csr_transpose(const phsvds_csr *A, int64_t *t_rowptr, int32_t *t_colind,
                         double *t_val, void *ws, size_t ws_bytes, void *stream);

/* Device workspace needed by phsvds_svds for these sizes and options. */
int phsvds_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int k, const phsvds_opts *opts,
                           size_t *bytes);

/* The k smallest (opts->which = 0) or largest singular triplets of A to
 * sqrt(||r_u||^2 + ||r_v||^2) <= tol ||A|| (Section 5 stopping test).
 *   sigma   host, k      singular values, ascending (descending if largest)
 *   U       device, m x k column-major left vectors
 *   V       device, n x k column-major right vectors; the largest-magnitude
 *           entry of each v_i is positive
 *   resnorm host, k      explicit float64 residuals of the returned triplets
 *   stats   host, may be NULL
 * Returns PHSVDS_OK, PHSVDS_NOT_CONVERGED, or an error.  1 <= k <= 64,
 * m >= n, tol > 0.  On PHSVDS_NOT_CONVERGED (restart or product budget
 * spent) every triplet is still filled: the pairs not locked are the
 * leading Ritz approximations of the final basis, u = A v / ||A v||, with
 * their explicit residuals in resnorm.  Device memory comes only from the
 * workspace; the call allocates one 64 KB pinned host buffer for its
 * per-iteration status reads and frees it before returning. */
int phsvds_svds(const phsvds_csr *A, int k, double tol, const phsvds_precond *P,
                const phsvds_opts *opts, void *workspace, size_t ws_bytes, void *stream,
                double *sigma, double *U, double *V, double *resnorm, phsvds_stats *stats);

/* phsvds_svds with the caller's operator for A instead of a CSR (Section
 * 3.3): every product with A and A^T of both stages, the transition and the
 * final check goes through A->apply.  Workspace: phsvds_workspace_bytes(
 * A->m, A->n, 0, k, opts).  Preconditioners NONE, USER and USER_A (JACOBI
 * and GNN need the entries of A) and float64 only (stage1_fp32 = 1);
 * otherwise PHSVDS_EINVAL. */
int phsvds_svds_op(const phsvds_operator *A, int k, double tol, const phsvds_precond *P,
                   const phsvds_opts *opts, void *workspace, size_t ws_bytes, void *hip_stream,
                   double *sigma, double *U, double *V, double *resnorm, phsvds_stats *stats);

/* ---- Learned preconditioner (message-passing network over the graph of
 * C = A^T A, float32).  Not in the paper: a preconditioner for C of the kind
 * Section 4 admits.  Per node j, width w in {8, 16, 32}, three layers:
 *   h0_j = [u_j, u_j d_j / max(d_j - tau, d_j/10), d_j, tau],  u = rh / sqrt(d),
 *          rh = r sqrt(n)/||r||, d = diag(C)/mean diag(C), tau = theta/mean diag(C)
 *   h^l = relu(h^{l-1} Ws_l + b_l + Ch (h^{l-1} Wm_l)), Ch = D^-1/2 A^T A D^-1/2
 *   t   = (I - x x^T) t~,
 *   t~_j = (h^3 wo + h0_1)_j ||r|| / (sqrt(n) mean diag(C) sqrt(d_j))
 * Input and output both carry D^-1/2, so the linear part of the network (a
 * polynomial q in Ch) acts as the symmetric operator D^-1/2 q(Ch) D^-1/2.
 * h0_1 through the readout is the Jacobi step r / max(C_jj - theta,
 * C_jj / 10): the zero network is the Jacobi preconditioner and the network
 * learns a correction to it.
 * Weights: one float32 array, row-major blocks in the order
 * Ws1, Wm1 (4 x w), b1 (w), Ws2, Wm2 (w x w), b2, Ws3, Wm3, b3, wo (w).
 * A per-matrix workspace `gws` (phsvds_gnn_workspace_bytes) holds the
 * prepared graph and activations; phsvds_gnn_prepare fills it once.
 * r, x, t, tstar are device float32 vectors of length n. */
int64_t phsvds_gnn_nweights(int width);
size_t phsvds_gnn_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int width);
int phsvds_gnn_prepare(const phsvds_csr *A, int width, void *gws, size_t gws_bytes,
                       void *stream);
/* t = network(r; x, theta). */
int phsvds_gnn_forward(const phsvds_csr *A, int width, void *gws, size_t gws_bytes,
                       const float *w, const float *r, const float *x, double theta, float *t,
                       void *stream);
/* Adds ||t - tstar||^2 / ||tstar||^2 to *loss and its gradient with respect to
 * the weights to grad (device float64, phsvds_gnn_nweights entries). */
int phsvds_gnn_loss_grad(const phsvds_csr *A, int width, void *gws, size_t gws_bytes,
                         const float *w, const float *r, const float *x, double theta,
                         const float *tstar, double *grad, double *loss, void *stream);
/* Adds ||C t - r||^2 / ||r||^2 for the network's output t = M(r) to *loss
 * and its gradient with respect to the weights to grad: how far the
 * correction is from solving C t = r, the criterion the polynomial start
 * fits (Section 4 leaves the preconditioner open; this objective needs no
 * exact corrections).  C t uses the float32 values of A.  Arguments as
 * for phsvds_gnn_loss_grad without tstar. */
int phsvds_gnn_residual_loss_grad(const phsvds_csr *A, int width, void *gws, size_t gws_bytes,
                                  const float *w, const float *r, const float *x, double theta,
                                  double *grad, double *loss, void *stream);
/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8) on the
 * float32 weights w with moments m, v (device, nw floats), gradient
 * grad * grad_scale; step counts from 1. */
int phsvds_gnn_adam(float *w, float *m, float *v, const double *grad, int64_t nw, int step,
                    double lr, double grad_scale, void *stream);

/* Training pairs from a float64 stage-1 run on A (k smallest, opts->block):
 * every `every` iterations, each targeted Ritz pair (theta, x) with residual
 * r gets the exact target t of
 *   (I-QQ^T)(C - rho theta I)(I-QQ^T) t = r,  t orthogonal to Q,
 * i.e. t = M r for M the inverse of the projected operator: the sign of a
 * preconditioned residual, which the network's output takes (the
 * Jacobi-Davidson correction is -t),
 * Q = [locked vectors, Ritz block], by projected CG (relative tolerance
 * cg_tol, at most cg_maxit steps); pairs with non-positive curvature or no
 * convergence are skipped.  rho = shift_scale in [0, 1]: 1 is the
 * Jacobi-Davidson correction equation, 0 the projected C^-1 r.  Outputs
 * (device, n x max_pairs column-major): R, X, T; theta (host, max_pairs, the
 * Ritz values); *count pairs written.  Stage 1 stops at tolerance `tol`,
 * once max_pairs are written, or after 50 every (ceil(max_pairs / block) + 1)
 * iterations (it need not converge).  cg_maxit = 0 runs no CG: every sampled pair is written with
 * T = 0, for training objectives that need no exact targets
 * (phsvds_gnn_residual_loss_grad). */
int phsvds_harvest_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int k,
                                   const phsvds_opts *opts, size_t *bytes);
int phsvds_harvest(const phsvds_csr *A, int k, int every, int max_pairs, double tol,
                   double cg_tol, int cg_maxit, double shift_scale, const phsvds_opts *opts,
                   void *workspace, size_t ws_bytes, void *stream, double *R, double *X,
                   double *T, double *theta, int *count, phsvds_stats *stats);

/* Values of A D^-1/2, D = diag(A^T A) (the squared column norms; a zero
 * column keeps its values): the symmetric Jacobi scaling of C, whose
 * largest singular value squared bounds the spectrum of the learned
 * preconditioner's operator Ch = D^-1/2 A^T A D^-1/2.  val_out (device,
 * nnz) in A's sparsity; `ws` holds phsvds_jacobi_ws_bytes(A) bytes (D is
 * formed from the CSR of A^T, rows summed in column order); A is checked as
 * for phsvds_spmm. */
size_t phsvds_jacobi_ws_bytes(const phsvds_csr *A);
int phsvds_jacobi_scaled_values(const phsvds_csr *A, double *val_out, void *ws, size_t ws_bytes,
                                void *stream);

/* Kernel timing for benchmarks: HIP event pairs recorded on the launching
 * stream around each operation of a kind.  Kinds: 0 float64 SpMM,
 * 1 float32 SpMM, 2 tall X^T Y, 3 tall X S, 4 Ritz block.
 * phsvds_profile(enable) clears the counters and starts recording when
 * enable != 0: enable = 1 records every kind, any other value is a bit mask
 * of kinds shifted left by one (bit k+1 = kind k, e.g. 2 = float64 SpMM
 * only); phsvds_profile(0) stops.
 * phsvds_profile_sample(every), called after phsvds_profile, times only
 * the first pair of consecutive operations of a kind in every `every` pairs
 * (each event record idles the stream for a few microseconds, so sampling
 * keeps the timed run close to an untimed one); phsvds_profile resets it to
 * 1, and every < 1 is PHSVDS_EINVAL.  Inside the solver the two SpMM
 * launches of one product with C = A^T A (A X, then A^T Y) are timed by a
 * single event pair and counted as two operations.
 * phsvds_profile_read returns the number of timed operations, their summed
 * device time (s) and their summed algorithmic HBM bytes.  Not thread-safe
 * against concurrent solves. */
int phsvds_profile(int enable);
int phsvds_profile_sample(int every);
int phsvds_profile_read(int kind, int64_t *launches, double *seconds, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* PHSVDS_H */
