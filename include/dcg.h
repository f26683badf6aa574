/*
 * dcg.h -- C ABI of the MI355X deflated-CG library (libdcg.so).
 *
 * Deflated conjugate gradients with Krylov subspace recycling for sequences
 * of SPD kernel systems A_i x_i = b_i, A_i = K_theta_i(X, X) + sigma_i^2 I
 * (de Roos & Hennig, arXiv 1706.00241: sequence of Eq. 1, deflated CG of
 * section 2.2 / Algorithm 1, harmonic Ritz extraction of section 2.3 /
 * Eq. 7).
 *
 * Conventions (apply to every entry point):
 *  - Array arguments are DEVICE pointers unless the comment says "host".
 *    Vectors are FP64 and have n entries; blocks of vectors are FP64,
 *    column-major n x m (leading dimension n).  X is FP64, row-major n x d.
 *  - All device memory is owned by the caller (allocated e.g. with
 *    PyTorch).  The library never allocates device memory: each handle
 *    lives in a caller-provided workspace whose size the *_workspace_bytes
 *    query returns.  A workspace must stay valid and untouched by the caller
 *    until the handle is destroyed.  Handles themselves are small host
 *    objects freed by the matching *_destroy call.
 *  - Every function returns a status code (dcg_status) and never aborts or
 *    throws across the ABI.  On an error, output arrays are unspecified
 *    unless stated otherwise.
 *  - Work is enqueued on the stream given to dcg_create_operator.  Calls
 *    that return results to host memory (dcg_solve, dcg_recycle_get_*)
 *    synchronise that stream before returning; dcg_matvec* do not.
 *  - One operator belongs to one stream.  Calls on different operators and
 *    streams may run concurrently; calls on one operator (or one recycle
 *    handle) must not overlap.
 */
#ifndef DCG_H
#define DCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dcg_operator_s *dcg_op_t;      /* opaque */
typedef struct dcg_recycle_s *dcg_recycle_t;  /* opaque */

/* Covariance functions.  RBF is the kernel of the paper's experiments
 * (section 3): s2 exp(-r^2 / (2 ell^2)).  The Matern kernels are the
 * textbook forms s2 (1 + t) e^-t, t = sqrt3 r/ell, and
 * s2 (1 + t + t^2/3) e^-t, t = sqrt5 r/ell. */
enum dcg_kernel { DCG_RBF = 0, DCG_MATERN32 = 1, DCG_MATERN52 = 2 };

/* Compute precision of the distance GEMM (points are rounded to it once, at
 * operator creation; the operator is the exact kernel matrix of the rounded
 * points evaluated with FP32 accumulation).  FP64 is the exact operator. */
enum dcg_prec {
  DCG_PREC_FP32 = 0,    /* fp32 points, fp32 MFMA                              */
  DCG_PREC_BF16 = 1,    /* bf16 points (8 significant bits), bf16 MFMA.  With
                           bf16 or fp16 points d may exceed 64 (up to 4096):
                           the product then runs an LDS-staged MFMA tile loop
                           over the points of 256-point block pairs, single
                           vectors only (dcg_matvec with m > 1 forms one
                           column at a time); there is no FP64 operator and no
                           multi-column sweep: dcg_matvec_exact, refinement,
                           dcg_solve_block and dcg_solve_batched return
                           DCG_E_ARG                                           */
  DCG_PREC_BF16X2 = 2,  /* points as a pair hi + lo of bf16 (16 significant
                           bits); the distance GEMM takes the four bf16
                           products hi.hi, hi.lo, lo.hi, lo.lo on MFMA         */
  DCG_PREC_FP64 = 3,    /* exact FP64 operator                                 */
  DCG_PREC_FP16 = 4,    /* fp16 points (11 significant bits), fp16 MFMA; the
                           scaled points and their squared norms must stay
                           inside the fp16 range (dcg_create_operator and
                           dcg_set_hyper return DCG_E_ARG otherwise)          */
  DCG_PREC_STORED = 5   /* the unit-amplitude kernel matrix formed once in
                           FP64 from the unrounded points and stored in FP32,
                           its block upper triangle only (128 x 128 tiles:
                           about 2 n_pad^2 bytes of workspace, n_pad = n
                           rounded up to 256; 1 <= d <= 4096): every product
                           streams it from HBM once, each off-diagonal tile
                           serving its rows and its columns, with FP64
                           accumulation.  For FP32-accurate kernel values
                           beyond 64 point dimensions and for sequences that
                           keep the kernel and lengthscale
                           (s2, sigma2 and a diagonal scaling apply at product
                           time; a new ell rebuilds the matrix).  No FP64
                           operator: dcg_matvec_exact, refinement, the
                           batched and gradient entry points return DCG_E_ARG
                           (dcg_solve_block and dcg_slq_logdet accept it);
                           its product has one plan (dcg_set_sweep_items
                           returns DCG_E_ARG, dcg_tune_operator times it and
                           returns the tile size, 128)                        */
};

enum dcg_status {
  DCG_OK = 0,
  DCG_NOT_CONVERGED = 1,   /* max_iter reached; x and stats are valid      */
  DCG_E_ARG = -1,          /* invalid argument (size, pointer, enum value)  */
  DCG_E_NOT_SPD = -2,      /* p^T A p <= 0 in the iteration                 */
  DCG_E_NONFINITE = -3,    /* NaN/Inf met in the iteration, or in W^T A W   */
  DCG_E_W_RANK = -4,       /* recycled basis numerically rank deficient: a
                              Cholesky pivot of W^T A W is at most 1e-12 of
                              the diagonal entry it started from (e.g. W with
                              repeated columns); found when a solve starts,
                              before its first CG step                      */
  DCG_E_HIP = -5,          /* a HIP runtime call failed                     */
  DCG_E_WORKSPACE = -6     /* workspace too small or misaligned             */
};

/* Solver parameters (host struct). */
typedef struct {
  double tol;          /* stop when |r_j|_2 / |b|_2 <= tol (recursive residual,
                          the relative error of section 3)                   */
  int max_iter;        /* CG steps per solve (<= 0: 10 n)                   */
  int L;               /* leading iterations stored for the extraction; the
                          "l" of def-CG(k, l) (section 2.2); <= rc's L       */
  int select_largest;  /* 1: keep the largest harmonic Ritz values (the
                          paper's experiments), 0: the smallest              */
  int check_every;     /* iterations between host convergence checks (>= 1) */
  int refine;          /* 0: none; 1: iterative refinement against the FP64
                          operator; 2: flexible-CG (Krylov-accelerated)
                          refinement; DCG_E_ARG otherwise                     */
  double inner_tol;    /* relative tolerance of each inner solve (refine)   */
  int refine_max;      /* maximum outer refinement steps                    */
  int use_graph;       /* 1: capture each chunk of iterations in a hipGraph */
  int true_residual;   /* 1: also compute |b - A x| / |b| at exit (one more
                          product; always done when refine > 0)              */
  int profile;         /* 1: time every matvec sweep with HIP events on the
                          operator's stream (recorded inside the iteration
                          graph when use_graph = 1), and with refine = 1 the
                          FP64 pair sweep of every refinement residual      */
  int refresh_every;   /* refine > 0 only, when the inner solves refresh W:
                          0 after the first inner solve of each dcg_solve
                          call (the operator does not change between them),
                          1 after every one, 2 once after the last one, from
                          the directions of all inner solves in order (up to
                          L; W unchanged meanwhile); DCG_E_ARG otherwise     */
  int ritz_route;      /* reduction of F in the harmonic Ritz problem (Eq. 7):
                          0: Cholesky when a bound shows that no direction of
                          F would be dropped as numerically null, else the
                          eigendecomposition; 1: always the eigendecomposition
                          (both give the same pairs when nothing is dropped);
                          DCG_E_ARG otherwise                                 */
  int extraction;      /* the next basis from span(Z), Z = [W, P_L] (section
                          2.3): 0 harmonic Ritz, G u = theta F u (Eq. 7),
                          W' A-orthonormal; 1 Rayleigh-Ritz,
                          (Z^T A Z) y = theta (Z^T Z) y, W' orthonormal;
                          2 harmonic Ritz with F and G formed from the
                          scalars of the first L steps (d_j, alpha_j,
                          beta_j, rho_j, mu_j and the re-projection's
                          coefficients; section 2.3, after Saad et al.)
                          instead of tall products; the solve stores the
                          FP64 directions p_0 .. p_L and no products A p_j.
                          AW' comes from the residual recurrence on the
                          FP64 operator and from k' products of W' on the
                          others (a second harmonic problem on span(W')
                          then drops pairs the scalars could not resolve).
                          dcg_solve only (the batched solve and
                          dcg_extract_basis refuse it), not with the pooled
                          refresh of refine (refresh_every = 2);
                          DCG_E_ARG otherwise                                 */
} dcg_params;

/* Per-solve statistics (host struct, filled by dcg_solve). */
typedef struct {
  int iters;                 /* CG steps (sum over inner solves if refine)   */
  int matvecs;               /* products with the low-precision operator     */
  int matvecs_exact;         /* products with the FP64 operator (refine)     */
  int k_used;                /* columns of W used in this solve              */
  int k_next;                /* columns of W' extracted for the next solve   */
  int outer_steps;           /* refinement steps                             */
  int status;                /* dcg_status of the solve                      */
  double rel_res_recursive;  /* final |r_j| / |b|, recursive residual        */
  double rel_res_true;       /* |b - A x| / |b| with the FP64 operator if
                                refine, else with the solve's operator       */
  double t_init_ms, t_loop_ms, t_refresh_ms, t_total_ms;
  int sweeps_timed;          /* profile = 1: matvec sweeps timed             */
  double t_sweeps_ms;        /* profile = 1: their summed device time        */
  int refresh_dim;           /* columns of Z = [W, P] in the last extraction */
  int refresh_rank;          /* of them kept after dropping F's null space   */
  int refresh_sweeps[2];     /* Jacobi sweeps of its two eigenproblems (the
                                first is 0 when F was reduced by Cholesky)  */
  int exact_sweeps_timed;    /* profile = 1, refine = 1: FP64 pair sweeps of
                                the refinement residuals timed              */
  double t_exact_sweeps_ms;  /* profile = 1, refine = 1: their summed device
                                time (HIP events on the operator's stream
                                around each sweep kernel)                   */
} dcg_stats;

/* ---------------------------------------------------------------- operator
 * The matrix A = K_theta(X, X) + sigma2 I of the paper's sequence (Eq. 1,
 * Gram matrix over X of section 1), applied matrix-free. */

/* Bytes of workspace the operator needs (256-byte aligned base required). */
size_t dcg_operator_workspace_bytes(int64_t n, int64_t d, int prec);

/* Scale X by the kernel's lengthscale factor, round it to prec, store it
 * with its squared norms in the workspace, and keep (kernel, ell, s2,
 * sigma2).  X: device FP64 row-major n x d, read only here (a copy is
 * kept).  stream: a hipStream_t (NULL = default).  Requires n >= 1,
 * ell > 0, s2 > 0, sigma2 >= 0, and 1 <= d <= 64 (fp32, bf16x2 and FP64
 * operators) or 1 <= d <= 4096 (bf16, fp16 and the stored operator).
 * Returns DCG_E_NONFINITE if X holds NaN/Inf, DCG_E_ARG if fp16 operands
 * would leave the fp16 range. */
int dcg_create_operator(const double *X, int64_t n, int64_t d, int kernel,
                        double ell, double s2, double sigma2, int prec,
                        void *workspace, size_t ws_bytes, void *stream,
                        dcg_op_t *out);

/* Change the hyperparameters (the next system of a sequence).  A new ell
 * rebuilds the operands on the operator's stream; for fp16 operands that
 * leave the fp16 range the call returns DCG_E_ARG and keeps the previous
 * hyperparameters. */
int dcg_set_hyper(dcg_op_t op, double ell, double s2, double sigma2);

/* Diagonal scaling of the operator: A = D K D + sigma2 I, the form of the
 * Laplace-approximation systems of section 3 (Eq. 10, D = H^{1/2}).
 * D: device FP64 n-vector of finite entries >= 0, copied into the operator
 * workspace (the caller's buffer is free on return), or NULL to remove the
 * scaling.  Every product of dcg_matvec, dcg_matvec_exact and dcg_solve then
 * applies it; the low-precision sweep multiplies fp32(D v).  dcg_solve_block,
 * dcg_solve_batched and dcg_mll_grad reject a scaled operator (DCG_E_ARG).
 * A recycled AW is recomputed at the next solve.  Returns DCG_E_NONFINITE
 * (and leaves the operator unscaled) for a negative or non-finite entry. */
int dcg_set_diag(dcg_op_t op, const double *D);

/* Y = A V with the operator's compute precision; V, Y device FP64
 * column-major n x m, m >= 1, V and Y must not overlap (Algorithm 1's
 * products A p_j; m > 1 is the block product used for AW). */
int dcg_matvec(dcg_op_t op, const double *V, double *Y, int64_t m);

/* Y = A V with the FP64 operator on the unrounded points (residuals of the
 * iterative refinement).  Same layout rules as dcg_matvec. */
int dcg_matvec_exact(dcg_op_t op, const double *V, double *Y, int64_t m);

/* Work-item target of the operator's low-precision pair sweep (256..8192,
 * default 2048): the sweep groups block offsets into work items so that one
 * launch has about this many.  More items balance the 256 compute units
 * better; fewer items read fewer row partials when the product is finished.
 * Any value gives the same product up to the FP64 summation order of the
 * row partials.  DCG_E_ARG outside the range. */
int dcg_set_sweep_items(dcg_op_t op, int items);

/* Autotuner of the sweep plans: times `reps` single-vector sweeps (1..1000)
 * for each distinct plan of the targets 256, 512, ..., 8192 on the
 * operator's stream, keeps the fastest (a larger target replaces a smaller
 * one only when it is more than 1% faster, so that timing noise does not
 * pick between nearly equal plans, which differ in the summation order of
 * the partial sums) and returns it in *items_out with its time per sweep in
 * *ms_out (either may be NULL); the FP64 sweep (refinement residuals, FP64
 * operators) gets its own plan the same way, timed max(2, reps / 2) times
 * (for an FP64 operator *items_out and *ms_out describe that one).
 * Overwrites the operator's staged vectors and partial sums, so it must not
 * overlap a solve with the same operator. */
int dcg_tune_operator(dcg_op_t op, int reps, int *items_out, double *ms_out);

void dcg_destroy_operator(dcg_op_t op);

/* ---------------------------------------------------------- recycle handle
 * Holds the recycled basis W (n x k) of section 2.1, its product AW with the
 * operator it was last used with, and the storage for the first L search
 * directions P_L and A P_L of a solve (section 2.3, Z = [W, P_L]).  A new
 * handle has no W, so the first solve is plain CG (Fig. 1). */

size_t dcg_recycle_workspace_bytes(int64_t n, int k, int L);

/* k >= 1, L >= k (the first extraction draws k vectors from P_L alone). */
int dcg_recycle_create(int64_t n, int k, int L, void *workspace,
                       size_t ws_bytes, dcg_recycle_t *out);

/* Set W from a device FP64 n x kw block (kw <= k, kw = 0 clears it); AW is
 * recomputed for the operator of the next solve.  The columns are not
 * checked here: the next solve returns DCG_E_W_RANK, before any CG step,
 * if they are numerically dependent against A (repeated columns, say), and
 * DCG_E_NONFINITE if W^T A W holds a NaN or Inf. */
int dcg_recycle_set_W(dcg_recycle_t rc, const double *W, int kw);

/* Copy the current W (n x k_used) to the device array W_out (may be NULL)
 * and write k_used to *k_used (host). */
int dcg_recycle_get_W(dcg_recycle_t rc, double *W_out, int *k_used);

/* Copy AW (n x k_used), the product of W with the operator of the last
 * solve, to the device array AW_out.  Returns DCG_E_ARG if no AW is held
 * (no solve since the last dcg_recycle_set_W). */
int dcg_recycle_get_AW(dcg_recycle_t rc, double *AW_out);

/* Host copy of the harmonic Ritz values selected at the last extraction
 * (theta_out holds at least k doubles; *count receives how many). */
int dcg_recycle_get_theta(dcg_recycle_t rc, double *theta_out, int *count);

void dcg_recycle_destroy(dcg_recycle_t rc);

/* ------------------------------------------------------------------- solve */

size_t dcg_solve_workspace_bytes(int64_t n, int k, int L);

/* Solve A x = b by deflated CG (Algorithm 1).
 *  b   device FP64 n-vector.
 *  x   device FP64 n-vector: on entry x_{-1} if x_given, else ignored
 *      (x_{-1} = 0); on exit the solution (also on DCG_NOT_CONVERGED).
 *  rc  recycle handle, or NULL for plain CG without extraction.  With a
 *      handle the solve starts from its W (if any) and ends by extracting
 *      the next W' = Z U from the harmonic Ritz problem G u = theta F u
 *      (Eq. 7), keeping the k largest (or smallest) theta.
 *  p   host parameters; st host statistics (may be NULL).
 *  ws  solve workspace of dcg_solve_workspace_bytes(n, k, L) bytes, where
 *      k and L are those of rc (0, 0 for rc = NULL).
 * With p->refine = 1 the solve runs iterative refinement: residuals with the
 * FP64 operator, inner deflated solves to p->inner_tol with the operator's
 * precision, until |b - A x| / |b| <= p->tol (the recycled W carries over
 * between the inner solves).  With p->refine = 2 the outer loop is flexible
 * CG with full A-orthogonalisation (Notay 2000) in FP64, the inner deflated
 * solve being its variable preconditioner: one FP64 product per outer step
 * for the direction's product, the residual updated recursively and
 * confirmed with one more FP64 product at the end (at most
 * min(refine_max, 32) directions are kept; the loop restarts from the FP64
 * residual beyond that). */
int dcg_solve(dcg_op_t op, const double *b, double *x, int x_given,
              dcg_recycle_t rc, const dcg_params *p, dcg_stats *st, void *ws,
              size_t ws_bytes);

/* --------------------------------------------- extraction on its own
 * The refresh step of section 2.3 on caller-given Z and AZ, with the kernels
 * that refresh W at the end of dcg_solve.  Harmonic Ritz (extraction = 0,
 * Eq. 7): F = (AZ)^T Z and G = (AZ)^T AZ; Rayleigh-Ritz (extraction = 1):
 * F = Z^T Z and G = (AZ)^T Z (all symmetrised).  G u = theta F u is solved
 * in the range of F (directions of the diagonally scaled F with eigenvalue
 * <= 1e-12 of the largest dropped), the k largest (largest != 0) or
 * smallest theta kept, W' = Z U with U^T F U = I.
 *  Z, AZ      device FP64 n x m, column-major (ld n); 1 <= m <= 192.
 *  k          columns wanted, 1..64.
 *  route      reduction of F, as dcg_params.ritz_route (0 or 1).
 *  W_out      device FP64 n x k, column-major; the first *k_out columns are
 *             written, *k_out = min(k, number of kept directions).
 *  theta_out  host double[k]: the kept values in selection order.
 *  rank_out   host int (may be NULL): directions of F kept.
 *  stream     HIP stream of the call (NULL: the null stream); the call
 *             returns once the results are in place.
 *  ws         device workspace of dcg_extract_basis_workspace_bytes(n, m)
 *             bytes, 256-byte aligned, caller-owned.
 * Errors: DCG_E_ARG (null pointer, sizes, extraction or route out of
 * range), DCG_E_WORKSPACE, DCG_E_HIP. */
size_t dcg_extract_basis_workspace_bytes(int64_t n, int m);
int dcg_extract_basis(const double *Z, const double *AZ, int64_t n, int m, int k, int largest,
                      int extraction, int route, double *W_out, double *theta_out, int *k_out,
                      int *rank_out, void *stream, void *ws, size_t ws_bytes);

/* ------------------------------------- extraction without any allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * extraction as dcg_extract_basis, with the same kernels and the same results
 * bit for bit, but its scratch (F, G and their split-K partial sums, the
 * eigensolver's work arrays, U, theta, status words) lives in a library-held
 * device array of dcg_extract_basis_noalloc_max_bytes() bytes (about 20 MiB,
 * the workspace of the largest pencil, m = 192), one per device, held until
 * the process ends.  The call allocates nothing (no hipMalloc, no allocating
 * library routine); the caller passes Z, AZ and W_out as for
 * dcg_extract_basis.
 *  stream  must belong to the current device (NULL: its null stream); the
 *          scratch used is the current device's.
 * Sizes beyond the scratch's reach (m > 192, k > 64) are DCG_E_ARG, as for
 * dcg_extract_basis; DCG_E_HIP if the device or the array's address cannot be
 * obtained.  Every call on one device shares that device's array, which keeps
 * the last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one device, from several host threads or on several streams,
 * race and must be serialised by the caller.  The call returns once its
 * results are in place. */
size_t dcg_extract_basis_noalloc_max_bytes(void);
int dcg_extract_basis_noalloc(const double *Z, const double *AZ, int64_t n, int m, int k,
                              int largest, int extraction, int route, double *W_out,
                              double *theta_out, int *k_out, int *rank_out, void *stream);

/* ------------------------------------------------ many right-hand sides
 * X = A^{-1} B for m <= 64 columns at once: every column runs its own
 * deflated CG (Algorithm 1) with the basis W held by rc (reused as it is, no
 * extraction; rc may be NULL or empty for plain CG).  The products of a step
 * are block sweeps over four columns at a time, so each kernel value is
 * evaluated once per four columns.  B, X: device FP64 n x m column-major;
 * x_{-1} = 0.  p->tol, max_iter, check_every apply per column; st->iters is
 * the largest column count, st->status the worst column status.  FP64 and
 * stored operators form each column's product on its own and accept a
 * diagonal scaling (dcg_set_diag); the low-precision operators refuse one
 * (DCG_E_ARG). */
size_t dcg_solve_block_workspace_bytes(int64_t n, int64_t m);
int dcg_solve_block(dcg_op_t op, const double *B, double *X, int64_t m,
                    dcg_recycle_t rc, const dcg_params *p, dcg_stats *st,
                    void *ws, size_t ws_bytes);

/* ------------------------------------------------ many independent systems
 * Solves A_s x_s = b_s for s < count (count <= 4096), each system with its
 * own operator (size, points, kernel, hyperparameters may all differ) and
 * its own recycle handle, by deflated CG (Algorithm 1) with the extraction
 * of section 2.3 per system, exactly as dcg_solve would one by one.  The
 * systems step in lockstep: one batched pair sweep over all of them, then
 * one launch per CG vector kernel; a converged system skips its share.
 *  ops    host array of count distinct operator handles, all created on the
 *         same stream (DCG_E_ARG otherwise).
 *  b, x   host arrays of count device FP64 vectors (length n of ops[s]);
 *         x[s] as in dcg_solve (x_{-1} given when x_given).
 *  rcs    host array of count recycle handles or NULL entries (plain CG for
 *         that system); a non-NULL handle appears once.  May itself be NULL.
 *  p      shared host parameters; p->refine must be 0.  p->tol, max_iter
 *         apply per system.
 *  stats  host array of count statistics (may be NULL); t_loop_ms is the
 *         time of the shared iteration.
 *  ws     workspace of dcg_solve_batched_workspace_bytes(count, n) bytes,
 *         n[s] the size of system s, 256-byte aligned.
 * Returns DCG_OK when every system converged, DCG_NOT_CONVERGED when one
 * ran out of iterations, else the first negative per-system status (every
 * system still finishes its solve; stats[s].status holds each one's). */
size_t dcg_solve_batched_workspace_bytes(int count, const int64_t *n);
int dcg_solve_batched(int count, const dcg_op_t *ops, const double *const *b,
                      double *const *x, int x_given, const dcg_recycle_t *rcs,
                      const dcg_params *p, dcg_stats *stats, void *ws,
                      size_t ws_bytes);

/* ------------------------------------------ GP hyperparameter gradient
 * For the operator A = s2 k(X, X) + sigma2 I, alpha = A^{-1} y and probe
 * solves U = A^{-1} Z (Z: P <= 16 probe vectors, e.g. Rademacher), writes to
 * grad3 (host) the gradient of the GP log marginal likelihood with respect to
 * (log ell, log s2, log sigma2) with the Hutchinson trace estimate:
 *   g_j = 1/2 sum_ij (dA/dtheta_j)_ij (alpha_i alpha_j - (1/P) sum_p U_ip Z_jp)
 * (GP model adaptation, section 1; Rasmussen & Williams eq. 5.9).  The two
 * kernel-matrix terms are taken in one symmetric sweep over the pairs.
 * alpha: device n-vector; U, Z: device FP64 n x P column-major.  Operators
 * of precision FP32 or BF16 only (DCG_E_ARG otherwise). */
size_t dcg_mll_grad_workspace_bytes(int64_t n);
int dcg_mll_grad(dcg_op_t op, const double *alpha, const double *U,
                 const double *Z, int64_t P, double *grad3, void *ws,
                 size_t ws_bytes);

/* ------------------------------------------ GP log marginal likelihood
 * The value of the GP log marginal likelihood of y under A = K + sigma2 I
 * (GP model adaptation, section 1; Rasmussen & Williams eq. 5.8) from
 * alpha = A^{-1} y, e.g. as dcg_solve returned it:
 *   *value = -1/2 y^T alpha - (n/2) log(2 pi) - 1/2 log det A,
 * the last term only when logdet is given (a host pointer to log det A, e.g.
 * dcg_slq_logdet's estimate; NULL leaves the term out).  y, alpha: device
 * FP64 n-vectors (n of the operator); value: host.  y^T alpha is summed on
 * the operator's stream in a fixed order (one workgroup), which the call
 * synchronises.  DCG_E_ARG for a null pointer or a non-finite *logdet,
 * DCG_E_NONFINITE when y^T alpha is not finite. */
int dcg_mll_value(dcg_op_t op, const double *y, const double *alpha, const double *logdet,
                  double *value);

/* ------------------------------------------------ log det by SLQ
 * Stochastic Lanczos quadrature: the forward value -1/2 log det A of the GP
 * log marginal likelihood (GP model adaptation, section 1), from the probe
 * solves the gradient already needs.  The P probe columns of Z run as one
 * block CG solve (no recycling: the coefficients must describe the Krylov
 * space of A and z alone) to p->tol (p->max_iter, p->check_every as for
 * dcg_solve_block); each column's alpha_j, beta_j give its Lanczos
 * tridiagonal T_j = 1/alpha_j + beta_{j-1}/alpha_{j-1} on the diagonal and
 * sqrt(beta_j)/alpha_j beside it (at most max_steps steps are used, 1..4096),
 * and quad[c] = |z_c|^2 e_1^T log(T) e_1 estimates z_c^T log(A) z_c (Gauss
 * quadrature).  *logdet (may be NULL) = mean of quad: log det A when
 * E[z z^T] = I (Rademacher probes).
 *  Z      device FP64 n x P column-major, 1 <= P <= 64.
 *  quad   host P doubles; steps host P ints (may be NULL): steps used.
 *  ws     dcg_slq_logdet_workspace_bytes(n, P, max_steps) bytes, aligned.
 * Operators as for dcg_solve_block (a diagonal scaling only on FP64 and
 * stored operators: then log det (D K D + sigma2 I), e.g. the Laplace
 * evidence term log det (I + D K D)).
 * Returns the block solve's status (DCG_NOT_CONVERGED if a column did not
 * reach p->tol: its quadrature still uses the steps taken), DCG_E_NOT_SPD
 * if a tridiagonal has a non-positive eigenvalue. */
size_t dcg_slq_logdet_workspace_bytes(int64_t n, int64_t P, int max_steps);
int dcg_slq_logdet(dcg_op_t op, const double *Z, int64_t P, const dcg_params *p,
                   int max_steps, double *quad, int *steps, double *logdet,
                   void *ws, size_t ws_bytes);

/* ------------------------------------------ Laplace GP classification
 * Newton's method for the mode of the latent function under a GP prior with
 * the operator's kernel (K = s2 K0) and the logistic likelihood
 * p(y_i | f_i) = 1 / (1 + exp(-y_i f_i)) (section 3, Eqs. 8-10).  From
 * f_0 = 0 each step forms, with pi = sigma(f), H = pi (1 - pi), D = H^{1/2}:
 *   b~ = H f + (y + 1)/2 - pi,  A = I + D K D,  b = D K b~,
 * solves A z = b with dcg_solve (x_{-1} = 0; W carried over from one step's
 * system to the next through rc, AW recomputed for each new A), then
 *   a = b~ - D z,  f = K a,  Psi = sum_i log sigma(y_i f_i) - a^T f / 2,
 * and stops once Psi grows by less than psi_tol (the paper uses 1).  The
 * products with K use the FP64 operator when the operator is FP64 or
 * p->refine > 0, else the operator's precision.  A stored operator
 * (DCG_PREC_STORED) has no FP64 operator: with p->refine != 0 the call
 * returns DCG_E_ARG before enqueuing any work.
 *  op          operator without a diagonal scaling (DCG_E_ARG otherwise);
 *              its sigma2 is not used (the systems have a unit shift) and
 *              is left as it was.
 *  y           device FP64 n-vector of labels, each -1 or +1 (DCG_E_ARG
 *              otherwise).
 *  rc, p       recycle handle (or NULL: plain CG) and solver parameters, as
 *              for dcg_solve.
 *  f, a        device FP64 n-vectors: on exit the last Newton iterate and
 *              its a (f = K a).
 *  psi         host array of max_newton + 1 doubles (may be NULL): Psi at
 *              f_0 and after every step taken.
 *  newton_steps host: steps taken.  stats: host array of max_newton
 *              dcg_stats (may be NULL), one per solve.
 *  ws          dcg_laplace_gpc_workspace_bytes(n) bytes, 256-byte aligned.
 * Returns DCG_OK when the Psi test stopped the loop, DCG_NOT_CONVERGED after
 * max_newton steps, or the first error of a solve or product (a solve that
 * ends DCG_NOT_CONVERGED does not stop the loop). */
size_t dcg_laplace_gpc_workspace_bytes(int64_t n);
int dcg_laplace_gpc(dcg_op_t op, const double *y, dcg_recycle_t rc,
                    const dcg_params *p, int max_newton, double psi_tol,
                    double *f, double *a, double *psi, int *newton_steps,
                    dcg_stats *stats, void *ws, size_t ws_bytes);

/* The Laplace approximation to the log evidence at a mode f (f = K a, as
 * dcg_laplace_gpc returns them): Psi(f) - 1/2 log det(I + D K D), D = H^{1/2}
 * at f (the third term of the objective, Eq. 8), the determinant by
 * stochastic Lanczos quadrature (dcg_slq_logdet) over the P probe columns of
 * Z on the operator scaled by D with a unit shift.  FP64 and stored operators
 * only, without a scaling of their own (DCG_E_ARG otherwise); the operator
 * leaves unscaled with its own shift.  evidence (host) required; psi and
 * logdet (host) may be NULL.  Returns the probe solve's status. */
size_t dcg_laplace_evidence_workspace_bytes(int64_t n, int64_t P, int max_steps);
int dcg_laplace_evidence(dcg_op_t op, const double *y, const double *f,
                         const double *a, const double *Z, int64_t P,
                         const dcg_params *p, int max_steps, double *evidence,
                         double *psi, double *logdet, void *ws, size_t ws_bytes);

/* Human-readable name of a status code (static string). */
const char *dcg_status_string(int status);

/* Library version string. */
const char *dcg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DCG_H */
