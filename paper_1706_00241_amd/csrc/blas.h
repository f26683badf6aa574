// Device-side state and kernel entry points shared by the HIP sources.
#pragma once

#include "common.h"

namespace dcg {

// One symmetric pair sweep (the low-precision product's first kernel).
struct SymvArgs {
  const void *xr, *xc;
  int kstride;
  const float *vin;   // n_pad x MV, leading dimension n_pad
  double *prow;
  float *pcol;
  int64_t n_pad;
  int nb, dmax, chunk, nchunk;
  const int *done;    // optional: skip the launch once the solve converged
};

// One system of a batched sweep.
struct BatchItem {
  SymvArgs a;
  int kernel;
  int64_t item0;      // first work item of this system in the batched grid
};

// Partial sums of the symmetric matvec and how to finish a product.
struct ReduceArgs {
  const double *prow;
  const float *pcol;
  int64_t n, n_pad;
  int nchunk, dmax, blk, nb, mv;
  double s2, sigma2;
  const double *dsc; // diagonal scaling D (A = D K D + sigma2 I), or null
  const double *V;   // n x mv (ld n)
  double *Y;         // n x mv (ld n)
};

// Row i of vector m: the row partials of every chunk, then the column
// partials of every block offset that owns a pair with row block i/blk (for
// even nb the offset nb/2 belongs to row blocks >= nb/2 only), in a fixed
// order.
__device__ __forceinline__ double sum_partials(const ReduceArgs &A, int m, int64_t i) {
  double s = 0.0;
  for (int c = 0; c < A.nchunk; ++c) s += A.prow[(int64_t(c) * A.mv + m) * A.n_pad + i];
  const int J = static_cast<int>(i / A.blk);
  const bool skip_last = (A.nb % 2 == 0) && (J < A.nb / 2);
  const int dlim = skip_last ? A.dmax - 1 : A.dmax;
  for (int dl = 1; dl <= dlim; ++dl) s += A.pcol[(int64_t(dl - 1) * A.mv + m) * A.n_pad + i];
  return s;
}

// Rows finished per block by cg_matvec_finish.
constexpr int kCgRows = 64;
// cg_update_xr: a grid of row blocks of kXrRows rows times groups of kXrCols
// columns of [AW | W]; its partial sums are per row block.
constexpr int kXrRows = 1024;
constexpr int kXrCols = 8;
__host__ __device__ inline int xr_groups(int k) { return k > 0 ? (2 * k + kXrCols - 1) / kXrCols : 1; }

// Scalars of one deflated-CG solve, resident on the device.
struct SolveState {
  double rho;       // r_j^T r_j
  double alpha, beta, d;
  double bnorm;     // |b|_2
  double relres;    // |r_j| / |b|
  int iter;         // CG steps done
  int done;         // 1 once converged, failed or out of iterations
  int status;       // 0 or a negative dcg_status
  int applied;      // iter as seen by the last cg_matvec_finish (see cg_update_p)
  double mu[kMaxK]; // mu_j of Algorithm 1
  double cvec[kMaxK];
};

struct CgArgs {
  SolveState *S;
  ReduceArgs red;
  const double *qdirect;  // FP64 operator: the finished product (else null)
  int mcol;               // which vector of red's partial layout (red.mv vectors)
  int64_t n;
  double *x, *r, *p, *q;
  float *p32;
  const double *W, *AW, *Minv;
  // FP32 copies of W and AW (exactly W's and AW's values), read instead of
  // them by cg_update_xr and cg_update_p when set
  const float *W32 = nullptr, *AW32 = nullptr;
  const double *N;  // (AW)^T AW, k x k
  int k;
  double *Z, *AZ;   // storage of p_j / A p_j for j < L at column koff + j
  int koff, L;
  double *part, *part2, *part_h;  // partials: d (finish), rho (update_xr), [h|g]
  int64_t nblk_q;                  // blocks of cg_matvec_finish (= its partials)
  int64_t nblk_xr;                 // row blocks of cg_update_xr (= its partials)
  int64_t nblk_p;                  // blocks of cg_update_p
  unsigned *counter;
  double *hist_d, *hist_alpha, *hist_beta, *hist_res;
  int hist_cap;
  double *lz_alpha, *lz_beta;  // every step's alpha_j, beta_j for j < lz_cap (or null)
  int lz_cap;
  double tol;
  int max_iter;
  // implicit extraction: rho_{j+1}, mu_{j+1} (rows of kMaxK) and the
  // re-projection's c_{j+1} (rows of kMaxK) recorded for j < L; Z then holds
  // the FP64 directions p_0 .. p_L and AZ is not written
  double *hist_rho = nullptr, *hist_mu = nullptr, *hist_c = nullptr;
  int implicit = 0;
};

// Block counts of the per-step kernels for a.n and a.k.
inline void cg_set_blocks(CgArgs &a) {
  a.nblk_q = (a.n + kCgRows - 1) / kCgRows;
  a.nblk_xr = (a.n + kXrRows - 1) / kXrRows;
  a.nblk_p = (a.n + 255) / 256;
}
inline int64_t xr_grid(const CgArgs &a) { return a.nblk_xr * xr_groups(a.k); }

__global__ void cg_matvec_finish(CgArgs a);
__global__ void cg_update_xr(CgArgs a);
__global__ void cg_update_xr_w32(CgArgs a);   // a.W32 set
__global__ void cg_update_p(CgArgs a);
__global__ void cg_finalize(CgArgs a);
__global__ void cg_matvec_finish_multi(const CgArgs *args);
__global__ void cg_update_xr_multi(const CgArgs *args);
__global__ void cg_finalize_multi(const CgArgs *args);
__global__ void cg_update_p_multi(const CgArgs *args);
__global__ void init_residual(const double *b, const double *Ax, double *x, double *r, int64_t n,
                              int x_given, double *part, unsigned *counter, SolveState *S);
__global__ void defl_start(double *x, double *t, const double *W, const double *cvec, int64_t n,
                           int k);
__global__ void init_direction(const double *r, const double *W, const double *mu, int64_t n,
                               int64_t n_pad, int k, const double *dsc, double *p, float *p32,
                               double *part,
                               unsigned *counter, SolveState *S, double tol, double *hist_res);

__global__ void residual_norms(const double *b, const double *Ax, int64_t n, double *out,
                               double *part, unsigned *counter, double *sums);
void enqueue_ts_dot(hipStream_t s, const double *Y, int64_t n, int m, const double *v,
                    double *part, unsigned *counter, const double *Minv, double *out);
void enqueue_tsgemm_tn(hipStream_t s, const double *A, const double *B, int64_t n, int ma, int mb,
                       double *part, size_t part_cap, double *C, int ldc, int symmetrise);
// Y (+)= X U; columns of X from round_from on are read as the FP32 copy the
// low-precision sweep multiplies (with the diagonal scaling dsc, if any).
void enqueue_ts_times_small(hipStream_t s, const double *X, int64_t n, int m, const double *U,
                            int ldu, int kout, double *Y, int round_from = 1 << 30,
                            const double *dsc = nullptr, int accumulate = 0);
// The implicit extraction (implicit.hip): the quantities of the first L
// steps of a solve, F and G from them, and the coefficients of AW'.
struct ImplicitHist {
  const double *d, *alpha, *beta;  // j < L
  const double *rho;               // j <= L
  const double *mu;                // rows j <= L of kMaxK doubles
  const double *cv;                // re-projection c_{j+1}, rows j < L of kMaxK doubles
};
void enqueue_implicit_pencil(hipStream_t s, const ImplicitHist &h, const double *M,
                             const double *N, int k, int L, double *scratch, double *F,
                             double *G);
void enqueue_implicit_aw_coef(hipStream_t s, const ImplicitHist &h, const double *U, int k, int L,
                              int kout, double *S1, double *S2);
void enqueue_block_axpy(hipStream_t s, double *Y, const double *X, double alpha, int64_t count);
void enqueue_round_to_fp32(hipStream_t s, double *Y, int64_t count);
// Y32 = (float) Y, element-wise.
void enqueue_to_float(hipStream_t s, const double *Y, float *Y32, int64_t count);
void enqueue_small_spd_inverse(hipStream_t s, const double *M, int k, double *Minv, double *work,
                               int *info);
void enqueue_harmonic_ritz(hipStream_t s, const double *F, const double *G, int m, int k,
                           int largest, int route, double tau, double *work, double *U,
                           double *theta, int *info);
size_t harmonic_ritz_work_doubles();

// matvec.hip
// Scale c applied to the points of the low-precision operands, so that the
// squared distance of the operands is (c r)^2 and the kernel needs no
// hyperparameter in its pair loop: sqrt(log2(e) / 2) / ell for RBF,
// sqrt(nu2) log2(e) / ell for Matern (nu2 = 3, 5).
double point_scale(int kernel, double ell);
// ln 2 and ln^2 2 / 3, the latter derived from the former at compile time
constexpr double kLn2d = 0.6931471805599453;   // the double nearest ln 2
constexpr double kLn2Sq3d = kLn2d * kLn2d / 3.0;
constexpr float kLn2 = static_cast<float>(kLn2d);
constexpr float kLn2Sq3 = static_cast<float>(kLn2Sq3d);
int launch_symv_sweep(const dcg_operator_s *op, int mv, const int *done);
// wide.hip: the LDS-staged sweep of bf16 / fp16 operands with d > kMaxD
int launch_symv_wide(const dcg_operator_s *op, const SymvArgs &a, int64_t grid);
int launch_symv_sweep_from(const dcg_operator_s *op, int mv, const float *vin, const int *done);
SymvArgs symv_args(const dcg_operator_s *op, int mv, const float *vin, const int *done,
                   int64_t *grid);
bool symv_batched_supported(int opk, int ksteps);
int launch_symv_batched(const BatchItem *d_items, int count, int64_t total, int ksteps, int opk,
                        hipStream_t s);
ReduceArgs reduce_args(const dcg_operator_s *op, int mv, const double *V, double *Y);
int matvec_lowprec(const dcg_operator_s *op, const double *V, double *Y, int64_t m);
// The block solve behind dcg_solve_block, optionally recording every
// column's CG coefficients (the Lanczos tridiagonal of stochastic Lanczos
// quadrature) and returning per-column step counts and |b_c|.
int solve_block_impl(dcg_operator_s *op, const double *B, double *X, int64_t m,
                     dcg_recycle_s *rc, const dcg_params *p, dcg_stats *st, void *ws,
                     size_t ws_bytes, double *lz, int lz_cap, int *col_iters, double *col_bnorm);
// The stored operator (DCG_PREC_STORED): build K0 from the points, products.
int stored_build_launch(const dcg_operator_s *op);
int stored_tune(dcg_operator_s *op, int reps, int *items_out, double *ms_out);
size_t stored_matrix_floats(int64_t n_pad);     // packed block upper triangle
size_t stored_partial_doubles(int64_t n_pad);   // row and column partials of a product
int matvec_stored_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                       const int *done);
int matvec_exact(const dcg_operator_s *op, const double *V, double *Y, int64_t m);
int matvec_exact_timed(const dcg_operator_s *op, const double *V, double *Y, hipEvent_t ev0,
                       hipEvent_t ev1);
int matvec_exact_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                      const int *done);
int prepare_operator(dcg_operator_s *op, const double *X);

// solver.hip
int deflation_setup(dcg_operator_s *op, dcg_recycle_s *rc, int *matvecs);

}  // namespace dcg
