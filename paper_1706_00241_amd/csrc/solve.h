// The phases of one deflated-CG solve (Algorithm 1 of the paper), shared by
// the single-system driver and the batched driver.
#pragma once

#include <chrono>

#include "blas.h"

namespace dcg {

using Clock = std::chrono::steady_clock;
inline double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

#define HIPCHK(x)                                      \
  do {                                                 \
    if ((x) != hipSuccess) return DCG_E_HIP;           \
  } while (0)

// Device buffers of one solve, carved from the caller's solve workspace.
struct SolveBuffers {
  SolveState *S;
  unsigned *counter;
  double *r, *p, *q, *part, *part_h, *hist_res, *hist_d, *hist_alpha, *hist_beta;
  double *hist_rho, *hist_mu, *hist_c;   // the implicit extraction's records
  double *tmp1, *tmp2, *tmp3;
  double *fD, *fQ;   // refinement directions (only with a refinement-sized workspace)
};

struct InnerResult {
  int iters = 0, matvecs = 0, k_used = 0, k_next = 0, status = DCG_OK;
  int sweeps_timed = 0;
  double t_sweeps = 0.0;
  double relres = 0.0;
  double t_init = 0.0, t_loop = 0.0, t_refresh = 0.0;
};

// Where a solve keeps its first directions p_j and A p_j: columns off,
// off + 1, ... of the recycle handle's Z and AZ, at most `count` of them
// (off < 0: right after W, count < 0: the handle's L); `extract`: refresh the
// basis from Z[:, :off + stored] when the solve ends.
struct StorePlan {
  int off = -1, count = -1;
  bool extract = true;
};

// State carried between the phases of one solve.
struct SolveCtx {
  SolveBuffers B;
  CgArgs a;
  int k = 0, L = 0, koff = 0, matvecs = 0;
  double tol = 0.0;
  bool extract = true;
};

// Bytes of one solve's workspace; without the refinement's direction blocks
// when refine is false.
size_t solve_workspace_total(int64_t n, bool refine);
SolveBuffers solve_buffers(void *ws, int64_t n);

// Phase 1: AW, (W^T A W)^{-1}, r_0, the deflated start and p_0 (ends with a
// stream synchronisation).
int solve_init(dcg_operator_s *op, const double *b, double *x, int x_given, dcg_recycle_s *rc,
               const dcg_params *p, double tol, void *ws, const StorePlan &sp, SolveCtx *ctx,
               InnerResult *out);
// Phase 2: the CG steps until the device state says done.
int solve_loop(dcg_operator_s *op, const dcg_params *p, SolveCtx *ctx, InnerResult *out);
// Phase 3: the harmonic Ritz extraction of the next basis (section 2.3).
int solve_extract(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p, SolveCtx *ctx,
                  InnerResult *out);
// The extraction itself: W' = Z U from the first mz columns of Z / AZ.
int extract_basis(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p, int mz,
                  InnerResult *out);
// |b - A x| / |b| with the low-precision (exact = 0) or FP64 operator.
int true_residual(dcg_operator_s *op, const double *b, const double *x, int exact,
                  const SolveBuffers &B, double *rel);

}  // namespace dcg
