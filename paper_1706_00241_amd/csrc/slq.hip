// Log-determinant by stochastic Lanczos quadrature, from the coefficients of
// the CG probe solves (the forward value of the GP log marginal likelihood,
// whose gradient the probe solves already serve).
//
// For SPD A and a probe z, m steps of CG on A x = z from x = 0 define the
// Lanczos tridiagonal T_m of (A, z / |z|) through their coefficients:
//   T_00 = 1 / alpha_0,  T_jj = 1 / alpha_j + beta_{j-1} / alpha_{j-1},
//   T_{j,j+1} = sqrt(beta_j) / alpha_j,
// and z^T log(A) z is approximated by the m-node Gauss quadrature
//   |z|^2 e_1^T log(T_m) e_1 = |z|^2 sum_i tau_i^2 log theta_i
// (theta_i the eigenvalues of T_m, tau_i the first components of its unit
// eigenvectors; Golub & Meurant).  With Rademacher probes the mean over
// probes estimates tr log A = log det A (Hutchinson).
//
// The probes run as one block solve without recycling (a recycled W would
// change the Krylov space the coefficients describe); each step records
// alpha_j and beta_j per column on the device.  The small eigenproblems are
// solved on the host by implicit symmetric QR steps with Wilkinson shifts
// (Golub & Van Loan, section 8.3), carrying only the first row of the
// eigenvector matrix.

#include <algorithm>
#include <cmath>
#include <vector>

#include "blas.h"
#include "common.h"
#include "host.h"

namespace dcg {

constexpr int kSlqMaxSteps = 4096;

static size_t slq_block_bytes(int64_t n, int64_t P) { return align256(dcg_solve_block_workspace_bytes(n, P)); }

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_slq_logdet_workspace_bytes(int64_t n, int64_t P, int max_steps) {
  if (n < 1 || P < 1 || P > kMaxBlockCols || max_steps < 1 || max_steps > kSlqMaxSteps) return 0;
  return slq_block_bytes(n, P) + align256(size_t(n) * P * 8) +
         align256(size_t(P) * 2 * max_steps * 8);
}

int dcg_slq_logdet(dcg_op_t op, const double *Z, int64_t P, const dcg_params *p, int max_steps,
                   double *quad, int *steps, double *logdet, void *ws, size_t ws_bytes) {
  if (op == nullptr || Z == nullptr || p == nullptr || quad == nullptr) return DCG_E_ARG;
  if (P < 1 || P > kMaxBlockCols || max_steps < 1 || max_steps > kSlqMaxSteps) return DCG_E_ARG;
  const int64_t n = op->g.n;
  const size_t need = dcg_slq_logdet_workspace_bytes(n, P, max_steps);
  if (ws == nullptr || ws_bytes < need) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  char *b = static_cast<char *>(ws);
  const size_t blk = slq_block_bytes(n, P);
  double *X = reinterpret_cast<double *>(b + blk);
  double *lz = reinterpret_cast<double *>(b + blk + align256(size_t(n) * P * 8));
  std::vector<int> its(static_cast<size_t>(P));
  std::vector<double> bn(static_cast<size_t>(P));
  dcg_stats st;
  int status = solve_block_impl(op, Z, X, P, nullptr, p, &st, ws, blk, lz, max_steps, its.data(),
                                bn.data());
  if (status < 0) return status;
  std::vector<double> h(size_t(P) * 2 * max_steps);
  if (hipMemcpyAsync(h.data(), lz, h.size() * sizeof(double), hipMemcpyDeviceToHost, op->stream) !=
          hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return DCG_E_HIP;
  double sum = 0.0;
  for (int64_t c = 0; c < P; ++c) {
    const int m = std::min(its[static_cast<size_t>(c)], max_steps);
    const double *al = h.data() + size_t(c) * 2 * max_steps;
    const double bn2 = bn[static_cast<size_t>(c)] * bn[static_cast<size_t>(c)];
    const int qs = slq_quadrature(al, al + max_steps, m, bn2, &quad[c]);
    if (qs != DCG_OK) return qs;
    if (steps != nullptr) steps[c] = m;
    sum += quad[c];
  }
  if (logdet != nullptr) *logdet = sum / static_cast<double>(P);
  return status;
}

}  // extern "C"
