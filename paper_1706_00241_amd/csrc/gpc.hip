// Gaussian process classification by the Laplace approximation (section 3,
// Eqs. 8-10): Newton's method for the mode of the latent function, each
// step solving A = I + D K D, b = D K b~ (D = H^{1/2}, H the diagonal of the
// negative Hessian of the logistic log-likelihood) by deflated CG, with W
// carried from one Newton system to the next.
//
// Per Newton step, with t = (y + 1) / 2 and pi = sigma(f):
//   H = pi (1 - pi),  D = sqrt(H),  b~ = H f + (t - pi),
//   b = D (K b~),  z = A^{-1} b,  a = b~ - D z,  f = K a,
//   Psi = sum_i log sigma(y_i f_i) - a^T f / 2,
// stopping when Psi grows by less than a tolerance.  D goes straight into
// the operator's diagonal scaling, so every product of the solve is the
// scaled pair sweep.

#include <algorithm>
#include <cmath>
#include <vector>

#include "blas.h"
#include "common.h"

namespace dcg {

constexpr int kPsiBlocks = 128;

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Labels must be -1 or +1.
__global__ __launch_bounds__(256) void gpc_check_labels(const double *y, int64_t n, int *flag) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n && y[i] != 1.0 && y[i] != -1.0) atomicOr(flag, 1);
}

// pi = sigma(f), H = pi (1 - pi): D = sqrt(H) into the operator's scaling
// (zero past n), b~ = H f + (t - pi).
__global__ __launch_bounds__(256) void gpc_terms(const double *y, const double *f, int64_t n,
                                                 int64_t n_pad, double *dsc, double *bt) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  if (i >= n) {
    dsc[i] = 0.0;
    return;
  }
  const double fi = f[i];
  const double pi = 1.0 / (1.0 + exp(-fi));
  const double h = pi * (1.0 - pi);
  dsc[i] = sqrt(h);
  bt[i] = h * fi + (0.5 * (y[i] + 1.0) - pi);
}

// out = D u.
__global__ __launch_bounds__(256) void gpc_scale(const double *dsc, const double *u, int64_t n,
                                                 double *out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) out[i] = dsc[i] * u[i];
}

// a = b~ - D z.
__global__ __launch_bounds__(256) void gpc_update_a(const double *bt, const double *dsc,
                                                    const double *z, int64_t n, double *a) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) a[i] = bt[i] - dsc[i] * z[i];
}

// Block partial sums of log sigma(y_i f_i) - a_i f_i / 2 (grid-stride over
// kPsiBlocks blocks; the host adds the partials in order).  log sigma(s) =
// -(max(-s, 0) + log1p(e^{-|s|})) stays finite for any s.
__global__ __launch_bounds__(256) void gpc_psi(const double *y, const double *f, const double *a,
                                               int64_t n, double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * 256) {
    const double s = y[i] * f[i];
    acc += -(fmax(-s, 0.0) + log1p(exp(-fabs(s)))) - 0.5 * a[i] * f[i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

struct GpcLayout {
  size_t solve, bt, u, z, part, flag, total;
};

static GpcLayout gpc_layout(int64_t n) {
  GpcLayout L;
  Carve c(nullptr, 0);
  L.solve = c.off = 0;
  c.off += dcg_solve_workspace_bytes(n, 0, 0);
  L.bt = c.off = align256(c.off); c.off += size_t(n) * 8;
  L.u = c.off = align256(c.off); c.off += size_t(n) * 8;
  L.z = c.off = align256(c.off); c.off += size_t(n) * 8;
  L.part = c.off = align256(c.off); c.off += kPsiBlocks * 8;
  L.flag = c.off = align256(c.off); c.off += 256;
  L.total = align256(c.off);
  return L;
}

// Y = K V (one vector): the kernel part s2 K0 alone, without the diagonal
// scaling and the shift, with the FP64 operator when `exact`.
static int k_product(dcg_operator_s *op, const double *V, double *Y, bool exact) {
  const double sigma2 = op->sigma2;
  const int has_dsc = op->has_dsc;
  op->sigma2 = 0.0;
  op->has_dsc = 0;
  // kernel arguments are taken at launch: the fields can be restored at once
  const int st = exact ? matvec_exact(op, V, Y, 1) : matvec_lowprec(op, V, Y, 1);
  op->sigma2 = sigma2;
  op->has_dsc = has_dsc;
  return st;
}

static int psi_value(const dcg_operator_s *op, const double *y, const double *f, const double *a,
                     double *part, double *out) {
  const int64_t n = op->g.n;
  const int blocks = static_cast<int>(std::min<int64_t>(kPsiBlocks, cdiv(n, 256)));
  hipLaunchKernelGGL(gpc_psi, dim3(blocks), dim3(256), 0, op->stream, y, f, a, n, part);
  if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  double h[kPsiBlocks];
  if (hipMemcpyAsync(h, part, sizeof(double) * blocks, hipMemcpyDeviceToHost, op->stream) !=
          hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return DCG_E_HIP;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += h[b];
  *out = s;
  return std::isfinite(s) ? DCG_OK : DCG_E_NONFINITE;
}

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_laplace_gpc_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return gpc_layout(n).total;
}

int dcg_laplace_gpc(dcg_op_t op, const double *y, dcg_recycle_t rc, const dcg_params *p,
                    int max_newton, double psi_tol, double *f, double *a, double *psi,
                    int *newton_steps, dcg_stats *stats, void *ws, size_t ws_bytes) {
  if (newton_steps != nullptr) *newton_steps = 0;
  if (op == nullptr || y == nullptr || p == nullptr || f == nullptr || a == nullptr)
    return DCG_E_ARG;
  if (max_newton < 1 || !(psi_tol >= 0.0) || op->has_dsc) return DCG_E_ARG;
  if (rc != nullptr && rc->n != op->g.n) return DCG_E_ARG;
  // refinement needs the FP64 operator, which the stored operator does not
  // have (checked before any work is enqueued)
  if (!has_exact(op) && p->refine != 0) return DCG_E_ARG;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  const GpcLayout L = gpc_layout(n);
  if (ws == nullptr || ws_bytes < L.total) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  char *b = static_cast<char *>(ws);
  double *bt = reinterpret_cast<double *>(b + L.bt);
  double *u = reinterpret_cast<double *>(b + L.u);
  double *z = reinterpret_cast<double *>(b + L.z);
  double *part = reinterpret_cast<double *>(b + L.part);
  int *flag = reinterpret_cast<int *>(b + L.flag);
  hipStream_t s = op->stream;
  const dim3 g1(static_cast<unsigned>(cdiv(n, 256))), gp(static_cast<unsigned>(cdiv(n_pad, 256)));
  const dim3 blk(256);

  int h = 0;
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return DCG_E_HIP;
  hipLaunchKernelGGL(gpc_check_labels, g1, blk, 0, s, y, n, flag);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DCG_E_HIP;
  if (h != 0) return DCG_E_ARG;

  // f_0 = 0, a_0 = 0
  if (hipMemsetAsync(f, 0, sizeof(double) * n, s) != hipSuccess ||
      hipMemsetAsync(a, 0, sizeof(double) * n, s) != hipSuccess)
    return DCG_E_HIP;
  const bool exact = op->g.prec == DCG_PREC_FP64 || p->refine > 0;
  const double sigma2_user = op->sigma2;
  double psi_prev = 0.0;
  int code = psi_value(op, y, f, a, part, &psi_prev);
  if (code != DCG_OK) return code;
  if (psi != nullptr) psi[0] = psi_prev;

  int steps = 0;
  code = DCG_NOT_CONVERGED;
  while (steps < max_newton) {
    // the system of this Newton step (Eqs. 9-10)
    hipLaunchKernelGGL(gpc_terms, gp, blk, 0, s, y, f, n, n_pad, op->dsc, bt);
    if (hipGetLastError() != hipSuccess) {
      code = DCG_E_HIP;
      break;
    }
    int st = k_product(op, bt, u, exact);
    if (st != DCG_OK) {
      code = st;
      break;
    }
    hipLaunchKernelGGL(gpc_scale, g1, blk, 0, s, op->dsc, u, n, u);
    // A = I + D K D: unit shift, the new scaling
    op->sigma2 = 1.0;
    op->has_dsc = 1;
    op->dsc_version += 1;
    op->generation += 1;
    dcg_stats local;
    dcg_stats *sst = (stats != nullptr) ? &stats[steps] : &local;
    st = dcg_solve(op, u, z, 0, rc, p, sst, b + L.solve, L.bt - L.solve);
    op->has_dsc = 0;
    op->sigma2 = sigma2_user;
    if (st < 0) {
      code = st;
      break;
    }
    hipLaunchKernelGGL(gpc_update_a, g1, blk, 0, s, bt, op->dsc, z, n, a);
    if (hipGetLastError() != hipSuccess) {
      code = DCG_E_HIP;
      break;
    }
    st = k_product(op, a, f, exact);
    if (st != DCG_OK) {
      code = st;
      break;
    }
    double psi_new = 0.0;
    st = psi_value(op, y, f, a, part, &psi_new);
    steps += 1;
    if (psi != nullptr) psi[steps] = psi_new;
    if (st != DCG_OK) {
      code = st;
      break;
    }
    const bool done = psi_new - psi_prev < psi_tol;
    psi_prev = psi_new;
    if (done) {
      code = DCG_OK;
      break;
    }
  }
  // the operator leaves as it came: no scaling, the caller's shift
  op->has_dsc = 0;
  op->sigma2 = sigma2_user;
  op->dsc_version += 1;
  op->generation += 1;
  if (newton_steps != nullptr) *newton_steps = steps;
  if (hipStreamSynchronize(s) != hipSuccess && code >= 0) code = DCG_E_HIP;
  return code;
}

size_t dcg_laplace_evidence_workspace_bytes(int64_t n, int64_t P, int max_steps) {
  const size_t slq = dcg_slq_logdet_workspace_bytes(n, P, max_steps);
  if (slq == 0) return 0;
  return align256(slq) + align256(size_t(n) * 8) + align256(kPsiBlocks * 8);
}

int dcg_laplace_evidence(dcg_op_t op, const double *y, const double *f, const double *a,
                         const double *Z, int64_t P, const dcg_params *p, int max_steps,
                         double *evidence, double *psi, double *logdet, void *ws,
                         size_t ws_bytes) {
  if (op == nullptr || y == nullptr || f == nullptr || a == nullptr || Z == nullptr ||
      p == nullptr || evidence == nullptr)
    return DCG_E_ARG;
  // the probe solves take the scaling only where each product is formed on
  // its own (FP64 and stored operators)
  if (op->has_dsc || (op->g.prec != DCG_PREC_FP64 && op->g.prec != DCG_PREC_STORED))
    return DCG_E_ARG;
  const size_t need = dcg_laplace_evidence_workspace_bytes(op->g.n, P, max_steps);
  if (need == 0) return DCG_E_ARG;
  if (ws == nullptr || ws_bytes < need) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  const size_t slq = align256(dcg_slq_logdet_workspace_bytes(n, P, max_steps));
  char *b = static_cast<char *>(ws);
  double *bt = reinterpret_cast<double *>(b + slq);
  double *part = reinterpret_cast<double *>(b + slq + align256(size_t(n) * 8));
  double ps = 0.0;
  int code = psi_value(op, y, f, a, part, &ps);
  if (code != DCG_OK) return code;
  // D = H^{1/2} at f into the operator's scaling; B = I + D K D
  hipLaunchKernelGGL(gpc_terms, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                     op->stream, y, f, n, n_pad, op->dsc, bt);
  if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  const double sigma2_user = op->sigma2;
  op->sigma2 = 1.0;
  op->has_dsc = 1;
  op->dsc_version += 1;
  op->generation += 1;
  std::vector<double> quad(static_cast<size_t>(P));
  double ld = 0.0;
  code = dcg_slq_logdet(op, Z, P, p, max_steps, quad.data(), nullptr, &ld, ws, slq);
  op->has_dsc = 0;
  op->sigma2 = sigma2_user;
  op->dsc_version += 1;
  op->generation += 1;
  if (code < 0) return code;
  *evidence = ps - 0.5 * ld;
  if (psi != nullptr) *psi = ps;
  if (logdet != nullptr) *logdet = ld;
  return code;
}

}  // extern "C"
