// The implicit extraction of the recycled basis (section 2.3: F and G of
// Eq. 7 formed from the quantities the iteration stores in its first L steps,
// as Saad et al. (2000) did, instead of from the tall products (AZ)^T Z and
// (AZ)^T AZ), and the coefficients that give AW' = (AZ) U without the stored
// products A P_L.
//
// Identities used (exact in exact arithmetic for the iterates of Algorithm 1
// with the library's re-projection; c_{j+1} its coefficients, zero in exact
// arithmetic):
//   F = blockdiag(M, diag(d_j))                (A-conjugacy of W, p_0, p_1, ...)
//   A p_j = (r_j - r_{j+1} - AW c_{j+1}) / alpha_j
//   (AW)^T r_j = M mu_j,  r_i^T r_j = 0 (i != j)
// with M = W^T A W and N = (AW)^T AW, so that
//   G_WW = N,  G_WP[:, j] = (M (mu_j - mu_{j+1}) - N c_{j+1}) / alpha_j,
//   G_PP[i, j] alpha_i alpha_j = R[i, j] - X[i, j] - X[j, i] + c_{i+1}^T N c_{j+1}
// where R is the residual Gram matrix of r_j - r_{j+1} (diagonal
// rho_j + rho_{j+1}, first off-diagonals -rho_{j+1}) and
// X[i, j] = (M (mu_i - mu_{i+1}))^T c_{j+1}.  The residuals follow from the
// directions, r_j = p_j - beta_{j-1} p_{j-1} + W mu_j, so
//   A p_j = [(1 + beta_j) p_j - beta_{j-1} p_{j-1} - p_{j+1}
//            + W (mu_j - mu_{j+1}) - AW c_{j+1}] / alpha_j
// and AW' = AW U_W + A P_L U_P = [W, P_{L+1}] S1 + AW S2 with small S1, S2.
#include "blas.h"

namespace dcg {

// Dm[j][c] = (M (mu_j - mu_{j+1}))_c and NC[j][c] = (N c_{j+1})_c, one block
// per step j (rows of kMaxK doubles in mu and cv).
__global__ __launch_bounds__(64) void implicit_terms(const double *M, const double *N, int k,
                                                     const double *mu, const double *cv,
                                                     double *Dm, double *NC) {
  const int j = blockIdx.x;
  __shared__ double dmu[kMaxK];
  __shared__ double cj[kMaxK];
  for (int e = threadIdx.x; e < k; e += 64) {
    dmu[e] = mu[int64_t(j) * kMaxK + e] - mu[int64_t(j + 1) * kMaxK + e];
    cj[e] = cv[int64_t(j) * kMaxK + e];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 64) {
    double s = 0.0, t = 0.0;
    for (int e = 0; e < k; ++e) {
      const double mce = 0.5 * (M[c * k + e] + M[e * k + c]);
      const double nce = 0.5 * (N[c * k + e] + N[e * k + c]);
      s += mce * dmu[e];
      t += nce * cj[e];
    }
    Dm[int64_t(j) * kMaxK + c] = s;
    NC[int64_t(j) * kMaxK + c] = t;
  }
}

// F and G (m x m row-major, m = k + L), one thread per entry; the entry
// (a, b) and (b, a) are formed by the same arithmetic, so both are exactly
// symmetric.
__global__ __launch_bounds__(256) void implicit_pencil(const double *M, const double *N, int k,
                                                       int L, const double *dv,
                                                       const double *alpha, const double *rho,
                                                       const double *cv, const double *Dm,
                                                       const double *NC, double *F, double *G) {
  const int m = k + L;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(m) * m) return;
  const int a = static_cast<int>(e / m), b = static_cast<int>(e % m);
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  double f = 0.0, g = 0.0;
  if (hi < k) {
    f = 0.5 * (M[lo * k + hi] + M[hi * k + lo]);
    g = 0.5 * (N[lo * k + hi] + N[hi * k + lo]);
  } else if (lo < k) {
    const int j = hi - k;
    g = (Dm[int64_t(j) * kMaxK + lo] - NC[int64_t(j) * kMaxK + lo]) / alpha[j];
  } else {
    const int i = lo - k, j = hi - k;
    if (i == j) f = dv[i];
    double s = 0.0;
    if (i == j) s = rho[i] + rho[i + 1];
    else if (j == i + 1) s = -rho[j];
    double x = 0.0;
    for (int c = 0; c < k; ++c) {
      const double ci = cv[int64_t(i) * kMaxK + c], cj = cv[int64_t(j) * kMaxK + c];
      x += Dm[int64_t(i) * kMaxK + c] * cj + Dm[int64_t(j) * kMaxK + c] * ci -
           ci * NC[int64_t(j) * kMaxK + c];
    }
    g = (s - x) / (alpha[i] * alpha[j]);
  }
  F[e] = f;
  G[e] = g;
}

// S1 ((k + L + 1) x kout, ld kMaxK) and S2 (k x kout, ld kMaxK) with
// AW' = [W, P_{L+1}] S1 + AW S2, from U (m x kout, ld kMaxK): the W rows of
// S1 are sum_j (mu_j - mu_{j+1}) / alpha_j U_P[j], its P rows the banded
// combination of U_P rows given by the residual recurrence, and
// S2 = U_W - sum_j c_{j+1} / alpha_j U_P[j].
__global__ __launch_bounds__(256) void implicit_aw_coef(const double *U, int k, int L, int kout,
                                                        const double *alpha, const double *beta,
                                                        const double *mu, const double *cv,
                                                        double *S1, double *S2) {
  const int rows = k + L + 1 + k;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(rows) * kout) return;
  const int row = static_cast<int>(e / kout), col = static_cast<int>(e % kout);
  auto up = [&](int j) { return U[int64_t(k + j) * kMaxK + col]; };
  double s = 0.0;
  if (row < k) {
    for (int j = 0; j < L; ++j)
      s += (mu[int64_t(j) * kMaxK + row] - mu[int64_t(j + 1) * kMaxK + row]) / alpha[j] * up(j);
    S1[int64_t(row) * kMaxK + col] = s;
  } else if (row < k + L + 1) {
    const int i = row - k;
    if (i < L) s += (1.0 + beta[i]) / alpha[i] * up(i);
    if (i + 1 < L) s -= beta[i] / alpha[i + 1] * up(i + 1);
    if (i >= 1) s -= up(i - 1) / alpha[i - 1];
    S1[int64_t(row) * kMaxK + col] = s;
  } else {
    const int c = row - (k + L + 1);
    s = U[int64_t(c) * kMaxK + col];
    for (int j = 0; j < L; ++j) s -= cv[int64_t(j) * kMaxK + c] / alpha[j] * up(j);
    S2[int64_t(c) * kMaxK + col] = s;
  }
}

void enqueue_implicit_pencil(hipStream_t s, const ImplicitHist &h, const double *M,
                             const double *N, int k, int L, double *scratch, double *F,
                             double *G) {
  double *Dm = scratch;
  double *NC = scratch + size_t(kMaxZ) * kMaxK;
  if (k > 0 && L > 0)
    hipLaunchKernelGGL(implicit_terms, dim3(static_cast<unsigned>(L)), dim3(64), 0, s, M, N, k,
                       h.mu, h.cv, Dm, NC);
  const int m = k + L;
  const int64_t cnt = int64_t(m) * m;
  hipLaunchKernelGGL(implicit_pencil, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0,
                     s, M, N, k, L, h.d, h.alpha, h.rho, h.cv, Dm, NC, F, G);
}

void enqueue_implicit_aw_coef(hipStream_t s, const ImplicitHist &h, const double *U, int k, int L,
                              int kout, double *S1, double *S2) {
  const int64_t cnt = int64_t(k + L + 1 + k) * kout;
  hipLaunchKernelGGL(implicit_aw_coef, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256),
                     0, s, U, k, L, kout, h.alpha, h.beta, h.mu, h.cv, S1, S2);
}

}  // namespace dcg
