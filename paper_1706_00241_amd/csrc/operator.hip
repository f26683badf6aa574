// Operator set-up (point rounding, augmented MFMA operands) and the exact
// FP64 product used for the residuals of iterative refinement.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "blas.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int dp_bucket(int d) { return d <= 8 ? 8 : d <= 16 ? 16 : d <= 32 ? 32 : 64; }

// Round an FP64 value to bfloat16, to nearest with ties to even, in one
// rounding step from the FP64 value (8 significant bits).  Values below the
// smallest normal bfloat16 are flushed to zero.
__device__ __forceinline__ uint16_t bf16_from_double(double x) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
  const uint64_t sign = u >> 63;
  const uint64_t mag = u & 0x7fffffffffffffffull;
  const int e = static_cast<int>(mag >> 52) - 1023;
  if (mag == 0 || e < -126) return static_cast<uint16_t>(sign << 15);
  uint64_t comb = (uint64_t(e + 127) << 52) | (mag & ((1ull << 52) - 1));
  comb += ((1ull << 44) - 1) + ((comb >> 45) & 1ull);
  uint64_t r = comb >> 45;
  if (r >= 0x7f80) r = 0x7f80;
  return static_cast<uint16_t>((sign << 15) | r);
}

__device__ __forceinline__ double bf16_to_double(uint16_t h) {
  return static_cast<double>(__uint_as_float(uint32_t(h) << 16));
}

__global__ __launch_bounds__(256) void check_finite(const double *X, int64_t count, int *flag) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * 256)
    if (!isfinite(X[e])) atomicOr(flag, 1);
}

// One thread per (padded) point: rounded coordinates, squared norm from the
// rounded coordinates, and the augmented row / column operands.
__global__ __launch_bounds__(256) void prepare_points(const double *X, int64_t n, int64_t n_pad,
                                                      int d, int prec, int kstride, int dp,
                                                      void *xr, void *xc, double *X64) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const bool real = i < n;
  double a = 0.0;
  if (prec == DCG_PREC_FP64) {
    // exact operator: only the FP64 copy below
  } else if (prec == DCG_PREC_BF16) {
    uint16_t *r = static_cast<uint16_t *>(xr) + i * kstride;
    uint16_t *c = static_cast<uint16_t *>(xc) + i * kstride;
    for (int t = 0; t < d; ++t) {
      const uint16_t h = real ? bf16_from_double(X[i * d + t]) : uint16_t(0);
      const double xv = bf16_to_double(h);
      a += xv * xv;
      c[t] = h;
      r[t] = bf16_from_double(-2.0 * xv);  // exact: exponent + 1
    }
    const uint16_t ah = bf16_from_double(a);
    const double rem1 = a - bf16_to_double(ah);
    const uint16_t am = bf16_from_double(rem1);
    const uint16_t al = bf16_from_double(rem1 - bf16_to_double(am));
    const uint16_t one = 0x3F80;
    r[d + 0] = one; r[d + 1] = one; r[d + 2] = one;
    r[d + 3] = ah;  r[d + 4] = am;  r[d + 5] = al;
    c[d + 0] = ah;  c[d + 1] = am;  c[d + 2] = al;
    c[d + 3] = one; c[d + 4] = one; c[d + 5] = one;
    for (int t = d + 6; t < kstride; ++t) r[t] = c[t] = 0;
  } else {
    float *r = static_cast<float *>(xr) + i * kstride;
    float *c = static_cast<float *>(xc) + i * kstride;
    const int half = kstride / 2;
    for (int t = 0; t < kstride; ++t) r[t] = c[t] = 0.0f;
    for (int t = 0; t < d; ++t) {
      const float xv = real ? static_cast<float>(X[i * d + t]) : 0.0f;
      a += double(xv) * double(xv);
      c[(t & 1) * half + (t >> 1)] = xv;
      r[(t & 1) * half + (t >> 1)] = -2.0f * xv;
    }
    const float af = static_cast<float>(a);
    r[(d & 1) * half + (d >> 1)] = 1.0f;
    r[((d + 1) & 1) * half + ((d + 1) >> 1)] = af;
    c[(d & 1) * half + (d >> 1)] = af;
    c[((d + 1) & 1) * half + ((d + 1) >> 1)] = 1.0f;
  }
  for (int t = 0; t < dp; ++t) X64[i * dp + t] = (real && t < d) ? X[i * d + t] : 0.0;
}

// ------------------------------------------------------ exact FP64 product

template <int KERN>
__device__ __forceinline__ double kval64(double r2, double ell) {
  if constexpr (KERN == DCG_RBF) {
    return exp(-r2 / (2.0 * ell * ell));
  } else if constexpr (KERN == DCG_MATERN32) {
    const double t = sqrt(3.0 * r2) / ell;
    return (1.0 + t) * exp(-t);
  } else {
    const double t = sqrt(5.0 * r2) / ell;
    return (1.0 + t + t * t / 3.0) * exp(-t);
  }
}

// Y = s2 K V + sigma2 V in FP64 from the unrounded points (difference-form
// distances), up to 4 vectors; one thread per row, column tiles in LDS.
template <int KERN, int DP>
__global__ __launch_bounds__(256) void exact_matvec_kernel(const double *Xp, int64_t n,
                                                           int64_t n_pad, const double *V,
                                                           double *Y, int m, double ell, double s2,
                                                           double sigma2, const int *done) {
  if (done != nullptr && *done != 0) return;
  __shared__ double xs[64][DP + 1];
  __shared__ double vs[4][64];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double xi[DP];
#pragma unroll
  for (int t = 0; t < DP; ++t) xi[t] = (i < n_pad) ? Xp[i * DP + t] : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t j0 = 0; j0 < n; j0 += 64) {
    for (int e = threadIdx.x; e < 64 * DP; e += 256) {
      const int jj = e / DP, t = e % DP;
      const int64_t j = j0 + jj;
      xs[jj][t] = (j < n_pad) ? Xp[j * DP + t] : 0.0;
    }
    for (int e = threadIdx.x; e < 4 * 64; e += 256) {
      const int mm = e / 64, jj = e % 64;
      const int64_t j = j0 + jj;
      vs[mm][jj] = (mm < m && j < n) ? V[mm * n + j] : 0.0;
    }
    __syncthreads();
    const int jn = static_cast<int>(std::min<int64_t>(64, n - j0));
    for (int jj = 0; jj < jn; ++jj) {
      double r2 = 0.0;
#pragma unroll
      for (int t = 0; t < DP; ++t) {
        const double df = xi[t] - xs[jj][t];
        r2 = fma(df, df, r2);
      }
      const double kv = kval64<KERN>(r2, ell);
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) acc[mm] = fma(kv, vs[mm][jj], acc[mm]);
    }
    __syncthreads();
  }
  if (i < n) {
    for (int mm = 0; mm < m; ++mm) Y[mm * n + i] = s2 * acc[mm] + sigma2 * V[mm * n + i];
  }
}

template <int KERN>
static void launch_exact(const dcg_operator_s *op, const double *V, double *Y, int m,
                         const int *done) {
  const int dp = dp_bucket(op->g.d);
  const dim3 grid(static_cast<unsigned>(cdiv(op->g.n, 256)));
  const int64_t n = op->g.n, np = op->g.n_pad;
  switch (dp) {
    case 8: hipLaunchKernelGGL((exact_matvec_kernel<KERN, 8>), grid, dim3(256), 0, op->stream, op->X64, n, np, V, Y, m, op->ell, op->s2, op->sigma2, done); break;
    case 16: hipLaunchKernelGGL((exact_matvec_kernel<KERN, 16>), grid, dim3(256), 0, op->stream, op->X64, n, np, V, Y, m, op->ell, op->s2, op->sigma2, done); break;
    case 32: hipLaunchKernelGGL((exact_matvec_kernel<KERN, 32>), grid, dim3(256), 0, op->stream, op->X64, n, np, V, Y, m, op->ell, op->s2, op->sigma2, done); break;
    default: hipLaunchKernelGGL((exact_matvec_kernel<KERN, 64>), grid, dim3(256), 0, op->stream, op->X64, n, np, V, Y, m, op->ell, op->s2, op->sigma2, done); break;
  }
}

int matvec_exact_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                      const int *done) {
  for (int64_t c = 0; c < m; c += 4) {
    const int mm = static_cast<int>(std::min<int64_t>(4, m - c));
    const double *Vc = V + c * op->g.n;
    double *Yc = Y + c * op->g.n;
    if (op->kernel == DCG_RBF) launch_exact<DCG_RBF>(op, Vc, Yc, mm, done);
    else if (op->kernel == DCG_MATERN32) launch_exact<DCG_MATERN32>(op, Vc, Yc, mm, done);
    else launch_exact<DCG_MATERN52>(op, Vc, Yc, mm, done);
    if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  }
  return DCG_OK;
}

int matvec_exact(const dcg_operator_s *op, const double *V, double *Y, int64_t m) {
  return matvec_exact_done(op, V, Y, m, nullptr);
}

// ----------------------------------------------------------- workspace

struct OpLayout {
  size_t x64, xr, xc, vin, part, ytmp, flag, total;
};

static OpLayout op_layout(const Geometry &g) {
  const int dp = dp_bucket(g.d);
  const size_t esz = (g.prec == DCG_PREC_BF16) ? 2 : (g.prec == DCG_PREC_FP64 ? 0 : 4);
  Carve c(nullptr, 0);
  OpLayout L;
  L.x64 = c.off = align256(c.off); c.off += size_t(g.n_pad) * dp * 8;
  L.xr = c.off = align256(c.off); c.off += size_t(g.n_pad) * g.kstride * esz;
  L.xc = c.off = align256(c.off); c.off += size_t(g.n_pad) * g.kstride * esz;
  L.vin = c.off = align256(c.off); c.off += size_t(g.n_pad) * 4 * 4;
  L.part = c.off = align256(c.off);
  c.off += std::max(matvec_partial_floats(g.n_pad, 1), matvec_partial_floats(g.n_pad, 4)) * 4;
  L.ytmp = c.off = align256(c.off); c.off += size_t(g.n_pad) * 4 * 8;
  L.flag = c.off = align256(c.off); c.off += 256;
  L.total = align256(c.off);
  return L;
}

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_operator_workspace_bytes(int64_t n, int64_t d, int prec) {
  if (n < 1 || d < 1 || d > kMaxD) return 0;
  if (prec != DCG_PREC_FP32 && prec != DCG_PREC_BF16 && prec != DCG_PREC_FP64) return 0;
  return op_layout(make_geometry(n, static_cast<int>(d), prec)).total;
}

int dcg_create_operator(const double *X, int64_t n, int64_t d, int kernel, double ell, double s2,
                        double sigma2, int prec, void *workspace, size_t ws_bytes, void *stream,
                        dcg_op_t *out) {
  if (out == nullptr) return DCG_E_ARG;
  *out = nullptr;
  if (X == nullptr || n < 1 || d < 1 || d > kMaxD) return DCG_E_ARG;
  if (kernel < DCG_RBF || kernel > DCG_MATERN52) return DCG_E_ARG;
  if (prec != DCG_PREC_FP32 && prec != DCG_PREC_BF16 && prec != DCG_PREC_FP64) return DCG_E_ARG;
  if (!(ell > 0.0) || !(s2 > 0.0) || !(sigma2 >= 0.0) || !std::isfinite(ell) ||
      !std::isfinite(s2) || !std::isfinite(sigma2))
    return DCG_E_ARG;
  if (prec == DCG_PREC_BF16 && d + 6 > 80) return DCG_E_ARG;
  const Geometry g = make_geometry(n, static_cast<int>(d), prec);
  if (g.ksteps < 0) return DCG_E_ARG;
  const OpLayout L = op_layout(g);
  if (workspace == nullptr || ws_bytes < L.total) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return DCG_E_WORKSPACE;
  dcg_operator_s *op = new (std::nothrow) dcg_operator_s;
  if (op == nullptr) return DCG_E_ARG;
  char *base = static_cast<char *>(workspace);
  op->g = g;
  op->kernel = kernel;
  op->ell = ell;
  op->s2 = s2;
  op->sigma2 = sigma2;
  op->stream = static_cast<hipStream_t>(stream);
  op->generation = 1;
  op->X64 = reinterpret_cast<double *>(base + L.x64);
  op->xr = base + L.xr;
  op->xc = base + L.xc;
  op->vin = reinterpret_cast<float *>(base + L.vin);
  op->part = reinterpret_cast<float *>(base + L.part);
  op->ytmp = reinterpret_cast<double *>(base + L.ytmp);
  int *flag = reinterpret_cast<int *>(base + L.flag);
  int hflag = 0;
  bool ok = hipMemsetAsync(flag, 0, sizeof(int), op->stream) == hipSuccess;
  const int64_t count = n * d;
  hipLaunchKernelGGL(check_finite, dim3(static_cast<unsigned>(std::min<int64_t>(1024, cdiv(count, 256)))),
                     dim3(256), 0, op->stream, X, count, flag);
  hipLaunchKernelGGL(prepare_points, dim3(static_cast<unsigned>(cdiv(g.n_pad, 256))), dim3(256), 0,
                     op->stream, X, n, g.n_pad, g.d, g.prec, g.kstride, dp_bucket(g.d), op->xr,
                     op->xc, op->X64);
  ok = ok && hipGetLastError() == hipSuccess;
  ok = ok && hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, op->stream) == hipSuccess;
  ok = ok && hipStreamSynchronize(op->stream) == hipSuccess;
  if (!ok) {
    delete op;
    return DCG_E_HIP;
  }
  if (hflag != 0) {
    delete op;
    return DCG_E_NONFINITE;
  }
  *out = op;
  return DCG_OK;
}

int dcg_set_hyper(dcg_op_t op, double ell, double s2, double sigma2) {
  if (op == nullptr) return DCG_E_ARG;
  if (!(ell > 0.0) || !(s2 > 0.0) || !(sigma2 >= 0.0) || !std::isfinite(ell) ||
      !std::isfinite(s2) || !std::isfinite(sigma2))
    return DCG_E_ARG;
  op->ell = ell;
  op->s2 = s2;
  op->sigma2 = sigma2;
  op->generation += 1;
  return DCG_OK;
}

int dcg_matvec(dcg_op_t op, const double *V, double *Y, int64_t m) {
  if (op == nullptr || V == nullptr || Y == nullptr || m < 1) return DCG_E_ARG;
  return matvec_lowprec(op, V, Y, m);
}

int dcg_matvec_exact(dcg_op_t op, const double *V, double *Y, int64_t m) {
  if (op == nullptr || V == nullptr || Y == nullptr || m < 1) return DCG_E_ARG;
  return matvec_exact(op, V, Y, m);
}

void dcg_destroy_operator(dcg_op_t op) { delete op; }

const char *dcg_status_string(int status) {
  switch (status) {
    case DCG_OK: return "ok";
    case DCG_NOT_CONVERGED: return "not converged (max_iter reached)";
    case DCG_E_ARG: return "invalid argument";
    case DCG_E_NOT_SPD: return "operator not positive definite (p^T A p <= 0)";
    case DCG_E_NONFINITE: return "non-finite value";
    case DCG_E_W_RANK: return "recycled basis rank deficient";
    case DCG_E_HIP: return "HIP runtime error";
    case DCG_E_WORKSPACE: return "workspace too small or misaligned";
  }
  return "unknown status";
}

const char *dcg_version(void) { return "dcg-mi355x 0.1 (gfx950)"; }

}  // extern "C"
