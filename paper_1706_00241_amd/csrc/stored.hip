// The stored operator: the unit-amplitude kernel matrix K0 = K(X, X) / s2
// formed once in FP64 and kept in HBM as FP32 (n_pad x n_pad, row-major,
// zero rows and columns past n), for point dimensions too large for the
// matrix-free pair sweep (the classification data of section 3 has 784
// coordinates).  K0 is fixed while only s2, sigma2 or the diagonal scaling
// change (a Newton loop changes only D), so every product is one streaming
// pass over 4 n_pad^2 bytes: the HBM roofline, not the kernel evaluations.
//
//   y = s2 * D (K0 (D v)) + sigma2 v      (D = I without a scaling)
//
// Accumulation is FP64 (each FP32 entry widened before its fused
// multiply-add), so the product's error is the FP32 rounding of K0 alone.

#include <algorithm>
#include <cmath>

#include "blas.h"
#include "common.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBuildTile = 64;   // output tile of the build (64 x 64 per block)
constexpr int kBuildK = 16;      // coordinates per LDS stage

// Kernel value at squared scaled distance q = |x_i - x_j|^2 / ell^2 (FP64,
// unit amplitude): the textbook forms of the RBF and Matern kernels.
__device__ __forceinline__ double stored_kval(int kernel, double q) {
  if (kernel == DCG_RBF) return exp(-0.5 * q);
  const double r = sqrt(q);
  if (kernel == DCG_MATERN32) {
    const double t = 1.7320508075688772 * r;   // sqrt(3) r
    return (1.0 + t) * exp(-t);
  }
  const double t = 2.23606797749979 * r;       // sqrt(5) r
  return (1.0 + t + t * t / 3.0) * exp(-t);
}

// K0 in 64 x 64 tiles: squared distances in difference form (no
// cancellation, zero on the diagonal), coordinates staged through LDS 16 at
// a time, 4 x 4 outputs per thread.  x64: n_pad x d row-major FP64 with zero
// rows past n, so every tile's loads stay inside it.
__global__ __launch_bounds__(256) void stored_build(const double *x64, int64_t n, int64_t n_pad,
                                                   int d, int kernel, double inv_ell2,
                                                   float *K) {
  __shared__ double xa[kBuildK][kBuildTile + 1];
  __shared__ double xb[kBuildK][kBuildTile + 1];
  const int64_t i0 = int64_t(blockIdx.y) * kBuildTile, j0 = int64_t(blockIdx.x) * kBuildTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = 0; k0 < d; k0 += kBuildK) {
    for (int e = threadIdx.x; e < kBuildTile * kBuildK; e += 256) {
      const int r = e / kBuildK, k = e % kBuildK;
      const bool in = k0 + k < d;
      xa[k][r] = in ? x64[(i0 + r) * d + k0 + k] : 0.0;
      xb[k][r] = in ? x64[(j0 + r) * d + k0 + k] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < kBuildK; ++k) {
      double a[4], b[4];
      for (int u = 0; u < 4; ++u) {
        a[u] = xa[k][ty + 16 * u];
        b[u] = xb[k][tx + 16 * u];
      }
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
          const double df = a[u] - b[v];
          acc[u][v] = fma(df, df, acc[u][v]);
        }
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + ty + 16 * u;
    for (int v = 0; v < 4; ++v) {
      const int64_t j = j0 + tx + 16 * v;
      const float val =
          (i < n && j < n) ? static_cast<float>(stored_kval(kernel, acc[u][v] * inv_ell2)) : 0.0f;
      K[i * n_pad + j] = val;
    }
  }
}

// v (times the diagonal scaling if given) -> zero-padded FP64 copy.
__global__ __launch_bounds__(256) void stored_stage(const double *V, int64_t n, int64_t n_pad,
                                                    const double *dsc, double *out,
                                                    const int *done) {
  if (done != nullptr && *done != 0) return;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n_pad) out[i] = (i < n) ? ((dsc != nullptr) ? dsc[i] * V[i] : V[i]) : 0.0;
}

// y_i = s2 d_i (K0 xs)_i + sigma2 v_i for ROWS rows per block: every thread
// streams 16-byte pieces of the block's rows, UNROLL pieces per row at a
// time, so each thread keeps ROWS x UNROLL independent loads in flight;
// FP64 accumulators, then a wave shuffle and an LDS step across the 4 waves.
// K0 is read once per product with non-temporal loads, which keeps the
// caches for xs.  Fewer rows per block mean more blocks (a shorter tail on 256 compute
// units) but more re-reads of xs from L2; the tuner picks the variant.
template <int ROWS, int UNROLL>
__global__ __launch_bounds__(256) void stored_gemv(const float *K, int64_t n, int64_t n_pad,
                                                   const double *xs, double s2, double sigma2,
                                                   const double *dsc, const double *V, double *Y,
                                                   const int *done) {
  if (done != nullptr && *done != 0) return;
  __shared__ double red[4][ROWS];
  const int64_t r0 = int64_t(blockIdx.x) * ROWS;
  double acc[ROWS];
  for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
  const int64_t nq = n_pad / 4;
  const f32x4 *K4 = reinterpret_cast<const f32x4 *>(K + r0 * n_pad);
  const double2 *x2 = reinterpret_cast<const double2 *>(xs);
  int64_t q = threadIdx.x;
  for (; q + (UNROLL - 1) * 256 < nq; q += UNROLL * 256) {
    f32x4 kr[UNROLL][ROWS];
    double2 xa[UNROLL], xb[UNROLL];
    for (int u = 0; u < UNROLL; ++u) {
      xa[u] = x2[2 * (q + u * 256)];
      xb[u] = x2[2 * (q + u * 256) + 1];
      for (int r = 0; r < ROWS; ++r) kr[u][r] = __builtin_nontemporal_load(K4 + r * nq + q + u * 256);
    }
    for (int u = 0; u < UNROLL; ++u)
      for (int r = 0; r < ROWS; ++r) {
        double s = acc[r];
        s = fma(static_cast<double>(kr[u][r].x), xa[u].x, s);
        s = fma(static_cast<double>(kr[u][r].y), xa[u].y, s);
        s = fma(static_cast<double>(kr[u][r].z), xb[u].x, s);
        s = fma(static_cast<double>(kr[u][r].w), xb[u].y, s);
        acc[r] = s;
      }
  }
  for (; q < nq; q += 256) {
    const double2 xa = x2[2 * q], xb = x2[2 * q + 1];
    for (int r = 0; r < ROWS; ++r) {
      const f32x4 k = __builtin_nontemporal_load(K4 + r * nq + q);
      double s = acc[r];
      s = fma(static_cast<double>(k.x), xa.x, s);
      s = fma(static_cast<double>(k.y), xa.y, s);
      s = fma(static_cast<double>(k.z), xb.x, s);
      s = fma(static_cast<double>(k.w), xb.y, s);
      acc[r] = s;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < ROWS; ++r) {
    double s = acc[r];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wave][r] = s;
  }
  __syncthreads();
  if (threadIdx.x < ROWS) {
    const int r = threadIdx.x;
    const int64_t i = r0 + r;
    if (i < n) {
      const double s = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
      const double sc = (dsc != nullptr) ? s2 * dsc[i] : s2;
      Y[i] = fma(sc, s, sigma2 * V[i]);
    }
  }
}

// Rows per block of the product's variants (each divides n_pad, a multiple
// of 256), with the unrolling that keeps 16 loads in flight per thread.
constexpr int kGemvVariants[] = {16, 8, 4, 2};
constexpr int kGemvDefaultRows = 4;

static void launch_gemv(const dcg_operator_s *op, int rows, const double *dsc, const double *V,
                        double *Y, const int *done) {
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  const dim3 g(static_cast<unsigned>(n_pad / rows)), b(256);
#define DCG_GEMV(R, U)                                                                         \
  hipLaunchKernelGGL((stored_gemv<R, U>), g, b, 0, op->stream, op->kst, n, n_pad, op->vin64, \
                     op->s2, op->sigma2, dsc, V, Y, done)
  switch (rows) {
    case 16: DCG_GEMV(16, 1); break;
    case 8: DCG_GEMV(8, 2); break;
    case 2: DCG_GEMV(2, 8); break;
    default: DCG_GEMV(4, 4); break;
  }
#undef DCG_GEMV
}

int stored_build_launch(const dcg_operator_s *op) {
  const int64_t tiles = op->g.n_pad / kBuildTile;
  hipLaunchKernelGGL(stored_build, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(tiles)),
                     dim3(256), 0, op->stream, op->x64, op->g.n, op->g.n_pad, op->g.d, op->kernel,
                     1.0 / (op->ell * op->ell), op->kst);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

int matvec_stored_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                       const int *done) {
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  const double *dsc = op->has_dsc ? op->dsc : nullptr;
  for (int64_t c = 0; c < m; ++c) {
    hipLaunchKernelGGL(stored_stage, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                       op->stream, V + c * n, n, n_pad, dsc, op->vin64, done);
    launch_gemv(op, (op->gemv_rows > 0) ? op->gemv_rows : kGemvDefaultRows, dsc, V + c * n,
                Y + c * n, done);
    if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  }
  return DCG_OK;
}

// Time `reps` products with each variant (on a zero vector, so the operator
// workspace's staged vector is overwritten) and keep the fastest.
int stored_tune(dcg_operator_s *op, int reps, int *rows_out, double *ms_out) {
  hipStream_t s = op->stream;
  if (hipMemsetAsync(op->vin64, 0, size_t(op->g.n_pad) * sizeof(double), s) != hipSuccess)
    return DCG_E_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return DCG_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DCG_E_HIP;
  }
  int best = kGemvDefaultRows, status = DCG_OK;
  float best_ms = -1.0f;
  // the product writes Y = s2 K0 0 + sigma2 * V with V = Y = the zero vector
  double *Y = op->ytmp;
  if (hipMemsetAsync(Y, 0, size_t(op->g.n_pad) * sizeof(double), s) != hipSuccess)
    status = DCG_E_HIP;
  for (int rows : kGemvVariants) {
    if (status != DCG_OK) break;
    launch_gemv(op, rows, nullptr, Y, Y, nullptr);   // warm-up
    if (hipEventRecord(e0, s) != hipSuccess) { status = DCG_E_HIP; break; }
    for (int r = 0; r < reps; ++r) launch_gemv(op, rows, nullptr, Y, Y, nullptr);
    float ms = 0.0f;
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      status = DCG_E_HIP;
      break;
    }
    ms /= static_cast<float>(reps);
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = rows;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != DCG_OK) return status;
  op->gemv_rows = best;
  if (rows_out != nullptr) *rows_out = best;
  if (ms_out != nullptr) *ms_out = best_ms;
  return DCG_OK;
}

}  // namespace dcg
