// The stored operator: the unit-amplitude kernel matrix K0 = K(X, X) / s2
// formed once in FP64 and kept in HBM as FP32, for point dimensions too
// large for the matrix-free pair sweep (the classification data of section 3
// has 784 coordinates).  K0 is fixed while only s2, sigma2 or the diagonal
// scaling change (a Newton loop changes only D), so every product is one
// streaming pass over the stored matrix: the HBM roofline, not the kernel
// evaluations.
//
// Only the block upper triangle is kept: 128 x 128 tiles (I, J), I <= J,
// each contiguous (row-major inside), packed row by row of tiles.  A product
// reads every tile once and uses it twice, y_I += K_IJ x_J and (I < J)
// y_J += K_IJ^T x_I, so it streams 2 n_pad^2 (1 + 1/nb) bytes instead of
// 4 n_pad^2.  Each tile writes its row and column partial sums; a second
// kernel adds a row's partials in a fixed order (deterministic results).
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
constexpr int kSymB = 128;       // stored tile size
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

// Index of stored tile (I, J), I <= J, among nb x nb tiles.
__host__ __device__ __forceinline__ int64_t sym_tile(int64_t I, int64_t J, int64_t nb) {
  return I * nb - I * (I - 1) / 2 + (J - I);
}

size_t stored_matrix_floats(int64_t n_pad) {
  const int64_t nb = n_pad / kSymB;
  return size_t(nb * (nb + 1) / 2) * kSymB * kSymB;
}

size_t stored_partial_doubles(int64_t n_pad) {
  const int64_t nb = n_pad / kSymB;
  return size_t(nb * (nb + 1) / 2) * 2 * kSymB;
}

// K0 in 64 x 64 output tiles (those in the block upper triangle of 128 x 128
// tiles; the others return at once): squared distances in difference form
// (no cancellation, zero on the diagonal), coordinates staged through LDS 16
// at a time, 4 x 4 outputs per thread.  x64: n_pad x d row-major FP64 with
// zero rows past n, so every tile's loads stay inside it.
__global__ __launch_bounds__(256) void stored_build(const double *x64, int64_t n, int64_t n_pad,
                                                   int d, int kernel, double inv_ell2,
                                                   int64_t nb, float *K) {
  const int64_t I = int64_t(blockIdx.y) * kBuildTile / kSymB;
  const int64_t J = int64_t(blockIdx.x) * kBuildTile / kSymB;
  if (I > J) return;
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
      K[(sym_tile(I, J, nb) * kSymB + (i % kSymB)) * kSymB + (j % kSymB)] = val;
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

// One stored tile per block: thread (rg = t / 16, c = t % 16) reads the
// 16-byte pieces c and c + 16 of rows rg, rg + 16, ..., rg + 112 (each load
// instruction covers 256 contiguous bytes of a row across 16 lanes;
// non-temporal, since every tile is read once per product), all 16 loads in
// flight at once.  Each row's 8 values give a row partial (products with
// x_J) and 8 column partials (times x_I).  Row partials go to LDS and the
// first 128 threads add each row's 16; the column partials (off-diagonal
// tiles) go to LDS and the other 128 threads add each column's 16.  FP64
// accumulation throughout; no cross-lane shuffles.
__global__ __launch_bounds__(256) void stored_symv(const float *K, int64_t nb, const double *xs,
                                                   double *part, const int *done) {
  if (done != nullptr && *done != 0) return;
  constexpr int kGroups = 16, kRowsPer = kSymB / kGroups;
  __shared__ double rs[kSymB][kGroups + 1];   // row partials [row][lane], padded
  __shared__ double cs[kGroups][kSymB];       // column partials [row group][column]
  const int64_t t = blockIdx.x;
  // (I, J) of tile t: the largest I with sym_tile(I, I) <= t
  const double b2 = 2.0 * double(nb) + 1.0;
  int64_t I = static_cast<int64_t>((b2 - sqrt(fmax(b2 * b2 - 8.0 * double(t), 0.0))) * 0.5);
  I = (I < 0) ? 0 : (I >= nb ? nb - 1 : I);
  while (I > 0 && sym_tile(I, I, nb) > t) --I;
  while (I + 1 < nb && sym_tile(I + 1, I + 1, nb) <= t) ++I;
  const int64_t J = I + (t - sym_tile(I, I, nb));
  const int tid = threadIdx.x, c = tid & 15, rg = tid >> 4;
  const f32x4 *Kt = reinterpret_cast<const f32x4 *>(K + t * kSymB * kSymB);
  const double *xI = xs + I * kSymB, *xJ = xs + J * kSymB;
  f32x4 ka[kRowsPer], kb[kRowsPer];
  for (int k = 0; k < kRowsPer; ++k) {
    ka[k] = __builtin_nontemporal_load(Kt + (rg + kGroups * k) * 32 + c);
    kb[k] = __builtin_nontemporal_load(Kt + (rg + kGroups * k) * 32 + c + 16);
  }
  double xj[8], cp[8];
  for (int e = 0; e < 4; ++e) {
    xj[e] = xJ[4 * c + e];
    xj[4 + e] = xJ[64 + 4 * c + e];
    cp[e] = 0.0;
    cp[4 + e] = 0.0;
  }
  for (int k = 0; k < kRowsPer; ++k) {
    const double v[8] = {ka[k].x, ka[k].y, ka[k].z, ka[k].w, kb[k].x, kb[k].y, kb[k].z, kb[k].w};
    double r = v[0] * xj[0];
    for (int e = 1; e < 8; ++e) r = fma(v[e], xj[e], r);
    rs[rg + kGroups * k][c] = r;
    const double xi = xI[rg + kGroups * k];
    for (int e = 0; e < 8; ++e) cp[e] = fma(v[e], xi, cp[e]);
  }
  for (int e = 0; e < 4; ++e) {
    cs[rg][4 * c + e] = cp[e];
    cs[rg][64 + 4 * c + e] = cp[4 + e];
  }
  __syncthreads();
  double *rowp = part + t * 2 * kSymB;
  if (tid < kSymB) {
    double v = 0.0;
    for (int l = 0; l < kGroups; ++l) v += rs[tid][l];
    rowp[tid] = v;
  } else if (I != J) {
    // a diagonal tile holds both triangles: its rows cover it
    const int col = tid - kSymB;
    double v = 0.0;
    for (int g = 0; g < kGroups; ++g) v += cs[g][col];
    rowp[kSymB + col] = v;
  }
}

// y_i = s2 d_i (sum of row i's partials) + sigma2 v_i.  Row i of block I
// has one partial per tile column m: the column partial of tile (m, I) for
// m < I, the row partial of tile (I, m) for m >= I.  Eight independent
// accumulators (m mod 8) keep eight loads in flight per thread, added in a
// fixed order at the end; 64-thread blocks spread the rows over the chip.
__global__ __launch_bounds__(64) void stored_sym_reduce(const double *part, int64_t nb, int64_t n,
                                                        double s2, double sigma2,
                                                        const double *dsc, const double *V,
                                                        double *Y, const int *done) {
  if (done != nullptr && *done != 0) return;
  const int64_t i = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (i >= n) return;
  const int64_t I = i / kSymB, li = i % kSymB;
  double acc[8];
  for (int a = 0; a < 8; ++a) acc[a] = 0.0;
  int64_t m = 0;
  for (; m + 8 <= nb; m += 8)
    for (int a = 0; a < 8; ++a) {
      const int64_t mm = m + a;
      acc[a] += (mm < I) ? part[sym_tile(mm, I, nb) * 2 * kSymB + kSymB + li]
                         : part[sym_tile(I, mm, nb) * 2 * kSymB + li];
    }
  for (; m < nb; ++m)
    acc[m % 8] += (m < I) ? part[sym_tile(m, I, nb) * 2 * kSymB + kSymB + li]
                          : part[sym_tile(I, m, nb) * 2 * kSymB + li];
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  const double sc = (dsc != nullptr) ? s2 * dsc[i] : s2;
  Y[i] = fma(sc, s, sigma2 * V[i]);
}

int stored_build_launch(const dcg_operator_s *op) {
  const int64_t tiles = op->g.n_pad / kBuildTile;
  hipLaunchKernelGGL(stored_build, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(tiles)),
                     dim3(256), 0, op->stream, op->x64, op->g.n, op->g.n_pad, op->g.d, op->kernel,
                     1.0 / (op->ell * op->ell), op->g.n_pad / kSymB, op->kst);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

static int launch_stored_product(const dcg_operator_s *op, const double *V, double *Y,
                                 const int *done) {
  const int64_t n = op->g.n, n_pad = op->g.n_pad, nb = n_pad / kSymB;
  const double *dsc = op->has_dsc ? op->dsc : nullptr;
  hipLaunchKernelGGL(stored_stage, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                     op->stream, V, n, n_pad, dsc, op->vin64, done);
  hipLaunchKernelGGL(stored_symv, dim3(static_cast<unsigned>(nb * (nb + 1) / 2)), dim3(256), 0,
                     op->stream, op->kst, nb, op->vin64, op->kpart, done);
  hipLaunchKernelGGL(stored_sym_reduce, dim3(static_cast<unsigned>(cdiv(n, 64))), dim3(64), 0,
                     op->stream, op->kpart, nb, n, op->s2, op->sigma2, dsc, V, Y, done);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

int matvec_stored_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                       const int *done) {
  const int64_t n = op->g.n;
  for (int64_t c = 0; c < m; ++c) {
    const int st = launch_stored_product(op, V + c * n, Y + c * n, done);
    if (st != DCG_OK) return st;
  }
  return DCG_OK;
}

// Time `reps` products (of the zero vector into the operator's staging
// buffer); *items_out is the tile size, the product's fixed plan.
int stored_tune(dcg_operator_s *op, int reps, int *items_out, double *ms_out) {
  hipStream_t s = op->stream;
  double *Y = op->ytmp;
  if (hipMemsetAsync(Y, 0, size_t(op->g.n_pad) * sizeof(double), s) != hipSuccess)
    return DCG_E_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return DCG_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DCG_E_HIP;
  }
  int status = launch_stored_product(op, Y, Y, nullptr);   // warm-up
  float ms = 0.0f;
  if (status == DCG_OK && hipEventRecord(e0, s) != hipSuccess) status = DCG_E_HIP;
  for (int r = 0; r < reps && status == DCG_OK; ++r) status = launch_stored_product(op, Y, Y, nullptr);
  if (status == DCG_OK &&
      (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    status = DCG_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != DCG_OK) return status;
  if (items_out != nullptr) *items_out = kSymB;
  if (ms_out != nullptr) *ms_out = ms / static_cast<float>(reps);
  return DCG_OK;
}

}  // namespace dcg
