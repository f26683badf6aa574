// Fused derivative sweep of the GP log-marginal-likelihood gradient.
//
// For A = s2 k(X, X) + sigma2 I, alpha = A^{-1} y and probe solves
// U = A^{-1} Z (Z: P Rademacher probes), the gradient with respect to
// theta = (log ell, log s2, log sigma2) is (Rasmussen & Williams eq. 5.9 with
// the Hutchinson trace estimator)
//
//   g_j = 1/2 sum_ij (dA/dtheta_j)_ij w_ij,  w_ij = alpha_i alpha_j - (1/P) sum_p U_ip Z_jp.
//
// dA/dlog ell and dA/dlog s2 = K are kernel matrices, so both sums are taken
// in one symmetric pass over the pairs: each unique off-diagonal pair adds
// D_ij (w_ij + w_ji).  The squared distance comes from the augmented bf16 /
// fp32 MFMA of the matvec sweep; sum_p U_ip Z_jp and sum_p Z_ip U_jp come from
// two more bf16 MFMA products, exact in Z (entries +-1) and with U carried
// over three bf16 words (hi + mid + lo, 24 bits).  The sigma2 term is a pair
// of dot products done on the host side of this file's entry point.
#include <algorithm>
#include <cmath>

#include "blas.h"

namespace dcg {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kMaxProbes = 16;
constexpr int kProbeK = 48;  // 3 x 16 bf16 per point: [U hi | U mid | U lo] or [Z | Z | Z]

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ uint16_t bf16_bits(double x) {
  // round to nearest even, from FP64, one rounding (values here are finite)
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
__device__ __forceinline__ double bf16_val(uint16_t h) {
  return static_cast<double>(__uint_as_float(uint32_t(h) << 16));
}

// Probe operands per point: ur = [U hi | U mid | U lo], zr = [Z | Z | Z]
// (P <= 16 probes, zero padded), and alpha in FP32.
__global__ __launch_bounds__(256) void stage_probes(const double *alpha, const double *U,
                                                    const double *Z, int64_t n, int64_t n_pad,
                                                    int P, uint16_t *ur, uint16_t *zr,
                                                    float *a32) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const bool real = i < n;
  for (int p = 0; p < kMaxProbes; ++p) {
    const bool on = real && p < P;
    const double u = on ? U[int64_t(p) * n + i] : 0.0;
    const uint16_t hi = bf16_bits(u);
    const double r1 = u - bf16_val(hi);
    const uint16_t mid = bf16_bits(r1);
    const uint16_t lo = bf16_bits(r1 - bf16_val(mid));
    const uint16_t z = on ? bf16_bits(Z[int64_t(p) * n + i]) : uint16_t(0);
    ur[i * kProbeK + p] = hi;
    ur[i * kProbeK + 16 + p] = mid;
    ur[i * kProbeK + 32 + p] = lo;
    zr[i * kProbeK + p] = z;
    zr[i * kProbeK + 16 + p] = z;
    zr[i * kProbeK + 32 + p] = z;
  }
  a32[i] = real ? static_cast<float>(alpha[i]) : 0.0f;
}

template <bool BF16, int KS>
struct GOp;
template <int KS>
struct GOp<true, KS> {
  bf16x8 v[KS];
  __device__ __forceinline__ void load(const void *base, int64_t point, int kstride, int lh) {
    const uint4 *p = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(base) +
                                                     point * kstride + 8 * lh);
#pragma unroll
    for (int s = 0; s < KS; ++s) v[s] = __builtin_bit_cast(bf16x8, p[2 * s]);
  }
};
template <int KS>
struct GOp<false, KS> {
  static constexpr int KS4 = (KS + 3) / 4;
  float v[KS4 * 4];
  __device__ __forceinline__ void load(const void *base, int64_t point, int kstride, int lh) {
    const float4 *p = reinterpret_cast<const float4 *>(static_cast<const float *>(base) +
                                                       point * kstride + lh * (kstride / 2));
#pragma unroll
    for (int s = 0; s < KS4; ++s) {
      const float4 u = p[s];
      v[4 * s] = u.x; v[4 * s + 1] = u.y; v[4 * s + 2] = u.z; v[4 * s + 3] = u.w;
    }
  }
};

struct Probe {  // 3 K-steps of 16 bf16
  bf16x8 v[3];
  __device__ __forceinline__ void load(const uint16_t *base, int64_t point, int lh) {
    const uint4 *p = reinterpret_cast<const uint4 *>(base + point * kProbeK + 8 * lh);
#pragma unroll
    for (int s = 0; s < 3; ++s) v[s] = __builtin_bit_cast(bf16x8, p[2 * s]);
  }
};

__device__ __forceinline__ f32x16 probe_dot(const Probe &a, const Probe &b) {
  f32x16 acc = {};
#pragma unroll
  for (int s = 0; s < 3; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[s], b.v[s], acc, 0, 0, 0);
  return acc;
}

template <bool BF16, int KS>
__device__ __forceinline__ f32x16 dist_tile(const GOp<BF16, KS> &a, const GOp<BF16, KS> &b) {
  f32x16 acc = {};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    if constexpr (BF16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[s], b.v[s], acc, 0, 0, 0);
    else acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[s], b.v[s], acc, 0, 0, 0);
  }
  return acc;
}

// kappa (kernel without s2) and its derivative with respect to log ell, from
// the squared distance r2 = (c r)^2 of the operands (points scaled by
// c = point_scale(kernel, ell)).
template <int KERN>
__device__ __forceinline__ void kval_dlog(float r2, float *k, float *dk) {
  if constexpr (KERN == DCG_RBF) {
    // kappa = exp2(-r2); d kappa / d log ell = kappa r^2 / ell^2 = kappa 2 ln2 r2
    const float e = __builtin_amdgcn_exp2f(-r2);
    *k = e;
    *dk = e * fabsf(r2) * (2.0f * kLn2);
  } else {
    // u = c r, t = sqrt(nu2) r / ell = ln2 u, e^-t = 2^-u
    const float u = __builtin_amdgcn_sqrtf(fabsf(r2));
    const float e = __builtin_amdgcn_exp2f(-u);
    const float t = u * kLn2;
    if constexpr (KERN == DCG_MATERN32) {
      *k = (1.0f + t) * e;
      *dk = t * t * e;                              // t^2 e^-t
    } else {
      *k = fmaf(t, fmaf(t, 1.0f / 3.0f, 1.0f), 1.0f) * e;
      *dk = (t * t) * (1.0f + t) * (1.0f / 3.0f) * e;  // (t^2 + t^3)/3 e^-t
    }
  }
}

struct GradArgs {
  const void *xr, *xc;
  int kstride;
  const uint16_t *ur, *zr;
  const float *a32;
  double *partial;  // [grid][2]: sum kappa w, sum dkappa w
  int64_t n_pad;
  int nb, dmax, chunk, nchunk;
  float invP;
};

// One wave = 32 rows; 4 waves = 128-row blocks; circulant block pairs as in
// the matvec sweep.
template <int KERN, int KS, bool BF16>
__global__ __launch_bounds__(256, 2) void grad_sweep(GradArgs A) {
  constexpr int BLK = 128, NCT = 4;
  __shared__ double red[2][4];
  const int64_t item = blockIdx.x;
  const int I = static_cast<int>(item / A.nchunk);
  const int c = static_cast<int>(item % A.nchunk);
  const int nb = A.nb;
  const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? A.dmax : A.dmax + 1;
  const int d0 = c * A.chunk;
  const int d1 = min(d0 + A.chunk, ndel);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lc = l & 31, lh = l >> 5;
  const int64_t rowbase = int64_t(I) * BLK + 32 * w;

  GOp<BF16, KS> ra;
  ra.load(A.xr, rowbase + lc, A.kstride, lh);
  Probe ru, rz;
  ru.load(A.ur, rowbase + lc, lh);
  rz.load(A.zr, rowbase + lc, lh);
  float ai[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) ai[v] = A.a32[rowbase + 8 * (v >> 2) + 4 * lh + (v & 3)];

  double sk = 0.0, sd = 0.0;
  for (int dl = d0; dl < d1; ++dl) {
    int J = I + dl;
    if (J >= nb) J -= nb;
    const bool diag = (dl == 0);
    float tk = 0.0f, td = 0.0f;
    for (int ct = 0; ct < NCT; ++ct) {
      const int64_t cb = int64_t(J) * BLK + 32 * ct;
      GOp<BF16, KS> cbx;
      cbx.load(A.xc, cb + lc, A.kstride, lh);
      Probe cu, cz;
      cu.load(A.ur, cb + lc, lh);
      cz.load(A.zr, cb + lc, lh);
      const float aj = A.a32[cb + lc];
      f32x16 r2 = dist_tile<BF16, KS>(ra, cbx);
      const f32x16 uz = probe_dot(ru, cz);   // sum_p U_ip Z_jp
      f32x16 zu = {};
      if (!diag) zu = probe_dot(rz, cu);      // sum_p Z_ip U_jp
      if (diag && ct == w) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          if (8 * (v >> 2) + 4 * lh + (v & 3) == lc) r2[v] = 0.0f;
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float kv, dv;
        kval_dlog<KERN>(r2[v], &kv, &dv);
        // diagonal block: every ordered pair once; otherwise the pair and its mirror
        const float wv = diag ? fmaf(-A.invP, uz[v], ai[v] * aj)
                              : fmaf(-A.invP, uz[v] + zu[v], 2.0f * ai[v] * aj);
        tk = fmaf(kv, wv, tk);
        td = fmaf(dv, wv, td);
      }
    }
    sk += static_cast<double>(tk);
    sd += static_cast<double>(td);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sk += __shfl_xor(sk, o);
    sd += __shfl_xor(sd, o);
  }
  if (l == 0) {
    red[0][w] = sk;
    red[1][w] = sd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A.partial[2 * item] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    A.partial[2 * item + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// out[0..1] = column sums of partial[grid][2]; out[2] = alpha^T alpha,
// out[3] = sum_p U_p^T Z_p (one block, fixed order).
__global__ __launch_bounds__(256) void grad_finish(const double *partial, int64_t grid,
                                                   const double *alpha, const double *U,
                                                   const double *Z, int64_t n, int P,
                                                   double *out) {
  __shared__ double lds[4][4];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t g = threadIdx.x; g < grid; g += 256) {
    s0 += partial[2 * g];
    s1 += partial[2 * g + 1];
  }
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    s2 += alpha[i] * alpha[i];
    for (int p = 0; p < P; ++p) s3 += U[int64_t(p) * n + i] * Z[int64_t(p) * n + i];
  }
  double v[4] = {s0, s1, s2, s3};
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[q] += __shfl_xor(v[q], o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0)
    for (int q = 0; q < 4; ++q) lds[q][w] = v[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    out[q] = (lds[q][0] + lds[q][1]) + (lds[q][2] + lds[q][3]);
  }
}

size_t grad_workspace_bytes(int64_t n_pad) {
  const MatvecPlan p = make_plan(n_pad, 128);
  return align256(size_t(n_pad) * kProbeK * 2) * 2 + align256(size_t(n_pad) * 4) +
         align256(size_t(p.grid) * 2 * 8) + 256;
}

template <int KERN, bool BF16>
static int launch_grad(const dcg_operator_s *op, const GradArgs &a, int64_t grid) {
  const dim3 g(static_cast<unsigned>(grid)), b(256);
  const int ks = op->g.ksteps;
  if constexpr (BF16) {
    switch (ks) {
      case 1: hipLaunchKernelGGL((grad_sweep<KERN, 1, true>), g, b, 0, op->stream, a); return 0;
      case 2: hipLaunchKernelGGL((grad_sweep<KERN, 2, true>), g, b, 0, op->stream, a); return 0;
      case 3: hipLaunchKernelGGL((grad_sweep<KERN, 3, true>), g, b, 0, op->stream, a); return 0;
      case 4: hipLaunchKernelGGL((grad_sweep<KERN, 4, true>), g, b, 0, op->stream, a); return 0;
      case 5: hipLaunchKernelGGL((grad_sweep<KERN, 5, true>), g, b, 0, op->stream, a); return 0;
      case 7: hipLaunchKernelGGL((grad_sweep<KERN, 7, true>), g, b, 0, op->stream, a); return 0;
      case 9: hipLaunchKernelGGL((grad_sweep<KERN, 9, true>), g, b, 0, op->stream, a); return 0;
      case 13: hipLaunchKernelGGL((grad_sweep<KERN, 13, true>), g, b, 0, op->stream, a); return 0;
      case 17: hipLaunchKernelGGL((grad_sweep<KERN, 17, true>), g, b, 0, op->stream, a); return 0;
    }
  } else {
    switch (ks) {
      case 5: hipLaunchKernelGGL((grad_sweep<KERN, 5, false>), g, b, 0, op->stream, a); return 0;
      case 9: hipLaunchKernelGGL((grad_sweep<KERN, 9, false>), g, b, 0, op->stream, a); return 0;
      case 13: hipLaunchKernelGGL((grad_sweep<KERN, 13, false>), g, b, 0, op->stream, a); return 0;
      case 17: hipLaunchKernelGGL((grad_sweep<KERN, 17, false>), g, b, 0, op->stream, a); return 0;
    }
  }
  return -1;
}

// out[0] = y^T alpha, one block of 1024 threads: each thread sums a strided
// subsequence, then a fixed tree (bitwise reproducible).
__global__ __launch_bounds__(1024) void dot_one_block(const double *y, const double *alpha,
                                                      int64_t n, double *out) {
  __shared__ double lds[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += y[i] * alpha[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) lds[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += lds[i];
    out[0] = t;
  }
}

}  // namespace dcg

using namespace dcg;

extern "C" {

int dcg_mll_value(dcg_op_t op, const double *y, const double *alpha, const double *logdet,
                  double *value) {
  if (op == nullptr || y == nullptr || alpha == nullptr || value == nullptr) return DCG_E_ARG;
  if (logdet != nullptr && !std::isfinite(*logdet)) return DCG_E_ARG;
  const int64_t n = op->g.n;
  hipStream_t s = op->stream;
  // the operator's product staging holds the one-double result (calls on one
  // operator do not overlap)
  hipLaunchKernelGGL(dot_one_block, dim3(1), dim3(1024), 0, s, y, alpha, n, op->ytmp);
  double ya = 0.0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&ya, op->ytmp, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DCG_E_HIP;
  if (!std::isfinite(ya)) return DCG_E_NONFINITE;
  // -1/2 y^T A^{-1} y - n/2 log(2 pi) [- 1/2 log det A]
  const double two_pi = 6.283185307179586;
  double v = -0.5 * ya - 0.5 * static_cast<double>(n) * std::log(two_pi);
  if (logdet != nullptr) v -= 0.5 * (*logdet);
  *value = v;
  return DCG_OK;
}

size_t dcg_mll_grad_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return grad_workspace_bytes(((n + 255) / 256) * 256);
}

int dcg_mll_grad(dcg_op_t op, const double *alpha, const double *U, const double *Z, int64_t P,
                 double *grad3, void *ws, size_t ws_bytes) {
  if (op == nullptr || alpha == nullptr || U == nullptr || Z == nullptr || grad3 == nullptr)
    return DCG_E_ARG;
  if (P < 1 || P > kMaxProbes || op->has_dsc) return DCG_E_ARG;
  if (op->g.prec != DCG_PREC_FP32 && op->g.prec != DCG_PREC_BF16) return DCG_E_ARG;
  if (sweep_wide(op->g)) return DCG_E_ARG;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  if (ws == nullptr || ws_bytes < grad_workspace_bytes(n_pad)) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  const MatvecPlan p = make_plan(n_pad, 128);
  char *b = static_cast<char *>(ws);
  size_t off = 0;
  uint16_t *ur = reinterpret_cast<uint16_t *>(b + off);
  off += align256(size_t(n_pad) * kProbeK * 2);
  uint16_t *zr = reinterpret_cast<uint16_t *>(b + off);
  off += align256(size_t(n_pad) * kProbeK * 2);
  float *a32 = reinterpret_cast<float *>(b + off);
  off += align256(size_t(n_pad) * 4);
  double *partial = reinterpret_cast<double *>(b + off);
  off += align256(size_t(p.grid) * 2 * 8);
  double *out = reinterpret_cast<double *>(b + off);
  hipStream_t s = op->stream;
  hipLaunchKernelGGL(stage_probes, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0, s,
                     alpha, U, Z, n, n_pad, static_cast<int>(P), ur, zr, a32);
  GradArgs a;
  a.xr = op->xr;
  a.xc = op->xc;
  a.kstride = op->g.kstride;
  a.ur = ur;
  a.zr = zr;
  a.a32 = a32;
  a.partial = partial;
  a.n_pad = n_pad;
  a.nb = p.nb;
  a.dmax = p.dmax;
  a.chunk = p.chunk;
  a.nchunk = p.nchunk;
  a.invP = static_cast<float>(1.0 / double(P));
  // bf16 terms (bf16 points, or FP32 points as three bf16 terms) or FP32
  const bool bf = op->g.opk != kOpF32;
  int rc;
  if (op->kernel == DCG_RBF) rc = bf ? launch_grad<DCG_RBF, true>(op, a, p.grid) : launch_grad<DCG_RBF, false>(op, a, p.grid);
  else if (op->kernel == DCG_MATERN32) rc = bf ? launch_grad<DCG_MATERN32, true>(op, a, p.grid) : launch_grad<DCG_MATERN32, false>(op, a, p.grid);
  else rc = bf ? launch_grad<DCG_MATERN52, true>(op, a, p.grid) : launch_grad<DCG_MATERN52, false>(op, a, p.grid);
  if (rc != 0) return DCG_E_ARG;
  hipLaunchKernelGGL(grad_finish, dim3(1), dim3(256), 0, s, partial, p.grid, alpha, U, Z, n,
                     static_cast<int>(P), out);
  double h[4];
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DCG_E_HIP;
  const double invP = 1.0 / double(P);
  // g = 1/2 sum_ij (dA/dtheta)_ij w_ij; kernel sums exclude the s2 factor
  grad3[0] = 0.5 * op->s2 * h[1];
  grad3[1] = 0.5 * op->s2 * h[0];
  grad3[2] = 0.5 * op->sigma2 * (h[2] - invP * h[3]);
  return DCG_OK;
}

}  // extern "C"
