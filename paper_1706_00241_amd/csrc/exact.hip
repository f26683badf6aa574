// The FP64 operator A = K(X, X) + sigma2 I on the unrounded points: the
// residuals b - A x of iterative refinement and the FP64 operator mode.
//
// Same circulant block-pair schedule as the low-precision sweep (every
// unordered pair once, row and column sums from the same kernel value), with
// 128-point blocks and 16x16 FP64 MFMA tiles: the squared distance comes out
// of the augmented product <[-2x_i, a_i, 1], [x_j, 1, a_j]> in FP64 (lane l
// holds column l%16, rows l/16 + 4v for v < 4), the kernel value is
// evaluated in FP64 (exp and sqrt specialised to the arguments that occur),
// and all sums are FP64.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "blas.h"
#include "host.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

typedef __attribute__((ext_vector_type(4))) double f64x4;

// 2^x for x <= 0 (and small positive x), to about one ulp: k = rint(x) and
// f = x - k in [-1/2, 1/2] (the subtraction is exact), 2^f by its degree-11
// interpolating polynomial at the 12 Chebyshev nodes of [-1/2, 1/2]
// (coefficients solved in 60-digit decimal arithmetic; the FMA Horner
// evaluation stays within 1.3e-16 relative on the interval), and 2^k applied
// with ldexp.  Arguments below -1100 give 0.
__device__ __forceinline__ double exp2_nonpos(double x) {
  x = fmax(x, -1100.0);
  const double k = __builtin_rint(x);
  const double f = x - k;
  double p = 4.4558179083360645e-10;
  p = fma(p, f, 7.074194297288521e-09);
  p = fma(p, f, 1.0178057087733941e-07);
  p = fma(p, f, 1.3215432535912375e-06);
  p = fma(p, f, 1.5252733841556773e-05);
  p = fma(p, f, 0.00015403530463724353);
  p = fma(p, f, 0.001333355814640647);
  p = fma(p, f, 0.009618129107587256);
  p = fma(p, f, 0.055504108664821625);
  p = fma(p, f, 0.24022650695910158);
  p = fma(p, f, 0.6931471805599453);
  p = fma(p, f, 1.0);
  return __builtin_amdgcn_ldexp(p, static_cast<int>(k));
}

// sqrt(a) for a >= 0 (a = 0 returns 1e-150): the hardware reciprocal square
// root refined by one coupled Newton step on (sqrt a, 1 / (2 sqrt a)) and a
// final residual correction a - g^2 (Markstein's scheme); within half an ulp
// on the probed range.
__device__ __forceinline__ double sqrt_nonneg(double a) {
  a = fmax(a, 1e-300);
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, a);
  return fma(d, h, g);
}

// Kernel value without s2 from the squared distance r2 = (c r)^2 of the
// operands (points pre-scaled by c = point_scale(kernel, ell)):
//   RBF 2^-r2;  Matern (u = c r, t = sqrt(nu2) r / ell = ln2 u):
//   3/2: (1 + ln2 u) 2^-u,  5/2: (1 + ln2 u + ln2^2 r2 / 3) 2^-u.
template <int KERN>
__device__ __forceinline__ double kval64(double r2) {
  if constexpr (KERN == DCG_RBF) {
    return exp2_nonpos(-r2);
  } else {
    const double r2a = fabs(r2);
    const double u = sqrt_nonneg(r2a);
    const double e = exp2_nonpos(-u);
    if constexpr (KERN == DCG_MATERN32) return fma(kLn2d, u, 1.0) * e;
    else return fma(kLn2d, u, fma(kLn2Sq3d, r2a, 1.0)) * e;
  }
}

template <int KS>
struct Op64 {
  static constexpr int KSP = KS + (KS & 1);
  double v[KSP];
  __device__ __forceinline__ void load(const double *base, int64_t point, int lh) {
    const double2 *p = reinterpret_cast<const double2 *>(base + point * (4 * KSP) + lh * KSP);
#pragma unroll
    for (int s = 0; s < KSP / 2; ++s) {
      const double2 u = p[s];
      v[2 * s] = u.x;
      v[2 * s + 1] = u.y;
    }
  }
};

struct Symv64Args {
  const double *xr, *xc;
  const double *vin;  // n_pad, zero padded
  double *prow, *pcol;
  int64_t n_pad;
  int nb, dmax, chunk, nchunk;
  const int *done;
};

template <int KERN, int KS>
__global__ __launch_bounds__(256, 2) void symv64_kernel(Symv64Args A) {
  if (A.done != nullptr && *A.done != 0) return;
  constexpr int BLK = 128, NCT = 8, TR = 2;
  __shared__ double colpart[4][BLK];
  const int64_t G = int64_t(A.nb) * A.nchunk;
  const int64_t bid = blockIdx.x;
  const int64_t Gm = G - G % 8;
  const int64_t item = (bid < Gm) ? (bid % 8) * (Gm / 8) + bid / 8 : bid;
  const int I = static_cast<int>(item / A.nchunk);
  const int c = static_cast<int>(item % A.nchunk);
  const int nb = A.nb;
  const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? A.dmax : A.dmax + 1;
  const int d0 = c * A.chunk;
  const int d1 = min(d0 + A.chunk, ndel);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lc = l & 15, lg = l >> 4;
  const int64_t n_pad = A.n_pad;
  const int64_t rowbase = int64_t(I) * BLK + w * 16 * TR;

  Op64<KS> ra[TR];
  double pi[TR][4], accr[TR][4];
#pragma unroll
  for (int tr = 0; tr < TR; ++tr) {
    ra[tr].load(A.xr, rowbase + 16 * tr + lc, lg);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      pi[tr][v] = A.vin[rowbase + 16 * tr + lg + 4 * v];
      accr[tr][v] = 0.0;
    }
  }
  const int tiles = (d1 > d0) ? (d1 - d0) * NCT : 0;
  auto colbase_of = [&](int t) -> int64_t {
    t = min(t, tiles - 1);   // past the end: a valid tile, its result unused
    int J = I + d0 + t / NCT;
    if (J >= nb) J -= nb;
    return int64_t(J) * BLK + 16 * (t % NCT);
  };
  // Software pipeline: the MFMA products of tile t + 1 are issued before the
  // kernel values of tile t are evaluated, and the operand of tile t + 2 is
  // loaded meanwhile, so matrix and vector units work at the same time.
  Op64<KS> cbn, cbn2;
  double pjc = 0.0, pjn = 0.0, pjn2 = 0.0;
  f64x4 r2c[TR], r2n[TR];
  if (tiles > 0) {
    Op64<KS> cb0;
    const int64_t c0b = colbase_of(0);
    cb0.load(A.xc, c0b + lc, lg);
    pjc = A.vin[c0b + lc];
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      r2c[tr] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        r2c[tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[tr].v[s], cb0.v[s], r2c[tr], 0, 0, 0);
    }
    const int64_t c1b = colbase_of(1);
    cbn.load(A.xc, c1b + lc, lg);
    pjn = A.vin[c1b + lc];
  }
  // One column tile; DG: the tile lies in the diagonal block pair, where the
  // exact diagonal gets distance zero and no column partials are formed.
  // The diagonal block pair comes first in chunk 0 and runs as its own loop.
  auto step = [&](const int t, auto dg) {
    constexpr bool DG = decltype(dg)::value;
    const int dl = d0 + t / NCT;
    const int ct = t % NCT;
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      r2n[tr] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s)
        r2n[tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[tr].v[s], cbn.v[s], r2n[tr], 0, 0, 0);
    }
    const int64_t cx = colbase_of(t + 2);
    cbn2.load(A.xc, cx + lc, lg);
    pjn2 = A.vin[cx + lc];
    double cs = 0.0;
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      bool dz = false;
      if constexpr (DG) dz = (ct == w * TR + tr);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double r2v = r2c[tr][v];
        // the exact diagonal: distance zero by definition
        if constexpr (DG) r2v = (dz && lg + 4 * v == lc) ? 0.0 : r2v;
        const double kv = kval64<KERN>(r2v);
        accr[tr][v] = fma(kv, pjc, accr[tr][v]);
        if constexpr (!DG) cs = fma(kv, pi[tr][v], cs);
      }
    }
#pragma unroll
    for (int i = 0; i < TR * KS; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
    }
    if constexpr (!DG) {
      cs += __shfl_xor(cs, 16);
      cs += __shfl_xor(cs, 32);
      if (lg == 0) colpart[w][16 * ct + lc] = cs;
      if (ct == NCT - 1) {
        __syncthreads();
        int J = I + dl;
        if (J >= nb) J -= nb;
        for (int e = threadIdx.x; e < BLK; e += 256)
          A.pcol[int64_t(dl - 1) * n_pad + int64_t(J) * BLK + e] =
              (colpart[0][e] + colpart[1][e]) + (colpart[2][e] + colpart[3][e]);
        __syncthreads();
      }
    }
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) r2c[tr] = r2n[tr];
    cbn = cbn2;
    pjc = pjn;
    pjn = pjn2;
  };
  int t = 0;
  if (d0 == 0)
    for (const int tdiag = min(tiles, NCT); t < tdiag; ++t) step(t, std::true_type());
  for (; t < tiles; ++t) step(t, std::false_type());
#pragma unroll
  for (int tr = 0; tr < TR; ++tr) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double s = accr[tr][v];
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
      if (lc == v) A.prow[int64_t(c) * n_pad + rowbase + 16 * tr + lg + 4 * v] = s;
    }
  }
}

// v (times the diagonal scaling d if given) -> zero-padded FP64 copy (n_pad).
__global__ __launch_bounds__(256) void stage64(const double *V, int64_t n, int64_t n_pad,
                                               const double *dsc, double *out, const int *done) {
  if (done != nullptr && *done != 0) return;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n_pad) out[i] = (i < n) ? ((dsc != nullptr) ? dsc[i] * V[i] : V[i]) : 0.0;
}

// y = s2 * (row partials + column partials, fixed order) + sigma2 v; with a
// diagonal scaling, y = d * s2 * (partials) + sigma2 v.
__global__ __launch_bounds__(256) void reduce64(const double *prow, const double *pcol,
                                                int64_t n, int64_t n_pad, int nchunk, int dmax,
                                                int nb, double s2, double sigma2,
                                                const double *dsc, const double *V, double *Y,
                                                const int *done) {
  if (done != nullptr && *done != 0) return;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += prow[int64_t(c) * n_pad + i];
  const int J = static_cast<int>(i / 128);
  const int dlim = ((nb % 2) == 0 && J < nb / 2) ? dmax - 1 : dmax;
  for (int dl = 1; dl <= dlim; ++dl) s += pcol[int64_t(dl - 1) * n_pad + i];
  Y[i] = fma((dsc != nullptr) ? s2 * dsc[i] : s2, s, sigma2 * V[i]);
}

template <int KERN>
static void launch64(const dcg_operator_s *op, const Symv64Args &a, int64_t grid) {
  const dim3 g(static_cast<unsigned>(grid)), b(256);
  switch (exact_ksteps(op->g.d)) {
    case 3: hipLaunchKernelGGL((symv64_kernel<KERN, 3>), g, b, 0, op->stream, a); break;
    case 5: hipLaunchKernelGGL((symv64_kernel<KERN, 5>), g, b, 0, op->stream, a); break;
    case 9: hipLaunchKernelGGL((symv64_kernel<KERN, 9>), g, b, 0, op->stream, a); break;
    default: hipLaunchKernelGGL((symv64_kernel<KERN, 17>), g, b, 0, op->stream, a); break;
  }
}

static Symv64Args exact_args(const dcg_operator_s *op, const int *done, MatvecPlan *plan) {
  const int64_t n_pad = op->g.n_pad;
  const MatvecPlan p = exact_plan(n_pad, op->exact_items);
  Symv64Args a;
  a.xr = op->x64r;
  a.xc = op->x64c;
  a.vin = op->vin64;
  a.prow = op->part64;
  a.pcol = op->part64 + size_t(p.nchunk) * n_pad;
  a.n_pad = n_pad;
  a.nb = p.nb;
  a.dmax = p.dmax;
  a.chunk = p.chunk;
  a.nchunk = p.nchunk;
  a.done = done;
  *plan = p;
  return a;
}

// The FP64 pair sweep over the staged vector op->vin64 (partial sums only).
int launch_exact_sweep(const dcg_operator_s *op, const int *done) {
  MatvecPlan p;
  const Symv64Args a = exact_args(op, done, &p);
  if (op->kernel == DCG_RBF) launch64<DCG_RBF>(op, a, p.grid);
  else if (op->kernel == DCG_MATERN32) launch64<DCG_MATERN32>(op, a, p.grid);
  else launch64<DCG_MATERN52>(op, a, p.grid);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

// Y = A V with the FP64 operator, vector by vector; `done` (optional) turns
// every launch into a no-op once a solve has finished.
int matvec_exact_done(const dcg_operator_s *op, const double *V, double *Y, int64_t m,
                      const int *done) {
  // the stored operator keeps no FP64 operands (their workspace is not laid out)
  if (!has_exact(op)) return DCG_E_ARG;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  MatvecPlan p;
  const Symv64Args a = exact_args(op, done, &p);
  const double *dsc = op->has_dsc ? op->dsc : nullptr;
  for (int64_t col = 0; col < m; ++col) {
    const double *Vc = V + col * n;
    double *Yc = Y + col * n;
    hipLaunchKernelGGL(stage64, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                       op->stream, Vc, n, n_pad, dsc, op->vin64, done);
    const int st = launch_exact_sweep(op, done);
    if (st != DCG_OK) return st;
    hipLaunchKernelGGL(reduce64, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0,
                       op->stream, a.prow, a.pcol, n, n_pad, p.nchunk, p.dmax, p.nb, op->s2,
                       op->sigma2, dsc, Vc, Yc, done);
    if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  }
  return DCG_OK;
}

int matvec_exact(const dcg_operator_s *op, const double *V, double *Y, int64_t m) {
  return matvec_exact_done(op, V, Y, m, nullptr);
}

// One FP64 product (m = 1) with HIP events recorded on the operator's stream
// right before and after the pair sweep, so the caller can time the sweep
// kernel alone.
int matvec_exact_timed(const dcg_operator_s *op, const double *V, double *Y, hipEvent_t ev0,
                       hipEvent_t ev1) {
  if (!has_exact(op)) return DCG_E_ARG;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  MatvecPlan p;
  const Symv64Args a = exact_args(op, nullptr, &p);
  const double *dsc = op->has_dsc ? op->dsc : nullptr;
  hipLaunchKernelGGL(stage64, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                     op->stream, V, n, n_pad, dsc, op->vin64, nullptr);
  if (hipEventRecord(ev0, op->stream) != hipSuccess) return DCG_E_HIP;
  const int st = launch_exact_sweep(op, nullptr);
  if (st != DCG_OK) return st;
  if (hipEventRecord(ev1, op->stream) != hipSuccess) return DCG_E_HIP;
  hipLaunchKernelGGL(reduce64, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0,
                     op->stream, a.prow, a.pcol, n, n_pad, p.nchunk, p.dmax, p.nb, op->s2,
                     op->sigma2, dsc, V, Y, nullptr);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

}  // namespace dcg
