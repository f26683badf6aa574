// Operator set-up (point rounding, augmented MFMA operands) and the exact
// FP64 product used for the residuals of iterative refinement.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "blas.h"
#include "host.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int launch_exact_sweep(const dcg_operator_s *op, const int *done);

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

// Round an FP64 value to binary16, to nearest with ties to even, in one
// rounding step from the FP64 value (11 significant bits; subnormals below
// 2^-14, spacing 2^-24).  A value that rounds beyond the largest finite
// binary16 sets *ovf and gives infinity.
__device__ __forceinline__ uint16_t f16_from_double(double x, int *ovf) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
  const uint32_t sign = static_cast<uint32_t>(u >> 63) << 15;
  const uint64_t mag = u & 0x7fffffffffffffffull;
  const int e = static_cast<int>(mag >> 52) - 1023;
  if (mag == 0 || e < -25) return static_cast<uint16_t>(sign);   // below half of 2^-24
  if (e > 15) {
    *ovf = 1;
    return static_cast<uint16_t>(sign | 0x7c00);
  }
  const uint64_t m = (mag & ((1ull << 52) - 1)) | (1ull << 52);   // 53-bit significand
  // keep 11 bits (normal) or fewer (subnormal: spacing fixed at 2^-24)
  const int shift = (e >= -14) ? 42 : 42 + (-14 - e);
  uint64_t q = m >> shift;
  const uint64_t rem = m & ((1ull << shift) - 1);
  const uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1))) q += 1;
  if (e < -14) return static_cast<uint16_t>(sign | q);   // q <= 1024: 1024 is 2^-14 itself
  uint32_t eb = static_cast<uint32_t>(e + 15);
  if (q == 2048) {
    q = 1024;
    eb += 1;
  }
  if (eb >= 31) {
    *ovf = 1;
    return static_cast<uint16_t>(sign | 0x7c00);
  }
  return static_cast<uint16_t>(sign | (eb << 10) | (q & 0x3ff));
}

__device__ __forceinline__ double f16_to_double(uint16_t h) {
  const int eb = (h >> 10) & 0x1f;
  const double m = static_cast<double>(h & 0x3ff);
  const double v = (eb == 0) ? std::ldexp(m, -24) : std::ldexp(m + 1024.0, eb - 25);
  return (h & 0x8000) ? -v : v;
}

__global__ __launch_bounds__(256) void check_finite(const double *X, int64_t count, int *flag) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * 256)
    if (!isfinite(X[e])) atomicOr(flag, 1);
}

// Copy of a diagonal scaling (zero padded to n_pad); flags entries that are
// negative or not finite.
__global__ __launch_bounds__(256) void copy_diag(const double *D, int64_t n, int64_t n_pad,
                                                 double *out, int *flag) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  double v = 0.0;
  if (i < n) {
    v = D[i];
    if (!(v >= 0.0) || !isfinite(v)) atomicOr(flag, 8);
  }
  out[i] = v;
}

// The input points as an FP64 copy (n_pad x d, row-major, zero rows past
// n), once when the operator is created: the source of every operand build.
__global__ __launch_bounds__(256) void copy_points(const double *X, int64_t n, int64_t n_pad,
                                                   int d, double *x64) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n_pad * d) return;
  x64[e] = (e < n * d) ? X[e] : 0.0;
}

// FP64 operands of the exact operator, one thread per (padded) point:
// [-2y, a, 1] and [y, 1, a] with y = scale * x (point_scale of the kernel
// and lengthscale, so the MFMA gives (c r)^2) and a = |y|^2, element k
// stored at (k % 4) * ksp + k / 4 (the K-step layout of the 16x16x4 FP64
// MFMA).  Run at creation and whenever the lengthscale changes.
__global__ __launch_bounds__(256) void prepare_exact(const double *x64, int64_t n_pad, int d,
                                                     int stride64, double scale, double *x64r,
                                                     double *x64c) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const int ksp = stride64 / 4;
  double *r64 = x64r + i * stride64;
  double *c64 = x64c + i * stride64;
  double a64 = 0.0;
  for (int t = 0; t < stride64; ++t) r64[t] = c64[t] = 0.0;
  for (int t = 0; t < d; ++t) {
    const double yv = scale * x64[i * d + t];
    a64 += yv * yv;
    r64[(t & 3) * ksp + (t >> 2)] = -2.0 * yv;
    c64[(t & 3) * ksp + (t >> 2)] = yv;
  }
  r64[(d & 3) * ksp + (d >> 2)] = a64;
  r64[((d + 1) & 3) * ksp + ((d + 1) >> 2)] = 1.0;
  c64[(d & 3) * ksp + (d >> 2)] = 1.0;
  c64[((d + 1) & 3) * ksp + ((d + 1) >> 2)] = a64;
}

// Low-precision operands, one thread per (padded) point: the point scaled
// by `scale` (point_scale of the kernel and lengthscale) and rounded, the
// squared norm of the rounded scaled point, and the augmented row / column
// operands, from the FP64 copy of the points; run at creation and whenever
// the lengthscale changes.
__global__ __launch_bounds__(256) void prepare_lowprec(const double *x64, int64_t n,
                                                       int64_t n_pad, int d, int prec, int opk,
                                                       int kstride, double scale, void *xr,
                                                       void *xc, int *flag) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const bool real = i < n;
  double a = 0.0;
  if (prec == DCG_PREC_BF16X2) {
    // x = hi + lo, both bf16; the operand columns hold the four product
    // pairings so that <xr_i, xc_j> = a_i + a_j - 2 (hi_i + lo_i).(hi_j + lo_j)
    uint16_t *r = static_cast<uint16_t *>(xr) + i * kstride;
    uint16_t *c = static_cast<uint16_t *>(xc) + i * kstride;
    for (int t = 0; t < d; ++t) {
      const double xv0 = real ? scale * x64[i * d + t] : 0.0;
      const uint16_t hi = bf16_from_double(xv0);
      const uint16_t lo = bf16_from_double(xv0 - bf16_to_double(hi));
      const double xv = bf16_to_double(hi) + bf16_to_double(lo);
      a += xv * xv;
      const uint16_t h2 = bf16_from_double(-2.0 * bf16_to_double(hi));
      const uint16_t l2 = bf16_from_double(-2.0 * bf16_to_double(lo));
      r[t] = h2;          c[t] = hi;
      r[d + t] = h2;      c[d + t] = lo;
      r[2 * d + t] = l2;  c[2 * d + t] = hi;
      r[3 * d + t] = l2;  c[3 * d + t] = lo;
    }
    const uint16_t ah = bf16_from_double(a);
    const double rem1 = a - bf16_to_double(ah);
    const uint16_t am = bf16_from_double(rem1);
    const uint16_t al = bf16_from_double(rem1 - bf16_to_double(am));
    const uint16_t one = 0x3F80;
    const int o = 4 * d;
    r[o + 0] = one; r[o + 1] = one; r[o + 2] = one;
    r[o + 3] = ah;  r[o + 4] = am;  r[o + 5] = al;
    c[o + 0] = ah;  c[o + 1] = am;  c[o + 2] = al;
    c[o + 3] = one; c[o + 4] = one; c[o + 5] = one;
    for (int t = o + 6; t < kstride; ++t) r[t] = c[t] = 0;
  } else if (prec == DCG_PREC_BF16) {
    uint16_t *r = static_cast<uint16_t *>(xr) + i * kstride;
    uint16_t *c = static_cast<uint16_t *>(xc) + i * kstride;
    for (int t = 0; t < d; ++t) {
      const uint16_t h =
          real ? bf16_from_double(scale * x64[i * d + t]) : uint16_t(0);
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
  } else if (prec == DCG_PREC_FP16) {
    // as bf16, with binary16 terms (the same column layout)
    uint16_t *r = static_cast<uint16_t *>(xr) + i * kstride;
    uint16_t *c = static_cast<uint16_t *>(xc) + i * kstride;
    int ovf = 0;
    for (int t = 0; t < d; ++t) {
      const uint16_t h = real ? f16_from_double(scale * x64[i * d + t], &ovf) : uint16_t(0);
      const double xv = f16_to_double(h);
      a += xv * xv;
      c[t] = h;
      r[t] = f16_from_double(-2.0 * xv, &ovf);   // exact unless it overflows
    }
    const uint16_t ah = f16_from_double(a, &ovf);
    const double rem1 = a - f16_to_double(ah);
    const uint16_t am = f16_from_double(rem1, &ovf);
    const uint16_t al = f16_from_double(rem1 - f16_to_double(am), &ovf);
    const uint16_t one = 0x3C00;
    r[d + 0] = one; r[d + 1] = one; r[d + 2] = one;
    r[d + 3] = ah;  r[d + 4] = am;  r[d + 5] = al;
    c[d + 0] = ah;  c[d + 1] = am;  c[d + 2] = al;
    c[d + 3] = one; c[d + 4] = one; c[d + 5] = one;
    for (int t = d + 6; t < kstride; ++t) r[t] = c[t] = 0;
    if (ovf) atomicOr(flag, 4);
  } else if (opk == kOpBf16Acc64) {
    // FP32 coordinate x = h + m + l, three bf16 terms (exact for every FP32
    // value); one column per kept pairing (row term, column term): (h,h)
    // (h,m) (m,h) (h,l) (l,h) (m,m), the row side carrying the factor -2
    // (exact in bf16).  |m| <= 2^-8 |x| and |l| <= 2^-17 |x|, so the dropped
    // m.l, l.m, l.l add up to at most 2^-24 |x_i x_j|: one FP32 rounding.
    uint16_t *r = static_cast<uint16_t *>(xr) + i * kstride;
    uint16_t *c = static_cast<uint16_t *>(xc) + i * kstride;
    for (int t = 0; t < d; ++t) {
      const float xf =
          real ? static_cast<float>(scale * x64[i * d + t]) : 0.0f;
      const double xv = xf;
      a += xv * xv;
      const uint16_t h = bf16_from_double(xv);
      const double r1 = xv - bf16_to_double(h);
      const uint16_t m = bf16_from_double(r1);
      const uint16_t lo = bf16_from_double(r1 - bf16_to_double(m));
      const uint16_t h2 = bf16_from_double(-2.0 * bf16_to_double(h));
      const uint16_t m2 = bf16_from_double(-2.0 * bf16_to_double(m));
      const uint16_t l2 = bf16_from_double(-2.0 * bf16_to_double(lo));
      r[t] = h2;          c[t] = h;
      r[d + t] = h2;      c[d + t] = m;
      r[2 * d + t] = m2;  c[2 * d + t] = h;
      r[3 * d + t] = h2;  c[3 * d + t] = lo;
      r[4 * d + t] = l2;  c[4 * d + t] = h;
      r[5 * d + t] = m2;  c[5 * d + t] = m;
    }
    const uint16_t ah = bf16_from_double(a);
    const double rem1 = a - bf16_to_double(ah);
    const uint16_t am = bf16_from_double(rem1);
    const uint16_t al = bf16_from_double(rem1 - bf16_to_double(am));
    const uint16_t one = 0x3F80;
    const int o = 6 * d;
    r[o + 0] = one; r[o + 1] = one; r[o + 2] = one;
    r[o + 3] = ah;  r[o + 4] = am;  r[o + 5] = al;
    c[o + 0] = ah;  c[o + 1] = am;  c[o + 2] = al;
    c[o + 3] = one; c[o + 4] = one; c[o + 5] = one;
    for (int t = o + 6; t < kstride; ++t) r[t] = c[t] = 0;
  } else {
    float *r = static_cast<float *>(xr) + i * kstride;
    float *c = static_cast<float *>(xc) + i * kstride;
    const int half = kstride / 2;
    for (int t = 0; t < kstride; ++t) r[t] = c[t] = 0.0f;
    for (int t = 0; t < d; ++t) {
      const float xv =
          real ? static_cast<float>(scale * x64[i * d + t]) : 0.0f;
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
}

// Both operand sets for the operator's kernel and lengthscale.  fp16
// operands are checked for overflow (the call then waits for the stream and
// returns DCG_E_ARG if a scaled point or squared norm left the fp16 range).
static int launch_prepare(const dcg_operator_s *op) {
  const Geometry &g = op->g;
  if (g.prec == DCG_PREC_STORED) return stored_build_launch(op);
  const double c = point_scale(op->kernel, op->ell);
  const dim3 grid(static_cast<unsigned>(cdiv(g.n_pad, 256)));
  const bool check = g.prec == DCG_PREC_FP16;
  if (check && hipMemsetAsync(op->flag, 0, sizeof(int), op->stream) != hipSuccess) return DCG_E_HIP;
  if (!sweep_wide(g))
    hipLaunchKernelGGL(prepare_exact, grid, dim3(256), 0, op->stream, op->x64, g.n_pad, g.d,
                       exact_stride(g.d), c, op->x64r, op->x64c);
  if (g.prec != DCG_PREC_FP64)
    hipLaunchKernelGGL(prepare_lowprec, grid, dim3(256), 0, op->stream, op->x64, g.n, g.n_pad,
                       g.d, g.prec, g.opk, g.kstride, c, op->xr, op->xc, op->flag);
  if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
  if (check) {
    int h = 0;
    if (hipMemcpyAsync(&h, op->flag, sizeof(int), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
        hipStreamSynchronize(op->stream) != hipSuccess)
      return DCG_E_HIP;
    if (h & 4) return DCG_E_ARG;
  }
  return DCG_OK;
}

// ----------------------------------------------------------- workspace

// Point dimensions each precision's products take.
static int64_t max_dims(int prec) {
  if (prec == DCG_PREC_STORED) return kMaxStoredD;
  if (prec == DCG_PREC_BF16 || prec == DCG_PREC_FP16) return kMaxWideD;
  return kMaxD;
}

struct OpLayout {
  size_t x64, x64r, x64c, vin64, part64, xr, xc, vin, part, ytmp, dsc, flag, kst, kpart, total;
};

static OpLayout op_layout(const Geometry &g) {
  const bool stored = g.prec == DCG_PREC_STORED;
  // the stored operator keeps the points, the staged vector and K0 only;
  // wide points have no FP64 operator
  const bool no64 = stored || sweep_wide(g);
  const int st64 = no64 ? 0 : exact_stride(g.d);
  const size_t esz = (g.prec == DCG_PREC_FP64 || stored) ? 0 : (g.opk == kOpF32 ? 4 : 2);
  Carve c(nullptr, 0);
  OpLayout L;
  L.x64 = c.off = align256(c.off); c.off += size_t(g.n_pad) * g.d * 8;
  L.x64r = c.off = align256(c.off); c.off += size_t(g.n_pad) * st64 * 8;
  L.x64c = c.off = align256(c.off); c.off += size_t(g.n_pad) * st64 * 8;
  L.vin64 = c.off = align256(c.off); c.off += size_t(g.n_pad) * 8;
  L.part64 = c.off = align256(c.off); if (!no64) c.off += exact_partial_doubles(g.n_pad) * 8;
  L.xr = c.off = align256(c.off); c.off += size_t(g.n_pad) * g.kstride * esz;
  L.xc = c.off = align256(c.off); c.off += size_t(g.n_pad) * g.kstride * esz;
  L.vin = c.off = align256(c.off); c.off += size_t(g.n_pad) * 4 * 4;
  L.part = c.off = align256(c.off);
  if (sweep_wide(g))
    c.off += wide_partial_floats(g.n_pad) * 4;
  else if (g.prec != DCG_PREC_FP64 && !stored)
    c.off += std::max(matvec_partial_floats(g.n_pad, 1, sweep_blk(g, 1)),
                      matvec_partial_floats(g.n_pad, 4, sweep_blk(g, 4))) * 4;
  L.ytmp = c.off = align256(c.off); c.off += size_t(g.n_pad) * 4 * 8;
  L.dsc = c.off = align256(c.off); c.off += size_t(g.n_pad) * 8;
  L.flag = c.off = align256(c.off); c.off += 256;
  L.kst = c.off = align256(c.off); if (stored) c.off += stored_matrix_floats(g.n_pad) * 4;
  L.kpart = c.off = align256(c.off); if (stored) c.off += stored_partial_doubles(g.n_pad) * 8;
  L.total = align256(c.off);
  return L;
}

// Time `reps` launches of `run` for each distinct plan of the targets and
// keep the fastest in *field; returns the best target and its time.
template <class PlanOf, class Run>
static int tune_field(hipStream_t s, int reps, int *field, PlanOf plan_of, Run run, int *best_out,
                      float *ms_out) {
  static const int cand[] = {256, 512, 1024, 2048, 4096, 8192};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return DCG_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DCG_E_HIP;
  }
  const int keep = *field;
  int best = keep, last_chunk = -1, status = DCG_OK;
  float best_ms = -1.0f;
  for (int items : cand) {
    const MatvecPlan p = plan_of(items);
    if (p.chunk == last_chunk) continue;   // the same plan as the previous target
    last_chunk = p.chunk;
    *field = items;
    status = run();   // warm-up
    if (status != DCG_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { status = DCG_E_HIP; break; }
    for (int r = 0; r < reps && status == DCG_OK; ++r) status = run();
    if (status != DCG_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      status = DCG_E_HIP;
      break;
    }
    ms /= static_cast<float>(reps);
    // a later plan must be faster by more than the timing noise to replace
    // the best so far: plans within 1% of each other would otherwise be
    // chosen at random from run to run, and with them the summation order
    // of the partial sums (and so the rounding of every product)
    if (best_ms < 0.0f || ms < 0.99f * best_ms) {
      best_ms = ms;
      best = items;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *field = (status == DCG_OK) ? best : keep;
  *best_out = best;
  *ms_out = best_ms;
  return status;
}

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_operator_workspace_bytes(int64_t n, int64_t d, int prec) {
  if (prec < DCG_PREC_FP32 || prec > DCG_PREC_STORED) return 0;
  if (n < 1 || d < 1 || d > max_dims(prec)) return 0;
  return op_layout(make_geometry(n, static_cast<int>(d), prec)).total;
}

int dcg_create_operator(const double *X, int64_t n, int64_t d, int kernel, double ell, double s2,
                        double sigma2, int prec, void *workspace, size_t ws_bytes, void *stream,
                        dcg_op_t *out) {
  if (out == nullptr) return DCG_E_ARG;
  *out = nullptr;
  if (prec < DCG_PREC_FP32 || prec > DCG_PREC_STORED) return DCG_E_ARG;
  if (X == nullptr || n < 1 || d < 1 || d > max_dims(prec)) return DCG_E_ARG;
  if (kernel < DCG_RBF || kernel > DCG_MATERN52) return DCG_E_ARG;
  if (!(ell > 0.0) || !(s2 > 0.0) || !(sigma2 >= 0.0) || !std::isfinite(ell) ||
      !std::isfinite(s2) || !std::isfinite(sigma2))
    return DCG_E_ARG;
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
  op->sweep_items = kSweepItemsDefault;
  op->exact_items = kSweepItemsDefault;
  op->x64 = reinterpret_cast<double *>(base + L.x64);
  op->x64r = reinterpret_cast<double *>(base + L.x64r);
  op->x64c = reinterpret_cast<double *>(base + L.x64c);
  op->vin64 = reinterpret_cast<double *>(base + L.vin64);
  op->part64 = reinterpret_cast<double *>(base + L.part64);
  op->xr = base + L.xr;
  op->xc = base + L.xc;
  op->vin = reinterpret_cast<float *>(base + L.vin);
  op->part = reinterpret_cast<float *>(base + L.part);
  op->ytmp = reinterpret_cast<double *>(base + L.ytmp);
  op->dsc = reinterpret_cast<double *>(base + L.dsc);
  op->kst = reinterpret_cast<float *>(base + L.kst);
  op->kpart = reinterpret_cast<double *>(base + L.kpart);
  op->has_dsc = 0;
  op->dsc_version = 0;
  // flag word 0: non-finite input; word 1: operand preparation (fp16 range)
  int *flag = reinterpret_cast<int *>(base + L.flag);
  op->flag = flag + 1;
  int hflag = 0;
  bool ok = hipMemsetAsync(flag, 0, 2 * sizeof(int), op->stream) == hipSuccess;
  const int64_t count = n * d;
  hipLaunchKernelGGL(check_finite, dim3(static_cast<unsigned>(std::min<int64_t>(1024, cdiv(count, 256)))),
                     dim3(256), 0, op->stream, X, count, flag);
  hipLaunchKernelGGL(copy_points, dim3(static_cast<unsigned>(cdiv(g.n_pad * g.d, 256))), dim3(256),
                     0, op->stream, X, n, g.n_pad, g.d, op->x64);
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
  int st = launch_prepare(op);
  if (st == DCG_OK && hipStreamSynchronize(op->stream) != hipSuccess) st = DCG_E_HIP;
  if (st != DCG_OK) {
    (void)hipStreamSynchronize(op->stream);
    delete op;
    return st;   // DCG_E_ARG: fp16 operands out of range for this lengthscale
  }
  *out = op;
  return DCG_OK;
}

int dcg_set_hyper(dcg_op_t op, double ell, double s2, double sigma2) {
  if (op == nullptr) return DCG_E_ARG;
  if (!(ell > 0.0) || !(s2 > 0.0) || !(sigma2 >= 0.0) || !std::isfinite(ell) ||
      !std::isfinite(s2) || !std::isfinite(sigma2))
    return DCG_E_ARG;
  const bool rescale = ell != op->ell;
  const double old[3] = {op->ell, op->s2, op->sigma2};
  op->ell = ell;
  op->s2 = s2;
  op->sigma2 = sigma2;
  op->generation += 1;
  if (!rescale) return DCG_OK;
  // the operands carry the lengthscale (point_scale)
  const int st = launch_prepare(op);
  if (st == DCG_E_ARG) {
    // fp16 operands out of range for this lengthscale: keep the previous
    // hyperparameters and their operands
    op->ell = old[0];
    op->s2 = old[1];
    op->sigma2 = old[2];
    op->generation += 1;
    (void)launch_prepare(op);
  }
  return st;
}

int dcg_set_diag(dcg_op_t op, const double *D) {
  if (op == nullptr) return DCG_E_ARG;
  if (D == nullptr) {
    if (op->has_dsc) {
      op->has_dsc = 0;
      op->dsc_version += 1;
      op->generation += 1;
    }
    return DCG_OK;
  }
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  int h = 0;
  if (hipMemsetAsync(op->flag, 0, sizeof(int), op->stream) != hipSuccess) return DCG_E_HIP;
  hipLaunchKernelGGL(copy_diag, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0,
                     op->stream, D, n, n_pad, op->dsc, op->flag);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&h, op->flag, sizeof(int), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
      hipStreamSynchronize(op->stream) != hipSuccess)
    return DCG_E_HIP;
  op->dsc_version += 1;
  op->generation += 1;
  if (h & 8) {
    // the copy is unusable: the operator goes back to no scaling
    op->has_dsc = 0;
    return DCG_E_NONFINITE;
  }
  op->has_dsc = 1;
  return DCG_OK;
}

int dcg_matvec(dcg_op_t op, const double *V, double *Y, int64_t m) {
  if (op == nullptr || V == nullptr || Y == nullptr || m < 1) return DCG_E_ARG;
  return matvec_lowprec(op, V, Y, m);
}

int dcg_matvec_exact(dcg_op_t op, const double *V, double *Y, int64_t m) {
  if (op == nullptr || V == nullptr || Y == nullptr || m < 1) return DCG_E_ARG;
  if (!has_exact(op)) return DCG_E_ARG;   // no FP64 operator
  return matvec_exact(op, V, Y, m);
}

int dcg_set_sweep_items(dcg_op_t op, int items) {
  if (op == nullptr) return DCG_E_ARG;
  if (op->g.prec == DCG_PREC_STORED) return DCG_E_ARG;   // a fixed tile plan
  if (items < kSweepItemsMin || items > kSweepItemsMax) return DCG_E_ARG;
  op->sweep_items = items;
  return DCG_OK;
}

int dcg_tune_operator(dcg_op_t op, int reps, int *items_out, double *ms_out) {
  if (op == nullptr || reps < 1 || reps > 1000) return DCG_E_ARG;
  // the stored operator has one plan: time it
  if (op->g.prec == DCG_PREC_STORED) return stored_tune(op, reps, items_out, ms_out);
  hipStream_t s = op->stream;
  int best = op->sweep_items, best64 = op->exact_items;
  float ms = 0.0f, ms64 = 0.0f;
  // the sweeps' costs do not depend on the vector's values
  if (hipMemsetAsync(op->vin64, 0, size_t(op->g.n_pad) * sizeof(double), s) != hipSuccess)
    return DCG_E_HIP;
  // FP64 sweep (refinement residuals, FP64 operators): a few launches
  int st = DCG_OK;
  if (has_exact(op)) {
    st = tune_field(
        s, std::max(2, reps / 2), &op->exact_items,
        [&](int items) { return exact_plan(op->g.n_pad, items); },
        [&]() { return launch_exact_sweep(op, nullptr); }, &best64, &ms64);
    if (st != DCG_OK) return st;
  }
  if (op->g.prec != DCG_PREC_FP64) {
    if (hipMemsetAsync(op->vin, 0, size_t(op->g.n_pad) * 4 * sizeof(float), s) != hipSuccess)
      return DCG_E_HIP;
    st = tune_field(
        s, reps, &op->sweep_items,
        [&](int items) { return sweep_plan(op->g, 1, items); },
        [&]() { return launch_symv_sweep(op, 1, nullptr); }, &best, &ms);
    if (st != DCG_OK) return st;
  } else {
    best = best64;
    ms = ms64;
  }
  if (items_out != nullptr) *items_out = best;
  if (ms_out != nullptr) *ms_out = ms;
  return DCG_OK;
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
