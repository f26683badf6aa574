// Matrix-free kernel matvec Y = (K_theta(X, X) + sigma2 I) V.
//
// The products A p_j of Algorithm 1 (one per CG step) and the block products
// A W.  K is symmetric, so every unordered pair of points is evaluated once
// and feeds both its row sum and its column sum.
//
// Schedule.  Rows are cut into nb blocks of BLK points.  Block pairs (I, J)
// are visited in circulant order: row block I owns the column blocks
// J = I + delta (mod nb) for delta = 0 .. nb/2 (for even nb the offset nb/2
// is owned only by I < nb/2).  Every unordered block pair is then owned once
// and each row block owns the same amount of work.  A work item (one
// workgroup) is a row block and a contiguous range of offsets; its row sums
// go to prow[chunk], the column sums of each off-diagonal block pair to
// pcol[delta], and a second kernel adds the partials in a fixed order (the
// result is bitwise reproducible).
//
// Tile.  A wave owns 32*TR rows and steps through 32-column tiles.  The
// squared distances of a 32x32 tile come straight out of MFMA, because the
// operands are augmented: <[-2x_i, 1, a_i], [x_j, a_j, 1]> = |x_i - x_j|^2
// (a = |x|^2, split over three bf16 terms in bf16 mode).  The kernel value is
// evaluated in registers on the MFMA output layout (lane l holds column
// l%32, rows 8(v/4) + 4(l/32) + v%4 for v < 16) and folded into the row
// accumulators and a per-lane column sum.
#include <algorithm>
#include <cmath>

#include <type_traits>

#include "blas.h"
#include "host.h"
#include "sweep.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Operand registers of one tile row: 16-bit terms (bf16 or fp16 bit
// patterns, 8 per lane per K-step) or FP32 values.
template <int OPK, int KS>
struct Operand {
  uint4 v[KS];
  __device__ __forceinline__ void load(const void *base, int64_t point, int kstride, int lh) {
    const uint4 *p = reinterpret_cast<const uint4 *>(
        static_cast<const uint16_t *>(base) + point * kstride + 8 * lh);
#pragma unroll
    for (int s = 0; s < KS; ++s) v[s] = p[2 * s];
  }
};

template <int KS>
struct Operand<kOpF32, KS> {
  static constexpr int KS4 = (KS + 3) / 4;
  float v[KS4 * 4];
  __device__ __forceinline__ void load(const void *base, int64_t point, int kstride, int lh) {
    const float4 *p = reinterpret_cast<const float4 *>(
        static_cast<const float *>(base) + point * kstride + lh * (kstride / 2));
#pragma unroll
    for (int s = 0; s < KS4; ++s) {
      float4 u = p[s];
      v[4 * s + 0] = u.x;
      v[4 * s + 1] = u.y;
      v[4 * s + 2] = u.z;
      v[4 * s + 3] = u.w;
    }
  }
};

template <int OPK, int KS>
__device__ __forceinline__ f32x16 tile_r2(const Operand<OPK, KS> &a, const Operand<OPK, KS> &b) {
  f32x16 acc = {};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    if constexpr (OPK == kOpF32)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[s], b.v[s], acc, 0, 0, 0);
    else if constexpr (OPK == kOpF16)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a.v[s]),
                                                   __builtin_bit_cast(f16x8, b.v[s]), acc, 0, 0, 0);
    else
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a.v[s]),
                                                    __builtin_bit_cast(bf16x8, b.v[s]), acc, 0, 0, 0);
  }
  return acc;
}


template <int KERN, int KS, int MV, int OPK>
__device__ __forceinline__ void symv_body(const SymvArgs &A, const int64_t item) {
  constexpr int TR = sweep_tile_rows(MV, OPK, KS);
  constexpr int BLK = 4 * 32 * TR;
  constexpr int NCT = BLK / 32;
  __shared__ float colpart[MV][4][BLK];
  const int I = static_cast<int>(item / A.nchunk);
  const int c = static_cast<int>(item % A.nchunk);

  const int nb = A.nb;
  const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? A.dmax : A.dmax + 1;
  const int d0 = c * A.chunk;
  const int d1 = min(d0 + A.chunk, ndel);

  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int lc = l & 31, lh = l >> 5;
  const int64_t n_pad = A.n_pad;
  const int64_t rowbase = int64_t(I) * BLK + w * 32 * TR;

  // Row sums: FP32 runs over the column tiles of one block pair, then FP64
  // across block pairs for the FP32 operator (single-vector kernel).  With
  // bf16 or split-bf16 points the operator's own error (the rounding of the
  // points) is orders above FP32 summation over one work item's few block
  // pairs, and dropping the FP64 accumulators frees the registers for two
  // tile rows per wave and three waves per SIMD.  Work items are summed in
  // FP64 either way.
  constexpr bool ACC64 = (MV == 1) && (OPK == kOpBf16Acc64 || OPK == kOpF32);
  Operand<OPK, KS> ra[TR];
  float pi[MV][TR][16];
  float accr[MV][TR][16];
  double acc64[ACC64 ? MV : 1][TR][16];
#pragma unroll
  for (int tr = 0; tr < TR; ++tr) {
    ra[tr].load(A.xr, rowbase + 32 * tr + lc, A.kstride, lh);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t i = rowbase + 32 * tr + 8 * (v >> 2) + 4 * lh + (v & 3);
#pragma unroll
      for (int m = 0; m < MV; ++m) {
        pi[m][tr][v] = A.vin[m * n_pad + i];
        accr[m][tr][v] = 0.0f;
        if constexpr (ACC64) acc64[m][tr][v] = 0.0;
      }
    }
  }

  const int tiles = (d1 > d0) ? (d1 - d0) * NCT : 0;
  auto colbase_of = [&](int t) -> int64_t {
    int J = I + d0 + t / NCT;
    if (J >= nb) J -= nb;
    return int64_t(J) * BLK + 32 * (t % NCT);
  };

  Operand<OPK, KS> cb, cbn;
  float pj[MV], pjn[MV];
  if (tiles > 0) {
    const int64_t cb0 = colbase_of(0);
    cb.load(A.xc, cb0 + lc, A.kstride, lh);
#pragma unroll
    for (int m = 0; m < MV; ++m) pj[m] = A.vin[m * n_pad + cb0 + lc];
  }

  // One column tile.  DG: the tile lies in the diagonal block pair (offset
  // 0), where the exact diagonal gets distance zero and no column partials
  // are formed (the block's row sums already cover both triangles).  Only the
  // first block pair of chunk 0 is diagonal, so the two cases run as separate
  // loops and the plain one carries no diagonal test.
  auto step = [&](const int t, auto dg) {
    constexpr bool DG = decltype(dg)::value;
    const int dl = d0 + t / NCT;
    const int ct = t % NCT;
    if (t + 1 < tiles) {
      const int64_t cbx = colbase_of(t + 1);
      cbn.load(A.xc, cbx + lc, A.kstride, lh);
#pragma unroll
      for (int m = 0; m < MV; ++m) pjn[m] = A.vin[m * n_pad + cbx + lc];
    }
    float cs[MV];
#pragma unroll
    for (int m = 0; m < MV; ++m) cs[m] = 0.0f;
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
      f32x16 r2 = tile_r2<OPK, KS>(ra[tr], cb);
      if constexpr (DG) {
        if (ct == w * TR + tr) {
          // the exact diagonal: distance zero by definition
#pragma unroll
          for (int v = 0; v < 16; ++v)
            if (8 * (v >> 2) + 4 * lh + (v & 3) == lc) r2[v] = 0.0f;
        }
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float kv = kval<KERN>(r2[v]);
#pragma unroll
        for (int m = 0; m < MV; ++m) {
          accr[m][tr][v] = fmaf(kv, pj[m], accr[m][tr][v]);
          if constexpr (!DG) cs[m] = fmaf(kv, pi[m][tr][v], cs[m]);
        }
      }
    }
    if constexpr (!DG) {
#pragma unroll
      for (int m = 0; m < MV; ++m) {
        cs[m] += __shfl_xor(cs[m], 32);
        if (lh == 0) colpart[m][w][32 * ct + lc] = cs[m];
      }
      if (ct == NCT - 1) {
        __syncthreads();
        int J = I + dl;
        if (J >= nb) J -= nb;
        for (int e = threadIdx.x; e < MV * BLK; e += 256) {
          const int m = e / BLK, col = e % BLK;
          const float s = (colpart[m][0][col] + colpart[m][1][col]) +
                          (colpart[m][2][col] + colpart[m][3][col]);
          A.pcol[(int64_t(dl - 1) * MV + m) * n_pad + int64_t(J) * BLK + col] = s;
        }
        __syncthreads();
      }
    }
    if constexpr (ACC64) {
      if (ct == NCT - 1) {
#pragma unroll
        for (int m = 0; m < MV; ++m)
#pragma unroll
          for (int tr = 0; tr < TR; ++tr)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              acc64[m][tr][v] += static_cast<double>(accr[m][tr][v]);
              accr[m][tr][v] = 0.0f;
            }
      }
    }
    if (t + 1 < tiles) {
      cb = cbn;
#pragma unroll
      for (int m = 0; m < MV; ++m) pj[m] = pjn[m];
    }
  };
  int t = 0;
  if (d0 == 0)
    for (const int tdiag = min(tiles, NCT); t < tdiag; ++t) step(t, std::true_type());
  for (; t < tiles; ++t) step(t, std::false_type());

  // Row sums: reduce over the 32 lanes that hold the same rows.
#pragma unroll
  for (int m = 0; m < MV; ++m) {
#pragma unroll
    for (int tr = 0; tr < TR; ++tr) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        double s;
        if constexpr (ACC64) s = acc64[m][tr][v];
        else s = static_cast<double>(accr[m][tr][v]);
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 16);
        if (lc == v) {
          const int64_t i = rowbase + 32 * tr + 8 * (v >> 2) + 4 * lh + (v & 3);
          A.prow[(int64_t(c) * MV + m) * n_pad + i] = s;
        }
      }
    }
  }
}

template <int KERN, int KS, int MV, int OPK>
__global__ __launch_bounds__(256, 2) void symv_kernel(SymvArgs A) {
  if (A.done != nullptr && *A.done != 0) return;
  symv_body<KERN, KS, MV, OPK>(A, xcd_remap(blockIdx.x, int64_t(A.nb) * A.nchunk));
}

// Many operators in one launch: the grid is the concatenation of every
// system's work items; a workgroup finds its system by binary search over
// the first-item offsets and skips systems that have converged.
template <int KS, int OPK>
__global__ __launch_bounds__(256, 2) void symv_batched(const BatchItem *sys, int count,
                                                       int64_t total) {
  const int64_t g = xcd_remap(blockIdx.x, total);
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (sys[mid].item0 <= g) lo = mid;
    else hi = mid - 1;
  }
  const BatchItem &B = sys[lo];
  if (B.a.done != nullptr && *B.a.done != 0) return;
  const int64_t item = g - B.item0;
  if (B.kernel == DCG_RBF) symv_body<DCG_RBF, KS, 1, OPK>(B.a, item);
  else if (B.kernel == DCG_MATERN32) symv_body<DCG_MATERN32, KS, 1, OPK>(B.a, item);
  else symv_body<DCG_MATERN52, KS, 1, OPK>(B.a, item);
}

// Finish y = s2 * (sum of partials) + sigma2 v for the first `cols` vectors
// (with a diagonal scaling: y = d * s2 * (sum) + sigma2 v).
__global__ __launch_bounds__(256) void symv_reduce(ReduceArgs A, int cols) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= A.n * cols) return;
  const int m = static_cast<int>(e / A.n);
  const int64_t i = e % A.n;
  const double s = sum_partials(A, m, i);
  const double s2 = (A.dsc != nullptr) ? A.s2 * A.dsc[i] : A.s2;
  A.Y[m * A.n + i] = fma(s2, s, A.sigma2 * A.V[m * A.n + i]);
}

// FP64 -> FP32 staging of up to 4 vectors (times the diagonal scaling d if
// given), zero padded to n_pad.
__global__ __launch_bounds__(256) void stage_vectors(const double *V, int64_t n, int64_t n_pad,
                                                     int mv, int mvs, const double *dsc,
                                                     float *out) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n_pad * mvs) return;
  const int m = static_cast<int>(e / n_pad);
  const int64_t i = e % n_pad;
  float v = 0.0f;
  if (m < mv && i < n) v = static_cast<float>((dsc != nullptr) ? dsc[i] * V[m * n + i] : V[m * n + i]);
  out[e] = v;
}

// ----------------------------------------------------------------- dispatch

double point_scale(int kernel, double ell) {
  const double log2e = 1.4426950408889634;
  if (kernel == DCG_RBF) return std::sqrt(0.5 * log2e) / ell;
  return std::sqrt(kernel == DCG_MATERN32 ? 3.0 : 5.0) * log2e / ell;
}

template <int KERN, int KS, int MV, int OPK>
static void launch_symv(const SymvArgs &a, int64_t grid, hipStream_t s) {
  hipLaunchKernelGGL((symv_kernel<KERN, KS, MV, OPK>), dim3(static_cast<unsigned>(grid)),
                     dim3(256), 0, s, a);
}

template <int KERN, int MV, int OPK>
static int dispatch_bf16(int ks, const SymvArgs &a, int64_t grid, hipStream_t s) {
  if (OPK == kOpBf16Acc64 && ks > 13) return -1;
  switch (ks) {
    case 1: launch_symv<KERN, 1, MV, OPK>(a, grid, s); return 0;
    case 2: launch_symv<KERN, 2, MV, OPK>(a, grid, s); return 0;
    case 3: launch_symv<KERN, 3, MV, OPK>(a, grid, s); return 0;
    case 4: launch_symv<KERN, 4, MV, OPK>(a, grid, s); return 0;
    case 5: launch_symv<KERN, 5, MV, OPK>(a, grid, s); return 0;
    case 7: launch_symv<KERN, 7, MV, OPK>(a, grid, s); return 0;
    case 9: launch_symv<KERN, 9, MV, OPK>(a, grid, s); return 0;
    case 13: launch_symv<KERN, 13, MV, OPK>(a, grid, s); return 0;
    case 17:
      if constexpr (OPK == kOpBf16 || OPK == kOpF16) {
        launch_symv<KERN, 17, MV, OPK>(a, grid, s);
        return 0;
      }
  }
  return -1;
}

template <int KERN, int MV>
static int dispatch_ks(const dcg_operator_s *op, const SymvArgs &a, int64_t grid) {
  const int ks = op->g.ksteps;
  hipStream_t s = op->stream;
  if (op->g.opk == kOpBf16) return dispatch_bf16<KERN, MV, kOpBf16>(ks, a, grid, s);
  if (op->g.opk == kOpBf16Acc64) return dispatch_bf16<KERN, MV, kOpBf16Acc64>(ks, a, grid, s);
  if (op->g.opk == kOpF16) return dispatch_bf16<KERN, MV, kOpF16>(ks, a, grid, s);
  switch (ks) {
    case 5: launch_symv<KERN, 5, MV, kOpF32>(a, grid, s); return 0;
    case 9: launch_symv<KERN, 9, MV, kOpF32>(a, grid, s); return 0;
    case 13: launch_symv<KERN, 13, MV, kOpF32>(a, grid, s); return 0;
    case 17: launch_symv<KERN, 17, MV, kOpF32>(a, grid, s); return 0;
    case 25: launch_symv<KERN, 25, MV, kOpF32>(a, grid, s); return 0;
    case 33: launch_symv<KERN, 33, MV, kOpF32>(a, grid, s); return 0;
  }
  return -1;
}

// Arguments of the symmetric pair sweep of op over vin (mv = 1 or 4
// vectors) and its grid.
SymvArgs symv_args(const dcg_operator_s *op, int mv, const float *vin, const int *done,
                   int64_t *grid) {
  MatvecPlan p = sweep_plan(op->g, mv, op->sweep_items);
  SymvArgs a;
  a.xr = op->xr;
  a.xc = op->xc;
  a.kstride = op->g.kstride;
  a.vin = vin;
  a.prow = reinterpret_cast<double *>(op->part);
  a.pcol = op->part + size_t(2 * p.nchunk) * op->g.n_pad * mv;
  a.n_pad = op->g.n_pad;
  a.nb = p.nb;
  a.dmax = p.dmax;
  a.chunk = p.chunk;
  a.nchunk = p.nchunk;
  a.done = done;
  if (grid != nullptr) *grid = p.grid;
  return a;
}

// The batched sweep is built for the two-tile-row single-vector kernels.
bool symv_batched_supported(int opk, int ksteps) {
  if (opk == kOpBf16 || opk == kOpBf16Acc64 || opk == kOpF16)
    return (ksteps >= 1 && ksteps <= 5) || ksteps == 7 || ksteps == 9;
  if (opk == kOpF32) return ksteps == 5 || ksteps == 9 || ksteps == 13 || ksteps == 17;
  return false;
}

template <int OPK>
static void launch_batched_bf16(const BatchItem *d_items, int count, int64_t total, int ksteps,
                                hipStream_t s) {
  const dim3 g(static_cast<unsigned>(total)), b(256);
  switch (ksteps) {
    case 1: hipLaunchKernelGGL((symv_batched<1, OPK>), g, b, 0, s, d_items, count, total); break;
    case 2: hipLaunchKernelGGL((symv_batched<2, OPK>), g, b, 0, s, d_items, count, total); break;
    case 3: hipLaunchKernelGGL((symv_batched<3, OPK>), g, b, 0, s, d_items, count, total); break;
    case 4: hipLaunchKernelGGL((symv_batched<4, OPK>), g, b, 0, s, d_items, count, total); break;
    case 5: hipLaunchKernelGGL((symv_batched<5, OPK>), g, b, 0, s, d_items, count, total); break;
    case 7: hipLaunchKernelGGL((symv_batched<7, OPK>), g, b, 0, s, d_items, count, total); break;
    default: hipLaunchKernelGGL((symv_batched<9, OPK>), g, b, 0, s, d_items, count, total); break;
  }
}

int launch_symv_batched(const BatchItem *d_items, int count, int64_t total, int ksteps, int opk,
                        hipStream_t s) {
  if (!symv_batched_supported(opk, ksteps) || total < 1) return DCG_E_ARG;
  const dim3 g(static_cast<unsigned>(total)), b(256);
  if (opk == kOpBf16) {
    launch_batched_bf16<kOpBf16>(d_items, count, total, ksteps, s);
  } else if (opk == kOpBf16Acc64) {
    launch_batched_bf16<kOpBf16Acc64>(d_items, count, total, ksteps, s);
  } else if (opk == kOpF16) {
    launch_batched_bf16<kOpF16>(d_items, count, total, ksteps, s);
  } else {
    switch (ksteps) {
      case 5: hipLaunchKernelGGL((symv_batched<5, kOpF32>), g, b, 0, s, d_items, count, total); break;
      case 9: hipLaunchKernelGGL((symv_batched<9, kOpF32>), g, b, 0, s, d_items, count, total); break;
      case 13: hipLaunchKernelGGL((symv_batched<13, kOpF32>), g, b, 0, s, d_items, count, total); break;
      default: hipLaunchKernelGGL((symv_batched<17, kOpF32>), g, b, 0, s, d_items, count, total); break;
    }
  }
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

int launch_symv_sweep_from(const dcg_operator_s *op, int mv, const float *vin, const int *done) {
  int64_t grid = 0;
  const SymvArgs a = symv_args(op, mv, vin, done, &grid);
  if (sweep_wide(op->g)) return mv == 1 ? launch_symv_wide(op, a, grid) : DCG_E_ARG;
  int rc = -1;
  if (mv == 1) {
    if (op->kernel == DCG_RBF) rc = dispatch_ks<DCG_RBF, 1>(op, a, grid);
    else if (op->kernel == DCG_MATERN32) rc = dispatch_ks<DCG_MATERN32, 1>(op, a, grid);
    else rc = dispatch_ks<DCG_MATERN52, 1>(op, a, grid);
  } else {
    if (op->kernel == DCG_RBF) rc = dispatch_ks<DCG_RBF, 4>(op, a, grid);
    else if (op->kernel == DCG_MATERN32) rc = dispatch_ks<DCG_MATERN32, 4>(op, a, grid);
    else rc = dispatch_ks<DCG_MATERN52, 4>(op, a, grid);
  }
  if (rc != 0) return DCG_E_ARG;
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

int launch_symv_sweep(const dcg_operator_s *op, int mv, const int *done) {
  return launch_symv_sweep_from(op, mv, op->vin, done);
}

ReduceArgs reduce_args(const dcg_operator_s *op, int mv, const double *V, double *Y) {
  MatvecPlan p = sweep_plan(op->g, mv, op->sweep_items);
  ReduceArgs r;
  r.prow = reinterpret_cast<const double *>(op->part);
  r.pcol = op->part + size_t(2 * p.nchunk) * op->g.n_pad * mv;
  r.n = op->g.n;
  r.n_pad = op->g.n_pad;
  r.nchunk = p.nchunk;
  r.dmax = p.dmax;
  r.blk = p.blk;
  r.nb = p.nb;
  r.mv = mv;
  r.s2 = op->s2;
  r.sigma2 = op->sigma2;
  r.dsc = op->has_dsc ? op->dsc : nullptr;
  r.V = V;
  r.Y = Y;
  return r;
}

// Y = A V for m vectors (groups of 4, a last single vector group of 1).
int matvec_lowprec(const dcg_operator_s *op, const double *V, double *Y, int64_t m) {
  if (op->g.prec == DCG_PREC_FP64) return matvec_exact(op, V, Y, m);
  if (op->g.prec == DCG_PREC_STORED) return matvec_stored_done(op, V, Y, m, nullptr);
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  int64_t done_cols = 0;
  while (done_cols < m) {
    const int64_t left = m - done_cols;
    const int mv = (left >= 2 && !sweep_wide(op->g)) ? 4 : 1;
    const int cols = static_cast<int>(std::min<int64_t>(left, mv));
    const double *Vc = V + done_cols * n;
    double *Yc = Y + done_cols * n;
    hipLaunchKernelGGL(stage_vectors, dim3(static_cast<unsigned>(cdiv(n_pad * mv, 256))), dim3(256),
                       0, op->stream, Vc, n, n_pad, cols, mv, op->has_dsc ? op->dsc : nullptr,
                       op->vin);
    int rc = launch_symv_sweep(op, mv, nullptr);
    if (rc != DCG_OK) return rc;
    // only the first `cols` staged vectors are real; reduce those
    ReduceArgs r = reduce_args(op, mv, Vc, Yc);
    hipLaunchKernelGGL(symv_reduce, dim3(static_cast<unsigned>(cdiv(n * cols, 256))), dim3(256),
                       0, op->stream, r, cols);
    if (hipGetLastError() != hipSuccess) return DCG_E_HIP;
    done_cols += cols;
  }
  return DCG_OK;
}

}  // namespace dcg
