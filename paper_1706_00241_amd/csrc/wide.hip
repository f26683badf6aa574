// The pair sweep for wide points (65 to 4096 coordinates, bf16 or fp16
// operands): the product A p of Algorithm 1 without a stored kernel matrix
// when the distance contraction, not the kernel evaluation, dominates the
// pair cost (2 (d + 6) MFMA flops against ~10 VALU slots per pair).
//
// Same circulant schedule of 256-point block pairs, work items and partial
// layout as the narrow sweep (matvec.hip), so the product is finished by the
// same kernels.  A work item (one 512-thread workgroup, eight waves) takes a
// row block I and a run of offsets; for each block pair (I, J) the augmented
// operands of both blocks stream through LDS in 64-element slices of K
// (double-buffered: the next slice's global loads are in flight while the
// current one feeds the matrix cores), each wave accumulating a 64 x 128
// part of the 256 x 256 distance tile in eight 32x32x16 MFMA tiles.  The
// slices are stored with the 16-byte groups of a row XOR-swizzled by the row
// index, so that the rows a fragment read serves together fall in distinct
// LDS banks.  After the last slice the kernel values are formed in registers on
// the MFMA output layout and folded into FP32 row sums (accumulated in LDS
// across the work item's block pairs) and per-block-pair column sums.
#include <algorithm>
#include <cmath>

#include "blas.h"
#include "host.h"
#include "sweep.h"

namespace dcg {

constexpr int kWideRows = 256;  // points per block (rows and columns)
constexpr int kWideKC = 64;     // K elements per LDS slice (four MFMA K-steps)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int OPK>
__device__ __forceinline__ f32x16 wide_mfma(const u32x4 &a, const u32x4 &b, const f32x16 &c) {
  if constexpr (OPK == kOpF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Slot of the 16-byte group g (0..7) of row `row` in a slice.  A fragment
// read takes group g of 32 consecutive rows; the 128-byte rows put rows of
// equal parity on the same half of 256 bytes of banks, so the group is
// XOR-ed with row mod 8 and with bit 3 of the row: any 8 consecutive rows
// use 8 distinct 16-byte bank groups, and any 16 use 16 distinct groups of
// 256 bytes (rows r and r + 8 differ in the low bit of the XOR).
__device__ __forceinline__ int wide_slot(int row, int g) {
  return row * 8 + (g ^ (row & 7) ^ ((row >> 3) & 1));
}

template <int KERN, int OPK>
__global__ __launch_bounds__(512, 1) void symv_wide_kernel(SymvArgs A) {
  if (A.done != nullptr && *A.done != 0) return;
  const int64_t item = xcd_remap(blockIdx.x, int64_t(A.nb) * A.nchunk);
  const int I = static_cast<int>(item / A.nchunk);
  const int c = static_cast<int>(item % A.nchunk);
  const int nb = A.nb;
  const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? A.dmax : A.dmax + 1;
  const int d0 = c * A.chunk;
  const int d1 = min(d0 + A.chunk, ndel);

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lc = l & 31, lh = l >> 5;
  const int wr = w & 3, wc = w >> 2;     // rows 64 wr .., columns 128 wc .. of a block pair
  const int64_t n_pad = A.n_pad;
  const int kst = A.kstride;             // a multiple of kWideKC
  const int nkc = kst / kWideKC;

  __shared__ u32x4 As[2][kWideRows * 8];
  __shared__ u32x4 Bs[2][kWideRows * 8];
  __shared__ float rowacc[2][kWideRows];
  __shared__ float colpart[4][kWideRows];
  __shared__ float vrow[kWideRows];      // the input vector on this row block

  for (int e = tid; e < 2 * kWideRows; e += 512) rowacc[e / kWideRows][e % kWideRows] = 0.0f;
  for (int e = tid; e < kWideRows; e += 512) vrow[e] = A.vin[int64_t(I) * kWideRows + e];
  __syncthreads();

  const uint16_t *xr = static_cast<const uint16_t *>(A.xr);
  const uint16_t *xc = static_cast<const uint16_t *>(A.xc);
  // staging: this thread moves rows srow + 64 i (i < 4), group sg, of both
  // operand blocks
  const int srow = tid >> 3, sg = tid & 7;

  for (int dl = d0; dl < d1; ++dl) {
    int J = I + dl;
    if (J >= nb) J -= nb;
    const uint16_t *ablk = xr + int64_t(I) * kWideRows * kst + int64_t(srow) * kst + sg * 8;
    const uint16_t *bblk = xc + int64_t(J) * kWideRows * kst + int64_t(srow) * kst + sg * 8;
    const int64_t rstep = int64_t(64) * kst;
    f32x16 acc[2][4];
#pragma unroll
    for (int tr = 0; tr < 2; ++tr)
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) acc[tr][tc] = f32x16{};
    u32x4 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;
#define DCG_WIDE_GLOAD(kc)                                                        \
  do {                                                                            \
    const int64_t ko = int64_t(kc) * kWideKC;                                     \
    sa0 = *reinterpret_cast<const u32x4 *>(ablk + ko);                            \
    sb0 = *reinterpret_cast<const u32x4 *>(bblk + ko);                            \
    sa1 = *reinterpret_cast<const u32x4 *>(ablk + rstep + ko);                    \
    sb1 = *reinterpret_cast<const u32x4 *>(bblk + rstep + ko);                    \
    sa2 = *reinterpret_cast<const u32x4 *>(ablk + 2 * rstep + ko);                \
    sb2 = *reinterpret_cast<const u32x4 *>(bblk + 2 * rstep + ko);                \
    sa3 = *reinterpret_cast<const u32x4 *>(ablk + 3 * rstep + ko);                \
    sb3 = *reinterpret_cast<const u32x4 *>(bblk + 3 * rstep + ko);                \
  } while (0)
#define DCG_WIDE_LSTORE(buf)                                                      \
  do {                                                                            \
    As[buf][wide_slot(srow, sg)] = sa0;                                           \
    Bs[buf][wide_slot(srow, sg)] = sb0;                                           \
    As[buf][wide_slot(srow + 64, sg)] = sa1;                                      \
    Bs[buf][wide_slot(srow + 64, sg)] = sb1;                                      \
    As[buf][wide_slot(srow + 128, sg)] = sa2;                                     \
    Bs[buf][wide_slot(srow + 128, sg)] = sb2;                                     \
    As[buf][wide_slot(srow + 192, sg)] = sa3;                                     \
    Bs[buf][wide_slot(srow + 192, sg)] = sb3;                                     \
  } while (0)
    DCG_WIDE_GLOAD(0);
    DCG_WIDE_LSTORE(0);
    __syncthreads();
    for (int kc = 0; kc < nkc; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nkc) DCG_WIDE_GLOAD(kc + 1);
#pragma unroll
      for (int ks = 0; ks < kWideKC / 16; ++ks) {
        const int g = 2 * ks + lh;   // this lane's 8 elements of the K-step
        u32x4 af[2], bf[4];
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) af[tr] = As[buf][wide_slot(64 * wr + 32 * tr + lc, g)];
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) bf[tc] = Bs[buf][wide_slot(128 * wc + 32 * tc + lc, g)];
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
          for (int tc = 0; tc < 4; ++tc) acc[tr][tc] = wide_mfma<OPK>(af[tr], bf[tc], acc[tr][tc]);
      }
      // the other slice buffer was last read before the previous barrier
      if (kc + 1 < nkc) DCG_WIDE_LSTORE(buf ^ 1);
      __syncthreads();
    }
#undef DCG_WIDE_GLOAD
#undef DCG_WIDE_LSTORE

    // kernel values on the MFMA output layout: lane l holds column l % 32
    // and rows 8 (v / 4) + 4 (l / 32) + v % 4 of each 32x32 tile
    const bool diag = (dl == 0);
    const int64_t cbase = int64_t(J) * kWideRows + 128 * wc;
    float pj[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) pj[tc] = A.vin[cbase + 32 * tc + lc];
    float cs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tr = 0; tr < 2; ++tr) {
      float rs[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) rs[v] = 0.0f;
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) {
        f32x16 r2 = acc[tr][tc];
        if (diag && 2 * wr + tr == 4 * wc + tc) {
          // the exact diagonal: distance zero by definition
#pragma unroll
          for (int v = 0; v < 16; ++v)
            if (8 * (v >> 2) + 4 * lh + (v & 3) == lc) r2[v] = 0.0f;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float kv = kval<KERN>(r2[v]);
          rs[v] = fmaf(kv, pj[tc], rs[v]);
          if (!diag)
            cs[tc] = fmaf(kv, vrow[64 * wr + 32 * tr + 8 * (v >> 2) + 4 * lh + (v & 3)], cs[tc]);
        }
      }
      // row sums of this tile row: over the 32 lanes that hold the same
      // rows, added into the work item's FP32 accumulator (one writer per row)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float s = rs[v];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 16);
        if (lc == v) rowacc[wc][64 * wr + 32 * tr + 8 * (v >> 2) + 4 * lh + (v & 3)] += s;
      }
    }
    // column sums of an off-diagonal block pair: the block's four row
    // quarters added in a fixed order
    if (!diag) {
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) {
        const float s = cs[tc] + __shfl_xor(cs[tc], 32);
        if (lh == 0) colpart[wr][128 * wc + 32 * tc + lc] = s;
      }
      __syncthreads();
      for (int e = tid; e < kWideRows; e += 512) {
        const float s = (colpart[0][e] + colpart[1][e]) + (colpart[2][e] + colpart[3][e]);
        A.pcol[int64_t(dl - 1) * n_pad + int64_t(J) * kWideRows + e] = s;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < kWideRows; e += 512)
    A.prow[int64_t(c) * n_pad + int64_t(I) * kWideRows + e] =
        static_cast<double>(rowacc[0][e]) + static_cast<double>(rowacc[1][e]);
}

template <int OPK>
static void launch_wide_kernel(int kernel, const SymvArgs &a, int64_t grid, hipStream_t s) {
  const dim3 g(static_cast<unsigned>(grid)), b(512);
  if (kernel == DCG_RBF) hipLaunchKernelGGL((symv_wide_kernel<DCG_RBF, OPK>), g, b, 0, s, a);
  else if (kernel == DCG_MATERN32)
    hipLaunchKernelGGL((symv_wide_kernel<DCG_MATERN32, OPK>), g, b, 0, s, a);
  else hipLaunchKernelGGL((symv_wide_kernel<DCG_MATERN52, OPK>), g, b, 0, s, a);
}

int launch_symv_wide(const dcg_operator_s *op, const SymvArgs &a, int64_t grid) {
  const Geometry &g = op->g;
  if (!sweep_wide(g) || g.kstride % kWideKC != 0 || sweep_blk(g, 1) != kWideRows ||
      g.n_pad % kWideRows != 0 || grid < 1)
    return DCG_E_ARG;
  if (g.opk == kOpF16) launch_wide_kernel<kOpF16>(op->kernel, a, grid, op->stream);
  else launch_wide_kernel<kOpBf16>(op->kernel, a, grid, op->stream);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

}  // namespace dcg
