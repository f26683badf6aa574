// Internal declarations shared by the HIP sources of libdcg.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/dcg.h"

namespace dcg {

constexpr int kMaxD = 64;          // point dimension of the register-operand pair sweep
constexpr int kMaxWideD = 4096;    // point dimension of the LDS-staged sweep (bf16, fp16)
constexpr int kMaxStoredD = 4096;  // point dimension of the stored operator
constexpr int kMaxK = 64;          // columns of W
constexpr int kMaxZ = 192;         // k + L (columns of Z)
constexpr int kRedBlocks = 256;    // blocks of the grid-stride FP64 reductions
constexpr int kMaxBatch = 4096;    // systems of one batched solve
constexpr int kMaxBlockCols = 64;  // right-hand sides of one block solve

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Simple bump allocator over a caller workspace.
struct Carve {
  char *base;
  size_t off = 0, cap;
  Carve(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
  template <class T>
  T *take(size_t count) {
    size_t o = align256(off);
    off = o + count * sizeof(T);
    return base ? reinterpret_cast<T *>(base + o) : nullptr;
  }
  bool fits() const { return off <= cap; }
};

// Geometry of the augmented point arrays used by the distance GEMM.
// Row operand  xr_i = [-2 x_i, 1.., a_i parts, 0 pad]
// Col operand  xc_j = [  x_j, a_j parts, 1.., 0 pad]
// so that <xr_i, xc_j> = a_i + a_j - 2 x_i.x_j = |x_i - x_j|^2.
//
// Operand kinds of the low-precision sweep:
//   kOpBf16       bf16 pieces (bf16: x~; bf16x2: hi, lo), FP32 row sums within
//                 a work item (the operator's own error is far above them);
//   kOpBf16Acc64  the FP32 operator's points, each FP32 coordinate split
//                 exactly into three bf16 terms h + m + l; the six products
//                 above 2^-24 (hh, hm, mh, hl, lh, mm) go through bf16 MFMA,
//                 and row sums carry FP64 accumulators across block pairs;
//   kOpF32        FP32 MFMA operands (the FP32 operator for d > 33, where
//                 6d + 6 terms need more than 13 bf16 K-steps);
//   kOpF16        fp16 points (11 significant bits) on fp16 MFMA, FP32 row
//                 sums within a work item as for bf16.
enum OperandKind { kOpBf16 = 0, kOpBf16Acc64 = 1, kOpF32 = 2, kOpF16 = 3 };

struct Geometry {
  int64_t n, n_pad;  // n_pad: multiple of the block size of both schedules
  int d;
  int prec;
  int opk;           // OperandKind of the low-precision operands
  int ksteps;        // MFMA K steps (bf16: 16 per step, fp32: 2 per step)
  int kstride;       // elements per point row in the stored operand arrays
};

Geometry make_geometry(int64_t n, int d, int prec);

struct MatvecPlan {
  int blk;      // rows per block
  int nb;       // number of blocks
  int dmax;     // largest block offset delta
  int chunk;    // column blocks per work item
  int nchunk;   // work items per row block
  int64_t grid;
};

// Tile rows (of 32) per wave in the symmetric sweep: two for the
// single-vector kernel unless its bf16 operands are wide (register budget;
// the FP64 row accumulators of kOpBf16Acc64 take 64 more).  The host plans
// and the device kernel's template parameters use this one rule.
__host__ __device__ constexpr int sweep_tile_rows(int mv, int opk, int ksteps) {
  return (mv == 1 && (opk == kOpF32 || ksteps <= (opk == kOpBf16Acc64 ? 4 : 9))) ? 2 : 1;
}
// bf16 and fp16 operands of more than kMaxD coordinates go through the
// LDS-staged sweep (wide.hip): single vectors, 256-point blocks, no FP64
// operator (the FP64 sweep holds its operands in registers).
inline bool sweep_wide(const Geometry &g) {
  return (g.prec == DCG_PREC_BF16 || g.prec == DCG_PREC_FP16) && g.d > kMaxD;
}
inline int sweep_blk(const Geometry &g, int mv) {
  return sweep_wide(g) ? 256 : 128 * sweep_tile_rows(mv, g.opk, g.ksteps);
}

// Work items of one pair sweep: the plan groups block offsets into chunks so
// that a sweep has about `items` work items.  The default suits one large
// operator; dcg_tune_operator picks the value per operator by timing.
constexpr int kSweepItemsMin = 256;
constexpr int kSweepItemsDefault = 2048;
constexpr int kSweepItemsMax = 8192;

MatvecPlan make_plan(int64_t n_pad, int blk, int items = kSweepItemsDefault);
// The wide sweep's tiled schedule (256-point blocks): groups of kWideGroup
// row blocks; tile (group, part) is kWideGroup x 4 work items (a, b), item
// (a, b) taking row block I = kWideGroup g + a and the pairs (I, I + u),
// u = 4 s + b - a in [0, ndel(I)), for the steps s of its part.  At a step
// the 32 items of a tile touch 8 row blocks and 4 column blocks, which they
// share in one XCD's L2.  Fields: chunk = steps per part, nchunk = 4 x parts
// (row-partial slots per row block: slot 4 part + b), grid = the tiles, padded
// to a multiple of 8, times 32.
constexpr int kWideGroup = 8;
MatvecPlan wide_plan(int64_t n_pad, int items);
int wide_steps(int nb);   // steps s per row block group
// The plan of the operator's single-vector (mv = 1) or four-vector sweep.
MatvecPlan sweep_plan(const Geometry &g, int mv, int items);
// Partial-sum floats of a sweep, for the largest plan any item target gives.
size_t matvec_partial_floats(int64_t n_pad, int mv, int blk);
size_t wide_partial_floats(int64_t n_pad);

}  // namespace dcg

struct dcg_operator_s {
  dcg::Geometry g;
  int kernel;
  double ell, s2, sigma2;
  hipStream_t stream;
  uint64_t generation;   // bumped by every hyperparameter change
  int sweep_items;       // work-item target of the low-precision pair sweep
  int exact_items;       // work-item target of the FP64 pair sweep
  double *x64;           // the points, FP64, n_pad x d row-major (operand source)
  int *flag;             // device flag word: operand preparation problems
  double *dsc;           // diagonal scaling D of A = D K D + sigma2 I (n_pad)
  int has_dsc;           // 1: dsc applies
  uint64_t dsc_version;  // bumped by every dcg_set_diag
  double *x64r, *x64c;   // FP64 augmented operands of the exact operator
  double *vin64;         // staged FP64 input vector, n_pad
  double *part64;        // partial sums of the FP64 sweep
  void *xr, *xc;         // augmented operands (bf16 or fp32)
  float *vin;            // staged FP32 input vectors, n_pad x 4
  float *part;           // partial sums of the symmetric matvec
  double *ytmp;          // n_pad x 4 FP64 staging for products
  float *kst;            // stored operator: K0's block upper triangle, packed FP32 tiles
  double *kpart;         // stored operator: row / column partial sums of a product
};

namespace dcg {
// Whether the operator has the FP64 operator of the unrounded points (the
// refinement residuals): not for the stored matrix, not for wide points.
inline bool has_exact(const dcg_operator_s *op) {
  return op->g.prec != DCG_PREC_STORED && !sweep_wide(op->g);
}
}  // namespace dcg

struct dcg_recycle_s {
  int64_t n;
  int k, L;
  int k_used;            // columns of W currently valid
  int L_eff;             // columns of Z used by the last extraction
  int aw_state;          // 0: AW invalid, 1: AW valid for (op, generation)
  const dcg_operator_s *aw_op;
  uint64_t aw_gen;
  double aw_ell, aw_s2, aw_sigma2;
  uint64_t aw_dsc;       // the operator's dsc_version when AW was formed
  int n_theta;
  double theta[dcg::kMaxK];
  double *Z;             // n x (k + L): [W | P_L]
  double *AZ;            // n x (k + L): [AW | A P_L]
  double *Wt, *AWt;      // n x k staging for W' = Z U, AW' = (AZ) U
  double *F, *G;         // (k+L)^2
  double *U;             // (k+L) x k
  double *eigw;          // eigen-solver workspace
  double *M, *Minv;      // k x k: W^T A W and its inverse
  double *Mwork;         // k x k scratch of the inverse
  double *N;             // k x k: (AW)^T AW
  double *small;         // misc small device scalars / vectors
  int *info;             // device status words of the extraction
  double *gemm;          // split-K partials of the tall-skinny products
  float *W32, *AW32;     // n x k: FP32 copies of W and AW for the per-step
                         // kernels of low-precision operators (w32_valid)
  int w32_valid;
  uint64_t w_version;    // bumped whenever W or AW changes
  uint64_t m_version;    // w_version when M, N, M^{-1} were formed
  int m_valid;
  int rank_F;            // numerical rank of F at the last extraction
  int sweeps[2];         // Jacobi sweeps of the last extraction
};
