// Device helpers shared by the pair sweeps (matvec.hip, wide.hip): MFMA
// operand and result vector types, the kernel value from the squared
// distance of pre-scaled operands, and the XCD-aware order of work items.
#pragma once

#include "blas.h"

namespace dcg {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// Kernel value without the s2 factor, from the squared distance of the
// operands, whose points are pre-scaled by c = point_scale(kernel, ell) so
// that r2 = (c r)^2 feeds exp2 directly:
//   RBF:        exp2(-r2)                              c^2 = log2(e) / (2 ell^2)
//   Matern-3/2: (1 + ln2 u) exp2(-u),          u = c r, c = sqrt3 log2(e) / ell
//   Matern-5/2: (1 + ln2 u + ln2^2 u^2 / 3) exp2(-u),   c = sqrt5 log2(e) / ell
// (for the Matern kernels t = sqrt(nu2) r / ell = u ln2, so e^-t = 2^-u).  No
// multiply by a hyperparameter is left in the pair loop.  |r2| absorbs the
// tiny negative values FP32 rounding can give at r ~ 0.
template <int KERN>
__device__ __forceinline__ float kval(float r2) {
  if constexpr (KERN == DCG_RBF) {
    return __builtin_amdgcn_exp2f(-r2);
  } else {
    const float r2a = fabsf(r2);
    const float u = __builtin_amdgcn_sqrtf(r2a);
    const float e = __builtin_amdgcn_exp2f(-u);
    if constexpr (KERN == DCG_MATERN32) {
      return fmaf(kLn2, u, 1.0f) * e;
    } else {
      return fmaf(kLn2, u, fmaf(kLn2Sq3, r2a, 1.0f)) * e;
    }
  }
}

// Work items are dealt to the 8 XCDs round-robin; the remap gives one XCD a
// run of consecutive items, i.e. neighbouring row blocks that share most
// column blocks, so they share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t G) {
  const int64_t Gm = G - G % 8;
  return (bid < Gm) ? (bid % 8) * (Gm / 8) + bid / 8 : bid;
}

}  // namespace dcg
