"""Rounding of the input points to the compute precision of the operator.

Test infrastructure only (see ``oracle/__init__``).

The precision form evaluates the distance GEMM on rounded points x~ = rnd(x)
and defines the low-precision operator as the exact kernel matrix on those
points, A~ = K(X~, X~) + sigma^2 I.  It therefore stays SPD, and iterative
refinement against the FP64 operator A = K(X, X) + sigma^2 I recovers the
FP64 solution.  The paper itself fixes no precision; this is the reading the
library implements, restated here from the number-format definitions:

* fp32: IEEE-754 binary32, round to nearest, ties to even (numpy's cast).
* bf16: bfloat16 = the upper 16 bits of binary32 (8 exponent bits, 7 stored
  mantissa bits).  Rounding is to nearest, ties to even, applied to the FP64
  value directly (one rounding, never via fp32 first).
* bf16x2: the pair hi + lo with hi = bf16(x), lo = bf16(x - hi).
"""

import numpy as np

PREC_FP32, PREC_BF16, PREC_BF16X2, PREC_FP64 = 0, 1, 2, 3


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), as FP64.

    A bfloat16 has 8 significant bits.  For a normal value with exponent e
    (2^e <= |x| < 2^(e+1)) the spacing is 2^(e-7); we scale so that spacing
    becomes 1, round half-to-even (numpy.rint), and scale back.  Values below
    the smallest normal bfloat16 (2^-126) are rejected: the synthetic inputs
    never reach them.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    if np.any(np.abs(x[nz]) < 2.0 ** -126):
        raise ValueError("subnormal bfloat16 inputs are outside the modelled range")
    m, e = np.frexp(x[nz])          # x = m 2^e with 0.5 <= |m| < 1
    # 8 significant bits: scale the mantissa to [128, 256)
    q = np.rint(m * 256.0)          # round half to even
    out[nz] = np.ldexp(q / 256.0, e)
    return out


def round_bf16x2(x):
    """A pair of bfloat16 values hi + lo: hi = bf16(x), lo = bf16(x - hi).

    The pair carries 16 significant bits (|x - (hi + lo)| <= 2^-17 |x| up to
    the bf16 spacing of lo), the representation of the split-bf16 operator.
    """
    x = np.asarray(x, dtype=np.float64)
    hi = round_bf16(x)
    lo = round_bf16(x - hi)
    return hi + lo


def round_points(X, prec):
    """Points in the operator's compute precision (returned as FP64)."""
    if prec == PREC_FP32:
        return round_fp32(X)
    if prec == PREC_BF16:
        return round_bf16(X)
    if prec == PREC_BF16X2:
        return round_bf16x2(X)
    if prec == PREC_FP64:
        return np.asarray(X, dtype=np.float64).copy()
    raise ValueError(f"unknown precision {prec}")
