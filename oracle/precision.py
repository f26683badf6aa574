"""Rounding of the input points to the compute precision of the operator.

Test infrastructure only (see ``oracle/__init__``).

The precision form evaluates the distance GEMM on rounded scaled points and
defines the low-precision operator as the exact kernel matrix on the points
they represent, x~ = rnd(c x) / c, A~ = K(X~, X~) + sigma^2 I.  It therefore
stays SPD, and iterative refinement against the FP64 operator
A = K(X, X) + sigma^2 I recovers the FP64 solution.  The scale c (see
``point_scale``) depends on the kernel and the lengthscale only: it makes the
squared distance of the scaled points the argument of a base-2 exponential,
so the product evaluates no hyperparameter per pair.  The paper itself fixes
no precision; this is the reading the library implements, restated here from
the number-format definitions:

* fp32: IEEE-754 binary32, round to nearest, ties to even (numpy's cast).
* bf16: bfloat16 = the upper 16 bits of binary32 (8 exponent bits, 7 stored
  mantissa bits).  Rounding is to nearest, ties to even, applied to the FP64
  value directly (one rounding, never via fp32 first).
* bf16x2: the pair hi + lo with hi = bf16(x), lo = bf16(x - hi).
* fp16: IEEE-754 binary16 (5 exponent bits, 10 stored mantissa bits,
  subnormals below 2^-14), round to nearest, ties to even, applied to the
  FP64 value directly.
"""

import math

import numpy as np

PREC_FP32, PREC_BF16, PREC_BF16X2, PREC_FP64, PREC_FP16 = 0, 1, 2, 3, 4
FP16_MAX = 65504.0
RBF, MATERN32, MATERN52 = 0, 1, 2
LOG2E = 1.4426950408889634     # the double nearest log2(e)


def point_scale(kernel, ell):
    """Scale c of the points before rounding (FP64, the operations in this
    order, so the value is the library's bit for bit).

    RBF: exp(-r^2 / (2 ell^2)) = 2^-((c r)^2) with c^2 = log2(e) / (2 ell^2).
    Matern with nu2 = 3 or 5: t = sqrt(nu2) r / ell, e^-t = 2^-(c r) with
    c = sqrt(nu2) log2(e) / ell.
    """
    if kernel == RBF:
        return math.sqrt(0.5 * LOG2E) / ell
    if kernel in (MATERN32, MATERN52):
        return math.sqrt(3.0 if kernel == MATERN32 else 5.0) * LOG2E / ell
    raise ValueError(f"unknown kernel id {kernel}")


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


def round_fp16(x):
    """Round FP64 values to the nearest binary16 (ties to even), as FP64.

    For |x| >= 2^-14 (normal range) the spacing is 2^(e-10) with
    2^e <= |x| < 2^(e+1); below it the spacing is 2^-24 (subnormals).  Scale
    so that the spacing is 1, round half-to-even (numpy.rint), scale back.
    Values whose rounding exceeds the largest finite binary16 are rejected.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    ax = np.abs(x[nz])
    _, fe = np.frexp(ax)                 # ax = m 2^fe with 0.5 <= m < 1
    e = np.maximum(fe - 1.0, -14.0)      # binade exponent, clamped at the subnormals
    q = np.rint(np.ldexp(ax, (10 - e).astype(int)))
    val = np.ldexp(q, (e - 10).astype(int))
    if np.any(val > FP16_MAX):
        raise ValueError("values beyond the binary16 range")
    out[nz] = np.sign(x[nz]) * val
    return out


def round_points(X, prec, kernel, ell):
    """The points the operator of precision ``prec`` represents, as FP64:
    rnd(c X) / c with c = point_scale(kernel, ell) (X itself for FP64)."""
    X = np.asarray(X, dtype=np.float64)
    if prec == PREC_FP64:
        return X.copy()
    rnd = {PREC_FP32: round_fp32, PREC_BF16: round_bf16, PREC_BF16X2: round_bf16x2,
           PREC_FP16: round_fp16}.get(prec)
    if rnd is None:
        raise ValueError(f"unknown precision {prec}")
    c = point_scale(kernel, ell)
    return rnd(c * X) / c
