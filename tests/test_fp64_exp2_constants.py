"""CPU pin of the FP64 exponential the FP64 operator evaluates (no GPU).

The FP64 pair sweep computes 2^x for x <= 0 as 2^k * p(f), k = rint(x),
f = x - k in [-1/2, 1/2], with p the degree-11 polynomial whose coefficients
are written in the kernel source, evaluated by Horner's rule with fused
multiply-adds (one rounding per step).  This test reads those coefficients
from the source, evaluates the same FMA Horner scheme exactly (each step
computed in rational arithmetic and rounded once to the nearest double), and
compares with 2^f to 40 significant digits (Python's decimal module): the
relative error must stay within 1.3e-16 over [-1/2, 1/2], so the constants
are checked on their own and not only through the product's 1e-12 parity.
"""

import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1706_00241_amd", "csrc", "exact.hip")


def _coefficients():
    text = open(SRC).read()
    body = text[text.index("double exp2_nonpos(double x)"):]
    body = body[:body.index("return __builtin_amdgcn_ldexp")]
    lead = re.search(r"double p = ([0-9.eE+-]+);", body).group(1)
    rest = re.findall(r"p = fma\(p, f, ([0-9.eE+-]+)\);", body)
    return [float(lead)] + [float(c) for c in rest]   # highest degree first


def _fma_horner(coef, f):
    """Horner with one rounding per fused multiply-add, as the GPU does."""
    p = coef[0]
    F = Fraction(f)
    for c in coef[1:]:
        p = float(Fraction(p) * F + Fraction(c))    # exact, then one rounding
    return p


def _exp2_exact(f):
    getcontext().prec = 40
    return Decimal(2) ** Decimal(f)


def test_coefficients_read_from_source():
    c = _coefficients()
    assert len(c) == 12
    # the constant and linear terms of 2^f: 1 and ln 2
    assert c[-1] == 1.0
    assert c[-2] == pytest.approx(np.log(2.0), rel=1e-15)


def test_exp2_polynomial_within_1p3e16_on_the_reduced_interval():
    coef = _coefficients()
    fs = np.concatenate([np.linspace(-0.5, 0.5, 4001),
                         np.random.default_rng(5).uniform(-0.5, 0.5, 2000),
                         [0.0, -0.5, 0.5, 2.0 ** -30, -(2.0 ** -30)]])
    worst = 0.0
    for f in fs:
        got = _fma_horner(coef, float(f))
        ref = _exp2_exact(float(f))
        err = abs((Decimal(got) - ref) / ref)
        worst = max(worst, float(err))
    assert worst <= 1.3e-16, worst


def test_exp2_with_range_reduction():
    """2^x for x in [-1100, 0]: k = rint(x) (ties to even), f = x - k is
    exact, 2^k applied exactly; the result keeps the polynomial's accuracy
    (normal range) and underflows to zero below -1075."""
    coef = _coefficients()
    xs = list(np.random.default_rng(6).uniform(-1000.0, 0.0, 300)) + [-0.5, -1.5, -2.5, -37.25]
    for x in xs:
        k = float(np.rint(x))
        f = x - k
        assert Fraction(f) == Fraction(x) - Fraction(k)      # exact subtraction
        got = np.ldexp(_fma_horner(coef, f), int(k))
        ref = _exp2_exact(x)
        if ref > Decimal(2) ** -1022:
            assert abs((Decimal(got) - ref) / ref) <= 1.3e-16, x
    assert np.ldexp(_fma_horner(coef, 0.0), -1100) == 0.0
