"""Inexact products for emulating the library's operators on the CPU.

Test infrastructure (helpers of the test suite, not part of the oracle's
arithmetic): the oracle's dense FP64 matrix with a random error added to
every product, so that the oracle's iterations can be run as they behave
with a low-precision (or differently rounded) operator.

Error model: the product (A v)_i = sum_j A_ij v_j is formed from n terms,
each carrying an independent relative rounding error of size eta (the FP32
copy of v, the FP32 kernel value, FP32 partial sums), so the error of row i
is Gaussian with standard deviation eta * sqrt(sum_j (A_ij v_j)^2).  A fresh
error is drawn for every product, as the rounding of each new direction is.
``fit_eta`` measures eta for a given operator from one product it formed.
"""

import numpy as np


def per_term_scale(A, v):
    """sqrt(sum_j (A_ij v_j)^2) for every row i."""
    A = np.asarray(A, dtype=np.float64)
    return np.sqrt((A * A) @ (np.asarray(v, dtype=np.float64) ** 2))


def noisy_product(A, eta, seed):
    """v -> A v + eta * sqrt((A o A)(v o v)) o N(0, I), a new draw per call."""
    A = np.asarray(A, dtype=np.float64)
    A2 = A * A
    g = np.random.default_rng(seed)

    def mv(v):
        return A @ v + eta * np.sqrt(A2 @ (v * v)) * g.standard_normal(v.shape[0])
    return mv


def fit_eta(A, v, y):
    """The eta of the error model that fits the product y ~ A v: the RMS of
    (y - A v)_i / sqrt(sum_j (A_ij v_j)^2) over the rows."""
    s = per_term_scale(A, v)
    e = (np.asarray(y, dtype=np.float64) - np.asarray(A) @ v) / s
    return float(np.sqrt(np.mean(e * e)))
