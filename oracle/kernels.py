"""Covariance functions and the dense SPD operator A = K_theta(X, X) + sigma^2 I.

Test infrastructure only (see ``oracle/__init__``).

The paper's sequence of systems (section 1, Eq. 1) comes from GP model
adaptation, where the matrix is the kernel Gram matrix k_{theta,XX} over the
data set X = [x_1, ..., x_n]^T.  Its experiments use the Gaussian/RBF kernel
theta^2 exp(-|x_i - x_j|^2 / (2 lambda^2)) (section 3); here theta^2 is the
signal variance ``s2`` and lambda the lengthscale ``ell``.  The Matern-3/2 and
Matern-5/2 kernels are not in the paper; they are the textbook forms
(Rasmussen & Williams 2006, eq. 4.17) in terms of r = |x_i - x_j|:

    Matern-3/2: s2 (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)
    Matern-5/2: s2 (1 + sqrt(5) r / ell + 5 r^2 / (3 ell^2)) exp(-sqrt(5) r / ell)

Distances are formed in difference form, sum_t (x_it - x_jt)^2, so that there
is no cancellation and r_ii = 0 exactly.
"""

import numpy as np

RBF, MATERN32, MATERN52 = 0, 1, 2
KERNEL_NAMES = {RBF: "rbf", MATERN32: "matern32", MATERN52: "matern52"}


def sqdist(X, Y=None):
    """Pairwise squared Euclidean distances in difference form (FP64).

    Row block by row block, so memory stays O(block * n * d).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = X if Y is None else np.asarray(Y, dtype=np.float64)
    out = np.empty((X.shape[0], Y.shape[0]), dtype=np.float64)
    blk = max(1, 2 ** 22 // max(1, Y.shape[0] * X.shape[1]))
    for s in range(0, X.shape[0], blk):
        diff = X[s:s + blk, None, :] - Y[None, :, :]
        out[s:s + blk] = np.einsum("ijt,ijt->ij", diff, diff)
    return out


def kernel_from_r2(r2, kernel, ell, s2):
    """Covariance value as a function of the squared distance r2 (FP64)."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == RBF:
        return s2 * np.exp(-r2 / (2.0 * ell * ell))
    r = np.sqrt(r2)
    if kernel == MATERN32:
        t = np.sqrt(3.0) * r / ell
        return s2 * (1.0 + t) * np.exp(-t)
    if kernel == MATERN52:
        t = np.sqrt(5.0) * r / ell
        return s2 * (1.0 + t + t * t / 3.0) * np.exp(-t)
    raise ValueError(f"unknown kernel id {kernel}")


def gram(X, kernel, ell, s2, Y=None):
    """Kernel Gram matrix K_theta(X, Y) in FP64 (Y defaults to X)."""
    return kernel_from_r2(sqdist(X, Y), kernel, ell, s2)


def operator(X, kernel, ell, s2, sigma2):
    """Dense A = K_theta(X, X) + sigma2 I (FP64), the SPD matrix of Eq. 1."""
    A = gram(X, kernel, ell, s2)
    A[np.diag_indices_from(A)] += sigma2
    return A


def matvec_blocked(X, kernel, ell, s2, sigma2, V, block=1024):
    """A V without forming A: row blocks of K times V, plus sigma2 V.

    Used when n is too large for a dense n x n matrix.  V is n or n x m.
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    out = np.empty_like(V)
    for s in range(0, X.shape[0], block):
        out[s:s + block] = gram(X[s:s + block], kernel, ell, s2, X) @ V
    return out + sigma2 * V


def dgram_dlog_ell(X, kernel, ell, s2, Y=None):
    """Derivative of K(X, Y) with respect to log(ell), dense FP64 (Y
    defaults to X).

    For the RBF kernel dK/dlog(ell) = K * r^2 / ell^2 (chain rule on
    exp(-r^2 / (2 ell^2))).  For the Matern kernels, with t = c r / ell
    (c = sqrt 3 or sqrt 5), dt/dlog(ell) = -t, so
      Matern-3/2: dk/dlog(ell) = s2 t^2 exp(-t)
      Matern-5/2: dk/dlog(ell) = s2 (t^2 + t^3) / 3 exp(-t)
    """
    return dkernel_dlog_ell_from_r2(sqdist(X, Y), kernel, ell, s2)


def dkernel_dlog_ell_from_r2(r2, kernel, ell, s2):
    """dk/dlog(ell) as a function of the squared distance (formulas above)."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == RBF:
        return s2 * np.exp(-r2 / (2 * ell * ell)) * r2 / (ell * ell)
    r = np.sqrt(r2)
    if kernel == MATERN32:
        t = np.sqrt(3.0) * r / ell
        return s2 * t * t * np.exp(-t)
    if kernel == MATERN52:
        t = np.sqrt(5.0) * r / ell
        return s2 * (t * t + t ** 3) / 3.0 * np.exp(-t)
    raise ValueError(f"unknown kernel id {kernel}")


def sqdist_gemm(X, Y):
    """|x_i - y_j|^2 as |x_i|^2 + |y_j|^2 - 2 x_i . y_j in FP64 (clipped at
    0): one matrix product, for blocks too large for the difference form.
    The cancellation costs ~1e-16 (|x|^2 + |y|^2), far below what the
    comparisons that use it resolve."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    r2 = np.sum(X * X, axis=1)[:, None] + np.sum(Y * Y, axis=1)[None, :] - 2.0 * (X @ Y.T)
    return np.maximum(r2, 0.0)
