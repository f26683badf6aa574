"""GP log marginal likelihood and its hyperparameter gradient (FP64, dense).

Test infrastructure only (see ``oracle/__init__``).

GP model adaptation (section 1 of the paper) needs k_theta^{-1} y for a
sequence of hyperparameters theta.  The objective and its gradient are the
textbook ones (Rasmussen & Williams 2006, eqs. 5.8 and 5.9), with
A = K_theta + sigma^2 I and alpha = A^{-1} y:

    log p(y | X, theta) = -1/2 y^T alpha - 1/2 log|A| - n/2 log(2 pi)
    d/dtheta_j          =  1/2 alpha^T (dA/dtheta_j) alpha
                          - 1/2 tr(A^{-1} dA/dtheta_j)

for theta = (log ell, log s2, log sigma2):
    dA/dlog ell    = dK/dlog ell         (see kernels.dgram_dlog_ell)
    dA/dlog s2     = K
    dA/dlog sigma2 = sigma2 I

The Hutchinson estimator replaces the trace by (1/P) sum_p u_p^T dA z_p with
u_p = A^{-1} z_p for P Rademacher probes z_p.
"""

import numpy as np
import scipy.linalg

from . import kernels as _k


def dA_list(X, kernel, ell, s2, sigma2):
    K = _k.gram(X, kernel, ell, s2)
    return [_k.dgram_dlog_ell(X, kernel, ell, s2), K,
            sigma2 * np.eye(X.shape[0])]


def lml(X, y, kernel, ell, s2, sigma2):
    """Exact log marginal likelihood via a Cholesky factorisation."""
    A = _k.operator(X, kernel, ell, s2, sigma2)
    c = scipy.linalg.cho_factor(A, lower=True)
    alpha = scipy.linalg.cho_solve(c, y)
    logdet = 2.0 * np.sum(np.log(np.diag(c[0])))
    n = y.shape[0]
    return -0.5 * y @ alpha - 0.5 * logdet - 0.5 * n * np.log(2 * np.pi)


def lml_grad_exact(X, y, kernel, ell, s2, sigma2):
    """Exact gradient w.r.t. (log ell, log s2, log sigma2), dense trace."""
    A = _k.operator(X, kernel, ell, s2, sigma2)
    c = scipy.linalg.cho_factor(A, lower=True)
    alpha = scipy.linalg.cho_solve(c, y)
    Ainv = scipy.linalg.cho_solve(c, np.eye(A.shape[0]))
    g = []
    for D in dA_list(X, kernel, ell, s2, sigma2):
        g.append(0.5 * alpha @ D @ alpha - 0.5 * np.sum(Ainv * D.T))
    return np.array(g)


def lml_grad_hutchinson(X, y, kernel, ell, s2, sigma2, probes, alpha=None,
                        U=None):
    """Gradient with the trace term estimated from the given probe matrix.

    probes : n x P matrix of probe vectors z_p
    alpha  : A^{-1} y (solved exactly if None)
    U      : A^{-1} probes (solved exactly if None)
    """
    A = _k.operator(X, kernel, ell, s2, sigma2)
    if alpha is None or U is None:
        c = scipy.linalg.cho_factor(A, lower=True)
        if alpha is None:
            alpha = scipy.linalg.cho_solve(c, y)
        if U is None:
            U = scipy.linalg.cho_solve(c, probes)
    P = probes.shape[1]
    g = []
    for D in dA_list(X, kernel, ell, s2, sigma2):
        tr = np.sum(U * (D @ probes)) / P
        g.append(0.5 * alpha @ D @ alpha - 0.5 * tr)
    return np.array(g)


def lml_grad_hutchinson_blocked(X, kernel, ell, s2, sigma2, alpha, U, probes, block=2048,
                                with_scale=False):
    """lml_grad_hutchinson for given alpha and U without forming n x n
    matrices: the products dA alpha and dA probes are taken block of rows by
    block of rows (same formulas, O(n * block) memory; distances in the
    matrix-product form, kernels.sqdist_gemm)."""
    n = X.shape[0]
    P = probes.shape[1]
    V = np.column_stack([alpha, probes])          # the vectors dA is applied to
    Va = np.abs(V)
    dK_V, K_V = np.zeros_like(V), np.zeros_like(V)
    dK_Va, K_Va = np.zeros_like(V), np.zeros_like(V)
    for i0 in range(0, n, block):
        rows = slice(i0, min(n, i0 + block))
        r2 = _k.sqdist_gemm(X[rows], X)
        D = _k.dkernel_dlog_ell_from_r2(r2, kernel, ell, s2)
        Kb = _k.kernel_from_r2(r2, kernel, ell, s2)
        dK_V[rows] = D @ V
        K_V[rows] = Kb @ V
        if with_scale:   # both matrices are elementwise non-negative
            dK_Va[rows] = D @ Va
            K_Va[rows] = Kb @ Va
    g, scale = [], []
    for DV, DVa in ((dK_V, dK_Va), (K_V, K_Va), (sigma2 * V, sigma2 * Va)):
        tr = np.sum(U * DV[:, 1:]) / P
        g.append(0.5 * alpha @ DV[:, 0] - 0.5 * tr)
        # sum_ij |dA_ij| (|alpha_i alpha_j| + (1/P) sum_p |U_ip Z_jp|) / 2
        scale.append(0.5 * (np.abs(alpha) @ DVa[:, 0] + np.sum(np.abs(U) * DVa[:, 1:]) / P))
    if with_scale:
        return np.array(g), np.array(scale)
    return np.array(g)
