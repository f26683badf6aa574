"""log det A by stochastic Lanczos quadrature from the coefficients of CG.

Test infrastructure only (see ``oracle/__init__``).

Not in the paper: it is the forward value of the GP log marginal likelihood
(GP model adaptation, section 1), whose probe solves the differentiation
form already runs.  Textbook sources: the CG/Lanczos correspondence (Saad,
Iterative Methods for Sparse Linear Systems, section 6.7.3), Gauss
quadrature through the Lanczos tridiagonal (Golub & Meurant), and
Hutchinson's trace estimator (Ubaru, Chen & Saad 2017 for the combination).

For SPD A and a probe z, m steps of plain CG on A x = z from x = 0 give
coefficients alpha_j, beta_j; the Lanczos tridiagonal of (A, z / |z|) is
    T_00 = 1 / alpha_0,   T_jj = 1 / alpha_j + beta_{j-1} / alpha_{j-1},
    T_{j,j+1} = T_{j+1,j} = sqrt(beta_j) / alpha_j,
and z^T log(A) z ~ |z|^2 e_1^T log(T) e_1 = |z|^2 sum_i tau_i^2 log theta_i
(eigenpairs of T).  For probes with E[z z^T] = I the mean over probes
estimates tr log A = log det A.
"""

import numpy as np


def cg_coefficients(A, z, tol=1e-10, max_iter=None):
    """Plain CG on A x = z from x = 0, stopping when |r| <= tol |z|; returns
    the lists alpha_j, beta_j of the steps taken."""
    A = np.asarray(A, dtype=np.float64)
    r = np.array(z, dtype=np.float64)
    p = r.copy()
    rho = r @ r
    bnorm = np.sqrt(rho)
    max_iter = max_iter or 10 * len(r)
    alphas, betas = [], []
    while np.sqrt(rho) > tol * bnorm and len(alphas) < max_iter:
        q = A @ p
        alpha = rho / (p @ q)
        r = r - alpha * q
        rho_new = r @ r
        beta = rho_new / rho
        alphas.append(alpha)
        betas.append(beta)
        p = r + beta * p
        rho = rho_new
    return np.array(alphas), np.array(betas)


def lanczos_from_cg(alphas, betas):
    """The tridiagonal T (dense m x m) from m CG steps."""
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def quadrature(T, znorm2):
    """|z|^2 e_1^T log(T) e_1 through the eigen-decomposition of T."""
    if T.shape[0] == 0:
        return 0.0
    theta, V = np.linalg.eigh(T)
    return float(znorm2 * np.sum(V[0] ** 2 * np.log(theta)))


def probe_value(A, z, tol=1e-10, max_iter=None):
    """The quadrature estimate of z^T log(A) z and the CG steps it used."""
    al, be = cg_coefficients(A, z, tol=tol, max_iter=max_iter)
    z = np.asarray(z, dtype=np.float64)
    return quadrature(lanczos_from_cg(al, be), z @ z), len(al)


def logdet(A, Z, tol=1e-10, max_iter=None):
    """Mean over the probe columns of Z of z^T log(A) z (per-probe values too)."""
    vals = [probe_value(A, Z[:, p], tol, max_iter)[0] for p in range(Z.shape[1])]
    return float(np.mean(vals)), vals
