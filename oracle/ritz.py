"""Harmonic projection: harmonic Ritz extraction of the recycled basis.

Test infrastructure only (see ``oracle/__init__``).

Section 2.3 of the paper (Eq. 7, after Morgan 1995): with Z = [W, P_L] and
AZ its product with A, form F = (AZ)^T Z and G = (AZ)^T (AZ), solve the
generalized eigenproblem G u = theta F u, keep k of the k + L pairs in U and
set the next basis W' = Z U.  The paper's experiments keep the pairs of the
largest theta (Fig. 1 caption); selecting the smallest is an option.

F is symmetric in exact arithmetic (A is); it is symmetrised, as is G.  When
F is SPD the pairs are those of ``scipy.linalg.eigh(G, F)``.  When loss of
A-conjugacy makes F numerically singular the problem is solved in the range
of F (a reading where the paper is silent on this case):

    S = diag(F)^(-1/2),  S F S = Q Lam Q^T,  keep lam > drop_tol * max(lam),
    B = S Q_keep Lam_keep^(-1/2)      (B^T F B = I)
    C = B^T G B = Y Theta Y^T,        U = B Y   (U^T F U = I)

which reduces to the plain definition when nothing is dropped.  U is
F-orthonormal, so W'^T A W' = U^T F U = I for the operator that produced Z.
Ties in theta are broken by a stable sort on the original column index.

The standard Rayleigh-Ritz extraction, which section 2.3 sets the harmonic
one against, is offered too: the pairs of (Z^T A Z) y = theta (Z^T Z) y, the
Galerkin condition Z^T (A w - theta w) = 0 instead of the harmonic
(AZ)^T (A w - theta w) = 0.  It is solved by the same reduction with Z^T Z in
the role of F, so W' = Z U has orthonormal columns (U^T Z^T Z U = I).

The implicit extraction forms F and G without products of tall matrices,
from the quantities Algorithm 1 stores in its first L steps (d_j, alpha_j,
beta_j, mu_j, p_j) plus rho_j = r_j^T r_j, as section 2.3 says Saad et al.
(2000) did.  The identities it rests on, all exact in exact arithmetic for
the iterates of Algorithm 1 (with W empty: plain CG):
* A-conjugacy: (AW)^T p_j = 0 and p_i^T A p_j = 0 (i != j), so
  F = blockdiag(W^T A W, diag(d_j));
* the residual update r_{j+1} = r_j - alpha_j A p_j - (AW) c_{j+1} (c = 0 in
  Algorithm 1; the re-projection's coefficients otherwise), so
  A p_j = (r_j - r_{j+1} - (AW) c_{j+1}) / alpha_j;
* the definition of mu_j: (AW)^T r_j = (W^T A W) mu_j;
* mutually orthogonal residuals: r_i^T r_j = 0 for i != j.
Then (AW)^T A p_j = (M (mu_j - mu_{j+1}) - N c_{j+1}) / alpha_j with
M = W^T A W, N = (AW)^T AW, and (A p_i)^T (A p_j) expands into the residual
Gram matrix (diagonal rho_j + rho_{j+1}, first off-diagonals -rho_{j+1}),
the cross terms (M (mu_i - mu_{i+1}))^T c_{j+1} and c_{i+1}^T N c_{j+1}.
The products A p_j themselves follow from the directions: the direction
update p_j = beta_{j-1} p_{j-1} + r_j - W mu_j gives r_j from P and W, so
A P_L = [P_L, p_L] T + W (mu_j - mu_{j+1}) / alpha_j - (AW) c_{j+1} / alpha_j
with a tridiagonal-band T, and AW' = [AW, A P_L] U needs no stored A P_L.
In finite precision every identity holds only to the loss of orthogonality
and conjugacy of the iteration, so the implicit pencil is an approximation
of the explicit one, close in the first steps.
"""

import numpy as np


def harmonic_ritz_FG(Z, AZ):
    """F = (AZ)^T Z and G = (AZ)^T AZ, both symmetrised."""
    F = AZ.T @ Z
    G = AZ.T @ AZ
    return 0.5 * (F + F.T), 0.5 * (G + G.T)


def harmonic_ritz_pairs(F, G, drop_tol=1e-12):
    """All pairs (theta ascending, U with U^T F U = I) of G u = theta F u."""
    s = 1.0 / np.sqrt(np.diag(F))
    Fs = F * s[:, None] * s[None, :]
    lam, Q = np.linalg.eigh(Fs)
    keep = lam > drop_tol * lam.max()
    B = (s[:, None] * Q[:, keep]) / np.sqrt(lam[keep])[None, :]
    C = B.T @ G @ B
    C = 0.5 * (C + C.T)
    theta, Y = np.linalg.eigh(C)
    return theta, B @ Y


def select(theta, k, largest=True):
    """Indices of the k selected pairs (largest or smallest theta, stable)."""
    order = np.argsort(-theta if largest else theta, kind="stable")
    return order[:k]


def harmonic_ritz(Z, AZ, k, largest=True, drop_tol=1e-12):
    """Extract the next recycled basis.

    Returns (W_new, AW_new, theta_sel, U) with W_new = Z U, AW_new = (AZ) U
    (the product with the operator that produced AZ), theta_sel the selected
    harmonic Ritz values in selection order.
    """
    F, G = harmonic_ritz_FG(Z, AZ)
    theta, U = harmonic_ritz_pairs(F, G, drop_tol)
    idx = select(theta, min(k, theta.shape[0]), largest)
    U = U[:, idx]
    return Z @ U, AZ @ U, theta[idx], U


def rayleigh_ritz_FE(Z, AZ):
    """F = Z^T A Z (formed as (AZ)^T Z) and E = Z^T Z, both symmetrised."""
    F = AZ.T @ Z
    E = Z.T @ Z
    return 0.5 * (F + F.T), 0.5 * (E + E.T)


def rayleigh_ritz(Z, AZ, k, largest=True, drop_tol=1e-12):
    """Rayleigh-Ritz extraction of the next basis: the pairs of
    F y = theta E y solved in the range of E (same reduction as the harmonic
    problem, E in the role of F); returns (W_new, AW_new, theta_sel, U) as
    ``harmonic_ritz`` does, with U^T E U = I (orthonormal W_new)."""
    F, E = rayleigh_ritz_FE(Z, AZ)
    theta, U = harmonic_ritz_pairs(E, F, drop_tol)
    idx = select(theta, min(k, theta.shape[0]), largest)
    U = U[:, idx]
    return Z @ U, AZ @ U, theta[idx], U


HARMONIC, RAYLEIGH, IMPLICIT = 0, 1, 2


def extract(Z, AZ, k, largest=True, kind=HARMONIC, drop_tol=1e-12):
    """The extraction of the next basis by kind (harmonic or Rayleigh-Ritz)."""
    if kind == HARMONIC:
        return harmonic_ritz(Z, AZ, k, largest, drop_tol)
    if kind == RAYLEIGH:
        return rayleigh_ritz(Z, AZ, k, largest, drop_tol)
    raise ValueError(f"unknown extraction {kind}")


def implicit_pencil(M, N, d, alpha, rho, mu=None, c=None):
    """F and G of Eq. 7 for Z = [W, P_L] from the quantities of the first L
    steps (see the module notes).

    M, N   W^T A W and (AW)^T AW (k x k; ignored with k = 0)
    d      d_j = p_j^T A p_j, j = 0 .. L-1
    alpha  alpha_j, j = 0 .. L-1
    rho    rho_j = r_j^T r_j, j = 0 .. L
    mu     mu_j, j = 0 .. L (k-vectors), or None with k = 0
    c      re-projection coefficients c_{j+1}, j = 0 .. L-1, or None (zero)
    """
    L = len(d)
    k = 0 if mu is None or len(mu) == 0 else len(mu[0])
    m = k + L
    F = np.zeros((m, m))
    G = np.zeros((m, m))
    d = np.asarray(d, dtype=np.float64)
    al = np.asarray(alpha, dtype=np.float64)
    rh = np.asarray(rho, dtype=np.float64)
    F[k:, k:] = np.diag(d)
    # residual Gram terms of (A p_i)^T (A p_j) alpha_i alpha_j
    S = np.zeros((L, L))
    for j in range(L):
        S[j, j] = rh[j] + rh[j + 1]
        if j + 1 < L:
            S[j, j + 1] = S[j + 1, j] = -rh[j + 1]
    if k > 0:
        M = 0.5 * (M + M.T)
        N = 0.5 * (N + N.T)
        F[:k, :k] = M
        G[:k, :k] = N
        Mu = np.column_stack(mu)                     # k x (L + 1)
        Cc = np.zeros((k, L)) if c is None or len(c) == 0 else np.column_stack(c)
        Dm = M @ (Mu[:, :L] - Mu[:, 1:L + 1])        # (AW)^T (r_j - r_{j+1})
        G[:k, k:] = (Dm - N @ Cc) / al[None, :]
        G[k:, :k] = G[:k, k:].T
        # (r_i - r_{i+1})^T (AW) c_{j+1} and c_{i+1}^T N c_{j+1}
        X = Dm.T @ Cc
        S = S - X - X.T + Cc.T @ N @ Cc
    G[k:, k:] = S / (al[:, None] * al[None, :])
    return F, G


def implied_AP(P, p_next, W, AW, alpha, beta, mu=None, c=None):
    """A P_L from the recurrences (see the module notes): with
    r_j = p_j - beta_{j-1} p_{j-1} + W mu_j (r_0 = p_0 + W mu_0),
    A p_j = (r_j - r_{j+1} - (AW) c_{j+1}) / alpha_j."""
    n, L = P.shape
    Pe = np.hstack([P, p_next[:, None]])
    R = Pe.copy()
    R[:, 1:] -= Pe[:, :-1] * np.asarray(beta, dtype=np.float64)[None, :L]
    if W is not None and W.shape[1] > 0:
        R += W @ np.column_stack(mu)
    AP = (R[:, :L] - R[:, 1:]) / np.asarray(alpha, dtype=np.float64)[None, :]
    if c is not None and len(c) > 0:
        AP -= (AW @ np.column_stack(c)) / np.asarray(alpha, dtype=np.float64)[None, :]
    return AP


def implicit_extract(res, W, AW, k, largest=True, drop_tol=1e-12, cleanup=True):
    """The next basis by the implicit extraction, from a DefCGResult ``res``
    of the solve with basis W (n x k0, or None) and AW: F, G by
    ``implicit_pencil``, the pairs as for the harmonic extraction, W' = Z U
    and AW' = [AW, implied A P_L] U.  With ``cleanup`` the harmonic problem
    is solved once more on span(W') with its explicit metric (AW')^T W' and
    (AW')^T AW', which drops directions that came out numerically dependent
    (the implicit F assumes conjugate directions, and finite precision
    loses conjugacy; see test_oracle_implicit.py); in exact arithmetic the
    second problem returns W' itself.  Returns (W', AW', theta_sel, U)."""
    L = len(res.d)
    has_w = W is not None and W.shape[1] > 0
    if has_w:
        M, N = W.T @ AW, AW.T @ AW
        mu, Z, AWs = res.mu[:L + 1], np.hstack([W, res.P]), AW
    else:
        M = N = None
        mu, Z, AWs = None, res.P, None
    cv = res.cvec[:L] if has_w else None
    F, G = implicit_pencil(M, N, res.d, res.alpha, res.rho[:L + 1], mu, cv)
    AP = implied_AP(res.P, res.p_next, W if has_w else None, AWs, res.alpha, res.beta, mu, cv)
    AZ = np.hstack([AW, AP]) if has_w else AP
    theta, U = harmonic_ritz_pairs(F, G, drop_tol)
    idx = select(theta, min(k, theta.shape[0]), largest)
    U = U[:, idx]
    W1, AW1, th1 = Z @ U, AZ @ U, theta[idx]
    if not cleanup:
        return W1, AW1, th1, U
    F2, G2 = harmonic_ritz_FG(W1, AW1)
    theta2, U2 = harmonic_ritz_pairs(F2, G2, drop_tol)
    idx2 = select(theta2, theta2.shape[0], largest)
    U2 = U2[:, idx2]
    return W1 @ U2, AW1 @ U2, theta2[idx2], U @ U2
