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


HARMONIC, RAYLEIGH = 0, 1


def extract(Z, AZ, k, largest=True, kind=HARMONIC, drop_tol=1e-12):
    """The extraction of the next basis by kind (harmonic or Rayleigh-Ritz)."""
    if kind == HARMONIC:
        return harmonic_ritz(Z, AZ, k, largest, drop_tol)
    if kind == RAYLEIGH:
        return rayleigh_ritz(Z, AZ, k, largest, drop_tol)
    raise ValueError(f"unknown extraction {kind}")
