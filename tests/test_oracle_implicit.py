"""Pins of the implicit extraction (F and G of Eq. 7 from the quantities
Algorithm 1 stores, section 2.3): against the explicit definition
F = (AZ)^T Z, G = (AZ)^T AZ with the products A P_L the iteration formed,
and A P_L from the recurrences against those products.  The two are equal in
exact arithmetic; in FP64 on well-conditioned systems over the first L steps
they agree to rounding amplified by the loss of orthogonality, which the
bounds below allow.  A wrong sign, index or factor anywhere in the formulas
moves some entry by O(1) of its scale."""

import numpy as np
import pytest

from oracle import cg as OC
from oracle import kernels as OK
from oracle import ritz as ORZ
from oracle import sequence as OS


def _system(n, sigma2, seed=0, d=4, ell=0.5):
    """RBF systems with kappa of a few hundred: over the first 12 steps CG's
    residuals and directions stay orthogonal / conjugate to ~1e-13."""
    X = np.random.default_rng(seed).standard_normal((n, d))
    A = OK.operator(X, 0, ell, 1.0, sigma2)
    b = np.random.default_rng(seed + 1).standard_normal(n)
    return A, b


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("L", [1, 6, 12])
def test_plain_cg_pencil_and_products(L):
    """W empty: F = diag(d_j) and G is the tridiagonal residual form; both
    and the implied A P_L match the products of the run."""
    A, b = _system(300, 1e-1)
    res = OC.cg(A, b, tol=1e-12, L=L)
    F, G = ORZ.implicit_pencil(None, None, res.d, res.alpha, res.rho[:L + 1])
    Fd, Gd = ORZ.harmonic_ritz_FG(res.P, res.AP)
    assert _rel(F, Fd) < 1e-10 and _rel(G, Gd) < 1e-10
    assert np.count_nonzero(np.triu(G, 2)) == 0        # tridiagonal
    AP = ORZ.implied_AP(res.P, res.p_next, None, None, res.alpha, res.beta)
    assert _rel(AP, res.AP) < 1e-11


@pytest.mark.parametrize("reproject", [False, True])
def test_deflated_pencil_and_products(reproject):
    """W from a first solve's harmonic extraction (k = 8), the second system
    solved by def-CG(8, 12) (literal Algorithm 1, and with the library's
    re-projection whose coefficients enter the formulas): the implicit F, G
    and A P_L match the explicit ones of Z = [W, P_L], AZ = [AW, A P_L]."""
    A, b = _system(400, 5e-2, seed=3)
    first = OC.cg(A, b, tol=1e-10, L=12)
    W, AW, _, _ = ORZ.harmonic_ritz(first.P, first.AP, 8)
    A2 = A + 0.02 * np.eye(400)
    AW2 = AW + 0.02 * W
    b2 = np.random.default_rng(9).standard_normal(400)
    res = OC.defcg(A2, b2, W=W, AW=AW2, tol=1e-10, L=12, reproject=reproject)
    assert len(res.d) == 12 and len(res.mu) == 13 and len(res.rho) == 13
    M, N = W.T @ AW2, AW2.T @ AW2
    cv = res.cvec if reproject else None
    F, G = ORZ.implicit_pencil(M, N, res.d, res.alpha, res.rho, res.mu, cv)
    Fd, Gd = ORZ.harmonic_ritz_FG(np.hstack([W, res.P]), np.hstack([AW2, res.AP]))
    assert _rel(F, Fd) < 1e-9, _rel(F, Fd)
    assert _rel(G, Gd) < 1e-9, _rel(G, Gd)
    AP = ORZ.implied_AP(res.P, res.p_next, W, AW2, res.alpha, res.beta, res.mu, cv)
    assert _rel(AP, res.AP) < 1e-9
    # the extraction: the same pairs as the explicit harmonic one
    W1, AW1, th1, _ = ORZ.implicit_extract(res, W, AW2, 8)
    W2, AW2x, th2, _ = ORZ.harmonic_ritz(np.hstack([W, res.P]), np.hstack([AW2, res.AP]), 8)
    np.testing.assert_allclose(th1, th2, rtol=1e-8)
    for c in range(W1.shape[1]):      # columns equal up to sign
        e = min(np.linalg.norm(W1[:, c] - W2[:, c]), np.linalg.norm(W1[:, c] + W2[:, c]))
        assert e <= 1e-6 * np.linalg.norm(W2[:, c]), (c, e)
    assert _rel(AW1, A2 @ W1) < 1e-8


def test_reprojection_terms_matter():
    """With re-projection coefficients forced to a visible size (the product
    perturbed, so W^T r drifts), dropping them from the implicit G leaves an
    error the formula with them does not: the c-terms are the ones the
    recurrence actually has."""
    from emulation import noisy_product
    A, b = _system(300, 1e-2, seed=5)
    first = OC.cg(A, b, tol=1e-10, L=12)
    W, AW, _, _ = ORZ.harmonic_ritz(first.P, first.AP, 6)
    res = OC.defcg(noisy_product(A, 1e-6, 0), b, W=W, AW=AW, tol=1e-10, L=10, reproject=True)
    M, N = W.T @ AW, AW.T @ AW
    Fd, Gd = ORZ.harmonic_ritz_FG(np.hstack([W, res.P]), np.hstack([AW, res.AP]))
    _, G_with = ORZ.implicit_pencil(M, N, res.d, res.alpha, res.rho, res.mu, res.cvec)
    _, G_without = ORZ.implicit_pencil(M, N, res.d, res.alpha, res.rho, res.mu, None)
    e_with = np.max(np.abs(G_with[:6, 6:] - Gd[:6, 6:]))
    e_without = np.max(np.abs(G_without[:6, 6:] - Gd[:6, 6:]))
    assert e_with < 1e-3 * e_without, (e_with, e_without)


def test_implicit_sequence_counts():
    """The n = 1024 RBF sequence (five systems, def-CG(8, 12), tol 1e-8)
    with the implicit extraction: the same step counts as the explicit
    harmonic extraction to within one step, and the same Ritz values to
    1e-6."""
    import workloads
    w = workloads.small(n=1024)
    X = w["X"]
    kw = dict(k=w["k"], L=w["L"], tol=w["tol"])
    a = OS.Sequence(**kw)
    b_ = OS.Sequence(extraction=ORZ.IMPLICIT, **kw)
    for i, ell in enumerate(w["ells"]):
        A = OK.operator(X, w["kernel"], ell, 1.0, w["sigma2"])
        bb = A @ w["xstar"] + w["noise"][i]
        ra, rb = a.step(A, bb), b_.step(A, bb)
        assert abs(ra.iters - rb.iters) <= 1, (i, ra.iters, rb.iters)
        np.testing.assert_allclose(rb.theta, ra.theta, rtol=1e-6)


def test_implicit_pencil_ghosts_and_cleanup():
    """Where the implicit pencil breaks: the precision form's first system at
    n = 3000 (bf16-rounded points, Matern-5/2, sigma2 = 1e-3, kappa ~ 1e5),
    plain CG to 2e-2 storing 24 directions, k = 16, exact FP64 products.
    The largest eigenvalue converges within these steps, the stored
    directions lose conjugacy, and two of them become nearly parallel: the
    explicit F = P^T A P (formed from the vectors) has a null direction,
    which its drop rule removes, while the implicit F = diag(d_j) cannot show
    it.  The implicit pencil then reports the top harmonic Ritz value twice
    (a ghost pair) and W' has a null direction in the A-metric.  The second
    harmonic problem on span(W') (``cleanup``) removes the ghost: what is
    left is A-orthonormal and carries the explicit extraction's leading
    values."""
    import workloads
    from oracle import precision as OP
    w = workloads.bf16_shift(n=3000, systems=1)
    X, b, kern, ell = w["X"], w["b"], w["kernel"], w["ell"]
    Xr = OP.round_points(X, 1, kern, ell)
    A = OK.operator(Xr, kern, ell, 1.0, w["sigma2s"][0])
    res = OC.cg(A, b, tol=2e-2, L=24)
    Fx, _ = ORZ.harmonic_ritz_FG(res.P, res.AP)
    s = 1.0 / np.sqrt(np.diag(Fx))
    assert np.linalg.eigvalsh(Fx * s[:, None] * s[None, :])[0] < 1e-12
    W0, _, th0, _ = ORZ.implicit_extract(res, None, None, 16, cleanup=False)
    assert abs(th0[1] - th0[0]) <= 1e-10 * th0[0]            # the ghost
    M0 = W0.T @ A @ W0
    assert np.linalg.eigvalsh(0.5 * (M0 + M0.T))[0] < 1e-10   # W' rank deficient
    W1, AW1, th1, _ = ORZ.implicit_extract(res, None, None, 16)
    W2, _, th2, _ = ORZ.harmonic_ritz(res.P, res.AP, 16)
    k1 = W1.shape[1]
    assert 8 <= k1 < 16
    np.testing.assert_allclose(W1.T @ A @ W1, np.eye(k1), atol=1e-8)
    np.testing.assert_allclose(th1, th2[:k1], rtol=1e-8)
    assert _rel(AW1, A @ W1) < 1e-9
