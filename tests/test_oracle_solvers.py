"""Pins of the oracle's CG, def-CG, harmonic Ritz, sequence, refinement and
GP-gradient functions (CPU only).

What pins them (none of these re-types the oracle's own formulas):
* a Cholesky solve (LAPACK via scipy) for final solutions;
* finite termination of CG in at most (#distinct eigenvalues) steps, and of
  def-CG with exact eigenvectors in at most (#remaining distinct eigenvalues);
* the Galerkin optimality of the def-CG iterate, checked by a dense A-norm
  least-squares solve over the same search space;
* the invariants the method fixes: W^T r_j = 0, W^T A p_j = 0, r_i^T r_j = 0,
  p_i^T A p_j = 0;
* scipy.linalg.eigh(G, F) for the harmonic Ritz pairs, and exact eigenvalues
  when span(Z) holds an invariant subspace;
* central finite differences and a deterministic exact trace for the GP
  gradient.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import cg as C
from oracle import gp as GP
from oracle import kernels as K
from oracle import precision as P
from oracle import refine as R
from oracle import ritz as RZ
from oracle import sequence as S
import workloads


def _kernel_system(n=200, d=3, ell=1.0, sigma2=1e-2, seed=0, kern=K.RBF):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d))
    A = K.operator(X, kern, ell, 1.0, sigma2)
    b = g.standard_normal(n)
    return X, A, b


def test_cg_matches_cholesky():
    _, A, b = _kernel_system()
    res = C.cg(A, b, tol=1e-12)
    x_ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) / np.linalg.norm(b) <= 1.5e-12
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(res.x - x_ref) / np.linalg.norm(x_ref) <= 10 * kappa * 1e-12


def test_cg_finite_termination():
    eigs = np.repeat([1.0, 2.0, 5.0, 11.0, 40.0], 20)   # 5 distinct eigenvalues
    A, _ = workloads.spd_with_spectrum(eigs)
    b = np.random.default_rng(1).standard_normal(100)
    res = C.cg(A, b, tol=1e-10)
    assert res.converged and res.iters <= 5


def test_cg_invariants():
    _, A, b = _kernel_system(n=150)
    res = C.cg(A, b, tol=1e-10, store_all=True)
    Rm, Pm = res.all_r[:, :12], res.all_p[:, :12]
    Rn = Rm / np.linalg.norm(Rm, axis=0)
    G = Rn.T @ Rn
    assert np.abs(G - np.eye(12)).max() < 1e-8        # residuals orthogonal
    H = Pm.T @ A @ Pm
    dH = np.sqrt(np.diag(H))
    Hn = H / dH[:, None] / dH[None, :]
    # directions A-conjugate: exactly for neighbours, up to the slow FP64
    # loss of global conjugacy (grows like kappa * eps) otherwise
    assert np.abs(np.diag(Hn, 1)).max() < 1e-12
    assert np.abs(Hn - np.eye(12)).max() < 1e-6


def test_defcg_empty_W_is_cg_bitwise():
    _, A, b = _kernel_system(n=120, seed=3)
    r1 = C.cg(A, b, tol=1e-9, L=10)
    r2 = C.defcg(A, b, W=np.zeros((120, 0)), tol=1e-9, L=10)
    assert r1.iters == r2.iters
    assert np.array_equal(r1.x, r2.x)
    assert np.array_equal(r1.P, r2.P)


def _deflation_case():
    # k = 6 large outlying eigenvalues + 8 distinct small ones (each x10)
    big = [500.0, 420.0, 300.0, 250.0, 180.0, 120.0]
    small = np.repeat([1.0, 1.3, 1.7, 2.2, 2.8, 3.5, 4.1, 5.0], 10)
    eigs = np.concatenate([small, big])
    A, Q = workloads.spd_with_spectrum(eigs, seed=11)
    W = Q[:, -6:]          # exact eigenvectors of the 6 largest eigenvalues
    b = np.random.default_rng(5).standard_normal(len(eigs))
    return A, W, b


def test_defcg_exact_eigenvectors_finite_termination():
    A, W, b = _deflation_case()
    plain = C.cg(A, b, tol=1e-10)
    defl = C.defcg(A, b, W=W, tol=1e-10)
    assert defl.converged and defl.iters <= 8      # only the 8 small clusters remain
    assert plain.iters > defl.iters
    x_ref = np.linalg.solve(A, b)
    assert np.linalg.norm(defl.x - x_ref) / np.linalg.norm(x_ref) < 1e-9


def test_defcg_invariants_and_galerkin_optimality():
    X, A, b = _kernel_system(n=160, seed=7)
    g = np.random.default_rng(8)
    W = g.standard_normal((160, 5))
    x_init = g.standard_normal(160)
    res = C.defcg(A, b, x_init=x_init, W=W, tol=1e-10, store_all=True)
    R_, P_ = res.all_r, res.all_p
    nW = np.linalg.norm(W, axis=0)
    for j in range(min(15, R_.shape[1])):
        rj = R_[:, j]
        assert np.abs(W.T @ rj).max() <= 1e-9 * np.linalg.norm(rj) * nW.max()
        pj = P_[:, j]
        assert np.abs(W.T @ A @ pj).max() <= 1e-9 * np.linalg.norm(A @ pj) * nW.max()
    Pm = P_[:, :10]
    H = Pm.T @ A @ Pm
    dH = np.sqrt(np.diag(H))
    Hn = H / dH[:, None] / dH[None, :]
    assert np.abs(np.diag(Hn, 1)).max() < 1e-12
    assert np.abs(Hn - np.eye(10)).max() < 1e-6
    # x_j is the A-norm best approximation of x* over x_{-1} + span(W, p_0..p_{j-1})
    res_j = C.defcg(A, b, x_init=x_init, W=W, tol=0.0, max_iter=6)
    Sbasis = np.hstack([W, res.all_p[:, :6]])
    x_star = np.linalg.solve(A, b)
    y = np.linalg.solve(Sbasis.T @ A @ Sbasis, Sbasis.T @ A @ (x_star - x_init))
    x_best = x_init + Sbasis @ y
    assert np.linalg.norm(res_j.x - x_best) <= 1e-8 * np.linalg.norm(x_best)
    # true residual matches the recursive one
    assert np.linalg.norm(b - A @ res.x - res.r_final) <= 1e-9 * np.linalg.norm(b)


def test_harmonic_ritz_matches_scipy_eigh():
    _, A, b = _kernel_system(n=120, seed=9)
    res = C.cg(A, b, tol=1e-12, L=15)
    F, G = RZ.harmonic_ritz_FG(res.P, res.AP)
    theta, U = RZ.harmonic_ritz_pairs(F, G)
    ref = scipy.linalg.eigh(G, F, eigvals_only=True)
    np.testing.assert_allclose(theta, ref, rtol=1e-9)
    np.testing.assert_allclose(U.T @ F @ U, np.eye(U.shape[1]), atol=1e-9)
    # harmonic Ritz values of an SPD matrix lie inside its spectrum
    lam = np.linalg.eigvalsh(A)
    assert theta.min() >= lam.min() * (1 - 1e-9) and theta.max() <= lam.max() * (1 + 1e-9)


def test_harmonic_ritz_full_basis_gives_eigenvalues():
    A, _ = workloads.spd_with_spectrum(np.linspace(1.0, 9.0, 12), seed=3)
    Z = np.random.default_rng(0).standard_normal((12, 12))
    theta, _ = RZ.harmonic_ritz_pairs(*RZ.harmonic_ritz_FG(Z, A @ Z))
    np.testing.assert_allclose(theta, np.linspace(1.0, 9.0, 12), rtol=1e-10)


def test_harmonic_ritz_invariant_subspace_exact():
    A, W, _ = _deflation_case()
    g = np.random.default_rng(2)
    Z = np.hstack([W[:, :3], g.standard_normal((A.shape[0], 4))])
    Wn, AWn, theta, U = RZ.harmonic_ritz(Z, A @ Z, k=3)
    np.testing.assert_allclose(np.sort(theta), [300.0, 420.0, 500.0], rtol=1e-10)
    # W'^T A W' = I (U is F-orthonormal)
    np.testing.assert_allclose(Wn.T @ A @ Wn, np.eye(3), atol=1e-9)
    np.testing.assert_allclose(AWn, A @ Wn, rtol=1e-10, atol=1e-10)


def test_harmonic_ritz_rank_deficient_F():
    _, A, b = _kernel_system(n=80, seed=4)
    res = C.cg(A, b, tol=1e-12, L=6)
    Z = np.hstack([res.P, res.P[:, :2]])           # duplicated columns
    Wn, _, theta, U = RZ.harmonic_ritz(Z, A @ Z, k=4)
    F, G = RZ.harmonic_ritz_FG(res.P, res.AP)
    ref = np.sort(scipy.linalg.eigh(G, F, eigvals_only=True))[::-1][:4]
    np.testing.assert_allclose(theta, ref, rtol=1e-7)
    assert np.all(np.isfinite(Wn))


def test_rayleigh_ritz_full_basis_and_invariant_subspace():
    """With Z spanning the whole space the Ritz values are the spectrum; with
    an invariant subspace inside span(Z) its eigenvalues come out exactly."""
    A, _ = workloads.spd_with_spectrum(np.linspace(1.0, 9.0, 12), seed=3)
    Z = np.random.default_rng(0).standard_normal((12, 12))
    _, _, theta, _ = RZ.rayleigh_ritz(Z, A @ Z, k=12)
    np.testing.assert_allclose(np.sort(theta), np.linspace(1.0, 9.0, 12), rtol=1e-10)
    A, W, _ = _deflation_case()
    g = np.random.default_rng(2)
    Z = np.hstack([W[:, :3], g.standard_normal((A.shape[0], 4))])
    Wn, AWn, theta, _ = RZ.rayleigh_ritz(Z, A @ Z, k=3)
    np.testing.assert_allclose(np.sort(theta), [300.0, 420.0, 500.0], rtol=1e-10)
    np.testing.assert_allclose(Wn.T @ Wn, np.eye(3), atol=1e-10)     # orthonormal Ritz vectors
    np.testing.assert_allclose(AWn, A @ Wn, rtol=1e-10, atol=1e-10)


def test_ritz_galerkin_conditions_and_interlacing():
    """The defining conditions of the two extractions on a generic basis:
    Rayleigh-Ritz Z^T (A w - theta w) = 0, harmonic (AZ)^T (A w - theta w) = 0;
    the Rayleigh-Ritz values interlace the spectrum (Cauchy): the j-th
    largest lies between the j-th largest and the (n - m + j)-th largest
    eigenvalue; both sets lie inside [lambda_min, lambda_max]."""
    _, A, _ = _kernel_system(n=150, seed=12)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    m = 20
    Z = np.random.default_rng(5).standard_normal((150, m))
    AZ = A @ Z
    for kind, test_space in ((RZ.RAYLEIGH, Z), (RZ.HARMONIC, AZ)):
        Wn, AWn, theta, _ = RZ.extract(Z, AZ, k=m, kind=kind)
        R = AWn - Wn * theta[None, :]
        scale = np.linalg.norm(test_space) * np.linalg.norm(AWn)
        assert np.abs(test_space.T @ R).max() <= 1e-10 * scale, kind
        assert theta.min() >= lam[-1] * (1 - 1e-9) and theta.max() <= lam[0] * (1 + 1e-9)
    _, _, th_rr, _ = RZ.rayleigh_ritz(Z, AZ, k=m)
    th_rr = np.sort(th_rr)[::-1]
    n = 150
    for j in range(m):
        assert lam[n - m + j] * (1 - 1e-9) <= th_rr[j] <= lam[j] * (1 + 1e-9), j
    # largest selection is descending, smallest ascending
    assert np.all(np.diff(RZ.rayleigh_ritz(Z, AZ, 5)[2]) <= 0)
    assert np.all(np.diff(RZ.rayleigh_ritz(Z, AZ, 5, largest=False)[2]) >= 0)


def test_rayleigh_ritz_rank_deficient_Z():
    """Repeated columns make Z^T Z singular: the repeats are dropped and the
    values are those of the basis without them."""
    _, A, _ = _kernel_system(n=90, seed=13)
    Z0 = np.random.default_rng(6).standard_normal((90, 8))
    Z = np.hstack([Z0, Z0[:, :3]])
    _, _, th, _ = RZ.rayleigh_ritz(Z, A @ Z, k=5)
    _, _, th0, _ = RZ.rayleigh_ritz(Z0, A @ Z0, k=5)
    np.testing.assert_allclose(th, th0, rtol=1e-9)


def test_sequence_first_system_is_cg_and_deflation_helps():
    w = workloads.small(n=400, d=4, systems=4)
    mats = [K.operator(w["X"], w["kernel"], ell, w["s2"], w["sigma2"]) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i][:400] for i, A in enumerate(mats)]
    rec = S.solve_sequence(mats, bs, k=8, L=12, tol=1e-8)
    plain = S.solve_sequence(mats, bs, k=8, L=12, tol=1e-8, recycle=False)
    assert rec[0].iters == plain[0].iters
    assert np.array_equal(rec[0].x, plain[0].x)
    for r, p, A, b in zip(rec, plain, mats, bs):
        x_ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
        assert np.linalg.norm(b - A @ r.x) / np.linalg.norm(b) <= 1.01e-8
        assert np.linalg.norm(r.x - x_ref) <= 1e-5 * np.linalg.norm(x_ref)
    assert sum(r.iters for r in rec[1:]) < sum(p.iters for p in plain[1:])


def test_sequence_sigma_shift_update_equals_recompute():
    X, _, b = _kernel_system(n=150, seed=12, kern=K.MATERN52)
    s2s = [1e-2, 9e-3, 8.1e-3]
    mats = [K.operator(X, K.MATERN52, 1.0, 1.0, s) for s in s2s]
    upd = S.solve_sequence(mats, [b] * 3, k=6, L=9, tol=1e-9, sigma2s=s2s)
    rec = S.solve_sequence(mats, [b] * 3, k=6, L=9, tol=1e-9)
    # same method up to rounding: iteration counts within 2, same solution
    for a, c, A in zip(upd, rec, mats):
        assert abs(a.iters - c.iters) <= 2
        assert np.linalg.norm(b - A @ a.x) <= 1.01e-9 * np.linalg.norm(b)
        assert np.linalg.norm(a.x - c.x) <= 1e-6 * np.linalg.norm(c.x)


def test_refine_recovers_fp64_solution_from_bf16_operator():
    g = np.random.default_rng(13)
    X = g.uniform(-1, 1, (300, 6))
    ell = 0.5 * workloads.median_distance(X)
    A64 = K.operator(X, K.MATERN52, ell, 1.0, 1e-3)
    Xl = P.round_bf16(X)
    Alow = K.operator(Xl, K.MATERN52, ell, 1.0, 1e-3)
    b = g.standard_normal(300)
    x, hist, inner, _ = R.refine(A64, Alow, b, tol=1e-8, inner_tol=1e-4, k=6, L=9)
    assert hist[-1] <= 1e-8
    x_ref = np.linalg.solve(A64, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-6
    rho = np.abs(np.linalg.eigvals(np.linalg.solve(Alow, A64 - Alow))).max()
    for a, c in zip(hist[1:], hist[:-1]):
        assert a <= 3 * (rho + 1e-4) * np.linalg.cond(A64) ** 0.5 * c


def _pcg_residuals(A, M_inv, b, steps):
    """Textbook preconditioned CG (short recurrence), residual norms."""
    x = np.zeros_like(b)
    r = b.copy()
    z = M_inv @ r
    p = z.copy()
    rz = r @ z
    out = [np.linalg.norm(r) / np.linalg.norm(b)]
    for _ in range(steps):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        out.append(np.linalg.norm(r) / np.linalg.norm(b))
        z = M_inv @ r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return np.array(out)


def test_fcg_exact_preconditioner_one_step():
    X, A, b = _kernel_system(n=150, sigma2=1e-3, seed=21)
    x, hist, D, _ = R.fcg_outer(lambda v: A @ v, lambda r: np.linalg.solve(A, r), b, tol=1e-12)
    assert len(D) == 1 and hist[-1] <= 1e-12
    c = scipy.linalg.cho_factor(A)
    xc = scipy.linalg.cho_solve(c, b)
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 1e-9


def test_fcg_fixed_preconditioner_is_pcg():
    """With a fixed SPD preconditioner flexible CG with full orthogonalisation
    generates the PCG iterates: the same residual norms step by step."""
    X, A, b = _kernel_system(n=120, sigma2=1e-2, seed=22)
    g = np.random.default_rng(23)
    # a fixed SPD approximation of A^{-1}: the inverse of a perturbed A
    E = 0.05 * g.standard_normal(A.shape)
    M_inv = np.linalg.inv(A + 0.1 * (E @ E.T) + 1e-3 * np.eye(120))
    steps = 12
    _, hist, D, AD = R.fcg_outer(lambda v: A @ v, lambda r: M_inv @ r, b, tol=0.0,
                                 max_outer=steps)
    ref = _pcg_residuals(A, M_inv, b, steps)
    np.testing.assert_allclose(np.array(hist), ref, rtol=1e-6)


def test_fcg_directions_A_orthogonal_with_variable_preconditioner():
    X, A, b = _kernel_system(n=200, sigma2=1e-3, seed=24)
    # the preconditioner: CG to 1e-2 on the operator of bf16-rounded points
    Alow = K.operator(P.round_bf16(X), K.RBF, 1.0, 1.0, 1e-3)
    pre = lambda r: C.defcg(Alow, r, tol=1e-2).x
    x, hist, D, AD = R.fcg_outer(lambda v: A @ v, pre, b, tol=1e-10)
    Dm = np.column_stack(D)
    G = Dm.T @ A @ Dm
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 1e-8 * np.abs(np.diag(G)).max()
    # the products carried along are the products of the directions
    np.testing.assert_allclose(np.column_stack(AD), A @ Dm, rtol=0, atol=1e-10 * np.abs(A @ Dm).max())
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-9
    # the A-norm of the error never grows
    xs = np.linalg.solve(A, b)
    errs = []
    for t in range(1, len(D) + 1):
        xt = sum(((Dm[:, j] @ b) / G[j, j]) * Dm[:, j] for j in range(t))
        e = xt - xs
        errs.append(e @ A @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) for i in range(len(errs) - 1))


def test_fcg_zero_rhs():
    A = np.eye(5) * 2.0
    x, hist, D, _ = R.fcg_outer(lambda v: A @ v, lambda r: r / 2.0, np.zeros(5), tol=1e-8)
    assert len(D) == 0 and hist == [0.0] and not np.any(x)


def test_refine_fcg_beats_plain_refinement_on_bf16_operator():
    g = np.random.default_rng(13)
    X = g.uniform(-1, 1, (300, 6))
    ell = 0.5 * workloads.median_distance(X)
    A64 = K.operator(X, K.MATERN52, ell, 1.0, 1e-3)
    # 4-bit mantissas: an operator error large enough that it, not the
    # inner tolerance, limits plain refinement
    mant, ex = np.frexp(X)
    Xl = np.ldexp(np.rint(mant * 16.0) / 16.0, ex)
    Alow = K.operator(Xl, K.MATERN52, ell, 1.0, 1e-3)
    b = g.standard_normal(300)
    x, hist, inner = R.refine_fcg(A64, Alow, b, tol=1e-8, inner_tol=1e-2, k=6, L=9)
    assert hist[-1] <= 1e-8
    assert np.linalg.norm(b - A64 @ x) / np.linalg.norm(b) <= 2e-8
    _, hist_ir, inner_ir, _ = R.refine(A64, Alow, b, tol=1e-8, inner_tol=1e-2, max_outer=60)
    assert hist_ir[-1] <= 1e-8
    assert len(inner) < len(inner_ir)


def test_refine_extraction_modes():
    """When the recycled basis is refreshed inside refinement: every mode
    converges; with a single inner solve all modes extract from the same Z;
    "accum" extracts once from the directions of all inner solves in order
    (up to L), giving an A~-orthonormal basis equal to the harmonic Ritz
    extraction of that concatenated subspace."""
    g = np.random.default_rng(14)
    X = g.uniform(-1, 1, (400, 6))
    ell = 0.5 * workloads.median_distance(X)
    A64 = K.operator(X, K.MATERN52, ell, 1.0, 1e-3)
    Alow = K.operator(P.round_bf16(X), K.MATERN52, ell, 1.0, 1e-3)
    b = g.standard_normal(400)
    outs = {m: R.refine(A64, Alow, b, tol=1e-8, inner_tol=1e-2, k=6, L=30, extract=m)
            for m in ("every", "first", "accum")}
    for m, (x, hist, inner, (W, AW)) in outs.items():
        assert hist[-1] <= 1e-8, m
        assert W.shape == (400, 6)
        np.testing.assert_allclose(W.T @ Alow @ W, np.eye(6), atol=1e-8)
        np.testing.assert_allclose(AW, Alow @ W, atol=1e-8 * np.abs(AW).max())
    # accum: the extraction over the first L directions of the inner solves
    _, _, inner, (W, _) = outs["accum"]
    P_all = np.hstack([r.P for r in inner])[:, :30]
    AP_all = np.hstack([r.AP for r in inner])[:, :30]
    assert sum(min(r.iters, 30) for r in inner) >= 30
    Wr, _, _, _ = RZ.harmonic_ritz(P_all, AP_all, 6)
    # same span (signs and order within equal values aside)
    s = np.linalg.svd(np.linalg.qr(W)[0].T @ np.linalg.qr(Wr)[0], compute_uv=False)
    assert s.min() > 1 - 1e-8
    # one inner solve: identical bases in all modes
    single = [R.refine(A64, Alow, b, tol=1e-8, inner_tol=1e-2, k=6, L=30, max_outer=1, extract=m)[3][0]
              for m in ("every", "first", "accum")]
    np.testing.assert_allclose(single[0], single[1], rtol=0, atol=0)
    np.testing.assert_allclose(single[0], single[2], rtol=0, atol=0)


@pytest.mark.parametrize("kern", [K.RBF, K.MATERN32, K.MATERN52])
def test_gp_blocked_gradient_equals_dense(kern):
    """The matrix-free, row-blocked Hutchinson gradient is the dense one
    (same alpha, U, probes), for blocks that do and do not divide n."""
    g = np.random.default_rng(41)
    X = g.standard_normal((333, 4))
    y = g.standard_normal(333)
    Z = np.where(g.random((333, 5)) < 0.5, -1.0, 1.0)
    A = K.operator(X, kern, 1.3, 0.8, 0.05)
    alpha = np.linalg.solve(A, y)
    U = np.linalg.solve(A, Z)
    dense = GP.lml_grad_hutchinson(X, y, kern, 1.3, 0.8, 0.05, Z, alpha=alpha, U=U)
    for block in (64, 100, 333, 1000):
        blk = GP.lml_grad_hutchinson_blocked(X, kern, 1.3, 0.8, 0.05, alpha, U, Z, block=block)
        np.testing.assert_allclose(blk, dense, rtol=1e-12, atol=1e-12 * np.abs(dense).max())


def test_gp_gradient_matches_finite_differences():
    g = np.random.default_rng(14)
    X = g.standard_normal((120, 3))
    y = np.sin(X[:, 0]) + 0.1 * g.standard_normal(120)
    th = np.array([np.log(1.2), np.log(0.9), np.log(0.05)])

    def f(t):
        return GP.lml(X, y, K.RBF, np.exp(t[0]), np.exp(t[1]), np.exp(t[2]))

    grad = GP.lml_grad_exact(X, y, K.RBF, *np.exp(th))
    h = 1e-5
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (f(th + e) - f(th - e)) / (2 * h)
        assert grad[j] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_gp_hutchinson_exact_with_unit_probes_and_unbiased():
    g = np.random.default_rng(15)
    X = g.standard_normal((90, 3))
    y = g.standard_normal(90)
    par = (K.RBF, 1.1, 1.0, 0.1)
    exact = GP.lml_grad_exact(X, y, *par)
    # probes = sqrt(n) e_i (E[z z^T] = I over the n of them): the trace is exact
    est = GP.lml_grad_hutchinson(X, y, *par, probes=np.sqrt(90.0) * np.eye(90))
    np.testing.assert_allclose(est, exact, rtol=1e-10, atol=1e-10)
    # Rademacher probes: unbiased, error within 4 standard errors
    Z = workloads.rademacher(90, 4000, step=0)
    est = GP.lml_grad_hutchinson(X, y, *par, probes=Z)
    A = K.operator(X, *par)
    Ainv = np.linalg.inv(A)
    for j, D in enumerate(GP.dA_list(X, *par)):
        samples = np.sum((Ainv @ Z) * (D @ Z), axis=0)
        se = 0.5 * samples.std() / np.sqrt(Z.shape[1])
        assert abs(est[j] - exact[j]) <= 4 * se + 1e-12
