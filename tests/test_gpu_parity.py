"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances:
* low-precision products: |y_gpu - y_ref|_i <= 2e-5 * (|A| |v|)_i, with y_ref
  the oracle's FP64 product on the *same rounded points* (the operator is the
  exact kernel matrix of the rounded points; the only error left is FP32
  evaluation and accumulation);
* the FP64 product: 1e-12 relative to (|A| |v|)_i;
* solves: the oracle's true residual of the GPU solution is at most
  tol + 2 * floor, floor = |(A_gpu - A_ref) x| / |b| measured per case.
"""

import numpy as np
import pytest

from oracle import cg as OC
from oracle import kernels as OK
from oracle import precision as OP
from oracle import ritz as ORZ
from oracle import sequence as OS
import workloads

from emulation import fit_eta, noisy_product

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _points(n, d, seed, dist="normal"):
    g = np.random.default_rng(seed)
    if dist == "uniform":
        return g.uniform(-1, 1, (n, d))
    return g.standard_normal((n, d))


@pytest.mark.parametrize("prec", [0, 1, 2, 4])
@pytest.mark.parametrize("kern", [0, 1, 2])
@pytest.mark.parametrize("n,d,m", [(1, 3, 1), (200, 3, 1), (777, 8, 2), (1500, 16, 5),
                                   (2500, 32, 1), (600, 33, 3), (300, 1, 1)])
def test_matvec_parity(lib, prec, kern, n, d, m):
    X = _points(n, d, seed=n + d)
    ell = max(0.5, workloads.median_distance(X)) if n > 1 else 1.0
    s2, sigma2 = 1.3, 1e-2
    op = lib.Operator(_dev(X), kern, ell, s2, sigma2, prec=prec)
    g = np.random.default_rng(5)
    V = g.standard_normal((n, m))
    Y = _np(op.matvec(_dev(V)))
    Xr = OP.round_points(X, prec, kern, ell)
    A = OK.operator(Xr, kern, ell, s2, sigma2)
    ref = A @ V
    scale = np.abs(A) @ np.abs(V)
    err = np.abs(Y - ref) / scale
    assert err.max() <= 2e-5, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("kern", [0, 1, 2])
def test_matvec_exact_parity(lib, kern):
    n, d = 1100, 7
    X = _points(n, d, seed=3)
    ell = workloads.median_distance(X)
    op = lib.Operator(_dev(X), kern, ell, 0.9, 1e-3, prec=1)
    V = np.random.default_rng(1).standard_normal((n, 3))
    Y = _np(op.matvec_exact(_dev(V)))
    A = OK.operator(X, kern, ell, 0.9, 1e-3)
    err = np.abs(Y - A @ V) / (np.abs(A) @ np.abs(V))
    assert err.max() <= 1e-12


def test_matvec_diagonal_exact(lib):
    # one point: A = s2 + sigma2 exactly (the distance to itself is zero)
    for kern in (0, 1, 2):
        for prec in (0, 1):
            op = lib.Operator(_dev([[0.3, -1.7, 2.2]]), kern, 0.7, 1.7, 0.25, prec=prec)
            y = _np(op.matvec(_dev([2.0])))
            assert abs(y[0] - 2.0 * (1.7 + 0.25)) <= 1e-6 * 3.9


def test_matvec_full_size_sampled_rows(lib):
    """n = 65536, d = 32, Matern-5/2, bf16: the launch configuration of the
    benchmark, checked on 48 sampled rows computed one by one."""
    w = workloads.bf16_shift()
    X = w["X"]
    n = X.shape[0]
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=1)
    v = np.random.default_rng(11).standard_normal(n)
    y = _np(op.matvec(_dev(v)))
    Xr = OP.round_points(X, 1, w["kernel"], w["ell"])
    rows = np.random.default_rng(12).choice(n, 48, replace=False)
    for i in rows:
        krow = OK.gram(Xr[i:i + 1], w["kernel"], w["ell"], 1.0, Xr)[0]
        ref = krow @ v + w["sigma2s"][0] * v[i]
        scale = np.abs(krow) @ np.abs(v) + w["sigma2s"][0] * abs(v[i])
        assert abs(y[i] - ref) <= 2e-5 * scale, (i, y[i], ref)


def _gpu_eta(op, A, seed=17):
    """The per-term error level of the GPU operator against the oracle's dense
    matrix of the same points (the error model of tests/emulation.py),
    measured on one random vector."""
    v = np.random.default_rng(seed).standard_normal(A.shape[0])
    return fit_eta(A, v, _np(op.matvec(_dev(v))))


def _floor(op, A, x, b):
    """|(A_gpu - A_ref) x| / |b|: how far the GPU operator is from the oracle's."""
    ax_gpu = _np(op.matvec(_dev(x)))
    return np.linalg.norm(ax_gpu - A @ x) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,tol,its_tol", [(3, 1e-8, 2), (0, 1e-5, 0)])
def test_plain_cg_parity(lib, prec, tol, its_tol):
    """Plain CG, n=1024 RBF system: FP64 operator at tol 1e-8 (iteration
    counts within 2 of the oracle), FP32 operator at 1e-5 (above its floor)."""
    w = workloads.small()
    X = w["X"]
    ell = w["ells"][0]
    Xr = OP.round_points(X, prec, w["kernel"], ell)
    A = OK.operator(Xr, w["kernel"], ell, 1.0, w["sigma2"])
    b = A @ w["xstar"] + w["noise"][0]
    op = lib.Operator(_dev(X), w["kernel"], ell, 1.0, w["sigma2"], prec=prec)
    x, st = lib.solve(op, _dev(b), tol=tol, true_residual=True)
    x = _np(x)
    ref = OC.cg(A, b, tol=tol)
    assert st["status"] == 0
    assert abs(st["iters"] - ref.iters) <= max(its_tol, 0.1 * ref.iters), (st["iters"], ref.iters)
    fl = _floor(op, A, x, b)
    res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert res <= tol + 2 * fl, (res, fl)
    assert st["rel_res_recursive"] <= tol
    if prec == 3:
        np.testing.assert_allclose(x, ref.x, rtol=0, atol=1e-6 * np.abs(ref.x).max())


def test_cg_graph_and_eager_bitwise_equal(lib):
    w = workloads.small(n=700)
    op = lib.Operator(_dev(w["X"]), 0, 1.0, 1.0, 1e-2, prec=0)
    b = _dev(np.random.default_rng(2).standard_normal(700))
    x1, s1 = lib.solve(op, b, tol=1e-9, use_graph=True)
    x2, s2 = lib.solve(op, b, tol=1e-9, use_graph=False, check_every=3)
    x3, s3 = lib.solve(op, b, tol=1e-9, use_graph=True)
    assert s1["iters"] == s2["iters"] == s3["iters"]
    assert torch.equal(x1, x2) and torch.equal(x1, x3)


@pytest.mark.parametrize("prec,tol,th_rtol", [(3, 1e-8, 1e-6), (0, 1e-6, 2e-3)])
def test_defcg_sequence_parity_small(lib, prec, tol, th_rtol):
    """The n=1024 five-system sequence: def-CG(8, 12) against the oracle's
    sequence (iteration counts, harmonic Ritz values, residuals)."""
    w = workloads.small()
    X = w["X"]
    n = X.shape[0]
    mats = [OK.operator(OP.round_points(X, prec, w["kernel"], ell), w["kernel"], ell, 1.0,
                        w["sigma2"]) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i] for i, A in enumerate(mats)]
    ref = OS.solve_sequence(mats, bs, k=8, L=12, tol=tol)
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], 1.0, w["sigma2"], prec=prec)
    rc = lib.Recycle(n, 8, 12)
    its = []
    for i, (ell, A, b) in enumerate(zip(w["ells"], mats, bs)):
        op.set_hyper(ell, 1.0, w["sigma2"])
        x, st = lib.solve(op, _dev(b), rc=rc, tol=tol)
        x = _np(x)
        assert st["status"] == 0
        its.append(st["iters"])
        fl = _floor(op, A, x, b)
        res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert res <= tol + 2 * fl
        # harmonic Ritz values of the extraction (largest first)
        th = np.array(rc.theta())
        assert len(th) == 8
        np.testing.assert_allclose(th, ref[i].theta, rtol=th_rtol)
    ref_its = [r.iters for r in ref]
    if prec == 3:
        # FP64 operator: the same iteration within rounding
        for a, c in zip(its, ref_its):
            assert abs(a - c) <= 2, (its, ref_its)
    else:
        # FP32 operator: its evaluation error delays CG.  The delay is bounded
        # by the oracle's own iteration with per-term product errors of 1e-7
        # and 3e-7 on this sequence (test_oracle_emulation.py: every system
        # within [exact - 1, 1.15 exact]); the GPU operator's error level is
        # measured here and must lie inside that range, and the counts inside
        # the band (two steps of margin for the error model)
        eta = _gpu_eta(op, mats[-1])
        print(f"FP32 operator per-term error {eta:.2e}; its {its} oracle {ref_its}", flush=True)
        assert eta <= 3e-7, eta
        for a, c in zip(its, ref_its):
            assert c - 3 <= a <= 1.15 * c + 2, (its, ref_its)
    # recycling pays: fewer steps than plain CG on the later systems
    plain = OS.solve_sequence(mats, bs, k=8, L=12, tol=tol, recycle=False)
    assert sum(its[1:]) < sum(p.iters for p in plain[1:])


@pytest.mark.parametrize("k,L,sigma2", [(8, 12, 1e-2), (16, 24, 1e-2), (32, 96, 1e-2),
                                        (64, 64, 3e-2)])
def test_ritz_routes_match_oracle(lib, k, L, sigma2):
    """Both reductions of F in the harmonic Ritz problem (Eq. 7): Cholesky,
    taken where a bound shows that nothing would be dropped, and the
    eigendecomposition, forced with ritz_route="eigen".  FP64 operator,
    three systems of the n = 1024 sequence: each route's harmonic Ritz values
    against the oracle's (rtol 1e-6), and the two routes' recycled spaces
    equal.  With (8, 12) the stored directions are A-conjugate to rounding
    and the automatic choice is always Cholesky.  In the two larger cases
    the first system's directions have lost A-conjugacy (F is numerically
    singular: the spectrum is a few large eigenvalues over a cluster at
    sigma2, whose early Ritz values converge), so the automatic choice must
    fall back to the eigendecomposition and drop F's null directions as the
    oracle does.  Z has more than 104 columns later in both (the instance
    that keeps its eigenvectors in global memory): with (32, 96) F stays
    singular there, with (64, 64) and sigma2 = 3e-2 it is well conditioned
    (110 and 119 columns), so that instance's Cholesky route runs.
    There GPU and oracle build Z from two FP64 CG runs that have lost
    conjugacy differently, and which borderline directions of the singular F
    (lam near 1e-12 lam_max) survive the drop differs by one or two between
    them; the trailing Ritz values depend on exactly those directions (seen
    to move by a few percent from the 16th value on), so only the leading 16
    are compared with the oracle's (rtol 1e-3, also on the later systems,
    whose W comes from that extraction), and the GPU basis is checked for the defining
    properties W^T A W = I and (AW)^T AW = diag(theta) with the dense FP64 A.
    Every Ritz value is compared (rtol 1e-6) on each system whose
    extraction, and every extraction before it in the sequence, kept all of
    F's directions: all systems of (8, 12) and of (16, 24) (whose F has
    smallest scaled eigenvalue ratios 0.14, 0.92, 0.93 in the oracle).
    The extraction itself on identical inputs is pinned by
    test_extraction_on_given_Z_matches_oracle.  The two routes' spaces
    agree to rounding in every case."""
    w = workloads.small(systems=3)
    X = w["X"]
    n = X.shape[0]
    tol = 1e-8
    mats = [OK.operator(X, w["kernel"], ell, 1.0, sigma2) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i] for i, A in enumerate(mats)]
    ref = OS.solve_sequence(mats, bs, k=k, L=L, tol=tol)
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], 1.0, sigma2, prec=3)
    rcs = {route: lib.Recycle(n, k, L) for route in ("auto", "eigen")}
    chosen = []
    full_rank_chain = {route: True for route in rcs}
    for i, (ell, A, b) in enumerate(zip(w["ells"], mats, bs)):
        op.set_hyper(ell, 1.0, sigma2)
        Ws, its = {}, {}
        for route, rc in rcs.items():
            x, st = lib.solve(op, _dev(b), rc=rc, tol=tol, ritz_route=route)
            print(f"system {i} {route}: {st['iters']} its, Z {st['refresh_dim']} rank "
                  f"{st['refresh_rank']} sweeps {st['refresh_sweeps']}", flush=True)
            assert st["status"] == 0
            assert np.linalg.norm(b - A @ _np(x)) / np.linalg.norm(b) <= 3 * tol
            cholesky = st["refresh_sweeps"][0] == 0
            if route == "auto":
                chosen.append((cholesky, st["refresh_rank"] < st["refresh_dim"],
                               st["refresh_dim"]))
            else:
                assert not cholesky
            if cholesky:
                assert st["refresh_rank"] == st["refresh_dim"]
            th = np.array(rc.theta())
            Wg = _np(rc.get_W())
            full_rank_chain[route] &= st["refresh_rank"] == st["refresh_dim"]
            if (k, L) in ((8, 12), (16, 24)):
                assert full_rank_chain[route]
            if full_rank_chain[route]:
                np.testing.assert_allclose(th, ref[i].theta, rtol=1e-6)
            else:
                np.testing.assert_allclose(th[:16], ref[i].theta[:16], rtol=1e-3)
                AWg = A @ Wg
                np.testing.assert_allclose(Wg.T @ AWg, np.eye(len(th)), atol=1e-3)
                np.testing.assert_allclose(np.sum(AWg * AWg, axis=0), th, rtol=1e-3)
            Ws[route], its[route] = Wg, st["iters"]
        assert abs(its["auto"] - its["eigen"]) <= 1
        Qa, _ = np.linalg.qr(Ws["auto"])
        Qb, _ = np.linalg.qr(Ws["eigen"])
        assert np.linalg.svd(Qa.T @ Qb, compute_uv=False).min() >= 1 - 1e-6
    if (k, L) in ((8, 12), (16, 24)):
        assert all(c for c, _, _ in chosen)
    else:
        assert not chosen[0][0] and chosen[0][1]
    if (k, L) == (64, 64):
        assert any(c and dim > 104 for c, _, dim in chosen[1:])


@pytest.mark.parametrize("kind", ["harmonic", "rayleigh"])
@pytest.mark.parametrize("route", ["auto", "eigen"])
@pytest.mark.parametrize("n,m,k,dup,largest", [(600, 40, 8, 0, True), (600, 40, 8, 0, False),
                                               (600, 60, 8, 20, True), (900, 150, 32, 0, True),
                                               (900, 150, 16, 30, True)])
def test_extraction_on_given_Z_matches_oracle(lib, kind, route, n, m, k, dup, largest):
    """The extraction kernels alone (dcg_extract_basis), fed a Z and AZ = A Z
    that the oracle also gets: the same Ritz values (rtol 1e-10) and the same
    W' = Z U column by column (up to sign), for harmonic and Rayleigh-Ritz
    extraction.  Z is Gaussian; with dup > 0 its last columns repeat earlier
    ones, so the metric (F, or Z^T Z) is singular and both sides drop the
    repeated directions (rank m - dup).  m = 150 runs the instance that keeps
    its eigenvectors in global memory."""
    g = np.random.default_rng(n + m + dup)
    A = OK.operator(g.standard_normal((n, 4)), 0, 1.0, 1.0, 1e-2)
    Z0 = g.standard_normal((n, m - dup))
    Z = np.hstack([Z0, Z0[:, :dup]]) if dup else Z0
    AZ = A @ Z
    Wg, thg, rank = lib.extract_basis(_dev(Z), _dev(AZ), k, largest=largest, extraction=kind,
                                      ritz_route=route)
    Wr, _, thr, _ = ORZ.extract(Z, AZ, k, largest=largest,
                                kind=ORZ.RAYLEIGH if kind == "rayleigh" else ORZ.HARMONIC)
    assert rank == m - dup
    assert len(thg) == k
    np.testing.assert_allclose(thg, thr, rtol=1e-10)
    Wg = _np(Wg)
    for i in range(k):
        w = Wg[:, i] * np.sign(Wg[:, i] @ Wr[:, i])
        assert np.linalg.norm(w - Wr[:, i]) <= 1e-8 * np.linalg.norm(Wr[:, i]), i
    # U^T F U = I: W' is A-orthonormal (harmonic) or orthonormal (Rayleigh-Ritz)
    metric = A if kind == "harmonic" else np.eye(n)
    np.testing.assert_allclose(Wg.T @ metric @ Wg, np.eye(k), atol=1e-9)


@pytest.mark.parametrize("largest", [True, False])
def test_rayleigh_ritz_sequence_matches_oracle(lib, largest):
    """The n = 1024 sequence with Rayleigh-Ritz extraction (FP64 operator,
    def-CG(8, 12), tol 1e-8), largest or smallest Ritz values kept: the
    oracle's iteration counts within 2, its Ritz values to rtol 1e-6, true
    residuals at the tolerance, and an orthonormal recycled basis."""
    w = workloads.small()
    X = w["X"]
    n = X.shape[0]
    tol = 1e-8
    mats = [OK.operator(X, w["kernel"], ell, 1.0, w["sigma2"]) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i] for i, A in enumerate(mats)]
    ref = OS.solve_sequence(mats, bs, k=8, L=12, tol=tol, largest=largest,
                            extraction=ORZ.RAYLEIGH)
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], 1.0, w["sigma2"], prec=3)
    rc = lib.Recycle(n, 8, 12)
    for i, (ell, A, b) in enumerate(zip(w["ells"], mats, bs)):
        op.set_hyper(ell, 1.0, w["sigma2"])
        x, st = lib.solve(op, _dev(b), rc=rc, tol=tol, extraction="rayleigh",
                          select_largest=largest)
        assert st["status"] == 0
        assert np.linalg.norm(b - A @ _np(x)) / np.linalg.norm(b) <= 3 * tol
        assert abs(st["iters"] - ref[i].iters) <= 2, (i, st["iters"], ref[i].iters)
        np.testing.assert_allclose(np.array(rc.theta()), ref[i].theta, rtol=1e-6)
        Wg = _np(rc.get_W())
        np.testing.assert_allclose(Wg.T @ Wg, np.eye(Wg.shape[1]), atol=1e-9)


def test_recycled_basis_is_A_orthonormal(lib):
    w = workloads.small(n=900)
    X = w["X"][:900]
    Xr = OP.round_points(X, 0, 0, 1.0)
    A = OK.operator(Xr, 0, 1.0, 1.0, 1e-2)
    op = lib.Operator(_dev(X), 0, 1.0, 1.0, 1e-2, prec=0)
    rc = lib.Recycle(900, 8, 12)
    b = np.random.default_rng(4).standard_normal(900)
    lib.solve(op, _dev(b), rc=rc, tol=1e-10)
    W = _np(rc.get_W())
    assert W.shape == (900, 8)
    M = W.T @ A @ W
    np.testing.assert_allclose(M, np.eye(8), atol=1e-5)
    # oracle extraction from the same directions: compare the spanned spaces
    ref = OC.cg(A, b, tol=1e-10, L=12)
    Wr, _, th, _ = ORZ.harmonic_ritz(ref.P, ref.AP, 8)
    Qa, _ = np.linalg.qr(W)
    Qb, _ = np.linalg.qr(Wr)
    s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    assert s.min() > 1 - 1e-4


@pytest.mark.parametrize("prec,sigma2,tol", [(3, 1e-2, 1e-8), (3, 1e-3, 1e-8), (0, 1e-2, 1e-6)])
def test_exact_eigenvector_deflation(lib, prec, sigma2, tol):
    """W = exact eigenvectors of the 8 largest eigenvalues (oracle eigh):
    def-CG needs fewer steps than plain CG, as many as the oracle def-CG up
    to the spread that the GPU operator's own error level causes: the
    oracle's iteration (with the library's re-projection) is rerun with
    per-term product errors of twice the level measured on the GPU operator
    (at least one FP64 rounding, 3e-16) over several seeds, and the GPU's
    counts must lie in the band those runs span, two steps of margin on
    either side (FP32: three).  test_oracle_emulation.py shows why a band is
    needed: at kappa 4.9e5 rounding alone moves FP64 counts by several
    steps, and FP32 evaluation error inflates them by 30-40% here."""
    n = 800
    X = _points(n, 4, seed=21)
    ell = workloads.median_distance(X)
    Xr = OP.round_points(X, prec, 0, ell)
    A = OK.operator(Xr, 0, ell, 1.0, sigma2)
    lam, Q = np.linalg.eigh(A)
    W = Q[:, -8:]
    b = np.random.default_rng(3).standard_normal(n)
    op = lib.Operator(_dev(X), 0, ell, 1.0, sigma2, prec=prec)
    rc = lib.Recycle(n, 8, 12)
    rc.set_W(_dev(W))
    x, st = lib.solve(op, _dev(b), rc=rc, tol=tol)
    plain_x, plain = lib.solve(op, _dev(b), tol=tol)
    ref = OC.defcg(A, b, W=W, tol=tol, reproject=True)
    ref_plain = OC.cg(A, b, tol=tol)
    assert st["status"] == 0 and st["k_used"] == 8
    assert st["iters"] < plain["iters"]
    eta = _gpu_eta(op, A)
    eta_e = max(2.0 * eta, 3e-16)
    seeds = range(6) if prec == 3 else range(4)
    emu = [OC.defcg(noisy_product(A, eta_e, s), b, W=W, AW=A @ W, tol=tol,
                    reproject=True).iters for s in seeds]
    margin = 2 if prec == 3 else 3
    lo, hi = min(emu + [ref.iters]) - margin, max(emu + [ref.iters]) + margin
    print(f"prec {prec} sigma2 {sigma2}: eta {eta:.2e}; GPU {st['iters']} / plain "
          f"{plain['iters']}; oracle {ref.iters} / {ref_plain.iters}; emulated {emu}", flush=True)
    assert lo <= st["iters"] <= hi, (st["iters"], lo, hi)
    if prec == 3 and ref_plain.iters <= n // 2:
        # (beyond n / 2 steps the count of finite-precision CG follows the
        # rounding order of its inner products, which no band pins down)
        emu_p = [OC.cg(noisy_product(A, eta_e, s), b, tol=tol).iters for s in seeds]
        lo, hi = min(emu_p + [ref_plain.iters]) - 2, max(emu_p + [ref_plain.iters]) + 2
        assert lo <= plain["iters"] <= hi, (plain["iters"], emu_p, ref_plain.iters)
    xn = _np(x)
    assert np.linalg.norm(b - A @ xn) / np.linalg.norm(b) <= tol + 2 * _floor(op, A, xn, b)


@pytest.mark.parametrize("prec", [1, 4])
def test_refinement_reaches_1e8_bf16(lib, prec):
    """Precision form at small size: bf16 (or fp16) distances, FP64
    refinement to 1e-8."""
    w = workloads.bf16_shift(n=3000)
    X = w["X"]
    A64 = OK.operator(X, w["kernel"], w["ell"], 1.0, w["sigma2s"][0])
    b = w["b"]
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=prec)
    rc = lib.Recycle(3000, 16, 24)
    x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=True, inner_tol=1e-4)
    x = _np(x)
    res = np.linalg.norm(b - A64 @ x) / np.linalg.norm(b)
    assert st["status"] == 0
    assert res <= 1.05e-8, res
    assert abs(res - st["rel_res_true"]) <= 1e-3 * res + 1e-15
    x_ref = np.linalg.solve(A64, b)
    err_A = np.sqrt((x - x_ref) @ A64 @ (x - x_ref) / (x_ref @ A64 @ x_ref))
    assert err_A <= 1e-7


def test_precision_form_reduced_headline_matches_oracle(lib):
    """The precision form at the headline's k, L and inner tolerance on a
    reduced size: n = 8192 points U[-1, 1]^32, Matern-5/2, ell = 0.5 x median
    distance, bf16 operands, def-CG(64, 96) inner solves to 2e-2, refinement
    against the FP64 operator to 1e-8, W refreshed after the first inner
    solve of each system, three systems of the sigma2 = 1e-3 * 0.9^i
    sequence.  The oracle runs the same refinement (oracle.refine, extract =
    "first", the library's re-projection) on the same rounded points, W and
    AW carried with the exact shift update.  Per system:
    * outer steps within one of the oracle's;
    * the oracle's dense FP64 true residual of the GPU solution <= 1.05e-8,
      and the library's own report of it within 1e-3 of that;
    * the A-norm error against the Cholesky solution <= 1e-7;
    * the extracted harmonic Ritz values (theta_i = |A w_i|^2 of the oracle's
      A-orthonormal basis): the leading 16 within the spread that the GPU
      operator's error level causes, measured by rerunning the oracle's
      first system with per-term product errors of twice that level (two
      seeds; tests/emulation.py), times three, and at least 1e-6 theta_1
      (Weyl's bound for the FP32 evaluation error of the operator)."""
    import scipy.linalg as sl
    from oracle import refine as ORF
    n, k, L = 8192, 64, 96
    w = workloads.bf16_shift(n=n, systems=3)
    X, b, kern, ell = w["X"], w["b"], w["kernel"], w["ell"]
    Xr = OP.round_points(X, 1, kern, ell)
    K64 = OK.gram(X, kern, ell, 1.0)
    Klo = OK.gram(Xr, kern, ell, 1.0)
    op = lib.Operator(_dev(X), kern, ell, 1.0, w["sigma2s"][0], prec=1)
    rc = lib.Recycle(n, k, L)
    bn = np.linalg.norm(b)
    W = AW = None
    s2_prev = None
    spread = None
    for i, s2 in enumerate(w["sigma2s"]):
        op.set_hyper(ell, 1.0, s2)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=True, inner_tol=2e-2,
                          refresh_every="first")
        x = _np(x)
        A64 = K64 + s2 * np.eye(n)
        Alo = Klo + s2 * np.eye(n)
        if W is not None:
            AW = AW + (s2 - s2_prev) * W
        W_in, AW_in = W, AW
        xr, hist, inner, (W, AW) = ORF.refine(A64, Alo, b, tol=1e-8, inner_tol=2e-2, k=k, L=L,
                                              extract="first", W=W_in, AW=AW_in, reproject=True)
        s2_prev = s2
        th_ref = np.sort(np.sum(AW * AW, axis=0))[::-1]
        th = np.array(rc.theta())
        if i == 0:
            eta = _gpu_eta(op, Alo)
            devs = []
            for seed in (0, 1):
                _, _, _, (We, AWe) = ORF.refine(A64, noisy_product(Alo, 2 * eta, seed), b,
                                                tol=1e-8, inner_tol=2e-2, k=k, L=L,
                                                extract="first", reproject=True, max_outer=1)
                th_e = np.sort(np.sum(AWe * AWe, axis=0))[::-1]
                devs.append(np.abs(th_e[:16] - th_ref[:16]) / th_ref[:16])
            spread = np.maximum(3 * np.max(devs, axis=0), 1e-9)
        res = np.linalg.norm(b - A64 @ x) / bn
        x_ref = sl.cho_solve(sl.cho_factor(A64), b)
        err_A = np.sqrt((x - x_ref) @ A64 @ (x - x_ref) / (x_ref @ A64 @ x_ref))
        print(f"system {i}: outer {st['outer_steps']} vs {len(inner)}, its {st['iters']} vs "
              f"{sum(r.iters for r in inner)}, k {st['k_used']}->{st['k_next']}, res {res:.2e}, "
              f"errA {err_A:.2e}, theta dev {np.abs(th[:16] - th_ref[:16]).max() / th_ref[0]:.1e}",
              flush=True)
        assert st["status"] == 0
        assert abs(st["outer_steps"] - len(inner)) <= 1, (st["outer_steps"], len(inner))
        assert res <= 1.05e-8, res
        assert abs(res - st["rel_res_true"]) <= 1e-3 * res + 1e-15
        assert err_A <= 1e-7, err_A
        assert len(th) == st["k_next"] and abs(len(th) - len(th_ref)) <= 2
        # Weyl: an operator error E moves every eigenvalue by at most
        # |E|_2 <= eps |A|_2 (entrywise positive kernel matrix, eps the
        # largest relative error of an FP32-evaluated entry, below 1e-6), so
        # no value is held closer than 1e-6 theta_1
        rel = np.abs(th[:16] - th_ref[:16]) / th_ref[:16]
        bound = np.maximum(spread if i == 0 else 3 * spread, 1e-6 * th_ref[0] / th_ref[:16])
        assert np.all(rel <= bound), (i, rel, bound)
        # the basis carried over is the previous extraction's (at this size the
        # first inner solve stops after fewer than k steps, so fewer than k
        # directions exist to keep)
        if i > 0:
            assert st["k_used"] == k_prev, (st["k_used"], k_prev)
        k_prev = st["k_next"]


def test_precision_form_full_size_residual_rows(lib):
    """The benchmark's configuration at full size (n = 65536, d = 32,
    Matern-5/2, bf16, def-CG(64, 96), inner tolerance 2e-2, refinement to
    1e-8, the sweep plan of 8192 work items), first two systems of the
    sequence: on 48 sampled rows the oracle forms (b - A64 x)_i one row at a
    time from the unrounded points; the library's FP64 product agrees with
    each row to 1e-12 of (|A64| |x|)_i, so the residual the library reports
    is the true residual, and every sampled |r_i| is below 1e-8 |b| plus the
    rows' FP64 rounding."""
    w = workloads.bf16_shift()
    X, b, kern, ell = w["X"], w["b"], w["kernel"], w["ell"]
    n = X.shape[0]
    op = lib.Operator(_dev(X), kern, ell, 1.0, w["sigma2s"][0], prec=1)
    op.set_sweep_items(8192)
    rc = lib.Recycle(n, w["k"], w["L"])
    rows = np.random.default_rng(13).choice(n, 48, replace=False)
    krows = OK.gram(X[rows], kern, ell, 1.0, X)
    bn = np.linalg.norm(b)
    for i, s2 in enumerate(w["sigma2s"][:2]):
        op.set_hyper(ell, 1.0, s2)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=True, inner_tol=2e-2)
        assert st["status"] == 0 and st["rel_res_true"] <= 1e-8
        y = _np(op.matvec_exact(x))
        x = _np(x)
        ax = krows @ x + s2 * x[rows]
        scale = np.abs(krows) @ np.abs(x) + s2 * np.abs(x[rows])
        assert np.all(np.abs(y[rows] - ax) <= 1e-12 * scale), np.max(np.abs(y[rows] - ax) / scale)
        r = b[rows] - ax
        assert np.all(np.abs(r) <= 1e-8 * bn + 1e-15 * scale), (np.abs(r).max() / bn)
        print(f"system {i}: {st['iters']} its, {st['outer_steps']} outer, reported residual "
              f"{st['rel_res_true']:.2e}, sampled max |r_i|/|b| {np.abs(r).max() / bn:.2e}",
              flush=True)


def test_fp16_operands_out_of_range(lib):
    """fp16 operands need the scaled points and their squared norms inside
    the fp16 range: creation with a lengthscale that breaks it returns
    DCG_E_ARG, and so does set_hyper, which then keeps the previous
    hyperparameters (the product is unchanged)."""
    g = np.random.default_rng(31)
    X = g.standard_normal((500, 16))
    with pytest.raises(lib.DcgError) as e:
        lib.Operator(_dev(X), 0, 1e-3, 1.0, 1e-2, prec=4)
    assert e.value.status == -1
    op = lib.Operator(_dev(X), 0, 2.0, 1.0, 1e-2, prec=4)
    v = _dev(g.standard_normal(500))
    y0 = op.matvec(v)
    with pytest.raises(lib.DcgError) as e:
        op.set_hyper(1e-3, 1.0, 1e-2)
    assert e.value.status == -1
    assert torch.equal(op.matvec(v), y0)
    A = OK.operator(OP.round_points(X, 4, 0, 2.0), 0, 2.0, 1.0, 1e-2)
    ref = A @ _np(v)
    assert np.abs(_np(y0) - ref).max() <= 2e-5 * (np.abs(A) @ np.abs(_np(v))).max()


@pytest.mark.parametrize("prec,inner_tol", [(1, 1e-2), (1, 1e-1), (0, 1e-3)])
def test_refinement_fcg_matches_oracle(lib, prec, inner_tol):
    """Flexible-CG refinement: FP64 outer directions around the inner
    deflated solve of the rounded-points operator, against the oracle's
    refine_fcg (same recycling: W extracted after the first inner solve)."""
    from oracle import refine as ORF
    w = workloads.bf16_shift(n=3000)
    X, b = w["X"], w["b"]
    s2 = w["sigma2s"][0]
    A64 = OK.operator(X, w["kernel"], w["ell"], 1.0, s2)
    Alow = OK.operator(OP.round_points(X, prec, w["kernel"], w["ell"]), w["kernel"], w["ell"], 1.0, s2)
    xr, hist, inner = ORF.refine_fcg(A64, Alow, b, tol=1e-8, inner_tol=inner_tol, k=16, L=24)
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, s2, prec=prec)
    rc = lib.Recycle(3000, 16, 24)
    x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine="fcg", inner_tol=inner_tol)
    x = _np(x)
    res = np.linalg.norm(b - A64 @ x) / np.linalg.norm(b)
    assert st["status"] == 0
    assert res <= 1.05e-8, res
    assert abs(res - st["rel_res_true"]) <= 1e-3 * res + 1e-15
    # outer steps as the oracle's, within one; one FP64 product per step plus
    # the final confirmation (the first residual from x = 0 is b)
    assert abs(st["outer_steps"] - len(inner)) <= 1, (st["outer_steps"], len(inner))
    assert st["matvecs_exact"] == st["outer_steps"] + 1
    x_ref = np.linalg.solve(A64, b)
    err_A = np.sqrt((x - x_ref) @ A64 @ (x - x_ref) / (x_ref @ A64 @ x_ref))
    assert err_A <= 1e-7
    rc2 = lib.Recycle(3000, 16, 24)
    _, st_ir = lib.solve(op, _dev(b), rc=rc2, tol=1e-8, refine=True, inner_tol=inner_tol)
    assert st_ir["status"] == 0
    print(f"prec {prec} inner_tol {inner_tol}: fcg {st['outer_steps']} outer / {st['iters']} its, "
          f"ir {st_ir['outer_steps']} outer / {st_ir['iters']} its", flush=True)


@pytest.mark.parametrize("refine", [True, "fcg"])
def test_refinement_accumulated_extraction_matches_oracle(lib, refine):
    """refresh_every = "accum": the inner solves of one system store their
    directions one after the other (up to L) and the basis is extracted once
    at the end.  With the FP64 operator inside the refinement the inner solves
    are those of the oracle step for step (the refinement converges by the
    inner tolerance, 1e-2 per outer step), so the stored subspace and its
    harmonic Ritz values match; two systems of the sigma^2 sequence.  (The
    oracle runs plain refinement; the flexible variant takes the same inner
    solves here, its outer directions being the inner solutions.)"""
    from oracle import refine as ORF
    w = workloads.bf16_shift(n=1200, systems=2)
    X, b = w["X"], w["b"]
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=3)
    rc = lib.Recycle(1200, 16, 24)
    W = AW = None
    for i, s2 in enumerate(w["sigma2s"]):
        op.set_hyper(w["ell"], 1.0, s2)
        A = OK.operator(X, w["kernel"], w["ell"], 1.0, s2)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=refine, inner_tol=1e-2,
                          refresh_every="accum")
        if W is not None:
            AW = A @ W
        xr, hist, inner, (W, AW) = ORF.refine(A, A, b, tol=1e-8, inner_tol=1e-2, k=16,
                                              L=24, extract="accum", W=W, AW=AW)
        x = _np(x)
        assert st["status"] == 0
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1.05e-8
        assert st["outer_steps"] == len(inner), (i, st["outer_steps"], len(inner))
        its = [r.iters for r in inner]
        assert abs(st["iters"] - sum(its)) <= len(its), (i, st["iters"], its)
        assert st["k_next"] == 16
        # theta_i = |A w_i|^2 for the A-orthonormal harmonic Ritz basis
        th_ref = np.sort(np.sum(AW * AW, axis=0))[::-1]
        np.testing.assert_allclose(np.array(rc.theta()), th_ref, rtol=1e-6)
        Wg = _np(rc.get_W())
        np.testing.assert_allclose(Wg.T @ A @ Wg, np.eye(16), atol=1e-8)


def test_refinement_accumulated_extraction_bf16(lib):
    """The accumulated schedule with the bf16 operator on a three-system
    sequence: every solve reaches 1e-8 in the FP64 residual, the basis is
    refreshed once per system and is A~-orthonormal for the rounded-points
    operator (which of the inner solves' directions fill the L slots depends
    on their iteration counts, so the Ritz values are not compared here)."""
    w = workloads.bf16_shift(n=3000, systems=3)
    X, b = w["X"], w["b"]
    Xr = OP.round_points(X, 1, w["kernel"], w["ell"])
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=1)
    rc = lib.Recycle(3000, 16, 24)
    for i, s2 in enumerate(w["sigma2s"]):
        op.set_hyper(w["ell"], 1.0, s2)
        A64 = OK.operator(X, w["kernel"], w["ell"], 1.0, s2)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=True, inner_tol=1e-2,
                          refresh_every="accum")
        x = _np(x)
        assert st["status"] == 0
        assert np.linalg.norm(b - A64 @ x) / np.linalg.norm(b) <= 1.05e-8
        assert st["k_used"] == (0 if i == 0 else 16) and st["k_next"] == 16
        Alow = OK.operator(Xr, w["kernel"], w["ell"], 1.0, s2)
        Wg = _np(rc.get_W())
        np.testing.assert_allclose(Wg.T @ Alow @ Wg, np.eye(16), atol=1e-4)


def test_refinement_fcg_from_given_start_and_zero_rhs(lib):
    w = workloads.bf16_shift(n=1500)
    X, b = w["X"], w["b"]
    s2 = w["sigma2s"][0]
    A64 = OK.operator(X, w["kernel"], w["ell"], 1.0, s2)
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], 1.0, s2, prec=1)
    x_ref = np.linalg.solve(A64, b)
    x0 = x_ref * (1.0 + 1e-3 * np.random.default_rng(3).standard_normal(1500))
    x, st = lib.solve(op, _dev(b), x0=_dev(x0), tol=1e-10, refine="fcg", inner_tol=1e-2)
    x = _np(x)
    assert st["status"] == 0
    assert np.linalg.norm(b - A64 @ x) / np.linalg.norm(b) <= 1.05e-10
    # the given start costs one FP64 product for r_0
    assert st["matvecs_exact"] == st["outer_steps"] + 2
    z, st0 = lib.solve(op, torch.zeros(1500, dtype=torch.float64, device="cuda"), tol=1e-8,
                       refine="fcg")
    assert st0["status"] == 0 and st0["outer_steps"] == 0 and torch.count_nonzero(z) == 0


def test_sigma_shift_sequence_reuses_AW(lib):
    """sigma^2-only changes: AW updated by the shift, no block product."""
    w = workloads.bf16_shift(n=2048, systems=3)
    op = lib.Operator(_dev(w["X"]), w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=1)
    rc = lib.Recycle(2048, 16, 24)
    Xr = OP.round_points(w["X"], 1, w["kernel"], w["ell"])
    for i, s2 in enumerate(w["sigma2s"]):
        op.set_hyper(w["ell"], 1.0, s2)
        x, st = lib.solve(op, _dev(w["b"]), rc=rc, tol=1e-6)
        if i > 0:
            assert st["k_used"] == 16
            # one product for r_0 after the deflated start, no AW recompute
            assert st["matvecs"] == st["iters"] + 1
        A = OK.operator(Xr, w["kernel"], w["ell"], 1.0, s2)
        x = _np(x)
        fl = _floor(op, A, x, w["b"])
        assert np.linalg.norm(w["b"] - A @ x) / np.linalg.norm(w["b"]) <= 1e-6 + 2 * fl


def test_deterministic(lib):
    w = workloads.fp32_walk(n=3000, systems=2)
    def run():
        op = lib.Operator(_dev(w["X"]), 0, w["ells"][0], 1.0, 1e-2, prec=0)
        rc = lib.Recycle(3000, 16, 24)
        xs = []
        for ell in w["ells"]:
            op.set_hyper(ell, 1.0, 1e-2)
            x, _ = lib.solve(op, _dev(w["b"]), rc=rc, tol=1e-6)
            xs.append(x.clone())
        return xs, rc.get_W().clone()
    a, Wa = run()
    b, Wb = run()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    assert torch.equal(Wa, Wb)


def test_edge_cases(lib):
    # converges before L directions are stored: k_next <= stored directions
    X = _points(40, 2, seed=1)
    op = lib.Operator(_dev(X), 0, 1.0, 1.0, 1.0, prec=0)
    rc = lib.Recycle(40, 8, 12)
    x, st = lib.solve(op, _dev(np.ones(40)), rc=rc, tol=1e-3)
    assert st["status"] == 0 and st["k_next"] <= min(8, st["iters"])
    # zero right-hand side: x = 0 at once
    x, st = lib.solve(op, _dev(np.zeros(40)), tol=1e-8)
    assert st["iters"] == 0 and float(x.abs().max()) == 0.0
    # NaN in the points
    Xn = X.copy()
    Xn[3, 1] = np.nan
    with pytest.raises(lib.DcgError) as e:
        lib.Operator(_dev(Xn), 0, 1.0, 1.0, 1.0)
    assert e.value.status == -3
    # bad hyperparameters
    with pytest.raises(lib.DcgError):
        op.set_hyper(-1.0, 1.0, 1.0)
    # max_iter reached: not converged, x still returned
    x, st = lib.solve(op, _dev(np.ones(40)), tol=1e-14, max_iter=2)
    assert st["status"] == 1 and st["iters"] == 2


def test_failure_injection_statuses(lib):
    """Failure paths as normal status returns (nothing faults): a recycled
    basis with repeated columns gives DCG_E_W_RANK before the first CG step
    (W^T A W is singular), a NaN or Inf in W gives DCG_E_NONFINITE, and a
    NaN or Inf in b gives DCG_E_NONFINITE from the iteration, with and
    without a basis and with refinement.  The handles stay usable: a
    full-rank basis afterwards solves as usual."""
    n = 600
    X = _points(n, 4, seed=41)
    ell = workloads.median_distance(X)
    A = OK.operator(X, 0, ell, 1.0, 1e-2)
    lam, Q = np.linalg.eigh(A)
    b = np.random.default_rng(5).standard_normal(n)
    for prec in (3, 0, 1):
        op = lib.Operator(_dev(X), 0, ell, 1.0, 1e-2, prec=prec)
        rc = lib.Recycle(n, 8, 12)
        Wdup = Q[:, -8:].copy()
        Wdup[:, 5] = Wdup[:, 2]                     # a repeated column
        rc.set_W(_dev(Wdup))
        with pytest.raises(lib.DcgError) as e:
            lib.solve(op, _dev(b), rc=rc, tol=1e-8)
        assert e.value.status == -4, (prec, e.value.status)
        with pytest.raises(lib.DcgError) as e:
            lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=prec != 3, inner_tol=1e-2)
        assert e.value.status == -4
        # nearly repeated: the columns differ by 1e-9 of their norm
        Wnear = Q[:, -8:].copy()
        Wnear[:, 5] = Wnear[:, 2] + 1e-9 * Q[:, 0]
        rc.set_W(_dev(Wnear))
        with pytest.raises(lib.DcgError) as e:
            lib.solve(op, _dev(b), rc=rc, tol=1e-8)
        assert e.value.status == -4
        Wnan = Q[:, -8:].copy()
        Wnan[7, 3] = np.nan
        rc.set_W(_dev(Wnan))
        with pytest.raises(lib.DcgError) as e:
            lib.solve(op, _dev(b), rc=rc, tol=1e-8)
        assert e.value.status == -3
        # a good basis: the handle works again
        rc.set_W(_dev(Q[:, -8:]))
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-6)
        assert st["status"] == 0 and st["k_used"] == 8
        for bad in (np.nan, np.inf):
            bb = b.copy()
            bb[123] = bad
            for kw in (dict(), dict(rc=rc), dict(refine=prec != 3, inner_tol=1e-2)):
                with pytest.raises(lib.DcgError) as e:
                    lib.solve(op, _dev(bb), tol=1e-8, **kw)
                assert e.value.status == -3, (prec, bad, kw, e.value.status)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-6)
        assert st["status"] == 0


def test_fp32_walk_full_size_matches_oracle(lib):
    """The FP32 log-lengthscale walk at full size (n = 16384, d = 16, RBF,
    sigma2 = 1e-2, 20 systems, def-CG(32, 48), tol 1e-6), the configuration
    of the fp32_walk benchmark, against the oracle's run of the same walk on
    the same FP32-rounded points (tests/golden/fp32_walk_n16384.json, written
    by tests/golden/make_fp32_walk.py from oracle/ alone):
    * step counts: within the band the oracle spans with exact products and
      with per-term product errors of 1e-7 (two seeds; the FP32 operator's
      level, checked here on the first operator), three steps of margin;
    * the leading 8 harmonic Ritz values: within three times the largest
      deviation the emulated runs show from the exact ones, and at least
      1e-6 relative;
    * the solutions: on 48 sampled rows per system the oracle forms A x one
      row at a time; the GPU operator's product agrees with each to 2e-5 of
      (|A| |x|)_i (its product bound), so the residual the library reports
      with its own operator is the operator's.
    Plain CG (the last five systems) against the oracle's plain runs, with
    the band widened by the spread of the two emulated plain runs."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "fp32_walk_n16384.json")))
    runs = gold["runs"]
    w = workloads.fp32_walk()
    X, b = w["X"], w["b"]
    n = X.shape[0]
    assert [round(v, 12) for v in gold["ells"]] == [round(v, 12) for v in w["ells"]]
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], w["s2"], w["sigma2"], prec=0)
    rc = lib.Recycle(n, w["k"], w["L"])
    rows = np.random.default_rng(19).choice(n, 48, replace=False)
    for i, ell in enumerate(w["ells"]):
        op.set_hyper(ell, w["s2"], w["sigma2"])
        x, st = lib.solve(op, _dev(b), rc=rc, tol=w["tol"], true_residual=True)
        assert st["status"] == 0
        exact = [runs["literal"]["iters"][i], runs["reproject"]["iters"][i]]
        emu = [runs[f"emulated{s}"]["iters"][i] for s in (0, 1)]
        lo, hi = min(exact + emu) - 3, max(exact + emu) + 3
        th = np.array(rc.theta())
        th_ref = np.array(runs["reproject"]["theta"][i])
        dev = max(np.max(np.abs(np.array(runs[f"emulated{s}"]["theta"][i][:8]) - th_ref[:8])
                         / th_ref[:8]) for s in (0, 1))
        rel = np.abs(th[:8] - th_ref[:8]) / th_ref[:8]
        Xr = OP.round_points(X[rows], 0, w["kernel"], ell)
        Xall = OP.round_points(X, 0, w["kernel"], ell)
        krows = OK.gram(Xr, w["kernel"], ell, w["s2"], Xall)
        xn = _np(x)
        ax = krows @ xn + w["sigma2"] * xn[rows]
        scale = np.abs(krows) @ np.abs(xn) + w["sigma2"] * np.abs(xn[rows])
        y = _np(op.matvec(x))
        print(f"system {i}: GPU {st['iters']} its, oracle exact {exact} emulated {emu}; "
              f"theta rel dev {rel.max():.1e} (emulated {dev:.1e}); "
              f"own residual {st['rel_res_true']:.1e}", flush=True)
        assert lo <= st["iters"] <= hi, (i, st["iters"], lo, hi)
        assert np.all(rel <= max(3 * dev, 1e-6)), (i, rel, dev)
        assert np.all(np.abs(y[rows] - ax) <= 2e-5 * scale)
    # the FP32 operator's error level is the one the band was drawn at
    # (measured on 2048 sampled rows of the last operator)
    Xr0 = OP.round_points(X, 0, w["kernel"], w["ells"][-1])
    sub = np.random.default_rng(3).choice(n, 2048, replace=False)
    A_sub = OK.gram(Xr0[sub], w["kernel"], w["ells"][-1], w["s2"], Xr0)
    v = np.random.default_rng(4).standard_normal(n)
    y = _np(op.matvec(_dev(v)))[sub] - w["sigma2"] * v[sub]
    e = (y - A_sub @ v) / np.sqrt((A_sub * A_sub) @ (v * v))
    eta = float(np.sqrt(np.mean(e * e)))
    print(f"FP32 operator per-term error {eta:.2e}", flush=True)
    assert eta <= 1e-7, eta
    for i in range(15, 20):
        op.set_hyper(w["ells"][i], w["s2"], w["sigma2"])
        _, st = lib.solve(op, _dev(b), tol=w["tol"])
        exact = runs["plain"]["iters"][i]
        emu = [runs[f"emulated_plain{s}"]["iters"][i] for s in (0, 1)]
        # plain CG's count at this error level is set by its loss of
        # orthogonality and moves with the rounding itself: the two
        # emulated seeds differ by up to 14 steps, so the band is widened
        # on each side by that spread (the deflated runs above stay tight)
        spread = max(3, max(emu) - min(emu))
        lo, hi = min([exact] + emu) - spread, max([exact] + emu) + spread
        print(f"plain system {i}: GPU {st['iters']}, oracle {exact}, emulated {emu}", flush=True)
        assert st["status"] == 0 and lo <= st["iters"] <= hi, (i, st["iters"], lo, hi)
