"""GPU parity of the LDS-staged pair sweep for wide points (bf16 / fp16
operands with more than 64 coordinates, up to the paper's 784-pixel data)
against the oracle's FP64 products on the same rounded points.

Product bound: the narrow sweep's products meet 2e-5 of (|A| |v|)_i with its
at most 80 augmented coordinates (five MFMA K-steps).  The squared distance
comes out of the MFMA with one FP32 rounding per 16-term K-step in the
worst case, so the bound on r^2 grows linearly with the number of K-steps;
the wide sweep is held to 2e-5 x K / 80 (K the augmented, padded width:
2.1e-4 at d = 784)."""

import numpy as np
import pytest

from oracle import gpc as OG
from oracle import kernels as OK
from oracle import precision as OP
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _bound(d):
    K = 64 * ((d + 6 + 63) // 64)
    return 2e-5 * max(1.0, K / 80.0)


def _points(n, d, seed):
    if d == 784:
        return workloads.gpc_pixels(n=n)["X"]
    return np.random.default_rng(seed).standard_normal((n, d))


@pytest.mark.parametrize("prec", [1, 4])
@pytest.mark.parametrize("kern", [0, 1, 2])
@pytest.mark.parametrize("n,d", [(300, 65), (1000, 130), (700, 170), (2600, 784), (256, 4090),
                                 (2, 100), (37, 785)])
def test_wide_matvec_parity(lib, prec, kern, n, d):
    """One product (and a four-column block, formed one column at a time)
    against A V of the rounded points; the plan spans 1 to 11 blocks of 256
    points with a ragged tail, down to two points in one block; the diagonal
    block pair gets distance zero.  The widths give 3, 4, 5, 6, 25 and 128
    stages of 32 K-elements (every remainder modulo the four stage
    buffers)."""
    print(f"wide matvec prec {prec} kern {kern} n {n} d {d}", flush=True)
    X = _points(n, d, seed=n + d)
    ell = workloads.median_distance(X)
    s2, sigma2 = 1.7, 1e-2
    op = lib.Operator(_dev(X), kern, ell, s2, sigma2, prec=prec)
    A = OK.operator(OP.round_points(X, prec, kern, ell), kern, ell, s2, sigma2)
    V = np.random.default_rng(5).standard_normal((n, 4))
    Y = _np(op.matvec(_dev(V)))
    err = np.abs(Y - A @ V) / (np.abs(A) @ np.abs(V))
    print(f"  max error {err.max():.2e} of (|A||v|)_i, bound {_bound(d):.1e}", flush=True)
    assert err.max() <= _bound(d), err.max()
    # symmetric: u^T (A v) = v^T (A u) to the same bound
    u = np.random.default_rng(6).standard_normal(n)
    v = V[:, 0]
    au, av = _np(op.matvec(_dev(u))), _np(op.matvec(_dev(v)))
    assert abs(u @ av - v @ au) <= _bound(d) * (np.abs(u) @ np.abs(A) @ np.abs(v))


def test_wide_plans_agree(lib):
    """Every work-item target gives the oracle's product (the plan only
    changes the grouping of block pairs and the order of the FP64 sums)."""
    n, d = 2600, 200
    X = _points(n, d, seed=1)
    ell = workloads.median_distance(X)
    op = lib.Operator(_dev(X), 2, ell, 1.0, 0.0, prec=1)
    A = OK.operator(OP.round_points(X, 1, 2, ell), 2, ell, 1.0, 0.0)
    v = np.random.default_rng(2).standard_normal(n)
    scale = np.abs(A) @ np.abs(v)
    for items in (256, 1024, 8192):
        op.set_sweep_items(items)
        y = _np(op.matvec(_dev(v)))
        assert np.max(np.abs(y - A @ v) / scale) <= _bound(d), items


def test_wide_laplace_gpc_matches_oracle(lib):
    """The Newton loop on the pixel-like data (n = 1500, d = 784) with bf16
    points through the wide sweep, against the oracle's loop with dense
    solves on the kernel matrix of the same rounded points: the same Newton
    steps, Psi to 4e-4 at every step and 2e-5 at the end, f to 1e-3 of
    max |f| (the bounds of the bf16 loop at tol 1e-6 in
    test_gpu_gpc.py, where the operator's error is the same kind)."""
    w = workloads.gpc_pixels(n=1500)
    X, y = w["X"], w["y"]
    n = X.shape[0]
    Xr = OP.round_points(X, 1, w["kernel"], w["ell"])
    Km = OK.gram(Xr, w["kernel"], w["ell"], w["s2"])
    f_ref, a_ref, psi_ref, _ = OG.laplace_mode(Km, y, psi_tol=w["psi_tol"])
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], w["s2"], 0.0, prec=1)
    rc = lib.Recycle(n, w["k"], w["L"])
    f, a, psi, stats, status = lib.laplace_gpc(op, _dev(y), rc=rc, tol=1e-6,
                                               psi_tol=w["psi_tol"])
    print(f"psi {psi} oracle {psi_ref}; its {[s['iters'] for s in stats]}", flush=True)
    assert status == 0 and len(psi) == len(psi_ref) >= 3, (psi, psi_ref)
    assert all(s["status"] == 0 for s in stats)
    np.testing.assert_allclose(psi, psi_ref, rtol=4e-4)
    assert abs(psi[-1] - psi_ref[-1]) <= 2e-5 * abs(psi_ref[-1])
    f = _np(f)
    assert np.abs(f - f_ref).max() <= 1e-3 * np.abs(f_ref).max()


def test_wide_deflated_sequence(lib):
    """A three-system lengthscale walk at n = 2600, d = 784 (fp16 points,
    RBF, sigma2 = 1e-2, def-CG(8, 12), tol 1e-6): each solution meets the
    tolerance in the oracle's residual up to the operator's floor, and the
    recycled systems take fewer steps than the first."""
    X = _points(2600, 784, seed=0)
    ell0 = workloads.median_distance(X)
    op = lib.Operator(_dev(X), 0, ell0, 1.0, 1e-2, prec=4)
    rc = lib.Recycle(2600, 8, 12)
    b = np.random.default_rng(3).standard_normal(2600)
    its = []
    for i, ell in enumerate(ell0 * np.exp(0.05 * np.arange(3))):
        op.set_hyper(ell, 1.0, 1e-2)
        x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-6)
        assert st["status"] == 0
        A = OK.operator(OP.round_points(X, 4, 0, ell), 0, ell, 1.0, 1e-2)
        xn = _np(x)
        floor = np.linalg.norm(_np(op.matvec(x)) - A @ xn) / np.linalg.norm(b)
        assert np.linalg.norm(b - A @ xn) / np.linalg.norm(b) <= 1e-6 + 2 * floor
        its.append(st["iters"])
    print(f"steps {its}", flush=True)
    assert its[1] < its[0] and its[2] < its[0]


def test_wide_refusals(lib):
    """Wide points have no FP64 operator (refinement, dcg_matvec_exact) and
    no multi-column sweep (block solve, batched solve): DCG_E_ARG, and the
    operator keeps working."""
    n, d = 600, 100
    X = _points(n, d, seed=4)
    op = lib.Operator(_dev(X), 0, workloads.median_distance(X), 1.0, 1e-2, prec=1)
    b = _dev(np.random.default_rng(1).standard_normal(n))
    for call in (lambda: lib.solve(op, b, tol=1e-8, refine=True),
                 lambda: op.matvec_exact(b),
                 lambda: lib.solve_block(op, torch.stack([b, b], 1), tol=1e-6),
                 lambda: lib.solve_batched([op], [b], tol=1e-6)):
        with pytest.raises(lib.DcgError) as e:
            call()
        assert e.value.status == -1
    _, st = lib.solve(op, b, tol=1e-6)
    assert st["status"] == 0


@pytest.mark.parametrize("prec", [1, 4])
def test_wide_full_size_sampled_rows(lib, prec):
    """The pixel workload at full size (n = 36551, d = 784, RBF, bf16 / fp16
    points) in the launch configurations of the GPC benchmark (its default
    plan) and of the plan limits: 24 sampled rows of the product, each row of
    the kernel matrix formed by the oracle from the same rounded points, to
    the wide bound; the diagonal block pairs, the last (ragged) row block
    and both ends of the block-offset range are among the rows."""
    w = workloads.gpc_pixels()
    X = w["X"]
    n = X.shape[0]
    s2, sigma2 = w["s2"], 0.5
    op = lib.Operator(_dev(X), w["kernel"], w["ell"], s2, sigma2, prec=prec)
    Xr = OP.round_points(X, prec, w["kernel"], w["ell"])
    v = np.random.default_rng(31).standard_normal(n)
    rows = np.random.default_rng(32).choice(n, 20, replace=False)
    rows = np.concatenate([rows, [0, 255, n - 256, n - 1]])
    Kr = OK.gram(Xr[rows], w["kernel"], w["ell"], s2, Xr)
    ref = Kr @ v + sigma2 * v[rows]
    scale = np.abs(Kr) @ np.abs(v) + sigma2 * np.abs(v[rows])
    for items in (256, 2048, 8192):
        op.set_sweep_items(items)
        y = _np(op.matvec(_dev(v)))[rows]
        err = np.abs(y - ref) / scale
        print(f"prec {prec} items {items}: max error {err.max():.2e}", flush=True)
        assert err.max() <= _bound(784), (items, err.max())
