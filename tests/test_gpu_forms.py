"""GPU parity of the differentiation form: the multi-right-hand-side
deflated solve, the fused gradient sweep and the autograd Function, against
the FP64 oracle (dense Cholesky solves, the Hutchinson gradient with the same
probes, the exact gradient and finite differences)."""

import math

import numpy as np
import pytest

from oracle import cg as OC
from oracle import gp as OG
from oracle import kernels as OK
from oracle import precision as OP
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec,tol", [(3, 1e-9), (0, 1e-6), (1, 1e-6)])
@pytest.mark.parametrize("deflate", [False, True])
def test_block_solve_columns(lib, prec, tol, deflate):
    n, m = 1500, 6
    g = np.random.default_rng(31)
    X = g.standard_normal((n, 5))
    ell = workloads.median_distance(X)
    Xr = OP.round_points(X, prec, 0, ell)
    A = OK.operator(Xr, 0, ell, 1.0, 1e-2)
    B = g.standard_normal((n, m))
    op = lib.Operator(_dev(X), 0, ell, 1.0, 1e-2, prec=prec)
    rc = None
    if deflate:
        rc = lib.Recycle(n, 8, 12)
        lib.solve(op, _dev(g.standard_normal(n)), rc=rc, tol=tol)   # fills W
    Xs, st = lib.solve_block(op, _dev(B), rc=rc, tol=tol)
    Xs = _np(Xs)
    assert st["status"] == 0
    if deflate:
        assert st["k_used"] == 8
    ref = np.linalg.solve(A, B)
    for c in range(m):
        x = Xs[:, c]
        floor = np.linalg.norm(_np(op.matvec(_dev(x))) - A @ x) / np.linalg.norm(B[:, c])
        res = np.linalg.norm(B[:, c] - A @ x) / np.linalg.norm(B[:, c])
        assert res <= tol + 2 * floor, (c, res, floor)
    # one column through the single-vector solve: same iteration count
    x1, st1 = lib.solve(op, _dev(B[:, 2]), rc=rc, tol=tol)
    if rc is None or prec == 3:
        its_ref = OC.defcg(A, B[:, 2], W=_np(rc.get_W()) if rc else None, tol=tol).iters
        assert st["iters"] >= its_ref - 3


@pytest.mark.parametrize("kern", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_mll_grad_sweep_matches_oracle(lib, kern, prec):
    """The fused sweep against the oracle's Hutchinson gradient with the same
    alpha, U and probes (dense FP64 on the same rounded points)."""
    w = workloads.gp_hyper(n=1200)
    X, y = w["X"], w["y"]
    ell, s2, sig2 = math.exp(w["log_ell"]), 1.3, 0.1
    Xr = OP.round_points(X, prec, kern, ell)
    A = OK.operator(Xr, kern, ell, s2, sig2)
    Z = workloads.rademacher(1200, 16, step=0)
    alpha = np.linalg.solve(A, y)
    U = np.linalg.solve(A, Z)
    op = lib.Operator(_dev(X), kern, ell, s2, sig2, prec=prec)
    g = np.array(lib.mll_grad(op, _dev(alpha), _dev(U), _dev(Z)))
    ref = OG.lml_grad_hutchinson(Xr, y, kern, ell, s2, sig2, Z, alpha=alpha, U=U)
    # scale: sum_ij |dA_ij| |w_ij| for each parameter
    W_abs = np.abs(np.outer(alpha, alpha)) + np.abs(U) @ np.abs(Z).T / 16
    scales = [0.5 * np.sum(np.abs(D) * W_abs) for D in OG.dA_list(Xr, kern, ell, s2, sig2)]
    for j in range(3):
        assert abs(g[j] - ref[j]) <= 2e-5 * scales[j] + 1e-9, (j, g[j], ref[j], scales[j])


def test_mll_value_matches_oracle(lib):
    """dcg_mll_value: -1/2 y^T alpha - n/2 log 2 pi (- 1/2 log det A) summed
    by the library, against the oracle's exact log marginal likelihood (dense
    Cholesky, Rasmussen & Williams eq. 5.8) when fed the exact alpha and the
    exact log det, and the determinant term left out when none is given."""
    w = workloads.gp_hyper(n=1300)
    X, y = w["X"], w["y"]
    ell, s2, sig2 = math.exp(w["log_ell"]), 1.1, 0.2
    op = lib.Operator(_dev(X), 0, ell, s2, sig2, prec=3)
    A = OK.operator(X, 0, ell, s2, sig2)
    alpha = np.linalg.solve(A, y)
    ld = np.linalg.slogdet(A)[1]
    ref = OG.lml(X, y, 0, ell, s2, sig2)
    v = lib.mll_value(op, _dev(y), _dev(alpha), logdet=ld)
    assert v == pytest.approx(ref, rel=1e-12, abs=1e-9)
    v0 = lib.mll_value(op, _dev(y), _dev(alpha))
    assert v0 - v == pytest.approx(0.5 * ld, rel=1e-12, abs=1e-9)
    with pytest.raises(lib.DcgError) as e:
        lib.mll_value(op, _dev(y), _dev(alpha), logdet=float("nan"))
    assert e.value.status == -1


def test_mll_backward_after_another_forward(lib):
    """The backward of a forward at theta_a, taken after a second forward at
    theta_b moved the operator: it runs at theta_a (the operator is set back
    to the first forward's hyperparameters), so it gives the gradient of a
    lone forward/backward at theta_a (to the probe solves' tolerance), not
    theta_b's."""
    w = workloads.gp_hyper(n=1500)
    X, y = w["X"], w["y"]
    Z = _dev(workloads.rademacher(1500, 16, step=2))
    th_a = [w["log_ell"], 0.0, math.log(0.1)]
    th_b = [w["log_ell"] + 0.3, 0.2, math.log(0.05)]

    def fresh():
        op = lib.Operator(_dev(X), 0, 1.0, 1.0, 0.1, prec=0)
        return lib.GPContext(op, _dev(y), lib.Recycle(1500, 16, 24), Z, tol=1e-8)

    def grad_alone(th):
        t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        lib.GPMarginalLikelihood.apply(t, fresh()).backward()
        return t.grad.numpy().copy()

    g_a, g_b = grad_alone(th_a), grad_alone(th_b)
    gpc = fresh()
    ta = torch.tensor(th_a, dtype=torch.float64, requires_grad=True)
    tb = torch.tensor(th_b, dtype=torch.float64, requires_grad=True)
    va = lib.GPMarginalLikelihood.apply(ta, gpc)
    lib.GPMarginalLikelihood.apply(tb, gpc)          # moves the operator to theta_b
    va.backward()
    g = ta.grad.numpy()
    # the probe solves start from different recycled bases, so they agree to
    # the solver tolerance on the FP32 operator (as GPU vs oracle elsewhere)
    np.testing.assert_allclose(g, g_a, rtol=1e-4, atol=1e-4 * np.abs(g_a).max())
    assert np.abs(g - g_b).max() > 1e-2 * np.abs(g_a).max()
    # the operator is at theta_a again
    assert gpc.op.ell == pytest.approx(math.exp(th_a[0]), rel=1e-15)


def test_mll_autograd_against_exact_gradient(lib):
    """torch.autograd.Function: the backward (probe solves reusing W, fused
    sweep) against the oracle's exact dense gradient within the Hutchinson
    error, and the forward value against the oracle's data-fit term."""
    w = workloads.gp_hyper(n=2048)
    X, y = w["X"], w["y"]
    op = lib.Operator(_dev(X), 0, 1.0, 1.0, 0.1, prec=0)
    rc = lib.Recycle(2048, 16, 24)
    theta = torch.tensor([w["log_ell"], 0.0, math.log(0.1)], dtype=torch.float64,
                         requires_grad=True)
    Z = workloads.rademacher(2048, 16, step=1)
    gpc = lib.GPContext(op, _dev(y), rc, _dev(Z), tol=1e-8)
    # two evaluations: the second one starts from a recycled W
    for _ in range(2):
        theta.grad = None
        val = lib.GPMarginalLikelihood.apply(theta, gpc)
        val.backward()
    assert gpc.last["probe_stats"]["k_used"] == 16
    ell, s2, sig2 = (math.exp(v) for v in theta.detach().tolist())
    Xr = OP.round_points(X, 0, 0, ell)
    exact = OG.lml_grad_exact(Xr, y, 0, ell, s2, sig2)
    hut = OG.lml_grad_hutchinson(Xr, y, 0, ell, s2, sig2, Z)
    g = theta.grad.numpy()
    # GPU vs the oracle's estimator with the same probes: solver tolerance level
    np.testing.assert_allclose(g, hut, rtol=1e-4, atol=1e-4 * np.abs(hut).max())
    # the estimator vs the exact gradient: within 4 standard errors
    A = OK.operator(Xr, 0, ell, s2, sig2)
    U = np.linalg.solve(A, Z)
    for j, D in enumerate(OG.dA_list(Xr, 0, ell, s2, sig2)):
        samples = 0.5 * np.sum(U * (D @ Z), axis=0)
        se = samples.std(ddof=1) / math.sqrt(Z.shape[1])
        assert abs(g[j] - exact[j]) <= 4 * se + 1e-6 * abs(exact[j]), (j, g[j], exact[j], se)
    # forward value: -1/2 y^T alpha - n/2 log 2 pi
    alpha = np.linalg.solve(A, y)
    assert float(val) == pytest.approx(-0.5 * y @ alpha - 0.5 * 2048 * math.log(2 * math.pi), rel=1e-6)
    # exact gradient pinned by finite differences of the exact LML
    h = 1e-5
    th = np.log([ell, s2, sig2])
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fp = OG.lml(Xr, y, 0, *np.exp(th + e))
        fm = OG.lml(Xr, y, 0, *np.exp(th - e))
        assert exact[j] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-6)


def test_mll_grad_full_size_differentiation_workload(lib):
    """The differentiation form at its stated size (n = 32768, d = 16, RBF,
    16 Rademacher probes, k = 32): the solves alpha = A^{-1} y and
    U = A^{-1} Z with recycling, then the fused gradient sweep against the
    oracle's row-blocked Hutchinson gradient on the same alpha, U and probes
    (FP32-rounded points), to the product tolerance of the small-size test."""
    w = workloads.gp_hyper()
    X, y = w["X"], w["y"]
    n = X.shape[0]
    ell, s2, sig2 = math.exp(w["log_ell"]), math.exp(w["log_s2"]), math.exp(w["log_sigma2"])
    op = lib.Operator(_dev(X), 0, ell, s2, sig2, prec=0)
    rc = lib.Recycle(n, w["k"], w["L"])
    alpha, st = lib.solve(op, _dev(y), rc=rc, tol=w["tol"], true_residual=True)
    assert st["status"] == 0 and st["k_next"] == w["k"]
    Z = workloads.rademacher(n, w["probes"], step=0)
    U, stb = lib.solve_block(op, _dev(Z), rc=rc, tol=w["tol"])
    assert stb["status"] == 0 and stb["k_used"] == w["k"]
    g = np.array(lib.mll_grad(op, alpha, U, _dev(Z)))
    print("full-size gradient", g, "alpha its", st["iters"], "probe its", stb["iters"], flush=True)
    ref, scale = OG.lml_grad_hutchinson_blocked(OP.round_points(X, 0, 0, ell), 0, ell, s2, sig2, _np(alpha),
                                                _np(U), Z, with_scale=True)
    for j in range(3):
        assert abs(g[j] - ref[j]) <= 2e-5 * scale[j] + 1e-9, (j, g[j], ref[j], scale[j])
