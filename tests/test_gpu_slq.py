"""GPU parity of the SLQ log-determinant (probe solves through the block CG,
Lanczos tridiagonals from their coefficients, host quadrature) against the
oracle's z^T log(A) z.

Per-probe bound: the quadrature of a converged CG is z^T log(A) z to ~1e-9
relative (oracle pins); the GPU run takes its own step count, so both are
compared with the dense eigendecomposition: 1e-7 relative for the FP64
operator (tol 1e-10), 1e-5 for FP32 operands (tol 1e-8; the operator's 1e-7
evaluation error moves log(A) by about that relative to its norm).
"""

import numpy as np
import pytest

from oracle import kernels as OK
from oracle import precision as OP
from oracle import slq as OS
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("prec,tol,rtol", [(3, 1e-10, 1e-7), (0, 1e-8, 1e-5)])
def test_slq_probe_values_match_dense(lib, prec, tol, rtol):
    w = workloads.small(n=1100)
    X = w["X"]
    n = X.shape[0]
    ell = w["ells"][0]
    Xr = OP.round_points(X, prec, w["kernel"], ell)
    A = OK.operator(Xr, w["kernel"], ell, 1.0, w["sigma2"])
    Z = workloads.rademacher(n, 6, step=0)
    op = lib.Operator(_dev(X), w["kernel"], ell, 1.0, w["sigma2"], prec=prec)
    est, quad, steps = lib.slq_logdet(op, _dev(Z), tol=tol, max_steps=2048)
    lam, V = np.linalg.eigh(A)
    ref = np.array([Z[:, p] @ (V @ (np.log(lam) * (V.T @ Z[:, p]))) for p in range(6)])
    np.testing.assert_allclose(quad, ref, rtol=rtol)
    assert abs(est - np.mean(quad)) <= 1e-12 * abs(est)
    # the oracle's own quadrature of the same probe
    o, o_steps = OS.probe_value(A, Z[:, 0], tol=tol)
    assert abs(quad[0] - o) <= rtol * abs(o)
    assert all(s > 0 for s in steps)


def test_slq_unit_probes_sum_to_logdet(lib):
    """Unit probes over all n coordinates: the quadratures add up to log det A
    (Gauss quadrature exact for the Krylov space), n = 96 in 2 blocks of 48."""
    g = np.random.default_rng(4)
    n = 96
    X = g.standard_normal((n, 3))
    op = lib.Operator(_dev(X), 0, 1.5, 1.0, 0.1, prec=3)
    A = OK.operator(X, 0, 1.5, 1.0, 0.1)
    total = 0.0
    for c0 in (0, 48):
        _, quad, _ = lib.slq_logdet(op, _dev(np.eye(n)[:, c0:c0 + 48]), tol=1e-13)
        total += sum(quad)
    ref = np.linalg.slogdet(A)[1]
    assert abs(total - ref) <= 1e-8 * abs(ref), (total, ref)


def test_slq_scaling_property_full_size(lib):
    """At the differentiation form's size (n = 32768, FP32 operands, 16
    Rademacher probes): doubling s2 and sigma2 doubles A exactly, so every
    probe's value moves by |z|^2 log 2 = n log 2 (CG's alphas halve, the
    betas and the steps stay)."""
    w = workloads.gp_hyper()
    X = w["X"]
    n = X.shape[0]
    ell, s2, sigma2 = np.exp(w["log_ell"]), 1.0, np.exp(w["log_sigma2"])
    Z = workloads.rademacher(n, 16, step=0)
    op = lib.Operator(_dev(X), w["kernel"], ell, s2, sigma2, prec=0)
    e1, q1, st1 = lib.slq_logdet(op, _dev(Z), tol=1e-6)
    op.set_hyper(ell, 2 * s2, 2 * sigma2)
    e2, q2, st2 = lib.slq_logdet(op, _dev(Z), tol=1e-6)
    assert st1 == st2
    np.testing.assert_allclose(np.array(q2) - np.array(q1), n * np.log(2.0), rtol=1e-9)
    assert abs((e2 - e1) - n * np.log(2.0)) <= 1e-9 * n


def test_slq_rejects_bad_arguments(lib):
    X = np.random.default_rng(0).standard_normal((100, 2))
    op = lib.Operator(_dev(X), 0, 1.0, 1.0, 0.1, prec=0)
    with pytest.raises(lib.DcgError):
        lib.slq_logdet(op, _dev(np.ones((100, 65))))        # more than 64 probes
    with pytest.raises(lib.DcgError):
        lib.slq_logdet(op, _dev(np.ones((100, 2))), max_steps=0)
    # a diagonal scaling on a low-precision operator: the four-column sweep
    # takes none
    op.set_diag(_dev(np.full(100, 0.5)))
    with pytest.raises(lib.DcgError):
        lib.slq_logdet(op, _dev(np.ones((100, 2))))


def test_marginal_likelihood_value_with_logdet(lib):
    """GPContext(logdet=True): the forward value is -1/2 y^T A^{-1} y
    - 1/2 (SLQ log det) - n/2 log 2 pi, the SLQ term matching the mean of the
    probes' dense z^T log(A) z."""
    import math
    w = workloads.small(n=900)
    X = w["X"]
    n = X.shape[0]
    ell, s2, sigma2 = 1.1, 1.3, 0.05
    y = np.random.default_rng(8).standard_normal(n)
    Z = workloads.rademacher(n, 8, step=1)
    op = lib.Operator(_dev(X), w["kernel"], ell, s2, sigma2, prec=3)
    rc = lib.Recycle(n, 8, 12)
    ctx = lib.GPContext(op, _dev(y), rc, _dev(Z), tol=1e-11, logdet=True)
    theta = torch.tensor([math.log(ell), math.log(s2), math.log(sigma2)], dtype=torch.float64)
    val = float(lib.GPMarginalLikelihood.apply(theta, ctx))
    A = OK.operator(X, w["kernel"], ell, s2, sigma2)
    lam, V = np.linalg.eigh(A)
    ld = np.mean([Z[:, p] @ (V @ (np.log(lam) * (V.T @ Z[:, p]))) for p in range(8)])
    ref = -0.5 * y @ np.linalg.solve(A, y) - 0.5 * ld - 0.5 * n * math.log(2 * math.pi)
    assert abs(ctx.last["logdet"] - ld) <= 1e-7 * abs(ld)
    assert abs(val - ref) <= 1e-7 * abs(ref), (val, ref)
