"""CPU emulation of deflated CG with inexact products (no GPU).

The library multiplies with a low-precision operator (FP32 or bf16 points,
FP32 kernel values) and re-projects the residual against W after every step
(``oracle.cg.defcg(reproject=True)``), which Algorithm 1 does not do.  These
tests pin what that choice rests on, with the oracle's dense FP64 matrix and
the per-term error model of ``emulation``:

* with exact products the re-projection changes nothing (the same iterates
  to rounding, the same step counts);
* with inexact products the literal Algorithm 1 loses W^T r_j = 0 and stops
  converging, while the re-projecting iteration converges;
* the step-count inflation the error causes at the FP32 level, which the GPU
  tests' bands on iteration counts are drawn from.
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


def _system(sigma2, prec=3, n=800):
    """An RBF system with a spread spectrum (kappa 4.9e4 at sigma2 = 1e-2,
    4.9e5 at 1e-3) and a recycled basis from a previous solve's harmonic Ritz
    extraction (the basis a sequence carries, not exact eigenvectors)."""
    X = np.random.default_rng(21).standard_normal((n, 4))
    ell = workloads.median_distance(X)
    A = OK.operator(OP.round_points(X, prec, 0, ell), 0, ell, 1.0, sigma2)
    prev = OC.cg(A, np.random.default_rng(4).standard_normal(n), tol=1e-10, L=24)
    W, AW, _, _ = ORZ.harmonic_ritz(prev.P, prev.AP, 8)
    b = np.random.default_rng(3).standard_normal(n)
    return A, W, AW, b


@pytest.mark.parametrize("sigma2", [1e-2, 1e-3])
def test_reprojection_is_algorithm1_with_exact_products(sigma2):
    A, W, AW, b = _system(sigma2)
    lit = OC.defcg(A, b, W=W, AW=AW, tol=1e-8, store_all=True)
    rep = OC.defcg(A, b, W=W, AW=AW, tol=1e-8, store_all=True, reproject=True)
    assert lit.converged and rep.converged
    assert abs(lit.iters - rep.iters) <= 1, (lit.iters, rep.iters)
    x = np.linalg.solve(A, b)
    for r in (lit, rep):
        err = np.sqrt((r.x - x) @ A @ (r.x - x) / (x @ A @ x))
        assert err <= 1e-7
    # the first steps agree to rounding, column by column
    for j in range(12):
        assert np.linalg.norm(rep.all_r[:, j] - lit.all_r[:, j]) <= \
            1e-9 * np.linalg.norm(lit.all_r[:, j]), j

    def wtr(R):
        return np.abs(W.T @ R).max(axis=0) / (np.linalg.norm(W, axis=0).max()
                                               * np.linalg.norm(R, axis=0))
    # even with FP64 products the literal iteration's W^T r_j / |r_j| grows
    # geometrically from rounding level; the re-projected one stays there
    assert wtr(lit.all_r)[-1] >= 1e-5 and wtr(lit.all_r)[1] <= 1e-10
    assert wtr(rep.all_r).max() <= 1e-14


def test_algorithm1_stalls_with_inexact_products_reprojection_converges():
    """Per-term product error 1e-8 (well below FP32 evaluation), kappa 4.9e4:
    the literal Algorithm 1 lets W^T r_j grow until the recursive residual
    stops falling (no convergence in 20x the exact count), the re-projecting
    iteration converges with a bounded delay."""
    A, W, AW, b = _system(1e-2)
    exact = OC.defcg(A, b, W=W, AW=AW, tol=1e-8).iters
    for seed in range(3):
        lit = OC.defcg(noisy_product(A, 1e-8, seed), b, W=W, AW=AW, tol=1e-8,
                       max_iter=20 * exact, store_all=True)
        assert not lit.converged, (seed, lit.iters)
        rel_WtR = np.abs(W.T @ lit.all_r[:, -1]).max() / np.linalg.norm(lit.all_r[:, -1])
        assert rel_WtR > 1e-3
        rep = OC.defcg(noisy_product(A, 1e-8, seed), b, W=W, AW=AW, tol=1e-8,
                       max_iter=20 * exact, reproject=True)
        assert rep.converged and rep.iters <= 1.6 * exact, (seed, rep.iters, exact)


def test_fp32_level_inflation_of_the_n1024_sequence():
    """The n = 1024 five-system sequence with FP32-rounded points, def-CG(8,
    12), tol 1e-6, solved with per-term product errors of 1e-7 and 3e-7 (the
    FP32 operator measures below 1e-7, see the GPU tests) over four seeds:
    every system needs at least its exact count minus 1 and at most 15% more
    than it.  This is the band the GPU sequence test draws."""
    w = workloads.small()
    X = w["X"]
    mats = [OK.operator(OP.round_points(X, 0, w["kernel"], ell), w["kernel"], ell, 1.0,
                        w["sigma2"]) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i] for i, A in enumerate(mats)]
    exact = [r.iters for r in OS.solve_sequence(mats, bs, k=8, L=12, tol=1e-6, reproject=True)]
    literal = [r.iters for r in OS.solve_sequence(mats, bs, k=8, L=12, tol=1e-6)]
    assert all(abs(a - c) <= 1 for a, c in zip(exact, literal)), (exact, literal)
    worst = 0.0
    for eta in (1e-7, 3e-7):
        for seed in range(4):
            mv = [noisy_product(A, eta, 100 * seed + i) for i, A in enumerate(mats)]
            its = [r.iters for r in OS.solve_sequence(mv, bs, k=8, L=12, tol=1e-6, reproject=True)]
            for a, c in zip(its, exact):
                assert c - 1 <= a <= 1.15 * c, (eta, seed, its, exact)
                worst = max(worst, a / c)
    assert worst > 1.05     # the delay is real, not an artefact of the bound


def test_rounding_level_spread_of_counts_at_kappa_5e5():
    """kappa 4.9e5 in FP64: a per-term error of 3e-16 (one rounding of each
    product term) moves the step counts of deflated and plain CG by several
    steps either way around the exact ones, so two correct FP64
    implementations that round differently need not agree step for step
    there; the GPU tests compare against such a band."""
    A, W, AW, b = _system(1e-3)
    ex = OC.defcg(A, b, W=W, AW=AW, tol=1e-8, reproject=True).iters
    exp = OC.cg(A, b, tol=1e-8).iters
    d = [OC.defcg(noisy_product(A, 3e-16, s), b, W=W, AW=AW, tol=1e-8, reproject=True).iters
         for s in range(6)]
    p = [OC.cg(noisy_product(A, 3e-16, s), b, tol=1e-8).iters for s in range(6)]
    assert max(d) - min(d) >= 2 and max(p) - min(p) >= 4, (d, p)
    assert max(abs(v - ex) for v in d) <= 0.05 * ex
    assert max(abs(v - exp) for v in p) <= 0.05 * exp


def test_fit_eta_recovers_the_model():
    """fit_eta inverts the error model: products drawn with eta give eta back."""
    A, _, _, _ = _system(1e-2, n=400)
    v = np.random.default_rng(9).standard_normal(400)
    for eta in (1e-15, 1e-7):
        y = noisy_product(A, eta, 3)(v)
        assert fit_eta(A, v, y) == pytest.approx(eta, rel=0.15)
