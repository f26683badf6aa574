"""Pins of the Laplace GPC oracle against the textbook Newton step and the
mode condition, not against a retyped copy of its own formulas."""

import numpy as np

from oracle import gpc as G
from oracle import kernels as K
import workloads


def _problem(n=150, d=3, seed=3):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d))
    y = np.sign(np.sin(X @ g.standard_normal(d)) + 0.1 * g.standard_normal(n))
    y[y == 0] = 1.0
    # a prior covariance with a 0.1 I term, so that K^{-1} (used by the
    # textbook Newton step below) is well conditioned
    Km = K.gram(X, K.RBF, workloads.median_distance(X), 2.0) + 0.1 * np.eye(n)
    return Km, y


def test_restructured_step_is_the_newton_step():
    """The step through A = I + D K D equals the plain Newton iterate
    f_new = f + (K^{-1} + H)^{-1} grad Psi(f), grad Psi = grad log p - K^{-1} f,
    formed by an explicit inverse."""
    Km, y = _problem()
    f = np.random.default_rng(1).standard_normal(len(y))
    A, b, D, bt = G.newton_system(Km, y, f)
    a = bt - D * np.linalg.solve(A, b)
    f_new = Km @ a
    _, H, g = G.newton_terms(y, f)
    Kinv = np.linalg.inv(Km)
    grad = g - Kinv @ f
    f_ref = f + np.linalg.solve(Kinv + np.diag(H), grad)
    np.testing.assert_allclose(f_new, f_ref, rtol=1e-9, atol=1e-9 * np.abs(f_ref).max())


def test_mode_condition_monotone_psi_and_spectrum():
    """At the returned mode f = K grad log p(y | f); Psi increases at every
    Newton step; the systems' eigenvalues lie in [1, 1 + n max K / 4]
    (the bound the restructuring guarantees)."""
    Km, y = _problem()
    f, a, psi, systems = G.laplace_mode(Km, y, psi_tol=1e-10)
    _, _, g = G.newton_terms(y, f)
    np.testing.assert_allclose(f, Km @ g, rtol=1e-6, atol=1e-8)
    assert np.all(np.diff(psi) > -1e-9)
    n = len(y)
    for A, _ in systems:
        lam = np.linalg.eigvalsh(A)
        assert lam.min() >= 1 - 1e-10 and lam.max() <= 1 + n * Km.max() / 4 + 1e-8


def test_log_lik_closed_form():
    y = np.array([1.0, -1.0, 1.0])
    f = np.array([0.0, 2.0, -30.0])
    ref = np.log(0.5) + np.log(1 / (1 + np.exp(2.0))) + np.log(1 / (1 + np.exp(30.0)))
    assert abs(G.log_lik(y, f) - ref) <= 1e-12


def test_laplace_evidence_matches_integral_one_point():
    """n = 1, prior N(0, k): the exact evidence is the integral of
    sigma(f) N(f; 0, k) df = 1/2 for every k (sigma(f) + sigma(-f) = 1 and the
    prior is symmetric).  The Laplace evidence approaches log 1/2 with an
    error of order k^2 (seen: 1.5e-6 at k = 0.01); without its log det term
    the error would be 1/2 log(1 + k/4) = 1.2e-3 at k = 0.01."""
    errs = []
    for k in (0.01, 0.03, 0.1):
        Km = np.array([[k]])
        y = np.array([1.0])
        f, a, _, _ = G.laplace_mode(Km, y, psi_tol=1e-14, max_newton=100)
        ev, _, _ = G.log_evidence(Km, y, f, a)
        errs.append(abs(ev - np.log(0.5)))
    assert errs[0] <= 2e-6
    # second order in k: the error grows like k^2 (seen 0.98 and 0.95 of it)
    for e0, e1, k0, k1 in ((errs[0], errs[1], 0.01, 0.03), (errs[1], errs[2], 0.03, 0.1)):
        assert 0.7 <= (e1 / e0) / (k1 / k0) ** 2 <= 1.3


def test_laplace_evidence_gaussian_limit():
    """At f = 0, a = 0 (pi = 1/2, H = 1/4): Psi = n log(1/2) and the
    determinant is that of I + K / 4, from its eigenvalues."""
    Km, y = _problem(n=40)
    f = np.zeros(40)
    ev, psi, ld = G.log_evidence(Km, y, f, np.zeros(40))
    ref_ld = np.sum(np.log(np.linalg.eigvalsh(np.eye(40) + Km / 4.0)))
    assert abs(psi - 40 * np.log(0.5)) <= 1e-12
    assert abs(ld - ref_ld) <= 1e-10 * abs(ref_ld)
