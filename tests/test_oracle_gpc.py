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
