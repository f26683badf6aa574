"""Gaussian process classification by the Laplace approximation: Newton's
method for the mode of the latent function (the paper's own test problem,
section 3, and its linear system after the restructuring of Kuss &
Rasmussen, the equations for b^(i) and A^(i) there).

Test infrastructure only (see ``oracle/__init__``).

Labels y_i in {-1, +1}, logistic likelihood p(y_i | f_i) = 1 / (1 + e^{-y_i f_i}).
With t = (y + 1) / 2 and pi = sigma(f) = 1 / (1 + e^{-f}):
    grad log p(y | f) = t - pi,     H = -grad grad log p(y | f) = diag(pi (1 - pi)).
One Newton step from f (D = H^(1/2)):
    b~ = H f + grad log p,
    A  = I + D K D,        b = D K b~,        z = A^{-1} b,
    a  = b~ - D z,         f_new = K a,
and f_new is the Newton iterate (K^{-1} + H)^{-1} b~.  The objective, up to
the terms that do not depend on f, is Psi(f) = log p(y | f) - a^T f / 2
(f^T K^{-1} f = a^T f for f = K a); the iteration stops when Psi grows by
less than psi_tol (the paper uses 1).
"""

import numpy as np


def log_lik(y, f):
    """sum_i log sigma(y_i f_i), computed as -log(1 + e^{-y f}) stably."""
    z = np.asarray(y, dtype=np.float64) * np.asarray(f, dtype=np.float64)
    return float(-np.sum(np.logaddexp(0.0, -z)))


def newton_terms(y, f):
    """(pi, H diagonal, grad log p) at f."""
    pi = 1.0 / (1.0 + np.exp(-np.asarray(f, dtype=np.float64)))
    t = 0.5 * (np.asarray(y, dtype=np.float64) + 1.0)
    return pi, pi * (1.0 - pi), t - pi


def newton_system(K, y, f):
    """A = I + D K D, b = D K b~ and the pieces to finish the step."""
    _, H, g = newton_terms(y, f)
    D = np.sqrt(H)
    bt = H * f + g
    A = np.eye(len(f)) + D[:, None] * K * D[None, :]
    b = D * (K @ bt)
    return A, b, D, bt


def laplace_mode(K, y, solve=None, psi_tol=1.0, max_newton=50, f0=None):
    """Newton's method for the Laplace mode.  ``solve(A, b)`` solves each
    system (default: a dense solve).  Returns (f, a, list of Psi, list of
    (A, b) systems solved)."""
    n = len(y)
    f = np.zeros(n) if f0 is None else np.asarray(f0, dtype=np.float64).copy()
    solve = solve or np.linalg.solve
    a = np.zeros(n)
    psi = [log_lik(y, f) - 0.5 * (a @ f)]
    systems = []
    for _ in range(max_newton):
        A, b, D, bt = newton_system(K, y, f)
        z = solve(A, b)
        systems.append((A, b))
        a = bt - D * z
        f = K @ a
        psi.append(log_lik(y, f) - 0.5 * (a @ f))
        if psi[-1] - psi[-2] < psi_tol:
            break
    return f, a, psi, systems


def log_evidence(K, y, f, a):
    """The Laplace approximation to log p(y | X) at the mode f (f = K a):
    Psi(f) - 1/2 log det(I + D K D), D = H^(1/2) (the third term of the
    objective whose first two terms stop the Newton loop)."""
    _, H, _ = newton_terms(y, f)
    D = np.sqrt(H)
    B = np.eye(len(f)) + D[:, None] * np.asarray(K) * D[None, :]
    sign, logdet = np.linalg.slogdet(B)
    assert sign > 0
    psi = log_lik(y, f) - 0.5 * (np.asarray(a) @ np.asarray(f))
    return psi - 0.5 * logdet, psi, logdet
