"""Pins of the SLQ log-determinant oracle: exact results where the
quadrature is exact, an independent Lanczos run, and the per-probe value
z^T log(A) z from a dense eigendecomposition."""

import numpy as np

from oracle import slq as S
import workloads


def _spd(n, cond, seed=7):
    eigs = np.geomspace(1.0, cond, n)
    A, _ = workloads.spd_with_spectrum(eigs, seed=seed)
    return A, eigs


def test_diagonal_unit_probes_exact():
    """A diagonal, z = e_i: CG stops after one step with alpha = 1 / a_ii, T =
    [a_ii], so the probe value is log a_ii and the unit probes sum to log det."""
    a = np.array([0.5, 2.0, 7.0, 1e3])
    A = np.diag(a)
    vals = [S.probe_value(A, np.eye(4)[:, i])[0] for i in range(4)]
    np.testing.assert_allclose(vals, np.log(a), rtol=1e-14)


def test_unit_probes_sum_to_logdet():
    """Gauss quadrature with as many nodes as A has eigenvalues in the Krylov
    space is exact: the unit probes' values add up to log det A."""
    A, eigs = _spd(30, 50.0)
    total = sum(S.probe_value(A, np.eye(30)[:, i], tol=1e-14)[0] for i in range(30))
    assert abs(total - np.sum(np.log(eigs))) <= 1e-8 * abs(np.sum(np.log(eigs)))


def test_tridiagonal_matches_explicit_lanczos():
    """T from the CG coefficients equals the tridiagonal of an explicit
    Lanczos run with full reorthogonalisation (up to the signs of the
    off-diagonal, which e_1^T f(T) e_1 does not see)."""
    A, _ = _spd(80, 1e3, seed=3)
    z = np.random.default_rng(1).standard_normal(80)
    al, be = S.cg_coefficients(A, z, tol=1e-30, max_iter=12)
    T = S.lanczos_from_cg(al, be)
    m = T.shape[0]
    Q = np.zeros((80, m + 1))
    Q[:, 0] = z / np.linalg.norm(z)
    a = np.zeros(m)
    b = np.zeros(m)
    for j in range(m):
        w = A @ Q[:, j]
        a[j] = Q[:, j] @ w
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        b[j] = np.linalg.norm(w)
        Q[:, j + 1] = w / b[j]
    np.testing.assert_allclose(np.diag(T), a, rtol=1e-9)
    np.testing.assert_allclose(np.abs(np.diag(T, 1)), b[:m - 1], rtol=1e-9)


def test_probe_value_converges_to_dense():
    """For a Rademacher probe the quadrature after CG to 1e-10 equals
    z^T log(A) z from the dense eigendecomposition (also past n steps, where
    finite-precision CG has lost orthogonality: the repeated Ritz values it
    then carries share the weight of the eigenvalue they copy)."""
    A, _ = _spd(200, 1e4, seed=5)
    w, V = np.linalg.eigh(A)
    g = np.random.default_rng(2)
    for _ in range(4):
        z = np.where(g.random(200) < 0.5, -1.0, 1.0)
        ref = z @ (V @ (np.log(w) * (V.T @ z)))
        val, steps = S.probe_value(A, z, tol=1e-10)
        assert abs(val - ref) <= 1e-8 * abs(ref), (val, ref)
