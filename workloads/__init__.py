"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws points,
right-hand sides, hyperparameter sequences and probe vectors.  Both the GPU
path's callers and the oracle's callers take their inputs from here; neither
side imports the other.

Workloads (kernel-regression systems A = K_theta(X, X) + sigma^2 I):

* ``small``      n=1024, d=8, X ~ N(0,1), RBF, ell_i = 1.05^i, sigma2 = 1e-2,
                 b_i = A_i x* + N(0, 1e-4) (x* ~ N(0,1)), 5 systems.  The
                 right-hand sides need A_i x*, so the caller supplies a matvec.
* ``fp32_walk``  n=16384, d=16, X ~ N(0,1) in fp32, RBF, sigma2 = 1e-2,
                 ell_0 = median pairwise distance, log-ell random walk with
                 step 0.05, fixed b ~ N(0,1), 20 systems.
* ``bf16_shift`` n=65536, d=32, X ~ U[-1,1], Matern-5/2, ell = 0.5 x median
                 pairwise distance (literal variant: ell = 0.5),
                 sigma2_i = 1e-3 * 0.9^i, fixed b ~ N(0,1), 10 systems.
* ``gp_hyper``   n=32768, d=16, X ~ N(0,1), y = sum_c a_c sin(X w_c) + 0.1 eps,
                 RBF, Rademacher probes.
* ``gpc``        Laplace GP classification (the systems A = I + D K D of the
                 Newton iteration): n=36551 points in d=64, two classes of
                 6 Gaussian modes each (centres ~ N(0, I), spread 0.7), 5%
                 of the labels flipped, RBF, ell = 0.5 x median pairwise
                 distance, s2 = 100; a stand-in for the 3-vs-5 digits set.
* ``gpc_pixels`` the same classification loop on paper-shaped data: n=36551
                 "images" of 28 x 28 = 784 pixels in (0, 1), x = logistic(3 B z
                 - 2) with z ~ N(0, I_16) and B 16 Gaussian blobs (centres
                 U[4, 24]^2, widths U[2, 5] pixels), labels the sign of a
                 smooth random function of z (sum of 3 sines), RBF, ell =
                 0.5 x median distance, s2 = 10.
* ``ragged``     64 sequences, n log-uniform in [2048, 32768], d=8, RBF or
                 Matern-3/2 (fair coin), sigma2 log-uniform [1e-4, 1e-1],
                 ell_0 = median heuristic, log-ell walk 0.05, 5 systems each.

Every generator takes the size as an argument so that tests can draw the same
structure at small n.  Seeds: numpy default_rng(170600241 + workload index).
"""

import numpy as np

SEED_BASE = 170600241
RBF, MATERN32, MATERN52 = 0, 1, 2


def rng(index, extra=0):
    return np.random.default_rng(SEED_BASE + index + 1000 * extra)


def median_distance(X, sample=2048, seed=0):
    """Median pairwise Euclidean distance of a random subsample of X (the
    'median heuristic' used to pick a lengthscale for the synthetic data)."""
    X = np.asarray(X, dtype=np.float64)
    g = np.random.default_rng(seed)
    idx = g.choice(X.shape[0], size=min(sample, X.shape[0]), replace=False)
    S = X[idx]
    sq = (S * S).sum(1)
    D2 = np.maximum(sq[:, None] + sq[None, :] - 2 * S @ S.T, 0.0)
    iu = np.triu_indices(S.shape[0], 1)
    return float(np.median(np.sqrt(D2[iu])))


def small(n=1024, d=8, systems=5):
    """Points, lengthscales, sigma2, x* and the noise to add to A_i x*."""
    g = rng(0)
    X = g.standard_normal((n, d))
    xstar = g.standard_normal(n)
    noise = 1e-2 * g.standard_normal((systems, n))   # variance 1e-4
    ells = [1.0 * 1.05 ** i for i in range(systems)]
    return dict(X=X, kernel=RBF, ells=ells, s2=1.0, sigma2=1e-2, xstar=xstar,
                noise=noise, k=8, L=12, tol=1e-8)


def fp32_walk(n=16384, d=16, systems=20):
    g = rng(1)
    X = g.standard_normal((n, d)).astype(np.float32).astype(np.float64)
    b = g.standard_normal(n)
    ell0 = median_distance(X)
    steps = g.standard_normal(systems)
    steps[0] = 0.0
    ells = list(ell0 * np.exp(0.05 * np.cumsum(steps)))
    return dict(X=X, kernel=RBF, ells=ells, s2=1.0, sigma2=1e-2, b=b, k=32,
                L=48, tol=1e-6)


def bf16_shift(n=65536, d=32, systems=10, literal=False):
    g = rng(2)
    X = g.uniform(-1.0, 1.0, (n, d))
    b = g.standard_normal(n)
    ell = 0.5 if literal else 0.5 * median_distance(X)
    sigma2s = [1e-3 * 0.9 ** i for i in range(systems)]
    return dict(X=X, kernel=MATERN52, ell=ell, s2=1.0, sigma2s=sigma2s, b=b,
                k=64, L=96, tol=1e-8, inner_tol=1e-4)


def gp_hyper(n=32768, d=16, probes=16, components=4):
    g = rng(3)
    X = g.standard_normal((n, d))
    a = g.standard_normal(components)
    Wc = g.standard_normal((d, components)) / np.sqrt(d)
    y = np.sin(X @ Wc) @ a + 0.1 * g.standard_normal(n)
    return dict(X=X, y=y, kernel=RBF, log_ell=np.log(median_distance(X)),
                log_s2=0.0, log_sigma2=np.log(0.1), probes=probes, k=32, L=48,
                tol=1e-6, lr=0.05)


def gpc(n=36551, d=64, modes=6, spread=0.7, flip=0.05):
    """Two-class point cloud and labels in {-1, +1} for Laplace GPC."""
    g = rng(5)
    centres = g.standard_normal((2, modes, d))
    cls = (g.random(n) < 0.5).astype(np.int64)
    mode = g.integers(modes, size=n)
    X = centres[cls, mode] + spread * g.standard_normal((n, d))
    y = np.where(cls == 1, 1.0, -1.0)
    y[g.random(n) < flip] *= -1.0
    return dict(X=X, y=y, kernel=RBF, ell=0.5 * median_distance(X), s2=100.0,
                k=8, L=12, tol=1e-5, psi_tol=1.0)


def gpc_pixels(n=36551, side=28, latent=16):
    """Pixel-like points in (0, 1)^(side^2) and labels in {-1, +1}."""
    g = rng(6)
    yy, xx = np.mgrid[0:side, 0:side]
    P = np.stack([yy.ravel(), xx.ravel()], 1).astype(np.float64)
    C = g.uniform(4.0, side - 4.0, (latent, 2))
    width = g.uniform(2.0, 5.0, latent)
    B = np.exp(-((P[:, None, :] - C[None]) ** 2).sum(-1) / (2.0 * width ** 2))
    Z = g.standard_normal((n, latent))
    X = 1.0 / (1.0 + np.exp(-(3.0 * Z @ B.T - 2.0)))
    Wc = g.standard_normal((latent, 3)) / np.sqrt(latent)
    a = g.standard_normal(3)
    y = np.where(np.sin(2.0 * Z @ Wc) @ a >= 0.0, 1.0, -1.0)
    return dict(X=X, y=y, kernel=RBF, ell=0.5 * median_distance(X), s2=10.0,
                k=8, L=12, tol=1e-5, psi_tol=1.0)


def rademacher(n, P, step, index=3):
    """Probe matrix (n x P, entries +-1) for optimisation step ``step``."""
    g = rng(index, extra=1 + step)
    return np.where(g.random((n, P)) < 0.5, -1.0, 1.0)


def ragged(count=64, d=8, systems=5, n_min=2048, n_max=32768):
    g = rng(4)
    seqs = []
    for s in range(count):
        n = int(round(np.exp(g.uniform(np.log(n_min), np.log(n_max)))))
        X = g.standard_normal((n, d))
        kernel = RBF if g.random() < 0.5 else MATERN32
        sigma2 = float(np.exp(g.uniform(np.log(1e-4), np.log(1e-1))))
        b = g.standard_normal(n)
        ell0 = median_distance(X, sample=1024, seed=s)
        steps = g.standard_normal(systems)
        steps[0] = 0.0
        ells = list(ell0 * np.exp(0.05 * np.cumsum(steps)))
        seqs.append(dict(X=X, kernel=kernel, sigma2=sigma2, b=b, ells=ells,
                         s2=1.0))
    return dict(seqs=seqs, k=16, L=24, tol=1e-6)


def spd_with_spectrum(eigs, seed=7):
    """Dense SPD matrix Q diag(eigs) Q^T with a random orthogonal Q (for
    exact-eigenvector deflation tests)."""
    g = np.random.default_rng(SEED_BASE + seed)
    n = len(eigs)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    return (Q * np.asarray(eigs)[None, :]) @ Q.T, Q
