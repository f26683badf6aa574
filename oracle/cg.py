"""Plain CG and deflated CG, def-CG(k, L), in FP64.

Test infrastructure only (see ``oracle/__init__``).

Follows section 2.2 and Algorithm 1 of the paper (the deflated CG of Saad et
al. 2000).  With W empty the iteration is the method of conjugate gradients
(Hestenes & Stiefel) and the two functions below produce bitwise-identical
iterates: ``cg`` simply calls ``defcg`` with no W, which is the paper's own
statement that the first system of a sequence is solved by normal CG (Fig. 1
caption).

Readings of the paper used here:
* residual sign r = b - A x (Algorithm 1), not the gradient sign of Eq. 2;
* stopping test on the recursive relative residual |r_j|_2 / |b|_2 <= tol,
  checked before each iteration (the relative error of section 3);
* W^T A r_j is formed as (AW)^T r_j (A is symmetric), so each iteration costs
  one product with A;
* r_0 after the deflated start is r_{-1} - (AW) c, no extra product;
* the first L directions p_0 .. p_{L-1} are stored together with A p_j and
  the scalars of that step (P_L of section 2.3).

``reproject=True`` adds one step that Algorithm 1 does not have: after each
update of x and r, the component of r that W^T r_j = 0 excludes in exact
arithmetic is removed again, c = (W^T A W)^{-1} W^T r, x += W c, r -= (AW) c,
before rho, beta, mu and the next direction are formed.  In exact arithmetic
c = 0 and the iterates are Algorithm 1's; with rounding or inexact products
it keeps W^T r_j at rounding level instead of letting it grow.  The library
iterates this way; the literal Algorithm 1 stays the default here.

``A`` may be a dense matrix or a callable v -> A v.
"""

import numpy as np


def _as_matvec(A):
    if callable(A):
        return A
    A = np.asarray(A, dtype=np.float64)
    return lambda v: A @ v


class DefCGResult:
    """Iterate, residual history and the quantities stored for the extraction."""

    def __init__(self):
        self.x = None
        self.iters = 0          # number of CG steps (products A p_j)
        self.matvecs = 0        # all products with A, including set-up
        self.converged = False
        self.res_hist = []      # |r_j| / |b| for j = 0, 1, ...
        self.P = None           # n x L_eff stored directions p_0..p_{L_eff-1}
        self.AP = None          # n x L_eff, A p_j
        self.d = []             # d_j = p_j^T A p_j
        self.alpha = []
        self.beta = []
        self.mu = []            # mu_j (k-vectors), j = 0 .. L_eff
        self.rho = []           # rho_j = r_j^T r_j, j = 0 .. L_eff
        self.cvec = []          # re-projection coefficients c_{j+1}, j < L_eff
        self.p_next = None      # p_{L_eff}, the direction after the stored ones
        self.r_final = None


def defcg(A, b, x_init=None, W=None, AW=None, tol=1e-8, L=0, max_iter=None,
          store_all=False, reproject=False):
    """Deflated CG (Algorithm 1).  W (n x k) empty or None gives plain CG.

    Parameters
    ----------
    A        dense SPD matrix or callable
    b        right-hand side (n,)
    x_init   x_{-1} (zero if None)
    W, AW    recycled basis and its product with A (AW computed if None)
    tol      relative residual tolerance
    L        number of leading iterations whose directions are stored
    store_all  also keep every residual (for invariant tests)
    reproject  remove W^T r from r after every step (see the module notes)
    """
    mv = _as_matvec(A)
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    if max_iter is None:
        max_iter = 10 * n
    res = DefCGResult()
    bnorm = np.linalg.norm(b)
    x = np.zeros(n) if x_init is None else np.array(x_init, dtype=np.float64)
    if x_init is None:
        r = b.copy()
    else:
        r = b - mv(x)
        res.matvecs += 1

    deflate = W is not None and W.shape[1] > 0
    if deflate:
        W = np.asarray(W, dtype=np.float64)
        if AW is None:
            AW = np.column_stack([mv(W[:, c]) for c in range(W.shape[1])])
            res.matvecs += W.shape[1]
        M = W.T @ AW
        M = 0.5 * (M + M.T)
        Mc = np.linalg.cholesky(M)

        def msolve(h):
            return np.linalg.solve(Mc.T, np.linalg.solve(Mc, h))

        # Algorithm 1, initialisation: x_0 = x_{-1} + W (W^T A W)^{-1} W^T r_{-1}
        c = msolve(W.T @ r)
        x = x + W @ c
        r = r - AW @ c
        # mu_0 from W^T A W mu_0 = W^T A r_0, p_0 = r_0 - W mu_0
        mu = msolve(AW.T @ r)
        p = r - W @ mu
        res.mu.append(mu)
    else:
        p = r.copy()

    rho = r @ r
    res.res_hist.append(np.sqrt(rho) / bnorm)
    res.rho.append(rho)
    Ps, APs = [], []
    all_r = [r.copy()] if store_all else None
    all_p = [p.copy()] if store_all else None
    j = 0
    while np.sqrt(rho) / bnorm > tol and j < max_iter:
        q = mv(p)
        res.matvecs += 1
        d = p @ q
        if not d > 0:
            raise np.linalg.LinAlgError("p^T A p <= 0: operator not SPD")
        alpha = rho / d
        if j < L:
            Ps.append(p.copy())
            APs.append(q.copy())
            res.d.append(d)
            res.alpha.append(alpha)
        x = x + alpha * p
        r = r - alpha * q
        if deflate and reproject:
            c = msolve(W.T @ r)
            x = x + W @ c
            r = r - AW @ c
            if j < L:
                res.cvec.append(c)
        rho_new = r @ r
        beta = rho_new / rho
        rho = rho_new
        if deflate:
            mu = msolve(AW.T @ r)
            p = beta * p + r - W @ mu
        else:
            p = beta * p + r
        if j < L:
            res.beta.append(beta)
            res.rho.append(rho)
            if deflate:
                res.mu.append(mu)
            if j + 1 == L:
                res.p_next = p.copy()
        j += 1
        res.res_hist.append(np.sqrt(rho) / bnorm)
        if store_all:
            all_r.append(r.copy())
            all_p.append(p.copy())
    if j < L:
        res.p_next = p.copy()
    res.x = x
    res.iters = j
    res.converged = np.sqrt(rho) / bnorm <= tol
    res.r_final = r
    res.P = np.column_stack(Ps) if Ps else np.zeros((n, 0))
    res.AP = np.column_stack(APs) if APs else np.zeros((n, 0))
    if store_all:
        res.all_r = np.column_stack(all_r)
        res.all_p = np.column_stack(all_p)
    return res


def cg(A, b, x_init=None, tol=1e-8, L=0, max_iter=None, store_all=False):
    """Plain CG: Algorithm 1 with W empty."""
    return defcg(A, b, x_init=x_init, W=None, tol=tol, L=L, max_iter=max_iter,
                 store_all=store_all)
