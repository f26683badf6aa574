"""Mixed-precision iterative refinement around the deflated solve.

Test infrastructure only (see ``oracle/__init__``).

Not in the paper: the precision form of the library.  The residual is taken
with the FP64 operator A, the correction solves the low-precision operator
A~ = K(X~, X~) + sigma^2 I (points rounded to bf16 or fp32) to a relative
tolerance eta, and the correction is added in FP64:

    x_0 = 0;  r_t = b - A x_t;  stop if |r_t| / |b| <= tol;
    A~ d_t = r_t  (def-CG, recycled basis carried across the inner solves);
    x_{t+1} = x_t + d_t.

Each step contracts the error by about rho(A~^{-1}(A - A~)) + eta, so it
converges to A^{-1} b whenever that is below one.  Here everything is FP64;
the only difference between A and A~ is the rounding of X.
"""

import numpy as np

from . import cg as _cg
from . import ritz as _ritz


def refine(A64, A_low, b, tol=1e-8, inner_tol=1e-4, k=0, L=0, max_outer=20, extract="every",
           W=None, AW=None, reproject=False):
    """Returns (x, history of |r_t|/|b|, list of inner DefCGResult, (W, AW)).

    extract (with k > 0) says when the recycled basis is refreshed (section
    2.3, Eq. 7) from Z = [W, stored directions]:
      "every": after every inner solve, from that solve's first L directions;
      "first": after the first inner solve only (the operator A~ is the same
               for all inner solves of one call);
      "accum": once, after the last inner solve, from the directions of the
               inner solves in order, up to L of them (W is unchanged meanwhile).
    W, AW: a basis carried in (AW its product with A~).
    reproject: passed to the inner ``defcg`` (remove W^T r after every step)."""
    mv64 = A64 if callable(A64) else (lambda v, A=np.asarray(A64): A @ v)
    mvl = A_low if callable(A_low) else (lambda v, A=np.asarray(A_low): A @ v)
    if extract not in ("every", "first", "accum"):
        raise ValueError(extract)
    b = np.asarray(b, dtype=np.float64)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist, inner = [], []
    P_acc, AP_acc = [], []
    for _ in range(max_outer + 1):
        r = b - mv64(x)
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol or len(inner) == max_outer:
            break
        if k == 0:
            store = 0
        elif extract == "every" or (extract == "first" and not inner):
            store = L
        elif extract == "accum":
            store = L - sum(P.shape[1] for P in P_acc)
        else:
            store = 0
        res = _cg.defcg(mvl, r, W=W, AW=AW, tol=inner_tol, L=store, reproject=reproject)
        inner.append(res)
        x = x + res.x
        if store > 0 and res.P.shape[1] > 0:
            if extract == "accum":
                P_acc.append(res.P)
                AP_acc.append(res.AP)
            else:
                Z = res.P if W is None else np.hstack([W, res.P])
                AZ = res.AP if W is None else np.hstack([AW, res.AP])
                W, AW, _, _ = _ritz.harmonic_ritz(Z, AZ, k)
    if extract == "accum" and P_acc:
        P = np.hstack(P_acc)
        AP = np.hstack(AP_acc)
        Z = P if W is None else np.hstack([W, P])
        AZ = AP if W is None else np.hstack([AW, AP])
        W, AW, _, _ = _ritz.harmonic_ritz(Z, AZ, k)
    return x, hist, inner, (W, AW)


def fcg_outer(mv64, precond, b, tol=1e-8, max_outer=20, x0=None):
    """Flexible conjugate gradients with full A-orthogonalisation (Notay,
    SIAM J. Sci. Comput. 22, 2000) around a variable preconditioner.

    Each outer step takes z_t = precond(r_t), A-orthogonalises it against
    every earlier direction, d_t = z_t - sum_j (d_j^T A z_t / d_j^T A d_j) d_j,
    and moves along it with the exact line search alpha_t = d_t^T r_t /
    d_t^T A d_t.  The products A d_t use the FP64 operator (one per step, A z_t
    updated by the same combination), the residual is updated recursively.
    With a fixed SPD preconditioner M^{-1} the iterates are those of PCG; with
    an exact solve (precond = A^{-1}) one step reaches A^{-1} b.

    Returns (x, history of |r_t|/|b|, directions D, products AD)."""
    b = np.asarray(b, dtype=np.float64)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if bn == 0.0:
        return np.zeros_like(b), [0.0], [], []
    r = b - mv64(x) if x0 is not None else b.copy()
    D, AD = [], []
    hist = [np.linalg.norm(r) / bn]
    while hist[-1] > tol and len(D) < max_outer:
        z = precond(r)
        d = np.array(z, dtype=np.float64)
        ad = mv64(d)
        for dj, adj in zip(D, AD):
            c = (adj @ z) / (adj @ dj)
            d = d - c * dj
            ad = ad - c * adj
        gamma = d @ ad
        if not gamma > 0.0:
            raise FloatingPointError("flexible CG: d^T A d <= 0")
        alpha = (d @ r) / gamma
        x = x + alpha * d
        r = r - alpha * ad
        D.append(d)
        AD.append(ad)
        hist.append(np.linalg.norm(r) / bn)
    return x, hist, D, AD


def refine_fcg(A64, A_low, b, tol=1e-8, inner_tol=1e-4, k=0, L=0, max_outer=20):
    """Krylov-accelerated refinement: flexible CG in FP64 whose
    preconditioner is the deflated solve of the low-precision operator to
    inner_tol (recycled basis extracted after the first inner solve and kept
    for the later ones).  Returns (x, history, list of inner DefCGResult)."""
    mv64 = A64 if callable(A64) else (lambda v, A=np.asarray(A64): A @ v)
    mvl = A_low if callable(A_low) else (lambda v, A=np.asarray(A_low): A @ v)
    inner = []
    state = {"W": None, "AW": None}

    def precond(r):
        res = _cg.defcg(mvl, r, W=state["W"], AW=state["AW"], tol=inner_tol,
                        L=L if (k > 0 and not inner) else 0)
        if k > 0 and not inner and res.P.shape[1] > 0:
            state["W"], state["AW"], _, _ = _ritz.harmonic_ritz(res.P, res.AP, k)
        inner.append(res)
        return res.x

    x, hist, _, _ = fcg_outer(mv64, precond, b, tol=tol, max_outer=max_outer)
    return x, hist, inner
