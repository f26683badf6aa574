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


def refine(A64, A_low, b, tol=1e-8, inner_tol=1e-4, k=0, L=0, max_outer=20):
    """Returns (x, history of |r_t|/|b|, list of inner DefCGResult)."""
    mv64 = A64 if callable(A64) else (lambda v, A=np.asarray(A64): A @ v)
    mvl = A_low if callable(A_low) else (lambda v, A=np.asarray(A_low): A @ v)
    b = np.asarray(b, dtype=np.float64)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist, inner = [], []
    W = AW = None
    for _ in range(max_outer + 1):
        r = b - mv64(x)
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol or len(inner) == max_outer:
            break
        res = _cg.defcg(mvl, r, W=W, AW=AW, tol=inner_tol, L=L if k > 0 else 0)
        inner.append(res)
        x = x + res.x
        if k > 0:
            Z = res.P if W is None else np.hstack([W, res.P])
            AZ = res.AP if W is None else np.hstack([AW, res.AP])
            if Z.shape[1] > 0:
                W, AW, _, _ = _ritz.harmonic_ritz(Z, AZ, k)
    return x, hist, inner
