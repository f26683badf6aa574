"""Sequences of related SPD systems solved with a recycled basis.

Test infrastructure only (see ``oracle/__init__``).

Section 1 (Eq. 1) poses the sequence A^(i) x^(i) = b^(i); Fig. 1 and
section 2.2 describe the scheme: the first system is solved by normal CG,
harmonic Ritz vectors (section 2.3) give W for the next system, and each
later system is solved by def-CG(k, L) with the basis extracted from the
previous solve.  AW must be the product with the *current* operator: it is
recomputed with k products for a new operator, or, when only sigma^2 changes
(A_{i+1} = A_i + (s_{i+1} - s_i) I), updated exactly as
(AZ) U + (sigma2_{i+1} - sigma2_i) W'.
"""

import numpy as np

from . import cg as _cg
from . import ritz as _ritz


def solve_sequence(matvecs, bs, k, L, tol, recycle=True, sigma2s=None,
                   x_inits=None, largest=True, max_iter=None, extraction=_ritz.HARMONIC):
    """Solve A_i x_i = b_i for i = 0..len-1.

    matvecs : list of callables v -> A_i v (or dense matrices)
    sigma2s : optional list of sigma^2 values; if given and recycle is on,
              consecutive operators are assumed to differ only by the shift
              and AW is updated exactly instead of recomputed.
    Returns list of DefCGResult with .theta (selected Ritz values) attached.
    """
    out = []
    W = AW_prev_op = None
    for i, (A, b) in enumerate(zip(matvecs, bs)):
        mv = A if callable(A) else (lambda v, A=np.asarray(A): A @ v)
        AW = None
        if recycle and W is not None:
            if sigma2s is not None:
                AW = AW_prev_op + (sigma2s[i] - sigma2s[i - 1]) * W
            else:
                AW = np.column_stack([mv(W[:, c]) for c in range(W.shape[1])])
        x0 = None if x_inits is None else x_inits[i]
        res = _cg.defcg(mv, b, x_init=x0, W=W if recycle else None, AW=AW,
                        tol=tol, L=L if recycle else 0, max_iter=max_iter)
        if recycle and AW is not None and sigma2s is None:
            res.matvecs += W.shape[1]
        res.theta = None
        if recycle:
            if W is not None:
                Z = np.hstack([W, res.P])
                AZ = np.hstack([AW, res.AP])
            else:
                Z, AZ = res.P, res.AP
            if Z.shape[1] > 0:
                W, AW_prev_op, theta, _ = _ritz.extract(Z, AZ, k, largest, extraction)
                res.theta = theta
        out.append(res)
    return out
