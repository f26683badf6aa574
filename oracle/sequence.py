"""Sequences of related SPD systems solved with a recycled basis.

Test infrastructure only (see ``oracle/__init__``).

Section 1 (Eq. 1) poses the sequence A^(i) x^(i) = b^(i); Fig. 1 and
section 2.2 describe the scheme: the first system is solved by normal CG,
harmonic Ritz vectors (section 2.3) give W for the next system, and each
later system is solved by def-CG(k, L) with the basis extracted from the
previous solve.  AW must be the product with the *current* operator: it is
recomputed with k products for a new operator, or, when only sigma^2 changes
(A_{i+1} = A_i + (s_{i+1} - s_i) I), updated exactly as
(AZ) U + (sigma2_{i+1} - sigma2_i) W'.  The implicit extraction
(``ritz.IMPLICIT``) takes F, G and A P_L from the solve's stored quantities
instead of its stored products.
"""

import numpy as np

from . import cg as _cg
from . import ritz as _ritz


class Sequence:
    """The recycling state carried from one system to the next (W and its
    product with the previous operator), advanced one system at a time by
    ``step``; ``solve_sequence`` runs it over a whole list.  The arguments
    are those of ``solve_sequence``; ``step(A, b, sigma2=None, x_init=None)``
    solves the next system (A a dense matrix or a callable) and returns its
    DefCGResult with .theta attached."""

    def __init__(self, k, L, tol, recycle=True, largest=True, max_iter=None,
                 extraction=_ritz.HARMONIC, reproject=False):
        self.k, self.L, self.tol = k, L, tol
        self.recycle, self.largest, self.max_iter = recycle, largest, max_iter
        self.extraction, self.reproject = extraction, reproject
        self.W = self.AW_prev_op = self.sigma2_prev = None

    def step(self, A, b, sigma2=None, x_init=None):
        mv = A if callable(A) else (lambda v, A=np.asarray(A): A @ v)
        W = self.W
        AW = None
        if self.recycle and W is not None:
            if sigma2 is not None:
                AW = self.AW_prev_op + (sigma2 - self.sigma2_prev) * W
            else:
                AW = np.column_stack([mv(W[:, c]) for c in range(W.shape[1])])
        res = _cg.defcg(mv, b, x_init=x_init, W=W if self.recycle else None, AW=AW,
                        tol=self.tol, L=self.L if self.recycle else 0, max_iter=self.max_iter,
                        reproject=self.reproject)
        if self.recycle and AW is not None and sigma2 is None:
            res.matvecs += W.shape[1]
        res.theta = None
        if self.recycle:
            if W is not None:
                Z = np.hstack([W, res.P])
                AZ = np.hstack([AW, res.AP])
            else:
                Z, AZ = res.P, res.AP
            if Z.shape[1] > 0 and self.extraction == _ritz.IMPLICIT:
                self.W, self.AW_prev_op, theta, _ = _ritz.implicit_extract(res, W, AW, self.k,
                                                                           self.largest)
                res.theta = theta
            elif Z.shape[1] > 0:
                self.W, self.AW_prev_op, theta, _ = _ritz.extract(Z, AZ, self.k, self.largest,
                                                                  self.extraction)
                res.theta = theta
        self.sigma2_prev = sigma2
        return res


def solve_sequence(matvecs, bs, k, L, tol, recycle=True, sigma2s=None,
                   x_inits=None, largest=True, max_iter=None, extraction=_ritz.HARMONIC,
                   reproject=False):
    """Solve A_i x_i = b_i for i = 0..len-1.

    matvecs : list of callables v -> A_i v (or dense matrices)
    sigma2s : optional list of sigma^2 values; if given and recycle is on,
              consecutive operators are assumed to differ only by the shift
              and AW is updated exactly instead of recomputed.
    reproject: passed to ``defcg`` (remove W^T r after every step).
    Returns list of DefCGResult with .theta (selected Ritz values) attached.
    """
    seq = Sequence(k, L, tol, recycle=recycle, largest=largest, max_iter=max_iter,
                   extraction=extraction, reproject=reproject)
    out = []
    for i, (A, b) in enumerate(zip(matvecs, bs)):
        out.append(seq.step(A, b, sigma2=None if sigma2s is None else sigma2s[i],
                            x_init=None if x_inits is None else x_inits[i]))
    return out
