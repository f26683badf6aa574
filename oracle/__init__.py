"""Reference oracle for deflated CG with Krylov subspace recycling.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of what the GPU library computes, written directly from the
paper (de Roos & Hennig, "Krylov Subspace Recycling for Fast Iterative
Least-Squares in Machine Learning", arXiv 1706.00241).  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  The
product path (``paper_1706_00241_amd``) never imports, calls or links it, and
this package never imports the product path: the two share no code.

Modules
-------
kernels    covariance functions and the dense operator A = K + sigma^2 I
           (Gram matrix over X, section 1; RBF kernel, section 3).
precision  rounding of the input points to the compute precision
           (bf16 / fp32), written from the IEEE/bfloat16 definitions.
cg         plain CG and deflated CG (section 2.2, Algorithm 1).
ritz       harmonic projection / harmonic Ritz extraction (section 2.3, Eq. 7).
sequence   sequences of related systems with the recycled basis carried
           from one solve to the next (section 1, Eq. 1; Fig. 1).
refine     mixed-precision iterative refinement around the deflated solve.
gp         GP log marginal likelihood, its exact gradient and the Hutchinson
           estimator of its trace term (GP model adaptation, section 1).
gpc        Laplace-approximation GP classification: the Newton iteration
           whose restructured systems A = I + H^1/2 K H^1/2 form the
           paper's own sequence (section 3).
slq        log det A by stochastic Lanczos quadrature from the coefficients
           of plain CG probe solves (the GP log marginal likelihood's value).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force on tiny inputs, library routines for
special cases, or invariants the mathematics fixes.  None is "parity
unpinned".
"""

from . import kernels, precision, cg, ritz, sequence, refine, gp  # noqa: F401
