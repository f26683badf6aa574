// Host-only arithmetic of the library (host.cpp): operand geometry, the
// work plans of the pair sweeps, and the tridiagonal eigenproblems of
// stochastic Lanczos quadrature.  Built by the host compiler alone.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.h"

namespace dcg {

// (Geometry make_geometry, MatvecPlan make_plan and matvec_partial_floats
// are declared in common.h.)

// The FP64 sweep: MFMA K steps (4 coordinates each) for d coordinates plus
// the two norm columns, the stored width per point, its plan (128-point
// blocks) and the doubles of its partial sums for the largest plan.
int exact_ksteps(int d);
int exact_stride(int d);
MatvecPlan exact_plan(int64_t n_pad, int items);
size_t exact_partial_doubles(int64_t n_pad);

// Eigenvalues (into d) and first eigenvector components (into q) of the
// symmetric tridiagonal matrix with diagonal d and off-diagonal e, by
// implicit QR steps with Wilkinson shifts; false if a block fails to
// converge.
bool tridiag_eig_first_row(std::vector<double> &d, std::vector<double> &e,
                           std::vector<double> &q);
// |z|^2 e_1^T log(T_m) e_1 for the Lanczos tridiagonal of m CG steps with
// coefficients alpha[0..m), beta[0..m-1); DCG_E_NOT_SPD for a non-positive
// alpha or Ritz value, DCG_E_NONFINITE if the eigenproblem fails.
int slq_quadrature(const double *alpha, const double *beta, int m, double znorm2, double *out);

}  // namespace dcg
