// Host-only arithmetic of the library, kept apart from the kernels so that it
// builds with the host compiler alone (and with its sanitizers, on a machine
// without a GPU): the operand geometry of each precision, the work plans of
// the two pair sweeps and the sizes of their partial sums, and the small
// tridiagonal eigenproblems of stochastic Lanczos quadrature.
#include "host.h"

#include <algorithm>
#include <cmath>

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int bf16_bucket(int ks) {
  const int b[] = {1, 2, 3, 4, 5, 7, 9, 13, 17};
  for (int v : b)
    if (ks <= v) return v;
  return -1;
}

static int fp32_bucket(int ks) {
  const int b[] = {5, 9, 13, 17, 25, 33};
  for (int v : b)
    if (ks <= v) return v;
  return -1;
}

Geometry make_geometry(int64_t n, int d, int prec) {
  Geometry g;
  g.n = n;
  g.d = d;
  g.prec = prec;
  g.n_pad = ((n + 255) / 256) * 256;
  g.opk = kOpBf16;
  if (prec == DCG_PREC_FP64 || prec == DCG_PREC_STORED) {
    g.ksteps = 0;  // the exact FP64 product and the stored matrix need no MFMA operands
    g.kstride = 0;
  } else if (prec == DCG_PREC_BF16 || prec == DCG_PREC_FP16) {
    g.opk = (prec == DCG_PREC_FP16) ? kOpF16 : kOpBf16;
    // the wide sweep streams K in stages of 32 (two K steps)
    g.ksteps = (d > kMaxD) ? 2 * ((d + 6 + 31) / 32) : (d + 6 + 15) / 16;
    g.kstride = 16 * g.ksteps;
  } else if (prec == DCG_PREC_BF16X2) {
    g.ksteps = bf16_bucket((4 * d + 6 + 15) / 16);
    g.kstride = 16 * g.ksteps;
  } else if (6 * d + 6 <= 16 * 13) {
    // FP32 points as three exact bf16 terms: six products per coordinate
    // and the squared norm in three terms on each side
    g.opk = kOpBf16Acc64;
    g.ksteps = bf16_bucket((6 * d + 6 + 15) / 16);
    g.kstride = 16 * g.ksteps;
  } else {
    g.opk = kOpF32;
    g.ksteps = fp32_bucket((d + 2 + 1) / 2);
    g.kstride = 2 * ((g.ksteps + 3) / 4) * 4;
  }
  return g;
}

MatvecPlan make_plan(int64_t n_pad, int blk, int items) {
  MatvecPlan p;
  p.blk = blk;
  p.nb = static_cast<int>(n_pad / p.blk);
  p.dmax = p.nb / 2;
  const int ndelta = p.dmax + 1;
  p.chunk = static_cast<int>(std::max<int64_t>(1, cdiv(int64_t(ndelta) * p.nb, items)));
  p.nchunk = static_cast<int>(cdiv(ndelta, p.chunk));
  p.grid = int64_t(p.nb) * p.nchunk;
  return p;
}

int wide_steps(int nb) {
  // u = 4 s + b - a must reach ndel - 1 <= nb / 2 for a = kWideGroup - 1
  const int ndel_max = nb / 2 + 1;
  return static_cast<int>(cdiv(int64_t(ndel_max) + kWideGroup - 1, 4));
}

MatvecPlan wide_plan(int64_t n_pad, int items) {
  MatvecPlan p;
  p.blk = 256;
  p.nb = static_cast<int>(n_pad / p.blk);
  p.dmax = p.nb / 2;
  const int S = wide_steps(p.nb);
  const int64_t groups = cdiv(p.nb, kWideGroup);
  // parts so that the sweep has about `items` work items of 32 per tile
  const int64_t want = std::max<int64_t>(1, items / (32 * groups));
  const int parts0 = static_cast<int>(std::min<int64_t>(want, S));
  p.chunk = static_cast<int>(cdiv(S, parts0));
  const int parts = static_cast<int>(cdiv(S, p.chunk));
  p.nchunk = 4 * parts;
  p.grid = cdiv(groups * parts, 8) * 8 * 32;
  return p;
}

MatvecPlan sweep_plan(const Geometry &g, int mv, int items) {
  if (sweep_wide(g)) return wide_plan(g.n_pad, items);
  return make_plan(g.n_pad, sweep_blk(g, mv), items);
}

size_t wide_partial_floats(int64_t n_pad) {
  // the most slots: one part per step
  const int nb = static_cast<int>(n_pad / 256);
  return size_t(2 * 4 * wide_steps(nb) + nb / 2) * size_t(n_pad);
}

size_t matvec_partial_floats(int64_t n_pad, int mv, int blk) {
  // chunks per row block grow with the item target
  MatvecPlan p = make_plan(n_pad, blk, kSweepItemsMax);
  // row partials are FP64 (two floats each), column partials FP32
  return size_t(2 * p.nchunk + p.dmax) * size_t(n_pad) * size_t(mv);
}

int exact_ksteps(int d) {
  const int ks = (d + 2 + 3) / 4;
  return ks <= 3 ? 3 : ks <= 5 ? 5 : ks <= 9 ? 9 : 17;
}
int exact_stride(int d) {
  const int ks = exact_ksteps(d);
  return 4 * (ks + (ks & 1));
}

MatvecPlan exact_plan(int64_t n_pad, int items) {
  MatvecPlan p;
  p.blk = 128;
  p.nb = static_cast<int>(n_pad / p.blk);
  p.dmax = p.nb / 2;
  const int ndelta = p.dmax + 1;
  p.chunk = static_cast<int>(std::max<int64_t>(1, cdiv(int64_t(ndelta) * p.nb, items)));
  p.nchunk = static_cast<int>(cdiv(ndelta, p.chunk));
  p.grid = int64_t(p.nb) * p.nchunk;
  return p;
}

size_t exact_partial_doubles(int64_t n_pad) {
  // chunks per row block grow with the item target
  const MatvecPlan p = exact_plan(n_pad, kSweepItemsMax);
  return size_t(p.nchunk + p.dmax) * size_t(n_pad);
}

// Eigenvalues (into d) and first eigenvector components (into q, starting
// from e_1) of the symmetric tridiagonal matrix with diagonal d[0..m) and
// off-diagonal e[0..m-1).  Returns false if a block fails to converge.
bool tridiag_eig_first_row(std::vector<double> &d, std::vector<double> &e,
                                  std::vector<double> &q) {
  const int m = static_cast<int>(d.size());
  q.assign(m, 0.0);
  if (m == 0) return true;
  q[0] = 1.0;
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  int steps = 0;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (++steps > 50 * m) return false;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer d[hi]
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double sg = (delta >= 0.0) ? 1.0 : -1.0;
    const double mu = d[hi] - eh * eh / (delta + sg * std::hypot(delta, eh));
    // implicit QR step on [lo, hi]: the first rotation brings in the shift,
    // the rest chase the bulge down the band
    double x = d[lo] - mu, y = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      const double c = (r == 0.0) ? 1.0 : x / r;
      const double s = (r == 0.0) ? 0.0 : -y / r;
      if (k > lo) e[k - 1] = r;
      const double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a - 2.0 * c * s * b + s * s * cc;
      d[k + 1] = s * s * a + 2.0 * c * s * b + c * c * cc;
      e[k] = c * s * (a - cc) + (c * c - s * s) * b;
      if (k + 1 < hi) {
        x = e[k];
        y = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      const double q0 = q[k], q1 = q[k + 1];
      q[k] = c * q0 - s * q1;
      q[k + 1] = s * q0 + c * q1;
    }
  }
  return true;
}

// |z|^2 e_1^T log(T) e_1 for the tridiagonal of m CG steps.
int slq_quadrature(const double *alpha, const double *beta, int m, double znorm2,
                          double *out) {
  if (m == 0) {
    *out = 0.0;
    return DCG_OK;
  }
  std::vector<double> d(m), e(std::max(m - 1, 0)), q;
  for (int j = 0; j < m; ++j) {
    if (!(alpha[j] > 0.0) || !std::isfinite(alpha[j])) return DCG_E_NOT_SPD;
    d[j] = 1.0 / alpha[j] + ((j > 0) ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < m) e[j] = std::sqrt(std::max(beta[j], 0.0)) / alpha[j];
  }
  if (!tridiag_eig_first_row(d, e, q)) return DCG_E_NONFINITE;
  double s = 0.0;
  for (int i = 0; i < m; ++i) {
    if (!(d[i] > 0.0)) return DCG_E_NOT_SPD;
    s += q[i] * q[i] * std::log(d[i]);
  }
  *out = znorm2 * s;
  return DCG_OK;
}

}  // namespace dcg
