// The extraction's small generalized eigenproblem G u = theta F u on the
// device (section 2.3): harmonic Ritz (Eq. 7) F = (AZ)^T Z, G = (AZ)^T AZ,
// or Rayleigh-Ritz F = Z^T Z, G = Z^T A Z.  Below, "F" is the matrix in the
// role of the metric.
//
// F is SPD in exact arithmetic but can be numerically singular when CG has
// lost A-conjugacy, so the problem is solved in the range of F:
//   S = diag(F)^-1/2,  S F S = Q Lam Q^T,  keep lam > tau max(lam),
//   B = S Q_keep Lam_keep^-1/2  (B^T F B = I),
//   C = B^T G B = Y Theta Y^T,  U = B Y   (U^T F U = I).
// With nothing dropped this is exactly the symmetric-definite problem, and
// then any B with B^T F B = I gives the same pairs.  The kernel first tries
// the cheap one, B = S R^-1 from the Cholesky factor S F S = R^T R, and keeps
// it when a bound proves that the drop rule would keep every direction:
// lam_min >= 1 / trace((S F S)^-1) = 1 / |R^-1|_F^2 and lam_max <= the
// largest absolute row sum, so 1 / |R^-1|_F^2 > tau * (row sum) means
// lam_min > tau lam_max.  Otherwise (or if a pivot is too small) it takes the
// eigendecomposition route above.  The symmetric eigenproblems are solved by
// cyclic Jacobi with the round-robin (tournament) ordering, so that the m/2
// rotations of a round are disjoint and applied in parallel by one
// workgroup.  The working matrix stays in LDS as a packed upper triangle.
#include <cmath>

#include "blas.h"

namespace dcg {

constexpr int kEigThreads = 1024;
// Problems up to this (even) size keep the eigenvectors in LDS:
// packed matrix 44 KB + V 87 KB.
constexpr int kEigSmall = 104;

__device__ __forceinline__ int pk_idx(int i, int j, int m2) {
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  return i * (2 * m2 - i + 1) / 2 + (j - i);
}

__device__ __forceinline__ void round_pair(int round, int pi, int m2, int *p, int *q) {
  *p = (pi == 0) ? 0 : ((pi - 1 + round) % (m2 - 1)) + 1;
  *q = ((m2 - 2 - pi + round) % (m2 - 1)) + 1;
}

// Block-wide sum (kEigThreads threads), result broadcast to all threads.
__device__ double eig_block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kEigThreads / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

struct JacobiLds {
  double cs[kMaxZ / 2 + 1], sn[kMaxZ / 2 + 1], tt[kMaxZ / 2 + 1];
  int pp[kMaxZ / 2 + 1], qq[kMaxZ / 2 + 1];
  double red[kEigThreads / 64];
};

// Eigen-decomposition of the packed symmetric m x m matrix Ap (LDS, padded
// to even m2 with zero rows).  On return Ap is diagonal (eigenvalues) and V
// (row-major, ld = ldv) holds the eigenvectors in its columns.  Returns the
// number of sweeps used.  MAXM bounds m2.  A round's work items are split
// into (a, b) = (e / P, e % P) with the quotient from an FP32 product:
// for e < 2^15 and P <= 96, (e + 1/2) / P is at least 1 / (2P) away from an
// integer, far above the FP32 rounding, so the floor is exact (checked for
// every P <= 96 and e < 20000).
__device__ __forceinline__ int div_small(int e, float inv) {
  return static_cast<int>((static_cast<float>(e) + 0.5f) * inv);
}

template <int MAXM>
__device__ int jacobi(double *Ap, int m, double *V, int ldv, JacobiLds &L) {
  const int m2 = m + (m & 1);
  const int P = m2 / 2;
  const float invP = 1.0f / static_cast<float>(P > 0 ? P : 1);
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += kEigThreads) V[(e / m) * ldv + e % m] = (e / m == e % m) ? 1.0 : 0.0;
  __syncthreads();
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int e = tid; e < m2 * m2; e += kEigThreads) {
      const int i = e / m2, j = e % m2;
      if (j < i) continue;
      const double v = Ap[pk_idx(i, j, m2)];
      if (i == j) dg += v * v;
      else off += v * v;
    }
    off = eig_block_sum(off, L.red);
    dg = eig_block_sum(dg, L.red);
    if (m2 <= 1 || off <= 1e-30 * dg || !(dg > 0.0)) break;
    for (int round = 0; round < m2 - 1; ++round) {
      for (int pi = tid; pi < P; pi += kEigThreads) {
        int p, q;
        round_pair(round, pi, m2, &p, &q);
        double c = 1.0, s = 0.0, t = 0.0;
        if (p < m && q < m) {
          const double apq = Ap[pk_idx(p, q, m2)];
          const double app = Ap[pk_idx(p, p, m2)], aqq = Ap[pk_idx(q, q, m2)];
          if (apq != 0.0 && fabs(apq) > 1e-300) {
            const double th = (aqq - app) / (2.0 * apq);
            t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + std::sqrt(th * th + 1.0));
            c = 1.0 / std::sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        L.cs[pi] = c;
        L.sn[pi] = s;
        L.tt[pi] = t;
        L.pp[pi] = p;
        L.qq[pi] = q;
      }
      __syncthreads();
      for (int e = tid; e < P * P; e += kEigThreads) {
        const int a = div_small(e, invP), b = e - a * P;
        if (a > b) continue;
        const double sa = L.sn[a], sb = L.sn[b];
        if (sa == 0.0 && sb == 0.0) continue;
        const int pa = L.pp[a], qa = L.qq[a], pb = L.pp[b], qb = L.qq[b];
        const double ca = L.cs[a], cb = L.cs[b];
        if (a == b) {
          const int ipp = pk_idx(pa, pa, m2), ipq = pk_idx(pa, qa, m2), iqq = pk_idx(qa, qa, m2);
          const double apq = Ap[ipq], t = L.tt[a];
          Ap[ipp] = Ap[ipp] - t * apq;
          Ap[iqq] = Ap[iqq] + t * apq;
          Ap[ipq] = 0.0;
        } else {
          const int i11 = pk_idx(pa, pb, m2), i12 = pk_idx(pa, qb, m2);
          const int i21 = pk_idx(qa, pb, m2), i22 = pk_idx(qa, qb, m2);
          const double x11 = Ap[i11], x12 = Ap[i12], x21 = Ap[i21], x22 = Ap[i22];
          // rows: J_a^T X
          const double y11 = ca * x11 - sa * x21, y12 = ca * x12 - sa * x22;
          const double y21 = sa * x11 + ca * x21, y22 = sa * x12 + ca * x22;
          // columns: (J_a^T X) J_b
          Ap[i11] = cb * y11 - sb * y12;
          Ap[i12] = sb * y11 + cb * y12;
          Ap[i21] = cb * y21 - sb * y22;
          Ap[i22] = sb * y21 + cb * y22;
        }
      }
      for (int e = tid; e < m * P; e += kEigThreads) {
        const int i = div_small(e, invP), b = e - i * P;
        const double sb = L.sn[b];
        if (sb == 0.0) continue;
        const int pb = L.pp[b], qb = L.qq[b];
        const double cb = L.cs[b];
        const double vp = V[i * ldv + pb], vq = V[i * ldv + qb];
        V[i * ldv + pb] = cb * vp - sb * vq;
        V[i * ldv + qb] = sb * vp + cb * vq;
      }
      __syncthreads();
    }
  }
  return sweep;
}

struct EigArgs {
  const double *F, *G;  // m x m row-major (ld = m)
  int m, k, largest;
  int route;            // 0: try Cholesky first, 1: eigendecomposition only
  double tau;
  double *V, *B, *T;    // kMaxZ x kMaxZ work (global)
  double *U;            // m x k out, row-major ld = kMaxK
  double *theta;        // k out
  int *info;            // [0] = columns kept (k_next), [1] = rank of F, [2..3] sweeps
                        // ([2] = 0: the Cholesky route)
};

// MAXM: the largest (even) m the instance takes.  VLDS: the eigenvector
// matrix V of the two Jacobi solves lives in LDS next to the packed matrix
// (small problems; every Jacobi round updates all of V), else in global work
// memory.
template <int MAXM, bool VLDS>
__global__ __launch_bounds__(kEigThreads) void harmonic_ritz_kernel(EigArgs A) {
  constexpr int kPacked = (MAXM * (MAXM + 1)) / 2;
  __shared__ double Ap[kPacked];
  __shared__ double Vl[VLDS ? MAXM * MAXM : 1];
  __shared__ double sc[MAXM];
  __shared__ double lam[MAXM];
  __shared__ int keep[MAXM];
  __shared__ int nkeep;
  __shared__ double lbound;
  __shared__ int sel[MAXM];
  __shared__ JacobiLds L;
  const int m = A.m, tid = threadIdx.x;
  const int m2 = m + (m & 1);
  constexpr int ld = kMaxZ;                   // B and T (global work)
  constexpr int ldv = VLDS ? MAXM : kMaxZ;    // V
  double *V = VLDS ? Vl : A.V;

  // 1. scaled F, and a bound on its largest eigenvalue (largest absolute
  // row sum)
  for (int i = tid; i < m; i += kEigThreads) {
    const double f = A.F[i * m + i];
    sc[i] = (f > 0.0) ? 1.0 / std::sqrt(f) : 0.0;
  }
  __syncthreads();
  auto load_scaled_f = [&]() {
    for (int e = tid; e < m2 * m2; e += kEigThreads) {
      const int i = e / m2, j = e % m2;
      if (i > j) continue;
      double v = 0.0;
      if (i < m && j < m) v = 0.5 * (A.F[i * m + j] + A.F[j * m + i]) * sc[i] * sc[j];
      Ap[pk_idx(i, j, m2)] = v;
    }
  };
  load_scaled_f();
  for (int i = tid; i < m; i += kEigThreads) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += fabs(0.5 * (A.F[i * m + j] + A.F[j * m + i]) * sc[i] * sc[j]);
    lam[i] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double b = 0.0;
    for (int i = 0; i < m; ++i) b = fmax(b, lam[i]);
    lbound = b;
  }
  __syncthreads();
  const double floor_lam = A.tau * lbound;

  // 2a. Cholesky S F S = R^T R in place (R in the packed upper triangle,
  // 1 / R_jj in lam).  Every thread reads the same pivot, so the exit is
  // uniform; a pivot at or below tau * bound means lam_min is too.
  bool chol = A.route == 0 && floor_lam > 0.0;
  for (int j = 0; chol && j < m; ++j) {
    const double piv = Ap[pk_idx(j, j, m2)];
    if (!(piv > floor_lam)) {
      chol = false;
      break;
    }
    const double rinv = 1.0 / std::sqrt(piv);
    for (int l = j + 1 + tid; l < m; l += kEigThreads) Ap[pk_idx(j, l, m2)] *= rinv;
    if (tid == 0) lam[j] = rinv;
    __syncthreads();
    const int w = m - j - 1;
    for (int e = tid; e < w * w; e += kEigThreads) {
      const int a = e / w, b = e - a * w;
      if (a > b) continue;
      const int i = j + 1 + a, l = j + 1 + b;
      Ap[pk_idx(i, l, m2)] -= Ap[pk_idx(j, i, m2)] * Ap[pk_idx(j, l, m2)];
    }
    __syncthreads();
  }
  // R^-1 (upper triangular) into V, one column per thread by back
  // substitution, and its squared Frobenius norm
  if (chol) {
    double tr = 0.0;
    for (int c = tid; c < m; c += kEigThreads) {
      const double xcc = lam[c];
      V[c * ldv + c] = xcc;
      tr += xcc * xcc;
      for (int i = c - 1; i >= 0; --i) {
        const int base = pk_idx(i, i, m2);
        double s = 0.0;
        for (int l = i + 1; l <= c; ++l) s += Ap[base + (l - i)] * V[l * ldv + c];
        const double x = -s * lam[i];
        V[i * ldv + c] = x;
        tr += x * x;
      }
      for (int i = c + 1; i < m; ++i) V[i * ldv + c] = 0.0;
    }
    tr = eig_block_sum(tr, L.red);
    chol = tr * floor_lam < 1.0;
  }

  int r, sw1 = 0;
  if (chol) {
    // B = S R^-1   (m x m, ld)
    r = m;
    for (int e = tid; e < m * m; e += kEigThreads) {
      const int i = e / m, t = e % m;
      A.B[i * ld + t] = sc[i] * V[i * ldv + t];
    }
  } else {
    // 2b. S F S = Q Lam Q^T; drop the numerically null directions of F
    __syncthreads();
    load_scaled_f();
    __syncthreads();
    sw1 = jacobi<MAXM>(Ap, m, V, ldv, L);
    for (int i = tid; i < m; i += kEigThreads) lam[i] = Ap[pk_idx(i, i, m2)];
    __syncthreads();
    if (tid == 0) {
      double lmax = 0.0;
      for (int i = 0; i < m; ++i) lmax = fmax(lmax, lam[i]);
      int nk = 0;
      for (int i = 0; i < m; ++i)
        if (lam[i] > A.tau * lmax && lam[i] > 0.0) keep[nk++] = i;
      nkeep = nk;
    }
    __syncthreads();
    r = nkeep;
    // B = S Q_keep Lam^-1/2   (m x r, ld)
    for (int e = tid; e < m * r; e += kEigThreads) {
      const int i = e / r, t = e % r;
      const int col = keep[t];
      A.B[i * ld + t] = sc[i] * V[i * ldv + col] / std::sqrt(lam[col]);
    }
  }
  const int r2 = r + (r & 1);
  __syncthreads();
  // T = G B   (m x r)
  for (int e = tid; e < m * r; e += kEigThreads) {
    const int i = e / r, t = e % r;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += 0.5 * (A.G[i * m + j] + A.G[j * m + i]) * A.B[j * ld + t];
    A.T[i * ld + t] = s;
  }
  __syncthreads();
  // C = B^T T, symmetrised, packed into Ap (r2 x r2)
  for (int e = tid; e < r2 * r2; e += kEigThreads) {
    const int t1 = e / r2, t2 = e % r2;
    if (t1 > t2) continue;
    double v = 0.0;
    if (t1 < r && t2 < r) {
      double s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < m; ++i) {
        s1 += A.B[i * ld + t1] * A.T[i * ld + t2];
        s2 += A.B[i * ld + t2] * A.T[i * ld + t1];
      }
      v = 0.5 * (s1 + s2);
    }
    Ap[pk_idx(t1, t2, r2)] = v;
  }
  __syncthreads();
  const int sw2 = jacobi<MAXM>(Ap, r, V, ldv, L);
  for (int t = tid; t < r; t += kEigThreads) lam[t] = Ap[pk_idx(t, t, r2)];
  __syncthreads();
  // 3. selection: stable rank by theta (descending if largest)
  const int kk = min(A.k, r);
  for (int t = tid; t < r; t += kEigThreads) {
    int rank = 0;
    for (int u = 0; u < r; ++u) {
      const bool before = A.largest ? (lam[u] > lam[t]) : (lam[u] < lam[t]);
      if (before || (lam[u] == lam[t] && u < t)) ++rank;
    }
    if (rank < kk) sel[rank] = t;
  }
  __syncthreads();
  // U = B Y_sel  (m x kk, ld kMaxK)
  for (int e = tid; e < m * kk; e += kEigThreads) {
    const int i = e / kk, s = e % kk;
    const int t = sel[s];
    double v = 0.0;
    for (int u = 0; u < r; ++u) v += A.B[i * ld + u] * V[u * ldv + t];
    A.U[i * kMaxK + s] = v;
  }
  for (int s = tid; s < kk; s += kEigThreads) A.theta[s] = lam[sel[s]];
  if (tid == 0) {
    A.info[0] = kk;
    A.info[1] = r;
    A.info[2] = sw1;
    A.info[3] = sw2;
  }
}

void enqueue_harmonic_ritz(hipStream_t s, const double *F, const double *G, int m, int k,
                           int largest, int route, double tau, double *work, double *U,
                           double *theta, int *info) {
  EigArgs a;
  a.F = F;
  a.G = G;
  a.m = m;
  a.k = k;
  a.largest = largest;
  a.route = route;
  a.tau = tau;
  a.V = work;
  a.B = work + kMaxZ * kMaxZ;
  a.T = work + 2 * kMaxZ * kMaxZ;
  a.U = U;
  a.theta = theta;
  a.info = info;
  if (m + (m & 1) <= kEigSmall)
    hipLaunchKernelGGL((harmonic_ritz_kernel<kEigSmall, true>), dim3(1), dim3(kEigThreads), 0, s, a);
  else
    hipLaunchKernelGGL((harmonic_ritz_kernel<kMaxZ, false>), dim3(1), dim3(kEigThreads), 0, s, a);
}

size_t harmonic_ritz_work_doubles() { return size_t(3) * kMaxZ * kMaxZ; }

}  // namespace dcg
