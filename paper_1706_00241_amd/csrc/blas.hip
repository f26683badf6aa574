// FP64 vector kernels of the deflated CG iteration (Algorithm 1), the
// deflation projections W (W^T A W)^{-1} W^T r, and the tall-skinny products
// of the harmonic Ritz extraction (F = (AZ)^T Z, G = (AZ)^T AZ, W' = Z U).
//
// Scalars of the iteration live on the device (SolveState); reductions are
// done in a fixed order by the last block to finish (a per-kernel counter),
// so results are bitwise reproducible and no host round trip is needed.
#include <algorithm>
#include <cmath>

#include "blas.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------- reductions

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += lds[i];
  }
  return s;  // valid in thread 0
}

// Block-wide sum broadcast to every thread (fixed reduction tree).
__device__ __forceinline__ double block_sum_all(double v, double *lds) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) s += lds[i];
  __syncthreads();
  return s;
}

// Sum of part[0 .. count) (stride 1) by the whole block, fixed order.
__device__ __forceinline__ double block_sum_array(const double *part, int64_t count, double *lds) {
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < count; b += blockDim.x) s += part[b];
  return block_sum_all(s, lds);
}

// out[c] = sum_b part[c * count + b] for c < m (column-major partials), one
// wave per column at a time; writes to LDS/global `out` (any address space).
__device__ __forceinline__ void column_sums(const double *part, int64_t count, int m, double *out) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  for (int c = w; c < m; c += nw) {
    double s = 0.0;
    for (int64_t b = l; b < count; b += 64) s += part[int64_t(c) * count + b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (l == 0) out[c] = s;
  }
}

// Returns true in every thread of the block that finished last.  The block's
// partial results must have been written before the call.
__device__ __forceinline__ bool last_block(unsigned *counter) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

// mu = Minv h (k x k dense, row-major), threads of the block over rows.
__device__ __forceinline__ void small_gemv(const double *Minv, const double *h, double *mu, int k) {
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += Minv[c * k + j] * h[j];
    mu[c] = s;
  }
}

// The same product with the matrix staged in LDS, rows padded to kMaxK + 1
// (so that the threads of a wave read distinct banks); same summation order.
__device__ __forceinline__ void small_gemv_lds(const double *Ms, const double *h, double *mu,
                                               int k) {
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0.0;
    // unrolled so that sixteen entries' LDS reads are in flight (the sum
    // still runs in column order)
#pragma unroll 16
    for (int j = 0; j < k; ++j) s += Ms[c * (kMaxK + 1) + j] * h[j];
    mu[c] = s;
  }
}

// ------------------------------------------------------ CG iteration kernels

// q = s2 * sum(partials) + sigma2 p and the block partials of d = p^T q.
// The fused multiply-add is written out so that every kernel built from
// this body (one system or many) rounds q the same way.
// Also stores p_j and q = A p_j into Z / AZ while j < L.  A block finishes
// kCgRows rows in groups of 64; each row's partials are split over 4 threads
// (memory parallelism), then added in a fixed order.  No cross-block step:
// the next kernel forms d and alpha itself from the block partials.
__device__ __forceinline__ void cg_matvec_finish_body(const CgArgs &a, const unsigned bid) {
  SolveState *S = a.S;
  // the step count when this step began: cg_update_p applies the step's
  // x / r update when the solve was still running at that point
  if (bid == 0 && threadIdx.x == 0) S->applied = S->iter;
  if (S->done) return;
  __shared__ double seg[4][64];
  __shared__ double lds[8];
  const int r = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int j = S->iter;  // index of the direction being multiplied
  double pq = 0.0;
  for (int grp = 0; grp < kCgRows / 64; ++grp) {
    const int64_t i = int64_t(bid) * kCgRows + grp * 64 + r;
    double s = 0.0;
    if (i < a.n) {
      if (a.qdirect != nullptr) {
        s = (sg == 0) ? a.qdirect[i] : 0.0;
      } else {
        const ReduceArgs &R = a.red;
        // vector a.mcol of an R.mv-vector partial layout
        const int64_t ps = int64_t(R.mv) * R.n_pad;
        const double *prow = R.prow + int64_t(a.mcol) * R.n_pad;
        const float *pcol = R.pcol + int64_t(a.mcol) * R.n_pad;
        // (the loops are unrolled so that several loads are in flight; each
        // accumulator still adds its terms in order)
#pragma unroll 4
        for (int c = sg; c < R.nchunk; c += 4) s += prow[int64_t(c) * ps + i];
        const int J = static_cast<int>(i / R.blk);
        const int dlim = ((R.nb % 2) == 0 && J < R.nb / 2) ? R.dmax - 1 : R.dmax;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int dl = 1 + sg;
#pragma unroll 2
        for (; dl + 12 <= dlim; dl += 16) {
          s += pcol[int64_t(dl - 1) * ps + i];
          s1 += pcol[int64_t(dl + 3) * ps + i];
          s2 += pcol[int64_t(dl + 7) * ps + i];
          s3 += pcol[int64_t(dl + 11) * ps + i];
        }
        for (; dl <= dlim; dl += 4) s += pcol[int64_t(dl - 1) * ps + i];
        s = (s + s1) + (s2 + s3);
      }
    }
    seg[sg][r] = s;
    __syncthreads();
    if (sg == 0 && i < a.n) {
      const double tot = (seg[0][r] + seg[1][r]) + (seg[2][r] + seg[3][r]);
      const double pi = a.p[i];
      const double di = (a.red.dsc != nullptr) ? a.red.dsc[i] : 1.0;
      const double qi =
          (a.qdirect != nullptr) ? tot : fma(a.red.s2 * di, tot, a.red.sigma2 * pi);
      a.q[i] = qi;
      pq += pi * qi;
      if (a.Z != nullptr && a.implicit && j <= a.L) {
        // the implicit extraction keeps the FP64 directions p_0 .. p_L (the
        // residuals, and so A p_j, follow from them) and no products
        a.Z[int64_t(a.koff + j) * a.n + i] = pi;
      } else if (a.Z != nullptr && j < a.L) {
        // store the direction the product was formed from: the low-precision
        // sweep multiplies the FP32 copy of p, so that copy (exact in FP64)
        // is the column of Z whose product is q; AZ then matches A~ Z to the
        // sweep's own evaluation error, and so does AW' = (AZ) U
        // (with a diagonal scaling the sweep multiplied fp32(d p): store
        // that copy divided by d, whose scaled product the sweep formed)
        double zi = pi;
        if (a.qdirect == nullptr) {
          zi = static_cast<double>(a.p32[i]);
          if (a.red.dsc != nullptr) zi = (di != 0.0) ? zi / di : pi;
        }
        a.Z[int64_t(a.koff + j) * a.n + i] = zi;
        a.AZ[int64_t(a.koff + j) * a.n + i] = qi;
      }
    }
    __syncthreads();
  }
  const double bs = block_sum_all(pq, lds);
  if (threadIdx.x == 0) a.part[bid] = bs;
}

// d = p^T q from the partials of cg_matvec_finish (every block forms it, in
// the same order), alpha = rho / d, and with r' = r - alpha q (formed here
// and again, identically, by cg_update_p, which writes x and r): per row
// block the partials of rho' = r'^T r' and of h = (AW)^T r', g = W^T r'.
// Block (row block rb, column group grp) takes rows rb * kXrRows ... and
// columns grp * kXrCols ... of [AW | W]; group 0 also forms rho'.  The
// kernel writes no vector, so the column groups of one row block never see
// each other's updates.
// kW32: the caller guarantees the FP32 copies of W and AW (a.W32 set), so
// the FP64 column path is compiled out and fewer registers are live.
template <bool kW32>
__device__ __forceinline__ void cg_update_xr_body(const CgArgs &a, const unsigned bid) {
  SolveState *S = a.S;
  if (S->done) return;
  const int64_t nrb = a.nblk_xr;
  const int rb = static_cast<int>(bid % nrb);
  const int grp = static_cast<int>(bid / nrb);
  const int k = a.k;
  if (grp >= xr_groups(k)) return;
  __shared__ double lds[8];
  __shared__ double cpart[4][kXrCols];
  constexpr int RPT = kXrRows / 256;
  const int64_t i0 = int64_t(rb) * kXrRows + threadIdx.x;
  // This block's rows of r, q and of its kXrCols columns of [AW | W] do not
  // depend on alpha: load them first, so that the reduction of d below runs
  // while they are in flight.  With a basis (k >= 1) the loads are
  // unconditional (rows past n and columns past 2k read row n - 1 / the
  // first column of W, which exists) so that none of them waits for another;
  // the out-of-range values are zeroed after the fact.  Without one (plain
  // CG: W and AW are null) no column is read.
  double rv[RPT], qv[RPT];
  double yv[kXrCols][RPT];
  float yf[kXrCols][RPT];
  int64_t ii[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int64_t i = i0 + 256 * u;
    ii[u] = (i < a.n) ? i : a.n - 1;
    rv[u] = a.r[ii[u]];
    qv[u] = a.q[ii[u]];
  }
  const bool w32 = kW32 || a.W32 != nullptr;
  if (k > 0 && w32) {
#pragma unroll
    for (int cc = 0; cc < kXrCols; ++cc) {
      const int c = grp * kXrCols + cc;
      const float *Y = (c < k) ? a.AW32 + int64_t(c) * a.n
                               : a.W32 + int64_t(c < 2 * k ? c - k : 0) * a.n;
#pragma unroll
      for (int u = 0; u < RPT; ++u) yf[cc][u] = Y[ii[u]];
    }
  } else if (k > 0) {
#pragma unroll
    for (int cc = 0; cc < kXrCols; ++cc) {
      const int c = grp * kXrCols + cc;
      const double *Y = (c < k) ? a.AW + int64_t(c) * a.n
                                : a.W + int64_t(c < 2 * k ? c - k : 0) * a.n;
#pragma unroll
      for (int u = 0; u < RPT; ++u) yv[cc][u] = Y[ii[u]];
    }
  }
  const double d = block_sum_array(a.part, a.nblk_q, lds);
  const bool bad = !(d > 0.0) || !isfinite(d);
  const double alpha = bad ? 0.0 : S->rho / d;
  if (bid == 0 && threadIdx.x == 0) {
    S->d = d;
    S->alpha = alpha;
    const int j = S->iter;
    if (j < a.L) {
      a.hist_d[j] = d;
      a.hist_alpha[j] = alpha;
    }
    if (a.lz_alpha != nullptr && j < a.lz_cap) a.lz_alpha[j] = alpha;
  }
  double ri[RPT];
  double rr = 0.0;
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int64_t i = i0 + 256 * u;
    ri[u] = 0.0;
    if (i < a.n) {
      ri[u] = rv[u] - alpha * qv[u];
      rr += ri[u] * ri[u];
    }
  }
  if (grp == 0) {
    const double bs = block_sum_all(rr, lds);
    if (threadIdx.x == 0) a.part2[rb] = bad ? (isfinite(d) ? -1.0 : -2.0) : bs;
  }
  if (k == 0) return;
#pragma unroll
  for (int cc = 0; cc < kXrCols; ++cc) {
    const bool colok = grp * kXrCols + cc < 2 * k;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const double y = w32 ? static_cast<double>(yf[cc][u]) : yv[cc][u];
      yv[cc][u] = (colok && i0 + 256 * u < a.n) ? y : 0.0;
    }
  }
  // partial dots with kXrCols columns of [AW | W]
  double sv[kXrCols];
#pragma unroll
  for (int cc = 0; cc < kXrCols; ++cc) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u)
      if (i0 + 256 * u < a.n) acc += yv[cc][u] * ri[u];
    sv[cc] = acc;
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int cc = 0; cc < kXrCols; ++cc) {
    double v = sv[cc];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (l == 0) cpart[w][cc] = v;
  }
  __syncthreads();
  if (threadIdx.x < kXrCols) {
    const int c = grp * kXrCols + threadIdx.x;
    if (c < 2 * k)
      a.part_h[int64_t(c) * nrb + rb] = (cpart[0][threadIdx.x] + cpart[1][threadIdx.x]) +
                                         (cpart[2][threadIdx.x] + cpart[3][threadIdx.x]);
  }
}

// One block: the sums of cg_update_xr's partials in a fixed order, then the
// re-projection c = (W^T A W)^{-1} g of the residual (zero in exact
// arithmetic, where W^T r_j = 0), and with r' = r - AW c:
// mu = (W^T A W)^{-1} (AW)^T r', beta = |r'|^2 / |r|^2 and the convergence
// test on |r'| / |b|.
__device__ __forceinline__ void cg_finalize_body(const CgArgs &a) {
  SolveState *S = a.S;
  if (S->done) return;
  __shared__ double lds[8];
  __shared__ double hg[2 * kMaxK];   // h = (AW)^T r, then g = W^T r
  __shared__ double cv[kMaxK];       // c = M^-1 g
  __shared__ double nc[kMaxK];       // N c
  __shared__ double hn[kMaxK];       // h - N c
  __shared__ double Ms[kMaxK * (kMaxK + 1)];   // M^-1 and N, rows padded by one
  __shared__ double Ns[kMaxK * (kMaxK + 1)];
  __shared__ int flag;
  const int k = a.k;
  const int64_t nblk = a.nblk_xr;
  const int jstep = S->iter;   // read before thread 0 advances it below
  const bool record = a.hist_rho != nullptr && jstep < a.L;
  if (threadIdx.x == 0) flag = 0;
  // Every load is issued before the first barrier, so that one memory
  // latency covers them all: the rows of M^-1 and N into LDS (coalesced),
  // this thread's share of the rho partials (a negative partial marks
  // p^T A p <= 0 (-1) or non-finite (-2)), and, for threads c < 2k, column
  // c of the [h | g] partials into eight accumulators (acc[u] sums the
  // entries u, u + 8, u + 16, ... in order; the outer loop is unrolled so
  // that several rounds of loads are in flight, not to change that order).
  // (the loads are unconditional, with clamped indices, so that none waits
  // for another; only in-range values are kept)
  constexpr int kStage = kMaxK * kMaxK / 256;
  const int kk = k * k;
  double mv[kStage], nv[kStage];
  if (kk > 0) {
#pragma unroll
    for (int t = 0; t < kStage; ++t) {
      const int e = min(static_cast<int>(threadIdx.x) + 256 * t, kk - 1);
      mv[t] = a.Minv[e];
      nv[t] = a.N[e];
    }
  }
  const double v0 = a.part2[min(static_cast<int64_t>(threadIdx.x), nblk - 1)];
  const int m2 = 2 * k;
  double csum = 0.0;
  if (threadIdx.x < m2) {
    const double *pc = a.part_h + int64_t(threadIdx.x) * nblk;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t b = 0;
#pragma unroll 8
    for (; b + 8 <= nblk; b += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += pc[b + u];
    for (; b < nblk; ++b) acc[0] += pc[b];
    csum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  double rr = 0.0;
  int fl = 0;
  if (threadIdx.x < nblk) {
    if (v0 < 0.0) fl = v0 < -1.5 ? 2 : 1;
    rr = v0;
  }
  for (int64_t b = threadIdx.x + 256; b < nblk; b += 256) {
    const double v = a.part2[b];
    if (v < 0.0) fl = max(fl, v < -1.5 ? 2 : 1);
    rr += v;
  }
  if (kk > 0) {
#pragma unroll
    for (int t = 0; t < kStage; ++t) {
      const int e = static_cast<int>(threadIdx.x) + 256 * t;
      if (e < kk) {
        const int r = e / k, c = e % k;
        Ms[r * (kMaxK + 1) + c] = mv[t];
        Ns[r * (kMaxK + 1) + c] = nv[t];
      }
    }
  }
  __syncthreads();   // flag's initial value is visible to every thread
  if (fl != 0) atomicMax(&flag, fl);
  __syncthreads();
  if (flag != 0) {
    if (threadIdx.x == 0) {
      S->status = (flag == 2) ? DCG_E_NONFINITE : DCG_E_NOT_SPD;
      S->done = 1;
    }
    return;
  }
  if (threadIdx.x < m2) hg[threadIdx.x] = csum;
  const double rho_raw = block_sum_all(rr, lds);   // includes barriers
  small_gemv_lds(Ms, hg + k, cv, k);
  __syncthreads();
  small_gemv_lds(Ns, cv, nc, k);
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 256) {
    hn[c] = hg[c] - nc[c];
    S->cvec[c] = cv[c];
    if (record) a.hist_c[int64_t(jstep) * kMaxK + c] = cv[c];
  }
  __syncthreads();
  small_gemv_lds(Ms, hn, S->mu, k);
  // each thread records the entries of mu it formed
  if (record)
    for (int c = threadIdx.x; c < k; c += blockDim.x)
      a.hist_mu[int64_t(jstep + 1) * kMaxK + c] = S->mu[c];
  if (threadIdx.x == 0) {
    // |r - AW c|^2 = |r|^2 - 2 c^T h + c^T N c
    double corr = 0.0;
    for (int c = 0; c < k; ++c) corr += cv[c] * (nc[c] - 2.0 * hg[c]);
    const double rho_new = fmax(rho_raw + corr, 0.0);
    const double beta = rho_new / S->rho;
    S->beta = beta;
    S->rho = rho_new;
    const int j = S->iter;
    if (j < a.L) a.hist_beta[j] = beta;
    if (record) a.hist_rho[j + 1] = rho_new;
    if (a.lz_beta != nullptr && j < a.lz_cap) a.lz_beta[j] = beta;
    S->iter = j + 1;
    const double rel = std::sqrt(rho_new) / S->bnorm;
    S->relres = rel;
    if (j + 1 < a.hist_cap) a.hist_res[j + 1] = rel;
    if (!isfinite(rho_new)) {
      S->status = DCG_E_NONFINITE;
      S->done = 1;
    } else if (rel <= a.tol || j + 1 >= a.max_iter) {
      S->done = 1;
    }
  }
}

// The step x += alpha p, r -= alpha q, then the re-projection (x += W c,
// r -= AW c) and the direction update p = beta p + r - W mu; the FP32 copy of
// p feeds the next matvec.
__device__ __forceinline__ void cg_update_p_body(const CgArgs &a, const unsigned bid) {
  SolveState *S = a.S;
  // A step that converges (or reaches max_iter) still applies its update:
  // cg_finalize has advanced iter past the count cg_matvec_finish recorded.
  // Steps after the end, and a step that failed (iter not advanced), do not.
  if (S->done && S->applied == S->iter) return;
  __shared__ double mu[kMaxK];
  __shared__ double cv[kMaxK];
  for (int c = threadIdx.x; c < a.k; c += 256) {
    mu[c] = S->mu[c];
    cv[c] = S->cvec[c];
  }
  __syncthreads();
  const int64_t i = int64_t(bid) * 256 + threadIdx.x;
  if (i >= a.n) return;
  const double alpha = S->alpha;
  const double pi = a.p[i];
  double ri = a.r[i] - alpha * a.q[i];
  double xn = a.x[i] + alpha * pi;
  double xi = 0.0;
  double wmu = 0.0;
  // unrolled so that eight columns' loads are in flight at once (each
  // accumulator still adds its terms in column order)
  if (a.W32 != nullptr) {
#pragma unroll 8
    for (int c = 0; c < a.k; ++c) {
      const double wv = static_cast<double>(a.W32[int64_t(c) * a.n + i]);
      ri -= static_cast<double>(a.AW32[int64_t(c) * a.n + i]) * cv[c];
      xi += wv * cv[c];
      wmu += wv * mu[c];
    }
  } else {
#pragma unroll 8
    for (int c = 0; c < a.k; ++c) {
      const double wv = a.W[int64_t(c) * a.n + i];
      ri -= a.AW[int64_t(c) * a.n + i] * cv[c];
      xi += wv * cv[c];
      wmu += wv * mu[c];
    }
  }
  if (a.k > 0) xn += xi;
  a.r[i] = ri;
  a.x[i] = xn;
  const double s = ri + S->beta * pi - wmu;
  a.p[i] = s;
  a.p32[i] = static_cast<float>((a.red.dsc != nullptr) ? a.red.dsc[i] * s : s);
}

// Kernels: one solve (arguments by value), or many columns / systems at once
// (blockIdx.y selects the arguments of a column or system).
__global__ __launch_bounds__(256) void cg_matvec_finish(CgArgs a) { cg_matvec_finish_body(a, blockIdx.x); }
__global__ __launch_bounds__(256) void cg_update_xr(CgArgs a) { cg_update_xr_body<false>(a, blockIdx.x); }
__global__ __launch_bounds__(256) void cg_update_xr_w32(CgArgs a) { cg_update_xr_body<true>(a, blockIdx.x); }
__global__ __launch_bounds__(256) void cg_finalize(CgArgs a) { cg_finalize_body(a); }
__global__ __launch_bounds__(256) void cg_update_p(CgArgs a) { cg_update_p_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void cg_matvec_finish_multi(const CgArgs *args) {
  const CgArgs &a = args[blockIdx.y];
  if (int64_t(blockIdx.x) * kCgRows >= a.n) return;
  cg_matvec_finish_body(a, blockIdx.x);
}
__global__ __launch_bounds__(256) void cg_update_xr_multi(const CgArgs *args) {
  const CgArgs &a = args[blockIdx.y];
  if (int64_t(blockIdx.x) >= a.nblk_xr * xr_groups(a.k)) return;
  cg_update_xr_body<false>(a, blockIdx.x);
}
__global__ __launch_bounds__(256) void cg_finalize_multi(const CgArgs *args) {
  cg_finalize_body(args[blockIdx.y]);
}
__global__ __launch_bounds__(256) void cg_update_p_multi(const CgArgs *args) {
  const CgArgs &a = args[blockIdx.y];
  if (int64_t(blockIdx.x) * 256 >= a.n) return;
  cg_update_p_body(a, blockIdx.x);
}

// -------------------------------------------------- initialisation kernels

// out[c] = sum_i Y[i, c] v[i] for c < m; with Minv != null, out = Minv * out.
// Grid-stride over rows; partials column-major [c][block]; the last block
// sums them in a fixed order.
__global__ __launch_bounds__(256) void ts_dot(const double *Y, int64_t n, int m, const double *v,
                                              double *part, unsigned *counter, const double *Minv,
                                              double *out) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t nblk = gridDim.x;
  for (int c = w; c < m; c += 4) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 64 + l; i < n; i += nblk * 64)
      s += Y[int64_t(c) * n + i] * v[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (l == 0) part[int64_t(c) * nblk + blockIdx.x] = s;
  }
  if (last_block(counter)) {
    __shared__ double h[kMaxZ];
    column_sums(part, nblk, m, h);
    __syncthreads();
    if (Minv != nullptr) small_gemv(Minv, h, out, m);
    else
      for (int c = threadIdx.x; c < m; c += 256) out[c] = h[c];
    if (threadIdx.x == 0) *counter = 0;
  }
}

// x += W c and t = W c (deflated start, Algorithm 1 initialisation; the
// residual is then formed with the product A t).
__global__ __launch_bounds__(256) void defl_start(double *x, double *t, const double *W,
                                                  const double *cvec, int64_t n, int k) {
  __shared__ double cc[kMaxK];
  for (int c = threadIdx.x; c < k; c += 256) cc[c] = cvec[c];
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double ts = 0.0;
  for (int c = 0; c < k; ++c) ts += W[int64_t(c) * n + i] * cc[c];
  x[i] += ts;
  t[i] = ts;
}

// r = b - Ax (or b when Ax is null), x = 0 unless given; partial |b|^2.
__global__ __launch_bounds__(256) void init_residual(const double *b, const double *Ax, double *x,
                                                     double *r, int64_t n, int x_given,
                                                     double *part, unsigned *counter,
                                                     SolveState *S) {
  __shared__ double lds[8];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double bb = 0.0;
  if (i < n) {
    const double bi = b[i];
    if (!x_given) x[i] = 0.0;
    r[i] = (Ax != nullptr) ? bi - Ax[i] : bi;
    bb = bi * bi;
  }
  const double bs = block_sum<256>(bb, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
  if (last_block(counter)) {
    const double s = block_sum_array(part, gridDim.x, lds);
    if (threadIdx.x == 0) {
      S->bnorm = std::sqrt(s);
      *counter = 0;
    }
  }
}

// p_0 = r_0 - W mu_0, rho = r_0^T r_0, FP32 copy of p (padded with zeros).
__global__ __launch_bounds__(256) void init_direction(const double *r, const double *W,
                                                      const double *mu, int64_t n, int64_t n_pad,
                                                      int k, const double *dsc, double *p,
                                                      float *p32, double *part,
                                                      unsigned *counter, SolveState *S,
                                                      double tol, double *hist_res) {
  __shared__ double lds[8];
  __shared__ double mm[kMaxK];
  for (int c = threadIdx.x; c < k; c += 256) mm[c] = mu[c];
  __syncthreads();
  double rr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n_pad;
       i += int64_t(gridDim.x) * 256) {
    if (i < n) {
      const double ri = r[i];
      double s = ri;
      for (int c = 0; c < k; ++c) s -= W[int64_t(c) * n + i] * mm[c];
      p[i] = s;
      p32[i] = static_cast<float>((dsc != nullptr) ? dsc[i] * s : s);
      rr += ri * ri;
    } else {
      p32[i] = 0.0f;
    }
  }
  const double bs = block_sum<256>(rr, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
  if (last_block(counter)) {
    const double s = block_sum_array(part, gridDim.x, lds);
    if (threadIdx.x == 0) {
      S->rho = s;
      S->iter = 0;
      S->applied = 0;
      S->status = 0;
      const double rel = (S->bnorm > 0.0) ? std::sqrt(s) / S->bnorm : 0.0;
      S->relres = rel;
      hist_res[0] = rel;
      S->done = (rel <= tol || !isfinite(s)) ? 1 : 0;
      if (!isfinite(s)) S->status = DCG_E_NONFINITE;
      *counter = 0;
    }
  }
}

// --------------------------------------------------- tall-skinny products

// part[chunk] = A[rows of chunk]^T B[rows of chunk] (ma x mb, row-major).
// Block: a 32x32 output tile over a 1024-row chunk, 64-row LDS sub-chunks.
__global__ __launch_bounds__(256) void tsgemm_tn(const double *A, const double *B, int64_t n,
                                                 int ma, int mb, double *part, int64_t chunk_rows) {
  __shared__ double As[64][33];
  __shared__ double Bs[64][33];
  const int tiles_b = (mb + 31) / 32;
  const int ta = blockIdx.x / tiles_b, tb = blockIdx.x % tiles_b;
  const int chunk = blockIdx.y;
  const int64_t r0 = int64_t(chunk) * chunk_rows;
  const int64_t r1 = std::min<int64_t>(n, r0 + chunk_rows);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // 16 x 16 threads, 2x2 outputs each
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t s = r0; s < r1; s += 64) {
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int rr = e % 64, cc = e / 64;
      const int64_t row = s + rr;
      const int ca = ta * 32 + cc, cb = tb * 32 + cc;
      As[rr][cc] = (row < r1 && ca < ma) ? A[int64_t(ca) * n + row] : 0.0;
      Bs[rr][cc] = (row < r1 && cb < mb) ? B[int64_t(cb) * n + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 64; ++rr) {
      const double a0 = As[rr][ty], a1 = As[rr][ty + 16];
      const double b0 = Bs[rr][tx], b1 = Bs[rr][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  double *out = part + int64_t(chunk) * ma * mb;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int ia = ta * 32 + ty + 16 * u, ib = tb * 32 + tx + 16 * v;
      if (ia < ma && ib < mb) out[int64_t(ia) * mb + ib] = acc[u][v];
    }
}

// C = sum over chunks of the partials (fixed order), optionally symmetrised.
__global__ __launch_bounds__(256) void tsgemm_sum(const double *part, int nchunk, int ma, int mb,
                                                  double *C, int ldc, int symmetrise) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ma * mb) return;
  const int i = e / mb, j = e % mb;
  double s = 0.0, t = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[int64_t(c) * ma * mb + e];
  if (symmetrise) {
    for (int c = 0; c < nchunk; ++c) t += part[int64_t(c) * ma * mb + j * mb + i];
    s = 0.5 * (s + t);
  }
  C[i * ldc + j] = s;
}

// Y[:, j] (+)= X[:, 0:m] U[:, j] for j < kout (U row-major m x ldu), 32
// columns per pass with U staged in LDS.  Columns c >= round_from of X are
// taken as the FP32 copy the low-precision sweep multiplies (fp32(x), or
// fp32(d x) / d with a diagonal scaling d, x itself where d = 0); accumulate
// adds to Y instead of overwriting it.
__global__ __launch_bounds__(256) void ts_times_small(const double *X, int64_t n, int m,
                                                      const double *U, int ldu, int kout,
                                                      double *Y, int round_from,
                                                      const double *dsc, int accumulate) {
  __shared__ double Us[kMaxZ + 1][32];
  const int j0 = blockIdx.y * 32;
  const int jn = std::min(32, kout - j0);
  for (int e = threadIdx.x; e < m * 32; e += 256) {
    const int c = e / 32, j = e % 32;
    Us[c][j] = (j < jn) ? U[c * ldu + j0 + j] : 0.0;
  }
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double di = (dsc != nullptr) ? dsc[i] : 1.0;
  double acc[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) acc[j] = 0.0;
  for (int c = 0; c < m; ++c) {
    double xv = X[int64_t(c) * n + i];
    if (c >= round_from) {
      if (dsc == nullptr) xv = static_cast<double>(static_cast<float>(xv));
      else if (di != 0.0) xv = static_cast<double>(static_cast<float>(di * xv)) / di;
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] += xv * Us[c][j];
  }
#pragma unroll
  for (int j = 0; j < 32; ++j)
    if (j < jn) {
      double *y = Y + int64_t(j0 + j) * n + i;
      *y = accumulate ? *y + acc[j] : acc[j];
    }
}

// Y += alpha X (n x m blocks, same layout).
__global__ __launch_bounds__(256) void block_axpy(double *Y, const double *X, double alpha,
                                                  int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e < count) Y[e] += alpha * X[e];
}

// Y = fp32(Y) elementwise, in place.
__global__ __launch_bounds__(256) void round_to_fp32(double *Y, int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e < count) Y[e] = static_cast<double>(static_cast<float>(Y[e]));
}

__global__ __launch_bounds__(256) void to_float(const double *Y, float *Y32, int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e < count) Y32[e] = static_cast<float>(Y[e]);
}

// Symmetrise M (k x k, row-major), Cholesky M = R R^T, Minv = M^{-1}.
// One block.  info = 0 on success; 2 if M holds a NaN or Inf; 1 if a pivot
// is at most kRankTol times the diagonal entry it started from (the square
// of the sine of the angle, in the A inner product, between that column of W
// and the span of the columns before it: W is numerically rank deficient
// against A, or M is not positive definite).
constexpr double kRankTol = 1e-12;
__global__ __launch_bounds__(256) void small_spd_inverse(const double *Min, int k, double *Minv,
                                                         double *work, int *info) {
  __shared__ double Ls[kMaxK][kMaxK + 1];
  __shared__ double diag0[kMaxK];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int i = e / k, j = e % k;
    const double v = 0.5 * (Min[i * k + j] + Min[j * k + i]);
    if (!isfinite(v)) atomicMax(&bad, 2);
    Ls[i][j] = v;
    if (i == j) diag0[i] = v;
  }
  __syncthreads();
  // right-looking Cholesky, lower triangle
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x == 0) {
      const double piv = Ls[j][j];
      const bool ok = piv > kRankTol * diag0[j] && diag0[j] > 0.0;
      if (!ok && bad == 0) bad = 1;
      Ls[j][j] = ok ? std::sqrt(piv) : 1.0;
    }
    __syncthreads();
    const double djj = Ls[j][j];
    for (int i = j + 1 + threadIdx.x; i < k; i += 256) Ls[i][j] /= djj;
    __syncthreads();
    for (int e = threadIdx.x; e < (k - j - 1) * (k - j - 1); e += 256) {
      const int i = j + 1 + e / (k - j - 1), c = j + 1 + e % (k - j - 1);
      if (c <= i) Ls[i][c] -= Ls[i][j] * Ls[c][j];
    }
    __syncthreads();
  }
  // inverse of L by columns (thread c solves L y = e_c), then Minv = L^-T L^-1
  for (int c = threadIdx.x; c < k; c += 256) {
    for (int i = 0; i < k; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int t = c; t < i; ++t) s -= Ls[i][t] * work[t * kMaxK + c];
      work[i * kMaxK + c] = (i < c) ? 0.0 : s / Ls[i][i];
    }
  }
  __syncthreads();
  __threadfence_block();
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int i = e / k, j = e % k;
    double s = 0.0;
    for (int t = std::max(i, j); t < k; ++t) s += work[t * kMaxK + i] * work[t * kMaxK + j];
    Minv[i * k + j] = s;
  }
  if (threadIdx.x == 0) *info = bad;
}

// ---------------------------------------------------------- host wrappers

void enqueue_ts_dot(hipStream_t s, const double *Y, int64_t n, int m, const double *v,
                    double *part, unsigned *counter, const double *Minv, double *out) {
  const int grid = static_cast<int>(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, cdiv(n, 256))));
  hipLaunchKernelGGL(ts_dot, dim3(grid), dim3(256), 0, s, Y, n, m, v, part, counter, Minv, out);
}

void enqueue_tsgemm_tn(hipStream_t s, const double *A, const double *B, int64_t n, int ma, int mb,
                       double *part, size_t part_cap, double *C, int ldc, int symmetrise) {
  int64_t chunk_rows = 1024;
  int64_t nchunk = cdiv(n, chunk_rows);
  while (size_t(nchunk) * ma * mb > part_cap) {
    chunk_rows *= 2;
    nchunk = cdiv(n, chunk_rows);
  }
  const int tiles = ((ma + 31) / 32) * ((mb + 31) / 32);
  hipLaunchKernelGGL(tsgemm_tn, dim3(tiles, static_cast<unsigned>(nchunk)), dim3(256), 0, s, A, B,
                     n, ma, mb, part, chunk_rows);
  hipLaunchKernelGGL(tsgemm_sum, dim3(static_cast<unsigned>(cdiv(int64_t(ma) * mb, 256))), dim3(256),
                     0, s, part, static_cast<int>(nchunk), ma, mb, C, ldc, symmetrise);
}

void enqueue_ts_times_small(hipStream_t s, const double *X, int64_t n, int m, const double *U,
                            int ldu, int kout, double *Y, int round_from, const double *dsc,
                            int accumulate) {
  if (kout <= 0 || n <= 0) return;
  hipLaunchKernelGGL(ts_times_small, dim3(static_cast<unsigned>(cdiv(n, 256)), (kout + 31) / 32),
                     dim3(256), 0, s, X, n, m, U, ldu, kout, Y, round_from, dsc, accumulate);
}

void enqueue_block_axpy(hipStream_t s, double *Y, const double *X, double alpha, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(block_axpy, dim3(static_cast<unsigned>(cdiv(count, 256))), dim3(256), 0, s, Y,
                     X, alpha, count);
}

void enqueue_to_float(hipStream_t s, const double *Y, float *Y32, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(to_float, dim3(static_cast<unsigned>(cdiv(count, 256))), dim3(256), 0, s, Y,
                     Y32, count);
}

void enqueue_round_to_fp32(hipStream_t s, double *Y, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(round_to_fp32, dim3(static_cast<unsigned>(cdiv(count, 256))), dim3(256), 0, s,
                     Y, count);
}

void enqueue_small_spd_inverse(hipStream_t s, const double *M, int k, double *Minv, double *work,
                               int *info) {
  hipLaunchKernelGGL(small_spd_inverse, dim3(1), dim3(256), 0, s, M, k, Minv, work, info);
}

}  // namespace dcg

namespace dcg {

// out = b - Ax; sums[0] = |out|^2, sums[1] = |b|^2 (last block, fixed order).
__global__ __launch_bounds__(256) void residual_norms(const double *b, const double *Ax, int64_t n,
                                                     double *out, double *part, unsigned *counter,
                                                     double *sums) {
  __shared__ double lds[8];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double bi = b[i];
    const double ri = (Ax != nullptr) ? bi - Ax[i] : bi;
    out[i] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  const double s1 = block_sum<256>(rr, lds);
  const double s2 = block_sum<256>(bb, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
  if (last_block(counter)) {
    if (threadIdx.x == 0) {
      double a = 0.0, c = 0.0;
      for (unsigned k = 0; k < gridDim.x; ++k) {
        a += part[2 * k];
        c += part[2 * k + 1];
      }
      sums[0] = a;
      sums[1] = c;
      *counter = 0;
    }
  }
}

}  // namespace dcg
