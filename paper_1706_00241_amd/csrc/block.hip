// Many right-hand sides with one operator (the probe solves of the GP
// gradient): every column runs its own deflated CG (Algorithm 1 with the
// per-step residual re-projection) on the basis W of the recycle handle,
// which is reused as it is (not refreshed).  The products of a step are one
// 4-vector block sweep per group of four columns, so each kernel value is
// evaluated once per group; the vector kernels take all columns at once
// (blockIdx.y = column).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "blas.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kBlockHist = 1024;

// C (k x m, ld m) = A (k x k, ld k) B (k x m, ld m); one block.
__global__ __launch_bounds__(256) void small_gemm(const double *A, const double *B, int k, int m,
                                                  double *C) {
  for (int e = threadIdx.x; e < k * m; e += 256) {
    const int i = e / m, j = e % m;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * m + j];
    C[e] = s;
  }
}

// Per column c (one block each): |b_c|, rho_c = |r_c|^2, the solve state,
// and the FP32 copy of p_c (zero padded; columns >= m of the last group zero).
__global__ __launch_bounds__(256) void block_init(const double *B, const double *R,
                                                  const double *P, int64_t n, int64_t n_pad,
                                                  int m, SolveState *S, float *P32, double tol) {
  __shared__ double lds[2][4];
  const int c = blockIdx.x;
  double bb = 0.0, rr = 0.0;
  for (int64_t i = threadIdx.x; i < n_pad; i += 256) {
    float pv = 0.0f;
    if (c < m && i < n) {
      const double bv = B[int64_t(c) * n + i], rv = R[int64_t(c) * n + i];
      bb += bv * bv;
      rr += rv * rv;
      pv = static_cast<float>(P[int64_t(c) * n + i]);
    }
    P32[int64_t(c) * n_pad + i] = pv;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    bb += __shfl_xor(bb, o);
    rr += __shfl_xor(rr, o);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    lds[0][w] = bb;
    lds[1][w] = rr;
  }
  __syncthreads();
  if (threadIdx.x == 0 && c < m) {
    const double b2 = (lds[0][0] + lds[0][1]) + (lds[0][2] + lds[0][3]);
    const double r2 = (lds[1][0] + lds[1][1]) + (lds[1][2] + lds[1][3]);
    SolveState &s = S[c];
    s.bnorm = std::sqrt(b2);
    s.rho = r2;
    s.iter = 0;
    s.applied = 0;
    s.status = 0;
    const double rel = (b2 > 0.0) ? std::sqrt(r2 / b2) : 0.0;
    s.relres = rel;
    s.done = (rel <= tol || !isfinite(r2)) ? 1 : 0;
    if (!isfinite(r2)) s.status = DCG_E_NONFINITE;
  }
}

struct BlockLayout {
  size_t args, S, R, P, Q, T, P32, part, part2, parth, hist, Cm, Cm2, gemm, total;
};

static BlockLayout block_layout(int64_t n, int64_t m) {
  BlockLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const int64_t n_pad = ((n + 255) / 256) * 256;
  const int64_t m4 = ((m + 3) / 4) * 4;
  const int64_t nq = cdiv(n, kCgRows), nx = cdiv(n, kXrRows);
  L.args = take(size_t(m) * sizeof(CgArgs));
  L.S = take(size_t(m) * sizeof(SolveState));
  L.R = take(size_t(n) * m * 8);
  L.P = take(size_t(n) * m * 8);
  L.Q = take(size_t(n) * m * 8);
  L.T = take(size_t(n) * m * 8);
  L.P32 = take(size_t(n_pad) * m4 * 4);
  L.part = take(size_t(m) * nq * 8);
  L.part2 = take(size_t(m) * nx * 8);
  L.parth = take(size_t(m) * 2 * kMaxK * nx * 8);
  L.hist = take(size_t(m) * (kBlockHist + 3 * kMaxZ) * 8);
  L.Cm = take(size_t(kMaxK) * m * 8);
  L.Cm2 = take(size_t(kMaxK) * m * 8);
  L.gemm = take(size_t(64) * kMaxK * m * 8);
  L.total = align256(off);
  return L;
}

#define HIPCHK(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return DCG_E_HIP; \
  } while (0)

}  // namespace dcg

using namespace dcg;

// The block solve; with lz (device, m x 2 x lz_cap doubles) it also records
// every column's alpha_j (first lz_cap) and beta_j (next lz_cap) for
// j < lz_cap, and with col_iters / col_bnorm (host, m each) it returns each
// column's step count and |b_c|.
int dcg::solve_block_impl(dcg_op_t op, const double *B, double *X, int64_t m, dcg_recycle_t rc,
                          const dcg_params *p, dcg_stats *st, void *ws, size_t ws_bytes,
                          double *lz, int lz_cap, int *col_iters, double *col_bnorm) {
  dcg_stats local;
  if (st == nullptr) st = &local;
  std::memset(st, 0, sizeof(*st));
  if (op == nullptr || B == nullptr || X == nullptr || p == nullptr) return st->status = DCG_E_ARG;
  // products finished per column (FP64 and stored operators) take any
  // diagonal scaling; the four-column low-precision sweep takes none
  const bool stored = op->g.prec == DCG_PREC_STORED;
  const bool direct = op->g.prec == DCG_PREC_FP64 || stored;
  if (op->has_dsc && !direct) return st->status = DCG_E_ARG;
  if (sweep_wide(op->g)) return st->status = DCG_E_ARG;   // single-vector sweep only
  if (m < 1 || m > kMaxBlockCols || !(p->tol >= 0.0)) return st->status = DCG_E_ARG;
  if (rc != nullptr && rc->n != op->g.n) return st->status = DCG_E_ARG;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  const BlockLayout Lb = block_layout(n, m);
  if (ws == nullptr || ws_bytes < Lb.total) return st->status = DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return st->status = DCG_E_WORKSPACE;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = op->stream;
  char *base = static_cast<char *>(ws);
  CgArgs *d_args = reinterpret_cast<CgArgs *>(base + Lb.args);
  SolveState *S = reinterpret_cast<SolveState *>(base + Lb.S);
  double *R = reinterpret_cast<double *>(base + Lb.R);
  double *P = reinterpret_cast<double *>(base + Lb.P);
  double *Q = reinterpret_cast<double *>(base + Lb.Q);
  double *T = reinterpret_cast<double *>(base + Lb.T);
  float *P32 = reinterpret_cast<float *>(base + Lb.P32);
  double *part = reinterpret_cast<double *>(base + Lb.part);
  double *part2 = reinterpret_cast<double *>(base + Lb.part2);
  double *parth = reinterpret_cast<double *>(base + Lb.parth);
  double *hist = reinterpret_cast<double *>(base + Lb.hist);
  double *Cm = reinterpret_cast<double *>(base + Lb.Cm);
  double *Cm2 = reinterpret_cast<double *>(base + Lb.Cm2);
  double *gemm = reinterpret_cast<double *>(base + Lb.gemm);
  const size_t gemm_cap = size_t(64) * kMaxK * m;
  const int max_iter = p->max_iter > 0 ? p->max_iter : static_cast<int>(std::min<int64_t>(10 * n, 1 << 30));

  int matvecs = 0;
  int k = 0;
  if (rc != nullptr && rc->k_used > 0) {
    const int rcode = deflation_setup(op, rc, &matvecs);
    if (rcode != DCG_OK) return st->status = rcode;
    k = rc->k_used;
  }
  HIPCHK(hipMemsetAsync(X, 0, size_t(n) * m * 8, s));
  HIPCHK(hipMemcpyAsync(R, B, size_t(n) * m * 8, hipMemcpyDeviceToDevice, s));
  if (k > 0) {
    // deflated start for every column: C = M^-1 W^T R, X = W C, R = B - A (W C)
    enqueue_tsgemm_tn(s, rc->Z, R, n, k, static_cast<int>(m), gemm, gemm_cap, Cm, static_cast<int>(m), 0);
    hipLaunchKernelGGL(small_gemm, dim3(1), dim3(256), 0, s, rc->Minv, Cm, k, static_cast<int>(m), Cm2);
    enqueue_ts_times_small(s, rc->Z, n, k, Cm2, static_cast<int>(m), static_cast<int>(m), T);
    HIPCHK(hipMemcpyAsync(X, T, size_t(n) * m * 8, hipMemcpyDeviceToDevice, s));
    int rcode = matvec_lowprec(op, T, Q, m);
    if (rcode != DCG_OK) return st->status = rcode;
    matvecs += static_cast<int>(m);
    enqueue_block_axpy(s, R, Q, -1.0, n * m);
    // P = R - W M^-1 (AW)^T R
    enqueue_tsgemm_tn(s, rc->AZ, R, n, k, static_cast<int>(m), gemm, gemm_cap, Cm, static_cast<int>(m), 0);
    hipLaunchKernelGGL(small_gemm, dim3(1), dim3(256), 0, s, rc->Minv, Cm, k, static_cast<int>(m), Cm2);
    enqueue_ts_times_small(s, rc->Z, n, k, Cm2, static_cast<int>(m), static_cast<int>(m), T);
    HIPCHK(hipMemcpyAsync(P, R, size_t(n) * m * 8, hipMemcpyDeviceToDevice, s));
    enqueue_block_axpy(s, P, T, -1.0, n * m);
  } else {
    HIPCHK(hipMemcpyAsync(P, R, size_t(n) * m * 8, hipMemcpyDeviceToDevice, s));
  }
  const int64_t m4 = ((m + 3) / 4) * 4;
  hipLaunchKernelGGL(block_init, dim3(static_cast<unsigned>(m4)), dim3(256), 0, s, B, R, P, n, n_pad,
                     static_cast<int>(m), S, P32, p->tol);
  HIPCHK(hipGetLastError());

  // per-column arguments of the vector kernels
  const int64_t nq = cdiv(n, kCgRows), nx = cdiv(n, kXrRows);
  std::vector<CgArgs> args(static_cast<size_t>(m));
  for (int64_t c = 0; c < m; ++c) {
    CgArgs &a = args[static_cast<size_t>(c)];
    std::memset(&a, 0, sizeof(a));
    a.S = S + c;
    if (!direct) a.red = reduce_args(op, 4, nullptr, nullptr);
    a.qdirect = direct ? Q + c * n : nullptr;
    a.mcol = static_cast<int>(c % 4);
    a.n = n;
    a.x = X + c * n;
    a.r = R + c * n;
    a.p = P + c * n;
    a.q = Q + c * n;
    a.p32 = P32 + c * n_pad;
    a.W = k > 0 ? rc->Z : nullptr;
    a.AW = k > 0 ? rc->AZ : nullptr;
    a.W32 = (k > 0 && rc->w32_valid) ? rc->W32 : nullptr;
    a.AW32 = (k > 0 && rc->w32_valid) ? rc->AW32 : nullptr;
    a.Minv = k > 0 ? rc->Minv : nullptr;
    a.N = k > 0 ? rc->N : nullptr;
    a.k = k;
    a.Z = nullptr;
    a.AZ = nullptr;
    a.koff = 0;
    a.L = 0;
    a.part = part + c * nq;
    a.part2 = part2 + c * nx;
    a.part_h = parth + c * 2 * kMaxK * nx;
    cg_set_blocks(a);
    a.counter = nullptr;
    double *h = hist + c * (kBlockHist + 3 * kMaxZ);
    a.hist_res = h;
    a.hist_cap = kBlockHist;
    a.hist_d = h + kBlockHist;
    a.hist_alpha = h + kBlockHist + kMaxZ;
    a.hist_beta = h + kBlockHist + 2 * kMaxZ;
    a.lz_alpha = (lz != nullptr) ? lz + c * 2 * lz_cap : nullptr;
    a.lz_beta = (lz != nullptr) ? lz + c * 2 * lz_cap + lz_cap : nullptr;
    a.lz_cap = lz_cap;
    a.tol = p->tol;
    a.max_iter = max_iter;
  }
  HIPCHK(hipMemcpyAsync(d_args, args.data(), sizeof(CgArgs) * m, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();

  const int chunk = std::max(1, p->check_every);
  std::vector<SolveState> hs(static_cast<size_t>(m));
  const int groups = static_cast<int>(m4 / 4);
  int sweeps = 0;
  while (true) {
    for (int step = 0; step < chunk; ++step) {
      if (direct) {
        for (int64_t c = 0; c < m; ++c) {
          const int rcode = stored ? matvec_stored_done(op, P + c * n, Q + c * n, 1, &S[c].done)
                                   : matvec_exact_done(op, P + c * n, Q + c * n, 1, &S[c].done);
          if (rcode != DCG_OK) return st->status = rcode;
        }
        hipLaunchKernelGGL(cg_matvec_finish_multi, dim3(static_cast<unsigned>(nq), static_cast<unsigned>(m)),
                           dim3(256), 0, s, d_args);
      } else {
        for (int g = 0; g < groups; ++g) {
          const int rcode = launch_symv_sweep_from(op, 4, P32 + int64_t(4 * g) * n_pad, nullptr);
          if (rcode != DCG_OK) return st->status = rcode;
          const int cols = static_cast<int>(std::min<int64_t>(4, m - 4 * g));
          hipLaunchKernelGGL(cg_matvec_finish_multi, dim3(static_cast<unsigned>(nq), static_cast<unsigned>(cols)),
                             dim3(256), 0, s, d_args + 4 * g);
          ++sweeps;
        }
      }
      hipLaunchKernelGGL(cg_update_xr_multi, dim3(static_cast<unsigned>(xr_grid(args[0])), static_cast<unsigned>(m)),
                         dim3(256), 0, s, d_args);
      hipLaunchKernelGGL(cg_finalize_multi, dim3(1, static_cast<unsigned>(m)), dim3(256), 0, s, d_args);
      hipLaunchKernelGGL(cg_update_p_multi, dim3(static_cast<unsigned>(args[0].nblk_p), static_cast<unsigned>(m)),
                         dim3(256), 0, s, d_args);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(hs.data(), S, sizeof(SolveState) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    for (const SolveState &x : hs) all = all && x.done;
    if (all) break;
  }
  int iters = 0, status = DCG_OK;
  double worst = 0.0;
  for (const SolveState &x : hs) {
    iters = std::max(iters, x.iter);
    worst = std::max(worst, x.relres);
    if (x.status < 0) status = x.status;
    else if (status == DCG_OK && x.relres > p->tol) status = DCG_NOT_CONVERGED;
  }
  st->iters = iters;
  st->matvecs = matvecs + (direct ? iters * static_cast<int>(m) : sweeps * 4);
  st->k_used = k;
  st->k_next = k;
  st->rel_res_recursive = worst;
  st->status = status;
  st->t_init_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  st->t_loop_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  st->t_total_ms = st->t_init_ms + st->t_loop_ms;
  for (int64_t c = 0; c < m; ++c) {
    if (col_iters != nullptr) col_iters[c] = hs[static_cast<size_t>(c)].iter;
    if (col_bnorm != nullptr) col_bnorm[c] = hs[static_cast<size_t>(c)].bnorm;
  }
  return status;
}

extern "C" {

size_t dcg_solve_block_workspace_bytes(int64_t n, int64_t m) {
  if (n < 1 || m < 1 || m > kMaxBlockCols) return 0;
  return block_layout(n, m).total;
}

int dcg_solve_block(dcg_op_t op, const double *B, double *X, int64_t m, dcg_recycle_t rc,
                    const dcg_params *p, dcg_stats *st, void *ws, size_t ws_bytes) {
  return solve_block_impl(op, B, X, m, rc, p, st, ws, ws_bytes, nullptr, 0, nullptr, nullptr);
}

}  // extern "C"
