// Host driver of deflated CG (Algorithm 1 of the paper) with the harmonic
// Ritz refresh of the recycled basis (section 2.3, Eq. 7), plus the
// mixed-precision iterative refinement around it.
//
// Per CG step five kernels run on the operator's stream: the symmetric pair
// sweep (q = A p partials), the product finish with the block partials of
// d = p^T q, the pass over r' = r - alpha q with the partials of rho' and
// h = (AW)^T r', g = W^T r', one block for the scalar step (re-projection,
// mu, beta, the convergence test), and the direction update
// p = beta p + r - W mu.  All scalars stay on the device; the host reads the
// solve state once per chunk of iterations (optionally replayed as one
// captured hipGraph), so the loop has one host round trip per chunk.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "solve.h"

namespace dcg {

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kHistCap = 1 << 16;
constexpr size_t kGemmPartDoubles = size_t(64) * kMaxZ * kMaxZ;

// Outer directions kept by the flexible-CG refinement.
constexpr int kFcgCap = 32;

struct SolveLayout {
  size_t S, counter, r, p, q, part, part_h, hist_res, hist_d, hist_alpha, hist_beta, hist_rho,
      hist_mu, hist_c, tmp1, tmp2, tmp3, core, fD, fQ, total;
};

static SolveLayout solve_layout(int64_t n) {
  SolveLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t nb = size_t(std::max<int64_t>(2 * cdiv(n, 64) + 2, kRedBlocks));
  L.S = take(sizeof(SolveState));
  L.counter = take(sizeof(unsigned) * 8);
  L.r = take(size_t(n) * 8);
  L.p = take(size_t(n) * 8);
  L.q = take(size_t(n) * 8);
  L.part = take(nb * 8);
  L.part_h = take(nb * kMaxZ * 8);
  L.hist_res = take(size_t(kHistCap) * 8);
  L.hist_d = take(size_t(kMaxZ) * 8);
  L.hist_alpha = take(size_t(kMaxZ) * 8);
  L.hist_beta = take(size_t(kMaxZ) * 8);
  L.hist_rho = take(size_t(kMaxZ + 1) * 8);
  L.hist_mu = take(size_t(kMaxZ + 1) * kMaxK * 8);
  L.hist_c = take(size_t(kMaxZ) * kMaxK * 8);
  L.tmp1 = take(size_t(n) * 8);
  L.tmp2 = take(size_t(n) * 8);
  L.tmp3 = take(size_t(n) * 8);
  L.core = align256(off);
  // the refinement's outer directions and their FP64 products
  L.fD = take(size_t(n) * kFcgCap * 8);
  L.fQ = take(size_t(n) * kFcgCap * 8);
  L.total = align256(off);
  return L;
}

size_t solve_workspace_total(int64_t n, bool refine) {
  const SolveLayout L = solve_layout(n);
  return refine ? L.total : L.core;
}

struct RecycleLayout {
  size_t Z, AZ, Wt, AWt, W32, AW32, F, G, U, eigw, M, Minv, Mwork, N, small, info, gemm, total;
};

static RecycleLayout recycle_layout(int64_t n, int k, int L) {
  RecycleLayout R;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t kz = size_t(k + L);
  R.Z = take(size_t(n) * (kz + 1) * 8);   // + p_L for the implicit extraction
  R.AZ = take(size_t(n) * kz * 8);
  R.Wt = take(size_t(n) * k * 8);
  R.AWt = take(size_t(n) * k * 8);
  R.W32 = take(size_t(n) * k * 4);
  R.AW32 = take(size_t(n) * k * 4);
  R.F = take(size_t(kMaxZ) * kMaxZ * 8);
  R.G = take(size_t(kMaxZ) * kMaxZ * 8);
  R.U = take(size_t(kMaxZ) * kMaxK * 8);
  R.eigw = take(harmonic_ritz_work_doubles() * 8);
  R.M = take(size_t(kMaxK) * kMaxK * 8);
  R.Minv = take(size_t(kMaxK) * kMaxK * 8);
  R.Mwork = take(size_t(kMaxK) * kMaxK * 8);
  R.N = take(size_t(kMaxK) * kMaxK * 8);
  R.small = take(size_t(kMaxZ) * 8);
  R.info = take(64);
  R.gemm = take(kGemmPartDoubles * 8);
  R.total = align256(off);
  return R;
}

SolveBuffers solve_buffers(void *ws, int64_t n) {
  const SolveLayout L = solve_layout(n);
  char *b = static_cast<char *>(ws);
  SolveBuffers B;
  B.S = reinterpret_cast<SolveState *>(b + L.S);
  B.counter = reinterpret_cast<unsigned *>(b + L.counter);
  B.r = reinterpret_cast<double *>(b + L.r);
  B.p = reinterpret_cast<double *>(b + L.p);
  B.q = reinterpret_cast<double *>(b + L.q);
  B.part = reinterpret_cast<double *>(b + L.part);
  B.part_h = reinterpret_cast<double *>(b + L.part_h);
  B.hist_res = reinterpret_cast<double *>(b + L.hist_res);
  B.hist_d = reinterpret_cast<double *>(b + L.hist_d);
  B.hist_alpha = reinterpret_cast<double *>(b + L.hist_alpha);
  B.hist_beta = reinterpret_cast<double *>(b + L.hist_beta);
  B.hist_rho = reinterpret_cast<double *>(b + L.hist_rho);
  B.hist_mu = reinterpret_cast<double *>(b + L.hist_mu);
  B.hist_c = reinterpret_cast<double *>(b + L.hist_c);
  B.tmp1 = reinterpret_cast<double *>(b + L.tmp1);
  B.tmp2 = reinterpret_cast<double *>(b + L.tmp2);
  B.tmp3 = reinterpret_cast<double *>(b + L.tmp3);
  B.fD = reinterpret_cast<double *>(b + L.fD);
  B.fQ = reinterpret_cast<double *>(b + L.fQ);
  return B;
}

// Make AZ[:, :k_used] the product of W with the current operator.
static int refresh_AW(dcg_operator_s *op, dcg_recycle_s *rc, int *matvecs) {
  const int k = rc->k_used;
  if (k == 0) return DCG_OK;
  const int64_t n = rc->n;
  const bool same_op = rc->aw_state == 1 && rc->aw_op == op;
  if (same_op && rc->aw_gen == op->generation) return DCG_OK;
  if (same_op && rc->aw_ell == op->ell && rc->aw_s2 == op->s2 && rc->aw_dsc == op->dsc_version) {
    // only the diagonal shift changed: A_new W = A_old W + (s_new - s_old) W
    enqueue_block_axpy(op->stream, rc->AZ, rc->Z, op->sigma2 - rc->aw_sigma2, n * k);
  } else {
    // the low-precision sweep multiplies the FP32 copy of W: make W that
    // copy (it is only a basis), so that AW is A~ W to the sweep's
    // evaluation error rather than to W's rounding
    if (op->g.prec != DCG_PREC_FP64 && op->g.prec != DCG_PREC_STORED && !op->has_dsc)
      enqueue_round_to_fp32(op->stream, rc->Z, n * k);
    const int st = matvec_lowprec(op, rc->Z, rc->AZ, k);
    if (st != DCG_OK) return st;
    *matvecs += k;
  }
  rc->aw_state = 1;
  rc->aw_op = op;
  rc->aw_gen = op->generation;
  rc->aw_ell = op->ell;
  rc->aw_s2 = op->s2;
  rc->aw_sigma2 = op->sigma2;
  rc->aw_dsc = op->dsc_version;
  rc->w_version += 1;
  return DCG_OK;
}

// AW for the current operator, then M = W^T A W, N = (AW)^T AW and M^{-1},
// recomputed only when W or AW changed since the last time.
int deflation_setup(dcg_operator_s *op, dcg_recycle_s *rc, int *matvecs) {
  const int k = rc->k_used;
  if (k == 0) return DCG_OK;
  int st = refresh_AW(op, rc, matvecs);
  if (st != DCG_OK) return st;
  if (rc->m_valid && rc->m_version == rc->w_version) return DCG_OK;
  hipStream_t s = op->stream;
  const int64_t n = rc->n;
  // With bf16 or fp16 points (8 or 11 significant bits: the operator is off
  // the kernel matrix by ~1e-3 relative) the per-step kernels read FP32
  // copies of W and AW, half the bytes of the two passes over them each
  // step.  W and AW are rounded to FP32 values first, so that M, N and
  // every later use see exactly the values the copies hold.  Not for FP32
  // or split-bf16 points, whose solves run to 1e-6 on the operator itself
  // (there the rounding added steps: 219 -> 224 on the 16384-point walk),
  // and not with a diagonal scaling, where the sweep multiplies fp32(D w)
  // rather than fp32(w) and W keeps its FP64 values (as in refresh_AW).
  const bool lowprec =
      (op->g.prec == DCG_PREC_BF16 || op->g.prec == DCG_PREC_FP16) && !op->has_dsc;
  if (lowprec) {
    enqueue_round_to_fp32(s, rc->Z, n * k);
    enqueue_round_to_fp32(s, rc->AZ, n * k);
  }
  enqueue_tsgemm_tn(s, rc->Z, rc->AZ, n, k, k, rc->gemm, kGemmPartDoubles, rc->M, k, 1);
  enqueue_tsgemm_tn(s, rc->AZ, rc->AZ, n, k, k, rc->gemm, kGemmPartDoubles, rc->N, k, 1);
  enqueue_small_spd_inverse(s, rc->M, k, rc->Minv, rc->Mwork, rc->info);
  rc->w32_valid = 0;
  if (lowprec) {
    enqueue_to_float(s, rc->Z, rc->W32, n * k);
    enqueue_to_float(s, rc->AZ, rc->AW32, n * k);
  }
  int info = 0;
  HIPCHK(hipMemcpyAsync(&info, rc->info, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // W^T A W is SPD for a full-rank W and an SPD operator: a failed
  // factorisation means W (against A) is numerically rank deficient
  if (info == 2) return DCG_E_NONFINITE;
  if (info != 0) return DCG_E_W_RANK;
  rc->m_valid = 1;
  rc->m_version = rc->w_version;
  rc->w32_valid = lowprec ? 1 : 0;
  return DCG_OK;
}

static CgArgs cg_args(dcg_operator_s *op, const SolveBuffers &B, double *x, dcg_recycle_s *rc,
                      const double *Minv, int k, int L, int koff, double tol, int max_iter) {
  CgArgs a;
  a.S = B.S;
  a.red = reduce_args(op, 1, nullptr, nullptr);
  a.qdirect = (op->g.prec == DCG_PREC_FP64 || op->g.prec == DCG_PREC_STORED) ? op->ytmp : nullptr;
  a.mcol = 0;
  a.n = op->g.n;
  a.x = x;
  a.r = B.r;
  a.p = B.p;
  a.q = B.q;
  a.p32 = op->vin;
  a.W = rc ? rc->Z : nullptr;
  a.AW = rc ? rc->AZ : nullptr;
  if (rc != nullptr && k > 0 && rc->w32_valid) {
    a.W32 = rc->W32;
    a.AW32 = rc->AW32;
  }
  a.Minv = Minv;
  a.N = rc ? rc->N : nullptr;
  a.k = k;
  a.Z = (rc && L > 0) ? rc->Z : nullptr;
  a.AZ = (rc && L > 0) ? rc->AZ : nullptr;
  a.koff = koff;
  a.L = L;
  cg_set_blocks(a);
  a.part = B.part;
  a.part2 = B.part + std::max<int64_t>(a.nblk_q, 1);
  a.part_h = B.part_h;
  a.counter = B.counter;
  a.hist_d = B.hist_d;
  a.hist_alpha = B.hist_alpha;
  a.hist_beta = B.hist_beta;
  a.hist_res = B.hist_res;
  a.hist_cap = kHistCap;
  a.lz_alpha = nullptr;
  a.lz_beta = nullptr;
  a.lz_cap = 0;
  a.tol = tol;
  a.max_iter = max_iter;
  return a;
}

// Timing events around the product: inside a stream capture they become
// event-record nodes of the graph, so replays time the graph's own launches.
static hipError_t record_event(hipEvent_t ev, hipStream_t s, bool in_graph) {
  return in_graph ? hipEventRecordWithFlags(ev, s, hipEventRecordExternal) : hipEventRecord(ev, s);
}

static int enqueue_cg_step(dcg_operator_s *op, const CgArgs &a, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr, bool in_graph = false) {
  if (ev0 != nullptr && record_event(ev0, op->stream, in_graph) != hipSuccess) return DCG_E_HIP;
  int st;
  if (op->g.prec == DCG_PREC_FP64) st = matvec_exact_done(op, a.p, op->ytmp, 1, &a.S->done);
  else if (op->g.prec == DCG_PREC_STORED) st = matvec_stored_done(op, a.p, op->ytmp, 1, &a.S->done);
  else st = launch_symv_sweep(op, 1, &a.S->done);
  if (ev1 != nullptr && record_event(ev1, op->stream, in_graph) != hipSuccess) return DCG_E_HIP;
  if (st != DCG_OK) return st;
  hipLaunchKernelGGL(cg_matvec_finish, dim3(static_cast<unsigned>(a.nblk_q)), dim3(256), 0,
                     op->stream, a);
  if (a.W32 != nullptr)
    hipLaunchKernelGGL(cg_update_xr_w32, dim3(static_cast<unsigned>(xr_grid(a))), dim3(256), 0,
                       op->stream, a);
  else
    hipLaunchKernelGGL(cg_update_xr, dim3(static_cast<unsigned>(xr_grid(a))), dim3(256), 0,
                       op->stream, a);
  hipLaunchKernelGGL(cg_finalize, dim3(1), dim3(256), 0, op->stream, a);
  hipLaunchKernelGGL(cg_update_p, dim3(static_cast<unsigned>(a.nblk_p)), dim3(256), 0,
                     op->stream, a);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

// Phase 1 of a solve (Algorithm 1 initialisation): AW, M^{-1}, r_0, the
// deflated start and p_0; leaves the device state ready for the iteration.
int solve_init(dcg_operator_s *op, const double *b, double *x, int x_given,
                      dcg_recycle_s *rc, const dcg_params *p, double tol, void *ws,
                      const StorePlan &sp, SolveCtx *ctx, InnerResult *out) {
  const auto t0 = Clock::now();
  hipStream_t s = op->stream;
  const int64_t n = op->g.n, n_pad = op->g.n_pad;
  SolveBuffers B = solve_buffers(ws, n);
  const int max_iter = p->max_iter > 0 ? p->max_iter : static_cast<int>(std::min<int64_t>(10 * n, 1 << 30));
  int L = 0;
  int k = 0;
  int koff = 0;
  if (rc != nullptr) {
    k = rc->k_used;
    koff = sp.off >= 0 ? sp.off : k;
    L = sp.count >= 0 ? sp.count : ((p->L > 0) ? std::min(p->L, rc->L) : rc->L);
    L = std::max(0, std::min(L, rc->k + rc->L - koff));
  }
  int matvecs = 0;
  const double *Minv = nullptr;
  HIPCHK(hipMemsetAsync(B.counter, 0, sizeof(unsigned) * 8, s));
  HIPCHK(hipMemsetAsync(B.S, 0, sizeof(SolveState), s));
  if (k > 0) {
    int st = deflation_setup(op, rc, &matvecs);
    if (st != DCG_OK) return st;
    Minv = rc->Minv;
  }
  // r = b - A x_{-1}
  const double *Ax = nullptr;
  if (x_given) {
    int st = matvec_lowprec(op, x, B.q, 1);
    if (st != DCG_OK) return st;
    Ax = B.q;
    matvecs += 1;
  }
  const dim3 grid(static_cast<unsigned>(cdiv(n, 256)));
  hipLaunchKernelGGL(init_residual, grid, dim3(256), 0, s, b, Ax, x, B.r, n, x_given, B.part,
                     B.counter, B.S);
  if (k > 0) {
    // x_0 = x_{-1} + W (W^T A W)^{-1} W^T r_{-1};  r_0 = b - A x_0, formed as
    // r_{-1} - A (W c) with one product, so that r_0 is the residual of the
    // operator itself and not of the stored AW (after an extraction whose
    // metric F was nearly singular, AW' = (AZ) U carries the products'
    // evaluation error amplified by U; with r_{-1} - (AW) c the n = 65536
    // sequence needed 348 steps and 13 refinement steps on such a system
    // instead of 169 and 9)
    enqueue_ts_dot(s, rc->Z, n, k, B.r, B.part_h, B.counter + 1, Minv, B.S->cvec);
    hipLaunchKernelGGL(defl_start, grid, dim3(256), 0, s, x, B.p, rc->Z, B.S->cvec, n, k);
    int st = matvec_lowprec(op, B.p, B.q, 1);
    if (st != DCG_OK) return st;
    matvecs += 1;
    enqueue_block_axpy(s, B.r, B.q, -1.0, n);
    // W^T A W mu_0 = (AW)^T r_0
    enqueue_ts_dot(s, rc->AZ, n, k, B.r, B.part_h, B.counter + 1, Minv, B.S->mu);
  }
  hipLaunchKernelGGL(init_direction, dim3(static_cast<unsigned>(cdiv(n_pad, 256))), dim3(256), 0, s,
                     B.r, rc ? rc->Z : nullptr, B.S->mu, n, n_pad, k,
                     op->has_dsc ? op->dsc : nullptr, B.p, op->vin, B.part,
                     B.counter, B.S, tol, B.hist_res);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  out->t_init = ms_since(t0);

  ctx->B = B;
  ctx->a = cg_args(op, B, x, rc, Minv, k, L, koff, tol, max_iter);
  if (rc != nullptr && sp.extract && p->extraction == 2 && L > 0) {
    // the implicit extraction: rho_0 and mu_0 of the start, then every step's
    // rho_{j+1}, mu_{j+1}, c_{j+1} (cg_finalize) and the FP64 directions
    ctx->a.implicit = 1;
    ctx->a.hist_rho = B.hist_rho;
    ctx->a.hist_mu = B.hist_mu;
    ctx->a.hist_c = B.hist_c;
    HIPCHK(hipMemcpyAsync(B.hist_rho, &B.S->rho, 8, hipMemcpyDeviceToDevice, s));
    if (k > 0) HIPCHK(hipMemcpyAsync(B.hist_mu, B.S->mu, size_t(k) * 8, hipMemcpyDeviceToDevice, s));
  }
  ctx->k = k;
  ctx->L = L;
  ctx->koff = koff;
  ctx->matvecs = matvecs;
  ctx->tol = tol;
  ctx->extract = sp.extract && rc != nullptr;
  return DCG_OK;
}

// Phase 2: the iteration, in chunks of check_every steps (one hipGraph per
// chunk unless profiling), until the device state says done.
int solve_loop(dcg_operator_s *op, const dcg_params *p, SolveCtx *ctx, InnerResult *out) {
  hipStream_t s = op->stream;
  const SolveBuffers &B = ctx->B;
  const CgArgs &a = ctx->a;
  const double tol = ctx->tol;
  const auto t1 = Clock::now();
  const int chunk = std::max(1, p->check_every);
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // profiling: one event pair per step of a chunk, read back at each chunk end
  hipEvent_t evs[2 * 64] = {};
  const bool prof = p->profile != 0;
  const int pchunk = prof ? std::min(chunk, 64) : chunk;
  if (prof)
    // no system-scope fence: the events only time device work on this stream
    for (int e = 0; e < 2 * pchunk; ++e)
      HIPCHK(hipEventCreateWithFlags(&evs[e], hipEventDisableSystemFence));
  if (p->use_graph) {
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int st = DCG_OK;
    for (int c = 0; c < pchunk && st == DCG_OK; ++c)
      st = prof ? enqueue_cg_step(op, a, evs[2 * c], evs[2 * c + 1], true) : enqueue_cg_step(op, a);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st == DCG_OK && e == hipSuccess) {
      HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    } else {
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      graph = nullptr;
      // a runtime that cannot capture timing events: time eager launches
      if (!prof) return st != DCG_OK ? st : DCG_E_HIP;
      (void)hipGetLastError();
    }
  }
  SolveState hs;
  hs.iter = 0;
  hs.done = 0;
  int status = DCG_OK;
  while (true) {
    if (gexec != nullptr) {
      if (hipGraphLaunch(gexec, s) != hipSuccess) { status = DCG_E_HIP; break; }
    } else {
      for (int c = 0; c < pchunk; ++c) {
        status = prof ? enqueue_cg_step(op, a, evs[2 * c], evs[2 * c + 1]) : enqueue_cg_step(op, a);
        if (status != DCG_OK) break;
      }
      if (status != DCG_OK) break;
    }
    const int prev_iter = hs.iter;
    if (hipMemcpyAsync(&hs, B.S, offsetof(SolveState, mu), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      status = DCG_E_HIP;
      break;
    }
    if (prof) {
      // sweeps that did work (those after convergence return at once)
      const int ran = std::min(pchunk, hs.iter - prev_iter);
      for (int c = 0; c < ran; ++c) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, evs[2 * c], evs[2 * c + 1]) == hipSuccess) {
          out->t_sweeps += ms;
          out->sweeps_timed += 1;
        }
      }
    }
    if (hs.done) break;
  }
  if (prof)
    for (int e = 0; e < 2 * pchunk; ++e) (void)hipEventDestroy(evs[e]);
  if (gexec != nullptr) (void)hipGraphExecDestroy(gexec);
  if (graph != nullptr) (void)hipGraphDestroy(graph);
  if (status != DCG_OK) return status;
  out->t_loop = ms_since(t1);
  out->iters = hs.iter;
  out->relres = hs.relres;
  ctx->matvecs += hs.iter;
  out->status = hs.status != 0 ? hs.status : (hs.relres <= tol ? DCG_OK : DCG_NOT_CONVERGED);
  out->k_used = ctx->k;
  out->k_next = ctx->k;
  return DCG_OK;
}


// The pencil (G, F) of the extraction from the m columns of Z and AZ:
// harmonic Ritz (Eq. 7) G = (AZ)^T AZ, F = (AZ)^T Z; Rayleigh-Ritz
// G = (AZ)^T Z, F = Z^T Z.  Both symmetrised, m x m.
static void enqueue_extraction_pencil(hipStream_t s, const double *Z, const double *AZ, int64_t n,
                                      int m, int extraction, double *part, double *F, double *G) {
  if (extraction == 1) {
    enqueue_tsgemm_tn(s, Z, Z, n, m, m, part, kGemmPartDoubles, F, m, 1);
    enqueue_tsgemm_tn(s, AZ, Z, n, m, m, part, kGemmPartDoubles, G, m, 1);
  } else {
    enqueue_tsgemm_tn(s, AZ, Z, n, m, m, part, kGemmPartDoubles, F, m, 1);
    enqueue_tsgemm_tn(s, AZ, AZ, n, m, m, part, kGemmPartDoubles, G, m, 1);
  }
}

// After the pencil's eigenproblem has been enqueued: read its status, form
// W' = Z U and AW' (by `form`, which enqueues both into rc->Wt, rc->AWt),
// move them into the first columns of Z and AZ and record the new basis.
template <class Form>
static int finish_extraction(dcg_operator_s *op, dcg_recycle_s *rc, int mz, InnerResult *out,
                             Form form) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  int info[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(info, rc->info, sizeof(info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(rc->theta, rc->small, sizeof(double) * kMaxK, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int knew = info[0];
  rc->rank_F = info[1];
  rc->sweeps[0] = info[2];
  rc->sweeps[1] = info[3];
  if (knew > 0) {
    form(knew);
    HIPCHK(hipMemcpyAsync(rc->Z, rc->Wt, size_t(n) * knew * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(rc->AZ, rc->AWt, size_t(n) * knew * 8, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  rc->k_used = knew;
  rc->n_theta = knew;
  rc->w_version += 1;
  rc->L_eff = mz;
  // AW' is the product with this operator
  rc->aw_state = 1;
  rc->aw_op = op;
  rc->aw_gen = op->generation;
  rc->aw_ell = op->ell;
  rc->aw_s2 = op->s2;
  rc->aw_sigma2 = op->sigma2;
  rc->aw_dsc = op->dsc_version;
  out->k_next = knew;
  return DCG_OK;
}

// The extraction of W' = Z U (section 2.3: harmonic Ritz, Eq. 7, or
// Rayleigh-Ritz) from the first mz columns of Z = [W, stored directions] and
// AZ.
int extract_basis(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p, int mz,
                  InnerResult *out) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  if (mz <= 0) return DCG_OK;
  enqueue_extraction_pencil(s, rc->Z, rc->AZ, n, mz, p->extraction, rc->gemm, rc->F, rc->G);
  enqueue_harmonic_ritz(s, rc->F, rc->G, mz, rc->k, p->select_largest, p->ritz_route, 1e-12,
                        rc->eigw, rc->U, rc->small, rc->info);
  return finish_extraction(op, rc, mz, out, [&](int knew) {
    enqueue_ts_times_small(s, rc->Z, n, mz, rc->U, kMaxK, knew, rc->Wt);
    enqueue_ts_times_small(s, rc->AZ, n, mz, rc->U, kMaxK, knew, rc->AWt);
  });
}

// The implicit extraction (section 2.3, the F and G that Saad et al. formed
// from the stored scalars): F, G from the records of the solve's first L_eff
// steps (implicit.hip), the same eigenproblem, W' = [W, P] U with P read as
// the FP32 copies the low-precision sweep multiplied, and AW' either from the
// residual recurrence, AW' = [W, P, p_L] S1 + AW S2 (FP64 operator), or as
// k' products of W' (every other operator), so that no product A p_j is
// stored.  Z holds the FP64 directions p_0 .. p_L after W.
//
// The implicit F = blockdiag(M, diag(d_j)) assumes A-conjugate directions;
// once the iteration has lost conjugacy (an extreme Ritz value converged) two
// stored directions can be nearly parallel, which the scalars do not show,
// and W' comes out numerically rank deficient.  A second harmonic problem on
// span(W') with its explicit metric (AW')^T W' and (AW')^T AW' (k-column
// products, against k + L for the explicit extraction) drops such
// directions; where W' is sound it returns W' itself (the harmonic Ritz
// vectors of span(Z) are those of span(W') with the same values).
static int extract_implicit(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p,
                            SolveCtx *ctx, int iters, InnerResult *out) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  const int k = ctx->k, Le = std::min(ctx->L, iters);
  const int mz = k + Le;
  if (mz <= 0) return DCG_OK;
  // p_{Le}: still the current direction unless step Le ran and stored it
  if (iters <= ctx->L)
    HIPCHK(hipMemcpyAsync(rc->Z + int64_t(ctx->koff + Le) * n, ctx->B.p, size_t(n) * 8,
                          hipMemcpyDeviceToDevice, s));
  ImplicitHist h;
  h.d = ctx->B.hist_d;
  h.alpha = ctx->B.hist_alpha;
  h.beta = ctx->B.hist_beta;
  h.rho = ctx->B.hist_rho;
  h.mu = ctx->B.hist_mu;
  h.cv = ctx->B.hist_c;
  // scratch in the split-K area the tall products would have used
  double *terms = rc->gemm;                                   // 2 x kMaxZ x kMaxK
  double *S1 = rc->gemm + 2 * size_t(kMaxZ) * kMaxK;          // (kMaxZ + 1) x kMaxK
  double *S2 = S1 + size_t(kMaxZ + 1) * kMaxK;                // kMaxK x kMaxK
  double *part = S2 + size_t(kMaxK) * kMaxK;                  // split-K partials (k x k)
  const size_t part_cap = kGemmPartDoubles - size_t(part - rc->gemm);
  enqueue_implicit_pencil(s, h, rc->M, rc->N, k, Le, terms, rc->F, rc->G);
  enqueue_harmonic_ritz(s, rc->F, rc->G, mz, rc->k, p->select_largest, p->ritz_route, 1e-12,
                        rc->eigw, rc->U, rc->small, rc->info);
  int info[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(info, rc->info, sizeof(info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int k1 = info[0];
  rc->rank_F = info[1];
  rc->sweeps[0] = info[2];
  rc->sweeps[1] = info[3];
  int knew = 0;
  if (k1 > 0) {
    const bool lowprec = ctx->a.qdirect == nullptr;
    enqueue_ts_times_small(s, rc->Z, n, mz, rc->U, kMaxK, k1, rc->Wt, lowprec ? k : (1 << 30),
                           op->has_dsc ? op->dsc : nullptr);
    if (op->g.prec == DCG_PREC_FP64) {
      enqueue_implicit_aw_coef(s, h, rc->U, k, Le, k1, S1, S2);
      enqueue_ts_times_small(s, rc->Z, n, mz + 1, S1, kMaxK, k1, rc->AWt);
      if (k > 0)
        enqueue_ts_times_small(s, rc->AZ, n, k, S2, kMaxK, k1, rc->AWt, 1 << 30, nullptr, 1);
    } else {
      // An FP32-accumulated product is exact only to ~1e-7 of (|A| |p|)_i,
      // and U, drawn from a metric that cannot see lost conjugacy, can
      // combine nearly parallel directions with large coefficients: the
      // implied products of such a combination are then dominated by those
      // errors (measured: 34% of |AW'| at n = 65536 with bf16 points after
      // one recycled system), and the harmonic problem below would pick
      // exactly those directions as its largest values.  Here AW' is the
      // operator's own product of W' (k1 columns), as in refresh_AW.
      if (op->g.prec != DCG_PREC_STORED && !op->has_dsc)
        enqueue_round_to_fp32(s, rc->Wt, n * k1);
      const int st = matvec_lowprec(op, rc->Wt, rc->AWt, k1);
      if (st != DCG_OK) return st;
      ctx->matvecs += k1;
    }
    // the second, explicit harmonic problem on span(W').  Its metric drops
    // a direction at tau times the largest eigenvalue of the scaled F, which
    // bounds the growth of the products' errors through U by 1/sqrt(tau):
    // FP32-accumulated products (~1e-7 relative) need tau = 1e-4 to keep
    // AW' at their own error level (at 1e-12, the n = 65536 bf16 sequence
    // kept an error of 2.5e-4 of |AW'|); columns that close to dependent are
    // the ghost pairs the cleanup is for.
    const double tau = (op->g.prec == DCG_PREC_FP64) ? 1e-12 : 1e-4;
    enqueue_tsgemm_tn(s, rc->AWt, rc->Wt, n, k1, k1, part, part_cap, rc->F, k1, 1);
    enqueue_tsgemm_tn(s, rc->AWt, rc->AWt, n, k1, k1, part, part_cap, rc->G, k1, 1);
    enqueue_harmonic_ritz(s, rc->F, rc->G, k1, k1, p->select_largest, p->ritz_route, tau,
                          rc->eigw, rc->U, rc->small, rc->info);
    int info2[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(info2, rc->info, sizeof(info2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rc->theta, rc->small, sizeof(double) * kMaxK, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    knew = info2[0];
    if (knew > 0) {
      enqueue_ts_times_small(s, rc->Wt, n, k1, rc->U, kMaxK, knew, rc->Z);
      enqueue_ts_times_small(s, rc->AWt, n, k1, rc->U, kMaxK, knew, rc->AZ);
    }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  rc->k_used = knew;
  rc->n_theta = knew;
  rc->w_version += 1;
  rc->L_eff = mz;
  rc->aw_state = 1;
  rc->aw_op = op;
  rc->aw_gen = op->generation;
  rc->aw_ell = op->ell;
  rc->aw_s2 = op->s2;
  rc->aw_sigma2 = op->sigma2;
  rc->aw_dsc = op->dsc_version;
  out->k_next = knew;
  return DCG_OK;
}

// Phase 3: the extraction from Z = [W, P_L] of this solve (the directions it
// stored follow any stored before it).
int solve_extract(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p, SolveCtx *ctx,
                  InnerResult *out) {
  const auto t2 = Clock::now();
  if (rc != nullptr && ctx->extract && out->status >= 0) {
    const int st = ctx->a.implicit
                       ? extract_implicit(op, rc, p, ctx, out->iters, out)
                       : extract_basis(op, rc, p, ctx->koff + std::min(ctx->L, out->iters), out);
    if (st != DCG_OK) return st;
  }
  out->t_refresh = ms_since(t2);
  out->matvecs = ctx->matvecs;
  return DCG_OK;
}

// One deflated-CG solve of A x = b (Algorithm 1), then the extraction of the
// next basis (section 2.3) when rc is given.
static int inner_solve(dcg_operator_s *op, const double *b, double *x, int x_given,
                       dcg_recycle_s *rc, const dcg_params *p, double tol, void *ws,
                       InnerResult *out, const StorePlan &sp = StorePlan()) {
  SolveCtx ctx;
  int st = solve_init(op, b, x, x_given, rc, p, tol, ws, sp, &ctx, out);
  if (st != DCG_OK) return st;
  st = solve_loop(op, p, &ctx, out);
  if (st != DCG_OK) return st;
  return solve_extract(op, rc, p, &ctx, out);
}


// |b - A x| / |b| with the low-precision (exact = 0) or FP64 operator.
int true_residual(dcg_operator_s *op, const double *b, const double *x, int exact,
                         const SolveBuffers &B, double *rel) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  int st = exact ? matvec_exact(op, x, B.tmp3, 1) : matvec_lowprec(op, x, B.tmp3, 1);
  if (st != DCG_OK) return st;
  HIPCHK(hipMemsetAsync(B.counter + 2, 0, sizeof(unsigned), s));
  hipLaunchKernelGGL(residual_norms, dim3(static_cast<unsigned>(std::min<int64_t>(kRedBlocks, cdiv(n, 256)))),
                     dim3(256), 0, s, b, B.tmp3, n, B.tmp2, B.part, B.counter + 2,
                     B.S->cvec);
  double h[2];
  HIPCHK(hipMemcpyAsync(h, B.S->cvec, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *rel = (h[1] > 0.0) ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return DCG_OK;
}

// When the inner solves of one refinement refresh the recycled basis:
// refresh_every = 0 after the first inner solve (the operator is the same for
// all of them), 1 after every inner solve, 2 once after the last one, from
// the directions of all the inner solves in order (up to L; W is unchanged
// meanwhile).
struct RefineStore {
  int mode = 0, Lcap = 0, stored = 0;
  RefineStore(const dcg_params *p, const dcg_recycle_s *rc) : mode(p->refresh_every) {
    if (rc != nullptr) Lcap = (p->L > 0) ? std::min(p->L, rc->L) : rc->L;
  }
  StorePlan plan(int t, const dcg_recycle_s *rc) const {
    StorePlan sp;
    if (rc == nullptr) {
      sp.count = 0;
      sp.extract = false;
    } else if (mode == 2) {
      sp.off = rc->k_used + stored;
      sp.count = std::max(0, Lcap - stored);
      sp.extract = false;
    } else if (mode == 0 && t > 0) {
      sp.count = 0;
      sp.extract = false;
    }
    return sp;
  }
  void after(const StorePlan &sp, int iters) {
    if (mode == 2) stored += std::min(iters, sp.count);
  }
  // the deferred extraction (mode 2)
  int finish(dcg_operator_s *op, dcg_recycle_s *rc, const dcg_params *p, dcg_stats *st) {
    if (mode != 2 || rc == nullptr || rc->k_used + stored == 0) return DCG_OK;
    const auto t0 = Clock::now();
    InnerResult R;
    R.k_next = rc->k_used;
    const int code = extract_basis(op, rc, p, rc->k_used + stored, &R);
    st->k_next = R.k_next;
    st->t_refresh_ms += ms_since(t0);
    return code;
  }
};

// ------------------------------------------------ flexible-CG refinement
//
// Krylov-accelerated refinement: flexible CG (full A-orthogonalisation) in
// FP64 around a variable preconditioner, the deflated solve of the
// low-precision operator to inner_tol.  Per outer step: z_t = inner solve of
// r_t (written straight into D_t), Q_t = A z_t with the FP64 operator, then
// D_t, Q_t -= sum_j c_j (D_j, Q_j) with c_j = Q_j^T z_t / gamma_j, and
// alpha = D_t^T r / gamma_t, gamma_t = D_t^T Q_t.  The residual is updated
// recursively with the FP64 products and confirmed with one FP64 product
// before the solve returns (a restart from that residual if it disagrees).

struct FcgCoef {
  double c[kFcgCap];
};

__global__ __launch_bounds__(256) void fcg_orth(double *D, double *Q, int t, int64_t n, FcgCoef cf) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  double d = D[int64_t(t) * n + i], q = Q[int64_t(t) * n + i];
  for (int j = 0; j < t; ++j) {
    d -= cf.c[j] * D[int64_t(j) * n + i];
    q -= cf.c[j] * Q[int64_t(j) * n + i];
  }
  D[int64_t(t) * n + i] = d;
  Q[int64_t(t) * n + i] = q;
}

// Column dots out[c] = Y[:, c]^T v, c < m, read back to the host.
static int host_dots(hipStream_t s, const double *Y, int64_t n, int m, const double *v,
                     const SolveBuffers &B, double *out) {
  enqueue_ts_dot(s, Y, n, m, v, B.part_h, B.counter + 1, nullptr, B.S->cvec);
  HIPCHK(hipMemcpyAsync(out, B.S->cvec, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return DCG_OK;
}

// r = b - A x with the FP64 operator (r = b when zero); returns |r|^2, |b|^2.
static int fp64_residual(dcg_operator_s *op, const double *b, const double *x, bool zero,
                         const SolveBuffers &B, double *r, double *rr, double *bb, int *exact) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  if (!zero) {
    const int st = matvec_exact(op, x, B.tmp3, 1);
    if (st != DCG_OK) return st;
    *exact += 1;
  }
  HIPCHK(hipMemsetAsync(B.counter + 2, 0, sizeof(unsigned), s));
  hipLaunchKernelGGL(residual_norms, dim3(static_cast<unsigned>(std::min<int64_t>(kRedBlocks, cdiv(n, 256)))),
                     dim3(256), 0, s, b, zero ? nullptr : B.tmp3, n, r, B.part, B.counter + 2,
                     B.S->cvec);
  double h[2];
  HIPCHK(hipMemcpyAsync(h, B.S->cvec, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *rr = h[0];
  *bb = h[1];
  return DCG_OK;
}

static int refine_fcg(dcg_operator_s *op, const double *b, double *x, int x_given,
                      dcg_recycle_s *rc, const dcg_params *p, dcg_stats *st, void *ws,
                      const SolveBuffers &B) {
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  double *r = B.tmp1;
  const int outer_max = p->refine_max > 0 ? p->refine_max : 20;
  HIPCHK(hipMemsetAsync(B.counter, 0, sizeof(unsigned) * 4, s));
  if (!x_given) HIPCHK(hipMemsetAsync(x, 0, size_t(n) * 8, s));
  double rr = 0.0, bb = 0.0;
  int code = fp64_residual(op, b, x, !x_given, B, r, &rr, &bb, &st->matvecs_exact);
  if (code != DCG_OK) return code;
  auto relof = [&](double v) { return bb > 0.0 ? std::sqrt(v / bb) : std::sqrt(v); };
  double rel = relof(rr);
  bool r_true = true;      // r is the FP64 residual of x (not the recursive one)
  double gamma[kFcgCap];
  RefineStore store(p, rc);
  int t = 0;               // directions kept
  int status = DCG_NOT_CONVERGED;
  while (true) {
    if (!std::isfinite(rel)) { status = DCG_E_NONFINITE; break; }
    if (rel <= p->tol || t == kFcgCap) {
      if (r_true && rel <= p->tol) { status = DCG_OK; break; }
      // confirm with the FP64 residual; continue from it (dropping the
      // directions) if the recursive residual drifted or the store is full
      code = fp64_residual(op, b, x, false, B, r, &rr, &bb, &st->matvecs_exact);
      if (code != DCG_OK) return code;
      rel = relof(rr);
      r_true = true;
      t = 0;
      continue;
    }
    if (st->outer_steps == outer_max) break;
    double *Dt = B.fD + int64_t(t) * n, *Qt = B.fQ + int64_t(t) * n;
    InnerResult R;
    const StorePlan sp = store.plan(st->outer_steps, rc);
    code = inner_solve(op, r, Dt, 0, rc, p, p->inner_tol, ws, &R, sp);
    if (code != DCG_OK) return code;
    store.after(sp, R.iters);
    st->iters += R.iters;
    st->matvecs += R.matvecs;
    if (st->outer_steps == 0) st->k_used = R.k_used;
    st->k_next = R.k_next;
    st->t_init_ms += R.t_init;
    st->t_loop_ms += R.t_loop;
    st->t_refresh_ms += R.t_refresh;
    st->sweeps_timed += R.sweeps_timed;
    st->t_sweeps_ms += R.t_sweeps;
    st->rel_res_recursive = R.relres;
    st->outer_steps += 1;
    if (R.status < 0) { status = R.status; break; }
    code = matvec_exact(op, Dt, Qt, 1);
    if (code != DCG_OK) return code;
    st->matvecs_exact += 1;
    if (t > 0) {
      double h[kFcgCap];
      code = host_dots(s, B.fQ, n, t, Dt, B, h);
      if (code != DCG_OK) return code;
      FcgCoef cf;
      for (int j = 0; j < t; ++j) cf.c[j] = h[j] / gamma[j];
      hipLaunchKernelGGL(fcg_orth, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0, s,
                         B.fD, B.fQ, t, n, cf);
      HIPCHK(hipGetLastError());
    }
    double g1[1], g2[1];
    code = host_dots(s, Qt, n, 1, Dt, B, g1);
    if (code == DCG_OK) code = host_dots(s, Dt, n, 1, r, B, g2);
    if (code != DCG_OK) return code;
    if (!std::isfinite(g1[0]) || !std::isfinite(g2[0])) { status = DCG_E_NONFINITE; break; }
    if (!(g1[0] > 0.0)) { status = DCG_E_NOT_SPD; break; }
    gamma[t] = g1[0];
    const double alpha = g2[0] / g1[0];
    enqueue_block_axpy(s, x, Dt, alpha, n);
    enqueue_block_axpy(s, r, Qt, -alpha, n);
    double rn[1];
    code = host_dots(s, r, n, 1, r, B, rn);
    if (code != DCG_OK) return code;
    rel = relof(rn[0]);
    r_true = false;
    t += 1;
  }
  if (status >= 0) {
    code = store.finish(op, rc, p, st);
    if (code != DCG_OK) return code;
  }
  st->rel_res_true = rel;
  st->status = status;
  return status;
}

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_recycle_workspace_bytes(int64_t n, int k, int L) {
  if (n < 1 || k < 1 || k > kMaxK || L < k || k + L > kMaxZ) return 0;
  return recycle_layout(n, k, L).total;
}

int dcg_recycle_create(int64_t n, int k, int L, void *workspace, size_t ws_bytes,
                       dcg_recycle_t *out) {
  if (out == nullptr) return DCG_E_ARG;
  *out = nullptr;
  if (n < 1 || k < 1 || k > kMaxK || L < k || k + L > kMaxZ) return DCG_E_ARG;
  const RecycleLayout R = recycle_layout(n, k, L);
  if (workspace == nullptr || ws_bytes < R.total) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return DCG_E_WORKSPACE;
  dcg_recycle_s *rc = new (std::nothrow) dcg_recycle_s;
  if (rc == nullptr) return DCG_E_ARG;
  std::memset(static_cast<void *>(rc), 0, sizeof(*rc));
  char *b = static_cast<char *>(workspace);
  rc->n = n;
  rc->k = k;
  rc->L = L;
  rc->Z = reinterpret_cast<double *>(b + R.Z);
  rc->AZ = reinterpret_cast<double *>(b + R.AZ);
  rc->Wt = reinterpret_cast<double *>(b + R.Wt);
  rc->AWt = reinterpret_cast<double *>(b + R.AWt);
  rc->F = reinterpret_cast<double *>(b + R.F);
  rc->G = reinterpret_cast<double *>(b + R.G);
  rc->U = reinterpret_cast<double *>(b + R.U);
  rc->eigw = reinterpret_cast<double *>(b + R.eigw);
  rc->M = reinterpret_cast<double *>(b + R.M);
  rc->Minv = reinterpret_cast<double *>(b + R.Minv);
  rc->Mwork = reinterpret_cast<double *>(b + R.Mwork);
  rc->N = reinterpret_cast<double *>(b + R.N);
  rc->small = reinterpret_cast<double *>(b + R.small);
  rc->info = reinterpret_cast<int *>(b + R.info);
  rc->gemm = reinterpret_cast<double *>(b + R.gemm);
  rc->W32 = reinterpret_cast<float *>(b + R.W32);
  rc->AW32 = reinterpret_cast<float *>(b + R.AW32);
  *out = rc;
  return DCG_OK;
}

int dcg_recycle_set_W(dcg_recycle_t rc, const double *W, int kw) {
  if (rc == nullptr || kw < 0 || kw > rc->k || (kw > 0 && W == nullptr)) return DCG_E_ARG;
  if (kw > 0 && hipMemcpy(rc->Z, W, size_t(rc->n) * kw * 8, hipMemcpyDeviceToDevice) != hipSuccess)
    return DCG_E_HIP;
  rc->k_used = kw;
  rc->aw_state = 0;
  rc->w_version += 1;
  rc->n_theta = 0;
  return DCG_OK;
}

int dcg_recycle_get_W(dcg_recycle_t rc, double *W_out, int *k_used) {
  if (rc == nullptr) return DCG_E_ARG;
  if (k_used != nullptr) *k_used = rc->k_used;
  if (W_out != nullptr && rc->k_used > 0 &&
      hipMemcpy(W_out, rc->Z, size_t(rc->n) * rc->k_used * 8, hipMemcpyDeviceToDevice) != hipSuccess)
    return DCG_E_HIP;
  return DCG_OK;
}

int dcg_recycle_get_AW(dcg_recycle_t rc, double *AW_out) {
  if (rc == nullptr || AW_out == nullptr || rc->aw_state != 1) return DCG_E_ARG;
  if (rc->k_used > 0 &&
      hipMemcpy(AW_out, rc->AZ, size_t(rc->n) * rc->k_used * 8, hipMemcpyDeviceToDevice) != hipSuccess)
    return DCG_E_HIP;
  return DCG_OK;
}

int dcg_recycle_get_theta(dcg_recycle_t rc, double *theta_out, int *count) {
  if (rc == nullptr) return DCG_E_ARG;
  if (count != nullptr) *count = rc->n_theta;
  if (theta_out != nullptr)
    for (int i = 0; i < rc->n_theta; ++i) theta_out[i] = rc->theta[i];
  return DCG_OK;
}

void dcg_recycle_destroy(dcg_recycle_t rc) { delete rc; }

size_t dcg_solve_workspace_bytes(int64_t n, int k, int L) {
  (void)k;
  (void)L;
  if (n < 1) return 0;
  return solve_layout(n).total;
}

// What the last extraction looked like (the handle keeps it).
static int with_refresh(dcg_stats *st, const dcg_recycle_s *rc, int status) {
  if (rc != nullptr) {
    st->refresh_dim = rc->L_eff;
    st->refresh_rank = rc->rank_F;
    st->refresh_sweeps[0] = rc->sweeps[0];
    st->refresh_sweeps[1] = rc->sweeps[1];
  }
  return status;
}

int dcg_solve(dcg_op_t op, const double *b, double *x, int x_given, dcg_recycle_t rc,
              const dcg_params *p, dcg_stats *st, void *ws, size_t ws_bytes) {
  dcg_stats local;
  std::memset(&local, 0, sizeof(local));
  if (st == nullptr) st = &local;
  std::memset(st, 0, sizeof(*st));
  if (op == nullptr || b == nullptr || x == nullptr || p == nullptr) return st->status = DCG_E_ARG;
  if (!(p->tol >= 0.0) || p->check_every < 0 || p->refine < 0 || p->refine > 2 ||
      p->refresh_every < 0 || p->refresh_every > 2 || p->ritz_route < 0 || p->ritz_route > 1 ||
      p->extraction < 0 || p->extraction > 2 ||
      // the implicit extraction describes one Krylov sequence, not the
      // pooled directions of several inner solves
      (p->extraction == 2 && p->refine != 0 && p->refresh_every == 2))
    return st->status = DCG_E_ARG;
  if (rc != nullptr && rc->n != op->g.n) return st->status = DCG_E_ARG;
  // the stored operator has no FP64 counterpart to refine against
  if (!has_exact(op) && p->refine != 0) return st->status = DCG_E_ARG;
  if (ws == nullptr || ws_bytes < solve_layout(op->g.n).total) return st->status = DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return st->status = DCG_E_WORKSPACE;
  const auto t0 = Clock::now();
  hipStream_t s = op->stream;
  const int64_t n = op->g.n;
  SolveBuffers B = solve_buffers(ws, n);
  if (!p->refine) {
    InnerResult R;
    int rcode = inner_solve(op, b, x, x_given, rc, p, p->tol, ws, &R);
    if (rcode != DCG_OK) return st->status = rcode;
    st->iters = R.iters;
    st->matvecs = R.matvecs;
    st->k_used = R.k_used;
    st->k_next = R.k_next;
    st->rel_res_recursive = R.relres;
    st->t_init_ms = R.t_init;
    st->t_loop_ms = R.t_loop;
    st->t_refresh_ms = R.t_refresh;
    st->status = R.status;
    st->sweeps_timed = R.sweeps_timed;
    st->t_sweeps_ms = R.t_sweeps;
    if (p->true_residual) {
      rcode = true_residual(op, b, x, 0, B, &st->rel_res_true);
      if (rcode != DCG_OK) return st->status = rcode;
      st->matvecs += 1;
    }
    st->t_total_ms = ms_since(t0);
    return with_refresh(st, rc, st->status);
  }
  if (p->refine == 2) {
    const int code = refine_fcg(op, b, x, x_given, rc, p, st, ws, B);
    st->t_total_ms = ms_since(t0);
    return with_refresh(st, rc, code);
  }
  // ---- iterative refinement: r_t = b - A64 x_t, A~ d_t = r_t, x += d_t
  double *rhs = B.tmp1, *delta = B.tmp2;
  if (!x_given) HIPCHK(hipMemsetAsync(x, 0, size_t(n) * 8, s));
  const int outer_max = p->refine_max > 0 ? p->refine_max : 20;
  double rel = 0.0;
  int status = DCG_NOT_CONVERGED;
  RefineStore store(p, rc);
  // profile: HIP events around each FP64 sweep, read after the residual's
  // host synchronisation below
  hipEvent_t pev[2] = {nullptr, nullptr};
  if (p->profile)
    for (int e = 0; e < 2; ++e)
      if (hipEventCreateWithFlags(&pev[e], hipEventDisableSystemFence) != hipSuccess)
        pev[e] = nullptr;
  const bool tex = pev[0] != nullptr && pev[1] != nullptr;
  struct EvFree {
    hipEvent_t *e;
    ~EvFree() {
      for (int i = 0; i < 2; ++i)
        if (e[i] != nullptr) (void)hipEventDestroy(e[i]);
    }
  } ev_free{pev};
  for (int t = 0; t <= outer_max; ++t) {
    // from x = 0 the first residual is b itself
    const bool zero_start = (t == 0 && !x_given);
    if (!zero_start) {
      int rcode = tex ? matvec_exact_timed(op, x, B.tmp3, pev[0], pev[1])
                      : matvec_exact(op, x, B.tmp3, 1);
      if (rcode != DCG_OK) return st->status = rcode;
      st->matvecs_exact += 1;
    }
    HIPCHK(hipMemsetAsync(B.counter + 2, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(residual_norms, dim3(static_cast<unsigned>(std::min<int64_t>(kRedBlocks, cdiv(n, 256)))),
                       dim3(256), 0, s, b, zero_start ? nullptr : B.tmp3, n, rhs, B.part,
                       B.counter + 2, B.S->cvec);
    double h[2];
    HIPCHK(hipMemcpyAsync(h, B.S->cvec, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tex && !zero_start) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, pev[0], pev[1]) == hipSuccess) {
        st->t_exact_sweeps_ms += ms;
        st->exact_sweeps_timed += 1;
      }
    }
    rel = (h[1] > 0.0) ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
    if (!std::isfinite(rel)) { status = DCG_E_NONFINITE; break; }
    if (rel <= p->tol) { status = DCG_OK; break; }
    if (t == outer_max) break;
    InnerResult R;
    const StorePlan sp = store.plan(st->outer_steps, rc);
    int rcode = inner_solve(op, rhs, delta, 0, rc, p, p->inner_tol, ws, &R, sp);
    if (rcode != DCG_OK) return st->status = rcode;
    store.after(sp, R.iters);
    st->iters += R.iters;
    st->matvecs += R.matvecs;
    if (t == 0) st->k_used = R.k_used;
    st->k_next = R.k_next;
    st->t_init_ms += R.t_init;
    st->t_loop_ms += R.t_loop;
    st->t_refresh_ms += R.t_refresh;
    st->sweeps_timed += R.sweeps_timed;
    st->t_sweeps_ms += R.t_sweeps;
    st->rel_res_recursive = R.relres;
    st->outer_steps += 1;
    if (R.status < 0) { status = R.status; break; }
    enqueue_block_axpy(s, x, delta, 1.0, n);
  }
  if (status >= 0) {
    const int rcode = store.finish(op, rc, p, st);
    if (rcode != DCG_OK) return st->status = rcode;
  }
  st->rel_res_true = rel;
  st->status = status;
  st->t_total_ms = ms_since(t0);
  return with_refresh(st, rc, status);
}

}  // extern "C"

namespace dcg {

// ------------------------------------------- extraction on given Z, AZ

static size_t ritz_ws_layout(int64_t n, int m, size_t *off) {
  Carve c(nullptr, 0);
  off[0] = c.off = align256(c.off); c.off += size_t(m) * m * 8;                 // F
  off[1] = c.off = align256(c.off); c.off += size_t(m) * m * 8;                 // G
  off[2] = c.off = align256(c.off); c.off += harmonic_ritz_work_doubles() * 8;  // eigensolver
  off[3] = c.off = align256(c.off); c.off += size_t(kMaxZ) * kMaxK * 8;         // U
  off[4] = c.off = align256(c.off); c.off += size_t(kMaxK) * 8;                 // theta
  off[5] = c.off = align256(c.off); c.off += 4 * sizeof(int);                   // info
  off[6] = c.off = align256(c.off); c.off += kGemmPartDoubles * 8;              // F, G partials
  (void)n;
  return align256(c.off);
}

static int extract_on_given(const double *Z, const double *AZ, int64_t n, int m, int k,
                            int largest, int extraction, int route, double *W_out,
                            double *theta_out, int *k_out, int *rank_out, hipStream_t s, char *b,
                            const size_t *off) {
  double *F = reinterpret_cast<double *>(b + off[0]);
  double *G = reinterpret_cast<double *>(b + off[1]);
  double *eigw = reinterpret_cast<double *>(b + off[2]);
  double *U = reinterpret_cast<double *>(b + off[3]);
  double *th = reinterpret_cast<double *>(b + off[4]);
  int *info_d = reinterpret_cast<int *>(b + off[5]);
  double *part = reinterpret_cast<double *>(b + off[6]);
  enqueue_extraction_pencil(s, Z, AZ, n, m, extraction, part, F, G);
  enqueue_harmonic_ritz(s, F, G, m, k, largest != 0, route, 1e-12, eigw, U, th, info_d);
  int info[4] = {0, 0, 0, 0};
  double theta[kMaxK];
  HIPCHK(hipMemcpyAsync(info, info_d, sizeof(info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(theta, th, sizeof(theta), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int knew = info[0];
  if (knew > 0) enqueue_ts_times_small(s, Z, n, m, U, kMaxK, knew, W_out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < knew; ++i) theta_out[i] = theta[i];
  *k_out = knew;
  if (rank_out != nullptr) *rank_out = info[1];
  return DCG_OK;
}

static bool extract_args_ok(const double *Z, const double *AZ, int64_t n, int m, int k,
                            int extraction, int route, const double *W_out,
                            const double *theta_out, const int *k_out) {
  return !(Z == nullptr || AZ == nullptr || W_out == nullptr || theta_out == nullptr ||
           k_out == nullptr || n < 1 || m < 1 || m > kMaxZ || k < 1 || k > kMaxK || route < 0 ||
           route > 1 || extraction < 0 || extraction > 1);
}

// ------------------------------------- extraction without any allocation
// The scratch of dcg_extract_basis_noalloc: the extraction's workspace at its
// largest pencil (m = kMaxZ), a file-scope device array.  Every device the
// library runs on holds its own copy until the process ends; host code uses
// the address hipGetSymbolAddress gives for the current device, never the
// array's name (which on the host is only a stand-in for the symbol).
static constexpr size_t a256c(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kExtractScratchBytes =
    2 * a256c(size_t(kMaxZ) * kMaxZ * 8) + a256c(size_t(3) * kMaxZ * kMaxZ * 8) +
    a256c(size_t(kMaxZ) * kMaxK * 8) + a256c(size_t(kMaxK) * 8) + a256c(4 * sizeof(int)) +
    a256c(kGemmPartDoubles * 8);
static __device__ __align__(256) char scratch[kExtractScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kScratchDevices];

// Address of the current device's scratch array, looked up once per device.
static int scratch_address(char **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return DCG_E_HIP;
  std::lock_guard<std::mutex> guard(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
      return DCG_E_HIP;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DCG_OK;
}

}  // namespace dcg

extern "C" {

using namespace dcg;

size_t dcg_extract_basis_workspace_bytes(int64_t n, int m) {
  if (n < 1 || m < 1 || m > kMaxZ) return 0;
  size_t off[7];
  return ritz_ws_layout(n, m, off);
}

int dcg_extract_basis(const double *Z, const double *AZ, int64_t n, int m, int k, int largest,
                      int extraction, int route, double *W_out, double *theta_out, int *k_out,
                      int *rank_out, void *stream, void *ws, size_t ws_bytes) {
  if (!extract_args_ok(Z, AZ, n, m, k, extraction, route, W_out, theta_out, k_out))
    return DCG_E_ARG;
  size_t off[7];
  if (ws == nullptr || ws_bytes < ritz_ws_layout(n, m, off)) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  return extract_on_given(Z, AZ, n, m, k, largest, extraction, route, W_out, theta_out, k_out,
                          rank_out, static_cast<hipStream_t>(stream), static_cast<char *>(ws),
                          off);
}

size_t dcg_extract_basis_noalloc_max_bytes(void) { return kExtractScratchBytes; }

int dcg_extract_basis_noalloc(const double *Z, const double *AZ, int64_t n, int m, int k,
                              int largest, int extraction, int route, double *W_out,
                              double *theta_out, int *k_out, int *rank_out, void *stream) {
  if (!extract_args_ok(Z, AZ, n, m, k, extraction, route, W_out, theta_out, k_out))
    return DCG_E_ARG;
  size_t off[7];
  if (ritz_ws_layout(n, m, off) > kExtractScratchBytes) return DCG_E_WORKSPACE;
  char *b = nullptr;
  const int rcode = scratch_address(&b);
  if (rcode != DCG_OK) return rcode;
  return extract_on_given(Z, AZ, n, m, k, largest, extraction, route, W_out, theta_out, k_out,
                          rank_out, static_cast<hipStream_t>(stream), b, off);
}

}  // extern "C"
