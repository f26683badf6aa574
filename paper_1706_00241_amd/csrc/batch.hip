// Batched deflated CG: many independent systems A_s x_s = b_s, each with its
// own operator (points, kernel, hyperparameters, size) and its own recycled
// basis, solved in lockstep.  The paper treats one sequence at a time
// (Algorithm 1 with the section 2.3 refresh); a batch runs many such
// sequences side by side, each one's step exactly the single-system step.
//
// Every system is initialised on its own; then one step of all of them is
// one batched pair sweep (the grid is the concatenation of every system's
// work items, grouped by operand layout) followed by one launch per CG
// vector kernel with blockIdx.y selecting the system.  A chunk of steps is
// captured as a hipGraph; the host reads the packed per-system state once per
// chunk.  Systems that converge inside a chunk skip the rest of its kernels;
// after the check they leave the tables and the chunk is re-captured for the
// systems still running.
// Each system's basis is refreshed on its own afterwards.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "solve.h"

namespace dcg {

static int64_t bdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// What the host needs of one system after a chunk.
struct StateHead {
  double relres;
  int iter, done, status, pad;
};

__global__ __launch_bounds__(256) void gather_states(const CgArgs *args, int count,
                                                     StateHead *out) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= count) return;
  const SolveState *S = args[s].S;
  StateHead h;
  h.relres = S->relres;
  h.iter = S->iter;
  h.done = S->done;
  h.status = S->status;
  h.pad = 0;
  out[s] = h;
}

struct BatchLayout {
  size_t items, args, heads, total;
  std::vector<size_t> sys;   // solve workspace of each system
};

static BatchLayout batch_layout(int count, const int64_t *n) {
  BatchLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t o = off;
    off += bytes;
    return o;
  };
  L.items = take(sizeof(BatchItem) * size_t(count));
  L.args = take(sizeof(CgArgs) * size_t(count));
  L.heads = take(sizeof(StateHead) * size_t(count));
  L.sys.resize(count);
  for (int s = 0; s < count; ++s) L.sys[s] = take(solve_workspace_total(n[s], false));
  L.total = align256(off);
  return L;
}

// One group of systems whose sweeps share a kernel instantiation.
struct SweepGroup {
  int opk, ksteps;
  int first, count;   // range in the device item table
  int64_t total;      // work items of the group
};

struct BatchPlan {
  std::vector<SweepGroup> groups;
  std::vector<int> direct;    // systems swept one by one (FP64 or unsupported shapes)
  int64_t nq_max = 1, nx_max = 1, np_max = 1;   // grids of the per-step kernels
};

static int enqueue_batch_step(hipStream_t s, int count, dcg_operator_s *const *ops,
                              const std::vector<SolveCtx> &ctx, const BatchPlan &plan,
                              const BatchItem *d_items, const CgArgs *d_args) {
  for (const SweepGroup &g : plan.groups) {
    const int st = launch_symv_batched(d_items + g.first, g.count, g.total, g.ksteps, g.opk, s);
    if (st != DCG_OK) return st;
  }
  for (int i : plan.direct) {
    dcg_operator_s *op = ops[i];
    const int *done = &ctx[i].B.S->done;
    const int st = (op->g.prec == DCG_PREC_FP64)
                       ? matvec_exact_done(op, ctx[i].a.p, op->ytmp, 1, done)
                       : launch_symv_sweep(op, 1, done);
    if (st != DCG_OK) return st;
  }
  const unsigned cy = static_cast<unsigned>(count);
  const dim3 gq(static_cast<unsigned>(plan.nq_max), cy), gx(static_cast<unsigned>(plan.nx_max), cy),
      gp(static_cast<unsigned>(plan.np_max), cy);
  hipLaunchKernelGGL(cg_matvec_finish_multi, gq, dim3(256), 0, s, d_args);
  hipLaunchKernelGGL(cg_update_xr_multi, gx, dim3(256), 0, s, d_args);
  hipLaunchKernelGGL(cg_finalize_multi, dim3(1, cy), dim3(256), 0, s, d_args);
  hipLaunchKernelGGL(cg_update_p_multi, gp, dim3(256), 0, s, d_args);
  return hipGetLastError() == hipSuccess ? DCG_OK : DCG_E_HIP;
}

// Device tables of the running systems `act` (positions in the tables are
// positions in act; blockIdx.y of the vector kernels indexes them).
static int build_tables(const std::vector<int> &act, dcg_operator_s *const *ops,
                        const std::vector<SolveCtx> &ctx, hipStream_t strm, BatchItem *d_items,
                        CgArgs *d_args, BatchPlan *plan) {
  *plan = BatchPlan();
  std::vector<BatchItem> items;
  std::vector<CgArgs> args(act.size());
  std::map<std::pair<int, int>, std::vector<int>> by_shape;
  for (size_t i = 0; i < act.size(); ++i) {
    const int s = act[i];
    const dcg_operator_s *op = ops[s];
    args[i] = ctx[s].a;
    plan->nq_max = std::max(plan->nq_max, ctx[s].a.nblk_q);
    plan->nx_max = std::max(plan->nx_max, xr_grid(ctx[s].a));
    plan->np_max = std::max(plan->np_max, ctx[s].a.nblk_p);
    // bf16 and bf16x2 operands share the bf16 kernels (one operand kind)
    if (op->g.prec != DCG_PREC_FP64 && symv_batched_supported(op->g.opk, op->g.ksteps))
      by_shape[{op->g.opk, op->g.ksteps}].push_back(s);
    else
      plan->direct.push_back(s);
  }
  for (const auto &kv : by_shape) {
    SweepGroup g;
    g.opk = kv.first.first;
    g.ksteps = kv.first.second;
    g.first = static_cast<int>(items.size());
    g.count = static_cast<int>(kv.second.size());
    g.total = 0;
    for (int s : kv.second) {
      BatchItem it;
      int64_t grid = 0;
      it.a = symv_args(ops[s], 1, ops[s]->vin, &ctx[s].B.S->done, &grid);
      it.kernel = ops[s]->kernel;
      it.item0 = g.total;
      g.total += grid;
      items.push_back(it);
    }
    if (g.total > int64_t(0x7fffffff)) return DCG_E_ARG;
    plan->groups.push_back(g);
  }
  if (!items.empty())
    HIPCHK(hipMemcpyAsync(d_items, items.data(), sizeof(BatchItem) * items.size(),
                          hipMemcpyHostToDevice, strm));
  HIPCHK(hipMemcpyAsync(d_args, args.data(), sizeof(CgArgs) * args.size(),
                        hipMemcpyHostToDevice, strm));
  // the host vectors go out of scope: the copies must have read them
  HIPCHK(hipStreamSynchronize(strm));
  return DCG_OK;
}

static void fill_stats(dcg_stats *st, const InnerResult &R) {
  st->iters = R.iters;
  st->matvecs = R.matvecs;
  st->k_used = R.k_used;
  st->k_next = R.k_next;
  st->rel_res_recursive = R.relres;
  st->t_init_ms = R.t_init;
  st->t_loop_ms = R.t_loop;
  st->t_refresh_ms = R.t_refresh;
  st->status = R.status;
}

}  // namespace dcg

using namespace dcg;

extern "C" {

size_t dcg_solve_batched_workspace_bytes(int count, const int64_t *n) {
  if (count < 1 || count > kMaxBatch || n == nullptr) return 0;
  for (int s = 0; s < count; ++s)
    if (n[s] < 1) return 0;
  return batch_layout(count, n).total;
}

int dcg_solve_batched(int count, const dcg_op_t *ops, const double *const *b, double *const *x,
                      int x_given, const dcg_recycle_t *rcs, const dcg_params *p,
                      dcg_stats *stats, void *ws, size_t ws_bytes) {
  if (stats != nullptr && count > 0 && count <= kMaxBatch)
    std::memset(stats, 0, sizeof(dcg_stats) * size_t(count));
  if (count < 1 || count > kMaxBatch || ops == nullptr || b == nullptr || x == nullptr ||
      p == nullptr)
    return DCG_E_ARG;
  if (!(p->tol >= 0.0) || p->check_every < 0 || p->refine != 0 || p->ritz_route < 0 ||
      p->ritz_route > 1 || p->extraction < 0 || p->extraction > 1)
    return DCG_E_ARG;
  std::vector<int64_t> ns(count);
  std::set<const void *> seen_op, seen_rc;
  for (int s = 0; s < count; ++s) {
    dcg_operator_s *op = ops[s];
    if (op == nullptr || b[s] == nullptr || x[s] == nullptr) return DCG_E_ARG;
    // not supported with a diagonal scaling, the stored operator or wide points
    if (op->has_dsc || op->g.prec == DCG_PREC_STORED || sweep_wide(op->g)) return DCG_E_ARG;
    // each system sweeps into its operator's own partial buffers
    if (!seen_op.insert(op).second) return DCG_E_ARG;
    if (op->stream != ops[0]->stream) return DCG_E_ARG;
    dcg_recycle_s *rc = rcs ? rcs[s] : nullptr;
    if (rc != nullptr && (rc->n != op->g.n || !seen_rc.insert(rc).second)) return DCG_E_ARG;
    ns[s] = op->g.n;
  }
  const BatchLayout BL = batch_layout(count, ns.data());
  if (ws == nullptr || ws_bytes < BL.total) return DCG_E_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return DCG_E_WORKSPACE;
  char *base = static_cast<char *>(ws);
  BatchItem *d_items = reinterpret_cast<BatchItem *>(base + BL.items);
  CgArgs *d_args = reinterpret_cast<CgArgs *>(base + BL.args);
  StateHead *d_heads = reinterpret_cast<StateHead *>(base + BL.heads);
  hipStream_t strm = ops[0]->stream;

  // ---- phase 1: every system's initialisation
  std::vector<SolveCtx> ctx(count);
  std::vector<InnerResult> R(count);
  for (int s = 0; s < count; ++s) {
    dcg_recycle_s *rc = rcs ? rcs[s] : nullptr;
    const int st = solve_init(ops[s], b[s], x[s], x_given, rc, p, p->tol, base + BL.sys[s], StorePlan(),
                              &ctx[s], &R[s]);
    if (st != DCG_OK) {
      if (stats != nullptr) stats[s].status = st;
      return st;
    }
  }

  // ---- phase 2: lockstep iteration over the systems still running.  The
  // device tables and the captured chunk cover only those; whenever a check
  // finds systems done, the tables are rebuilt and the chunk re-captured, so
  // converged systems stop costing launches.
  const auto t1 = Clock::now();
  const int chunk = std::max(1, p->check_every);
  std::vector<int> act(count);
  for (int s = 0; s < count; ++s) act[s] = s;
  std::vector<StateHead> heads(count), hact(count);
  for (int s = 0; s < count; ++s) {
    heads[s].done = 0;
    heads[s].iter = 0;
    heads[s].status = 0;
    heads[s].relres = 0.0;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  auto release = [&]() {
    if (gexec != nullptr) (void)hipGraphExecDestroy(gexec);
    if (graph != nullptr) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  };
  BatchPlan plan;
  int status = DCG_OK;
  bool rebuild = true;
  while (!act.empty()) {
    const int na = static_cast<int>(act.size());
    if (rebuild) {
      release();
      status = build_tables(act, ops, ctx, strm, d_items, d_args, &plan);
      if (status != DCG_OK) break;
      if (p->use_graph) {
        if (hipStreamBeginCapture(strm, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          status = DCG_E_HIP;
          break;
        }
        int st = DCG_OK;
        for (int c = 0; c < chunk && st == DCG_OK; ++c)
          st = enqueue_batch_step(strm, na, ops, ctx, plan, d_items, d_args);
        const hipError_t e = hipStreamEndCapture(strm, &graph);
        if (st != DCG_OK || e != hipSuccess) {
          status = st != DCG_OK ? st : DCG_E_HIP;
          break;
        }
        if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
          status = DCG_E_HIP;
          break;
        }
      }
      rebuild = false;
    }
    if (gexec != nullptr) {
      if (hipGraphLaunch(gexec, strm) != hipSuccess) { status = DCG_E_HIP; break; }
    } else {
      for (int c = 0; c < chunk && status == DCG_OK; ++c)
        status = enqueue_batch_step(strm, na, ops, ctx, plan, d_items, d_args);
      if (status != DCG_OK) break;
    }
    hipLaunchKernelGGL(gather_states, dim3(static_cast<unsigned>(bdiv(na, 256))), dim3(256), 0,
                       strm, d_args, na, d_heads);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hact.data(), d_heads, sizeof(StateHead) * size_t(na),
                       hipMemcpyDeviceToHost, strm) != hipSuccess ||
        hipStreamSynchronize(strm) != hipSuccess) {
      status = DCG_E_HIP;
      break;
    }
    std::vector<int> next;
    next.reserve(act.size());
    for (int i = 0; i < na; ++i) {
      heads[act[i]] = hact[i];
      if (!hact[i].done) next.push_back(act[i]);
    }
    rebuild = next.size() != act.size();
    act.swap(next);
  }
  release();
  if (status != DCG_OK) return status;
  const double t_loop = ms_since(t1);

  // ---- phase 3: per-system results and basis refresh
  int worst = DCG_OK;
  for (int s = 0; s < count; ++s) {
    InnerResult &r = R[s];
    const StateHead &h = heads[s];
    r.t_loop = t_loop;
    r.iters = h.iter;
    r.relres = h.relres;
    ctx[s].matvecs += h.iter;
    r.status = h.status != 0 ? h.status : (h.relres <= p->tol ? DCG_OK : DCG_NOT_CONVERGED);
    r.k_used = ctx[s].k;
    r.k_next = ctx[s].k;
    dcg_recycle_s *rc = rcs ? rcs[s] : nullptr;
    const int st = solve_extract(ops[s], rc, p, &ctx[s], &r);
    if (st != DCG_OK) return st;
    if (stats != nullptr) fill_stats(&stats[s], r);
    if (p->true_residual) {
      double rel = 0.0;
      const int tr = true_residual(ops[s], b[s], x[s], 0, ctx[s].B, &rel);
      if (tr != DCG_OK) return tr;
      if (stats != nullptr) {
        stats[s].rel_res_true = rel;
        stats[s].matvecs += 1;
      }
    }
    if (r.status < 0 && worst >= 0) worst = r.status;
    else if (r.status == DCG_NOT_CONVERGED && worst == DCG_OK) worst = DCG_NOT_CONVERGED;
  }
  return worst;
}

}  // extern "C"
