#!/usr/bin/env python3
"""Time-to-tolerance of deflated CG on a sequence of kernel systems, one MI355X.

Workload (the precision-form sequence): X is 65536 x 32 drawn U[-1, 1]; the
operator is Matern-5/2 with ell = 0.5 x median pairwise distance, distances on
bf16 MFMA with FP32 kernel evaluation and FP64 CG recurrences; the sequence
steps sigma2_i = 1e-3 * 0.9^i with a fixed b ~ N(0, 1); each system is solved
by deflated CG with k = 64 recycled harmonic Ritz vectors (L = 96 stored
directions) inside an iterative refinement against the FP64 operator, to a
relative residual of 1e-8.

One step = one system of the sequence: set sigma2_i, the deflated solve (all
CG iterations, deflation projections, refinement residuals with the exact
FP64 product) and the harmonic Ritz refresh of W.  Warm-up steps are the
first systems of the sequence (system 0 is plain CG, W is empty); the timed
steps are the systems after them.  The same timed systems are then solved by
plain CG (no recycling) for comparison.

Printed: one JSON line with value = time-to-tol per solve (ms), the plain-CG
time, matvec GFLOP/s = n^2 (2d + 2) / t_sweep, the roofline of the matvec
sweep (ALU-bound, measured live with HIP events on the operator's stream),
and the FP64 oracle timed on a bounded sample on the host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz of non-packed VALU issue
PEAK_VALU_SLOTS = 256 * 64 * 2.4e9
# VALU issue slots per unique pair of the symmetric sweep (transcendentals
# v_exp_f32 / v_sqrt_f32 count 2 slots: measured half rate on gfx950).  The
# compiled bf16 inner loop issues 7.56 VALU instructions per pair for
# Matern-5/2 (242 per iteration of 32 pairs a lane), 7 of them the formulation
# below.  The points are pre-scaled so that r2 = (c r)^2 needs no
# hyperparameter multiply:
#   RBF        exp2(-r2)                               exp(2) + 2 fma = 4
#   Matern-3/2 u = sqrt r2, (1 + ln2 u) 2^-u           sqrt(2) + exp(2) + fma + mul + 2 fma = 7
#   Matern-5/2 (1 + ln2 u + ln2^2 r2 / 3) 2^-u         sqrt(2) + exp(2) + 2 fma + mul + 2 fma = 9
SLOTS_PER_PAIR = {0: 4, 1: 7, 2: 9}
# FP64 issue slots per unique pair of the FP64 sweep (refinement residuals):
# the distance on FP64 MFMA, 9 K-steps of 4 = 36 FMAs per pair for d = 32
# (one 16x16x4 FP64 MFMA does 1024 FMAs, at the same DP rate as the VALU),
# plus the FP64 VALU instructions of the kernel's formulation: exp2 16 (max,
# rint, subtract, 11 Horner FMAs, convert, ldexp), sqrt 9 (max, rsq, 2 mul,
# 5 FMA), the Matern polynomial 3 (5/2) or 2 (3/2), the row and column FMAs 2.
# The compiled inner loop issues 33.5 / 32.5 / 21.5 VALU instructions per
# pair (Matern-5/2, 3/2, RBF): the formulation plus address and select work.
DP_SLOTS_PER_PAIR = {0: 36 + 18, 1: 36 + 29, 2: 36 + 30}
PEAK_DP_SLOTS = 256 * 64 * 2.4e9
# HBM bytes per launch of the sweep measured with rocprofv3 FETCH_SIZE /
# WRITE_SIZE (scaled by a 256 MiB copy) for this workload, valid while the
# sweep's source is the one the counters were taken from (its SHA-256 prefix);
# None for any other configuration or source.
SWEEP_TRAFFIC = {("bf16", 65536, 32, 2, 8192): (112.6e6, "73e7f4b4495c711d")}
# the same for the wide pair sweep (bf16 points, GPC pixel workload), keyed by
# (points, n, d, work items) and valid for the sources of csrc/wide.hip (the
# kernel) and csrc/host.cpp (its operand width) it was taken from
WIDE_TRAFFIC = {("bf16", 36551, 784, 8192): (2491.2e6, "52b46e8a7fcbbc28", "bdc84a605bc288b2"),
                ("bf16", 36551, 784, 4096): (2414.1e6, "52b46e8a7fcbbc28", "bdc84a605bc288b2")}


def _source_sha(name):
    import hashlib
    src = os.path.join(ROOT, "paper_1706_00241_amd", "csrc", name)
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def sweep_traffic(prec, n, d, kernel, items):
    entry = SWEEP_TRAFFIC.get((prec, n, d, kernel, items))
    if entry is None:
        return None
    value, sha = entry
    return value if sha is not None and _source_sha("matvec.hip") == sha else None


def wide_traffic(points, n, d, items):
    entry = WIDE_TRAFFIC.get((points, n, d, items))
    if entry is None:
        return None
    value, sha_kernel, sha_host = entry
    if _source_sha("wide.hip") != sha_kernel or _source_sha("host.cpp") != sha_host:
        return None
    return value


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--literal", action="store_true",
                    help="ell = 0.5 as written (an almost diagonal operator)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-literal", action="store_true",
                    help="skip the short ell = 0.5 (as written) line")
    ap.add_argument("--prec", choices=["bf16", "bf16x2", "fp32", "fp16"], default="bf16",
                    help="operator precision of the inner solves")
    ap.add_argument("--inner-tol", type=float, default=2e-2,
                    help="relative tolerance of each inner (low-precision) solve; the bf16 "
                         "operator contracts the refinement error by ~0.1 per step, so "
                         "tighter inner solves only add iterations")
    ap.add_argument("--refresh", choices=["first", "every", "accum"], default="first",
                    help="refresh W after the first inner solve, after every inner solve, or "
                         "once per system from the directions of all its inner solves")
    ap.add_argument("--extraction", choices=["harmonic", "rayleigh", "implicit"], default="harmonic",
                    help="next basis by harmonic Ritz (Eq. 7, F and G as tall products), by "
                         "Rayleigh-Ritz, or by harmonic Ritz with F and G from the stored "
                         "scalars of the first L steps (no stored A P_L)")
    ap.add_argument("--select", choices=["largest", "smallest"], default="largest",
                    help="keep the Ritz pairs of the largest or of the smallest values")
    ap.add_argument("--ritz-route", choices=["auto", "eigen"], default="auto",
                    help="reduction of F in the harmonic Ritz problem (Cholesky where a bound "
                         "allows it, or always the eigendecomposition)")
    ap.add_argument("--refine", choices=["ir", "fcg"], default="ir",
                    help="outer loop: iterative refinement or flexible CG in FP64")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default sweep plan instead of the autotuned one")
    ap.add_argument("--sweep-items", type=int, default=0, metavar="N",
                    help="use this sweep plan (work-item target) instead of tuning; for "
                         "profiling runs that should launch only the timed plan")
    ap.add_argument("--workload", choices=["bf16_shift", "ragged", "gp_hyper", "fp32_walk",
                                           "gpc", "gpc64"],
                    default="bf16_shift",
                    help="bf16_shift: the headline sequence; ragged: the batching form (64 "
                         "independent sequences, one batched solve per step); gp_hyper: the "
                         "differentiation form (Adam on the GP marginal likelihood); "
                         "fp32_walk: FP32 log-ell walk; gpc: Laplace GP classification "
                         "(the paper's own test problem, the whole Newton loop per step) on "
                         "784-pixel data with the stored kernel matrix; gpc64: the same loop "
                         "at d = 64 with the matrix-free FP32 operator")
    ap.add_argument("--refine-walk", action="store_true",
                    help="fp32_walk: refine against the FP64 operator so that the tolerance "
                         "holds for the true residual")
    ap.add_argument("--gpc-stored", action="store_true",
                    help="gpc64: use the stored kernel matrix instead of the matrix-free sweep")
    ap.add_argument("--gpc-points", choices=["stored", "bf16", "fp16"], default="stored",
                    help="gpc (784 coordinates): the stored kernel matrix, or the matrix-free "
                         "LDS-staged sweep of bf16 / fp16 points")
    ap.add_argument("--adam-steps", type=int, default=50,
                    help="gp_hyper: Adam steps in all (the first --warmup are not timed)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized device buffer (a kernel of known traffic "
                         "for scaling HBM counters)")
    return ap.parse_args()


_ORACLE = {}


def _oracle_init():
    # one BLAS thread per worker: the pool itself spreads over the cores
    from threadpoolctl import threadpool_limits
    _ORACLE["limits"] = threadpool_limits(1)


def _oracle_rows(bounds):
    from oracle import kernels as OK
    lo, hi = bounds
    X = _ORACLE["X"]
    return lo, OK.gram(X[lo:hi], _ORACLE["kernel"], _ORACLE["ell"], 1.0, X) @ _ORACLE["v"]


def oracle_product_seconds(w, block=256):
    """Wall time of one full product of the FP64 oracle, K(X, X) v over all n
    rows in its dense-row form (oracle.kernels.gram row blocks times v), on
    the host cores: a pool of one process per core (the cores this process
    may run on, at most 16: the host's CPU share per GPU), each taking
    blocks of `block` rows.  Called before anything touches the GPU (the
    pool forks).  Returns (seconds, processes, cores in the affinity mask)."""
    import multiprocessing as mp
    import numpy as np
    X = w["X"]
    n = X.shape[0]
    affinity = len(os.sched_getaffinity(0))
    procs = max(1, min(affinity, 16))
    _ORACLE.update(X=X, kernel=w["kernel"], ell=w["ell"],
                   v=np.random.default_rng(0).standard_normal(n))
    chunks = [(lo, min(n, lo + block)) for lo in range(0, n, block)]
    with mp.get_context("fork").Pool(procs, initializer=_oracle_init) as pool:
        pool.map(_oracle_rows, [(0, 8)] * procs)            # imports, first touch
        t0 = time.perf_counter()
        parts = pool.map(_oracle_rows, chunks, chunksize=1)
        t = time.perf_counter() - t0
    y = np.empty(n)
    for lo, part in parts:
        y[lo:lo + part.shape[0]] = part
    assert np.all(np.isfinite(y))
    return t, procs, affinity


def cpu_baseline(t_product, procs, affinity, n, products_per_solve):
    """The oracle's time per solve: one full oracle product (timed) times the
    products (low-precision and FP64 alike, the oracle has only FP64) that
    the GPU run needed per solve; the oracle's vector work per step is O(n)
    against the product's O(n^2 d) and is not counted."""
    total = t_product * products_per_solve
    return {"value": round(total * 1e3, 1), "unit": "ms/solve", "cores": procs, "kind": "oracle",
            "sample": f"one full FP64 oracle product (oracle.kernels.gram rows x v, all {n} rows) "
                      f"on {procs} processes ({affinity} cores in the affinity mask, the pool "
                      f"capped at 16): {t_product:.2f} s, times the {products_per_solve:.1f} "
                      f"products per solve of the GPU run"}


def main_ragged(args):
    """Batching form: 64 independent sequences (n log-uniform in [2048, 32768],
    d = 8, RBF / Matern-3/2, FP32 operator, k = 16, L = 24, tol 1e-6); one step
    = one batched deflated solve of every sequence's next system.  The same
    steps are then solved one system at a time for comparison."""
    import torch

    import paper_1706_00241_amd as dcg
    import workloads

    dcg.load()
    steps = min(args.steps, 4)
    warm = min(args.warmup, 5 - steps)
    w = workloads.ragged(systems=warm + steps)
    seqs = w["seqs"]
    stream = torch.cuda.Stream()

    def build():
        ops, rcs = [], []
        for q in seqs:
            ops.append(dcg.Operator(torch.as_tensor(q["X"], device="cuda"), q["kernel"],
                                    q["ells"][0], q["s2"], q["sigma2"], prec=dcg.PREC_FP32,
                                    stream=stream))
            rcs.append(dcg.Recycle(q["X"].shape[0], w["k"], w["L"]))
        return ops, rcs

    opsA, rcsA = build()
    opsB, rcsB = build()
    items = []
    for a, b in zip(opsA, opsB):
        it, _ = a.tune(reps=3)
        b.set_sweep_items(it)
        items.append(it)
    bs = [torch.as_tensor(q["b"], device="cuda") for q in seqs]

    def hyper(ops, t):
        for op, q in zip(ops, seqs):
            op.set_hyper(q["ells"][t], q["s2"], q["sigma2"])

    for t in range(warm):
        hyper(opsA, t)
        dcg.solve_batched(opsA, bs, rcs=rcsA, tol=w["tol"])
        hyper(opsB, t)
        for op, b, rc in zip(opsB, bs, rcsB):
            dcg.solve(op, b, rc=rc, tol=w["tol"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for t in range(warm, warm + steps):
        hyper(opsA, t)
        _, st = dcg.solve_batched(opsA, bs, rcs=rcsA, tol=w["tol"])
        stats.append(st)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    bad = sum(1 for st in stats for s in st if s["status"] != 0)
    t_single = None
    if not args.no_plain:
        t0 = time.perf_counter()
        for t in range(warm, warm + steps):
            hyper(opsB, t)
            for op, b, rc in zip(opsB, bs, rcsB):
                dcg.solve(op, b, rc=rc, tol=w["tol"])
        torch.cuda.synchronize()
        t_single = time.perf_counter() - t0
    matvecs = sum(s["matvecs"] for st in stats for s in st)
    ns = [q["X"].shape[0] for q in seqs]
    pairs = sum(s["iters"] * n * (n + 1) / 2 for st in stats for s, n in zip(st, ns))
    out = {
        "metric": "aggregate matvecs/s, 64 ragged sequences batched, 1 GPU",
        "value": round(matvecs / t_batched, 1),
        "unit": "matvecs/s",
        "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": round(t_batched * 1e3 / steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32 points (three bf16 terms on bf16 MFMA), f32 kernel values, f64 CG", "data": "synthetic",
        "config": {"workload": "ragged: 64 sequences, n log-uniform [2048, 32768], d=8, "
                               "RBF/Matern-3/2, sigma2 log-uniform [1e-4, 1e-1], k=16 L=24 tol 1e-6",
                   "sum_n": sum(ns), "sweep_items": sorted(set(items))},
        "unique_pairs_per_s": round(pairs / t_batched, 1),
        "one_by_one_ms_per_step": round(t_single * 1e3 / steps, 2) if t_single else None,
        "speedup_vs_one_by_one": round(t_single / t_batched, 3) if t_single else None,
        "iters_per_system": [[s["iters"] for s in st] for st in stats],
        "failed_solves": bad,
    }
    print(json.dumps(out), flush=True)
    if bad:
        sys.exit(1)


def main_walk(args):
    """FP32 sequence: n = 16384, d = 16, RBF, sigma2 = 1e-2, 20 systems on a
    log-ell random walk (step 0.05), fixed b, k = 32, L = 48, tol 1e-6.  One
    step = one system: set_hyper (the operands follow ell), AW for the new
    operator (a block product), the deflated solve and the refresh.  The same
    systems are then solved by plain CG.  Matvecs count the block product."""
    import torch

    import paper_1706_00241_amd as dcg
    import workloads

    dcg.load()
    w = workloads.fp32_walk()
    n = w["X"].shape[0]
    dev = torch.device("cuda:0")
    X = torch.as_tensor(w["X"], device=dev)
    b = torch.as_tensor(w["b"], device=dev)
    op = dcg.Operator(X, w["kernel"], w["ells"][0], w["s2"], w["sigma2"], prec=dcg.PREC_FP32)
    items, _ = op.tune(reps=5)
    ws = dcg.SolveWorkspace(n, dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    systems = len(w["ells"])
    warm = min(args.warmup, systems - 1)

    refine = args.refine_walk

    def run(rc):
        rows = []
        for t, ell in enumerate(w["ells"]):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.set_hyper(ell, w["s2"], w["sigma2"])
            if refine:
                # FP64 residuals: the 1e-6 tolerance holds for the true residual
                _, st = dcg.solve(op, b, rc=rc, tol=w["tol"], ws=ws, out=x, refine=True,
                                  inner_tol=1e-3)
            else:
                _, st = dcg.solve(op, b, rc=rc, tol=w["tol"], ws=ws, out=x, true_residual=True)
            torch.cuda.synchronize()
            rows.append((st["iters"], st["matvecs"], (time.perf_counter() - t0) * 1e3,
                         st["rel_res_true"], st["status"], st["matvecs_exact"]))
        return rows

    rows = run(dcg.Recycle(n, w["k"], w["L"], device=dev))
    for t, r in enumerate(rows):
        print(f"system {t}: {r[0]} its, {r[1]} matvecs, {r[2]:.2f} ms, res {r[3]:.2e}",
              file=sys.stderr, flush=True)
    timed = rows[warm:]
    ms = sum(r[2] for r in timed) / len(timed)
    res_true = sorted(r[3] for r in rows)
    out = {
        "metric": "ms per solve, FP32 deflated CG on a log-ell random walk, n=16384, 1 GPU",
        "value": round(ms, 3), "unit": "ms/solve", "n_gpus": 1,
        "steps": len(timed), "warmup": warm, "ms_per_step": round(ms, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32 points (three bf16 terms on bf16 MFMA), f32 kernel values, f64 CG",
        "data": "synthetic",
        "config": {"workload": "fp32_walk: n=16384 d=16 X~N(0,1) RBF sigma2=1e-2, 20 systems, "
                               "log-ell walk step 0.05, k=32 L=48, "
                               + ("tol 1e-6 on the FP64 true residual (refinement against the "
                                  "FP64 operator, inner tol 1e-3)" if refine else
                                  "tol 1e-6 on the recursive residual; the true residual "
                                  f"reached is {res_true[-1]:.1e} at most (the FP32 operator's "
                                  "evaluation floor, rel_res_true_*)"),
                   "sweep_items": items, "refine": bool(refine)},
        "matvecs_per_solve": round(sum(r[1] for r in timed) / len(timed), 1),
        "exact_matvecs_per_solve": round(sum(r[5] for r in timed) / len(timed), 1),
        "iters_per_solve": round(sum(r[0] for r in timed) / len(timed), 1),
        "rel_res_true_max": res_true[-1],
        "rel_res_true_median": _median(res_true),
        "rel_res_true_of": ("|b - A64 x| / |b|, FP64 operator on the unrounded points" if refine
                            else "|b - A x| / |b| with the solve's own FP32 operator"),
        "failed_solves": sum(1 for r in rows if r[4] != 0 or (refine and r[3] > w["tol"])),
    }
    if not args.no_plain:
        prow = run(None)[warm:]
        out["plain_ms_per_solve"] = round(sum(r[2] for r in prow) / len(prow), 3)
        out["plain_matvecs_per_solve"] = round(sum(r[1] for r in prow) / len(prow), 1)
        out["speedup_vs_plain"] = round(out["plain_ms_per_solve"] / ms, 3)
    print(json.dumps(out), flush=True)
    if out["failed_solves"]:
        sys.exit(1)


def main_gpc(args):
    """Laplace GP classification (section 3): Newton's method for the mode
    from f = 0 until Psi grows by less than 1, each system A = I + D K D
    solved to 1e-5 by def-CG(8, 12) with W carried from one Newton system to
    the next.  One step = one whole Newton loop (every system, its K products,
    Psi); the same loop is then run with plain CG.

    gpc: the paper-shaped data, n = 36551 pixel-like points in d = 784, RBF
    with s2 = 10; the stored operator (K0 formed once in FP64, kept in HBM as
    FP32, every product one streaming pass with FP64 accumulation; forming
    K0 is outside the timed loop, as it is fixed across the Newton steps).
    gpc64: n = 36551 two-class points in d = 64, s2 = 100, the matrix-free
    FP32 operator (FP32 MFMA distances, FP32 kernel values)."""
    import torch

    import paper_1706_00241_amd as dcg
    import workloads

    dcg.load()
    if args.copy_calibration > 0:
        # a plain copy of known size, for scaling the HBM counters of a profile
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wide = args.workload == "gpc" and args.gpc_points != "stored"
    stored = (args.workload == "gpc" and not wide) or args.gpc_stored
    w = workloads.gpc_pixels() if args.workload == "gpc" else workloads.gpc()
    n, d = w["X"].shape
    dev = torch.device("cuda:0")
    X = torch.as_tensor(w["X"], device=dev)
    y = torch.as_tensor(w["y"], device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if wide:
        prec = dcg.PREC_BF16 if args.gpc_points == "bf16" else dcg.PREC_FP16
    else:
        prec = dcg.PREC_STORED if stored else dcg.PREC_FP32
    op = dcg.Operator(X, w["kernel"], w["ell"], w["s2"], 0.0, prec=prec)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    items, _ = op.tune(reps=5)

    def run(rc_args, profile):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = dcg.Recycle(n, *rc_args, device=dev) if rc_args else None
        _, _, psi, stats, status = dcg.laplace_gpc(op, y, rc=rc, tol=w["tol"],
                                                   psi_tol=w["psi_tol"], profile=profile)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, psi, stats, status

    for _ in range(args.warmup):
        run((w["k"], w["L"]), False)
    # the timed runs carry HIP events around each CG step's sweep (as the
    # headline's timed solves do), for the sweep kernel's own duration
    runs = [run((w["k"], w["L"]), True) for _ in range(args.steps)]
    ms = sum(r[0] for r in runs) / len(runs)
    _, psi, stats, status = runs[-1]
    its = [s["iters"] for s in stats]
    for t, s in enumerate(stats):
        print(f"newton {t + 1}: {s['iters']} its, {s['matvecs']} matvecs, "
              f"{s['t_total_ms']:.2f} ms, psi {psi[t + 1]:.3f}", file=sys.stderr, flush=True)
    if args.workload == "gpc":
        data = (f"gpc: n={n} d={d} pixel-like points in (0,1) (logistic of 16 Gaussian blobs), "
                f"labels from a smooth random function, RBF ell=0.5 x median distance s2=10")
    else:
        data = (f"gpc64: n={n} d={d}, two classes of 6 Gaussian modes, 5% labels flipped, "
                f"RBF ell=0.5 x median distance s2=100")
    if stored:
        dtype = "f32 stored kernel matrix (formed in f64), f64 accumulation, CG and Newton terms"
    elif wide:
        dtype = (f"{args.gpc_points} points on {args.gpc_points} MFMA (LDS-staged), f32 kernel "
                 f"values, f64 CG and Newton terms")
    else:
        dtype = "fp32 points on fp32 MFMA, f32 kernel values, f64 CG and Newton terms"
    out = {
        "metric": f"ms per Laplace-GPC mode (whole Newton loop), def-CG(8,12) to 1e-5, "
                  f"n={n}, 1 GPU",
        "value": round(ms, 2), "unit": "ms/mode", "n_gpus": 1, "steps": len(runs),
        "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": data + ", Newton from f=0 until dPsi < 1, def-CG(8,12) tol 1e-5",
                   "sweep_items": items},
        "operator_build_ms": round(build_ms, 1),
        "newton_steps": len(stats), "iters_per_system": its,
        "matvecs_total": sum(s["matvecs"] for s in stats),
        "solve_ms_total": round(sum(s["t_total_ms"] for s in stats), 2),
        "psi": [round(v, 3) for v in psi], "status": status,
        "failed_solves": sum(1 for s in stats if s["status"] != 0),
    }
    if stored:
        # the dominant kernel: one product streams K0's packed block upper
        # triangle (nb (nb + 1) / 2 tiles of 128 x 128 FP32); timed with HIP
        # events on the operator's stream (stage, tile pass and row reduction)
        n_pad = (n + 255) // 256 * 256
        nb = n_pad // 128
        kbytes = nb * (nb + 1) // 2 * 128 * 128 * 4
        v = torch.ones(n, dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        op.matvec(v)
        e0.record(op.stream)
        for _ in range(reps):
            op.matvec(v)
        e1.record(op.stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / reps
        gbs = kbytes / (t * 1e-3) / 1e9
        out["product_ms"] = round(t, 4)
        out["stored_bytes_per_product"] = kbytes
        # HBM bytes per stored_symv launch from rocprofv3 FETCH_SIZE + WRITE_SIZE
        # (scaled by a 256 MiB copy) for this workload and this kernel version
        traffic = 2775.5e6 if (args.workload == "gpc" and n == 36551) else None
        out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                           "unit": "GB/s", "frac": round(gbs / 8000.0, 4), "traffic": traffic}
    if wide:
        # the dominant kernel: the LDS-staged pair sweep; algorithmic work 2 d
        # MFMA flops per unique pair (the distance contraction) over the
        # kernel's own duration (HIP events around each sweep launch of the
        # timed runs' CG steps); whole products (staging, sweep, row
        # reduction) are timed beside it
        sw_n = sum(st["sweeps_timed"] for r in runs for st in r[2])
        sw_ms = sum(st["t_sweeps_ms"] for r in runs for st in r[2]) / max(1, sw_n)
        v = torch.ones(n, dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        op.matvec(v)
        e0.record(op.stream)
        for _ in range(reps):
            op.matvec(v)
        e1.record(op.stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / reps
        flops = 2.0 * d * n * (n - 1) / 2
        if sw_n == 0:
            print("bench.py: no sweep timings from the profiled solves", file=sys.stderr)
            sys.exit(1)
        tf = flops / (sw_ms * 1e-3) / 1e12
        out["product_ms"] = round(t, 4)
        out["sweep_ms"] = round(sw_ms, 4)
        out["sweeps_timed"] = sw_n
        out["roofline"] = {"bound": "mfma", "achieved": round(tf, 1), "peak": 2500.0,
                           "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4),
                           "traffic": wide_traffic(args.gpc_points, n, d, items),
                           "traffic_unit": "bytes per launch of symv_wide_kernel (rocprofv3 "
                                           "FETCH_SIZE + WRITE_SIZE)",
                           "per_launch": f"{n * (n - 1) // 2:.3e} unique pairs x 2 d flops"}
    if not args.no_plain:
        prow = [run(None, False) for _ in range(max(1, min(args.steps, 3)))]
        out["plain_ms_per_mode"] = round(sum(r[0] for r in prow) / len(prow), 2)
        out["plain_iters_per_system"] = [s["iters"] for s in prow[-1][2]]
        out["plain_matvecs_total"] = sum(s["matvecs"] for s in prow[-1][2])
        out["speedup_vs_plain"] = round(out["plain_ms_per_mode"] / ms, 3)
    print(json.dumps(out), flush=True)
    if out["failed_solves"] or status != 0:
        sys.exit(1)


def main_gp(args):
    """Differentiation form: GP hyperparameter optimisation, n = 32768, d = 16,
    RBF, FP32 operator, Adam (lr 0.05) on theta = (log ell, log s2, log
    sigma2).  One step = the marginal likelihood and its gradient: alpha =
    A^{-1} y by deflated CG (the recycled W, k = 32, refreshed), 16 Rademacher
    probe solves reusing W, one fused gradient sweep, the Adam update.  The
    same steps (each step's recorded theta) are then run without recycling.""" 
    import math

    import torch

    import paper_1706_00241_amd as dcg
    import workloads

    dcg.load()
    w = workloads.gp_hyper()
    n = w["X"].shape[0]
    total = max(args.adam_steps, args.warmup + 1)
    dev = torch.device("cuda:0")
    X = torch.as_tensor(w["X"], device=dev)
    y = torch.as_tensor(w["y"], device=dev)
    probes = [torch.as_tensor(workloads.rademacher(n, w["probes"], step=t), device=dev)
              for t in range(total)]

    def run(steps, recycle, first=0, replay=None):
        """Adam from theta_0, or (replay) the given theta of every step."""
        theta = torch.tensor([w["log_ell"], w["log_s2"], w["log_sigma2"]], dtype=torch.float64,
                             requires_grad=True)
        opt = torch.optim.Adam([theta], lr=w["lr"])
        thetas = []
        op = dcg.Operator(X, w["kernel"], math.exp(w["log_ell"]), 1.0, math.exp(w["log_sigma2"]),
                          prec=dcg.PREC_FP32)
        op.tune(reps=3)
        rc = dcg.Recycle(n, w["k"], w["L"], device=dev) if recycle else None
        rows, t_timed = [], 0.0
        for t in range(steps):
            if replay is not None:
                with torch.no_grad():
                    theta.copy_(torch.tensor(replay[t], dtype=torch.float64))
            thetas.append(theta.detach().tolist())
            gpc = dcg.GPContext(op, y, rc, probes[t], tol=w["tol"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            opt.zero_grad()
            val = dcg.GPMarginalLikelihood.apply(theta, gpc)
            (-val).backward()
            if replay is None:
                opt.step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if t >= first:
                t_timed += dt
            rows.append((float(val), gpc.last["alpha_stats"]["iters"],
                         gpc.last["probe_stats"]["iters"], dt * 1e3))
        return rows, t_timed / max(1, steps - first), theta.detach().tolist(), thetas

    rows, ms, theta, thetas = run(total, True, first=args.warmup)
    for t, r in enumerate(rows):
        print(f"adam step {t}: data-fit {r[0]:.3f}, alpha its {r[1]}, probe its {r[2]}, "
              f"{r[3]:.1f} ms", file=sys.stderr, flush=True)
    out = {
        "metric": "ms per Adam step (marginal likelihood + gradient), GP hyper-optimisation "
                  "n=32768, 1 GPU",
        "value": round(ms * 1e3, 2), "unit": "ms/step", "n_gpus": 1,
        "steps": total - args.warmup, "warmup": args.warmup, "ms_per_step": round(ms * 1e3, 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32 points (three bf16 terms on bf16 MFMA), f32 kernel values, f64 CG", "data": "synthetic",
        "config": {"workload": "gp_hyper: n=32768 d=16 RBF, y = sin-sum + 0.1 noise, "
                               "16 Rademacher probes per step, k=32 L=48, tol 1e-6, Adam lr 0.05",
                   "adam_steps": total},
        "alpha_iters_per_step": round(sum(r[1] for r in rows[args.warmup:]) / (total - args.warmup), 1),
        "probe_iters_per_step": round(sum(r[2] for r in rows[args.warmup:]) / (total - args.warmup), 1),
        "theta_final": [round(v, 5) for v in theta],
    }
    if not args.no_plain:
        # the same steps (the recorded theta of each) without recycling
        prows, pms, _, _ = run(total, False, first=args.warmup, replay=thetas)
        out["plain_ms_per_step"] = round(pms * 1e3, 2)
        out["plain_alpha_iters_per_step"] = round(
            sum(r[1] for r in prows[args.warmup:]) / (total - args.warmup), 1)
        out["plain_probe_iters_per_step"] = round(
            sum(r[2] for r in prows[args.warmup:]) / (total - args.warmup), 1)
        out["speedup_vs_plain"] = round(pms / ms, 3)
    print(json.dumps(out), flush=True)


def _median(v):
    v = sorted(v)
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def run_sequence(dcg, op, rc, w, b, kw, first, count, profile=False):
    """Solve systems first .. first + count - 1 of the configured sigma2
    sequence, restarting it after its last system (system i has sigma2_{i mod
    10}); returns the per-solve stats with each solve's wall time."""
    sig = w["sigma2s"]
    out = []
    for i in range(first, first + count):
        t0 = time.perf_counter()
        op.set_hyper(w["ell"], 1.0, sig[i % len(sig)])
        _, st = dcg.solve(op, b, rc=rc, profile=profile, **kw)
        st["wall_ms"] = (time.perf_counter() - t0) * 1e3
        st["system"] = i
        out.append(st)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ragged":
        return main_ragged(args)
    if args.workload == "gp_hyper":
        return main_gp(args)
    if args.workload in ("gpc", "gpc64"):
        return main_gpc(args)
    if args.workload == "fp32_walk":
        return main_walk(args)
    import workloads

    # the configured sequence: ten systems sigma2_i = 1e-3 * 0.9^i
    w = workloads.bf16_shift(n=args.n, systems=10, literal=args.literal)
    n, d = w["X"].shape
    # the oracle's product on the host cores, before anything touches the GPU
    cpu = oracle_product_seconds(w) if not args.no_cpu else None

    import torch

    import paper_1706_00241_amd as dcg

    dcg.load()
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dev = torch.device("cuda:0")
    X = torch.as_tensor(w["X"], device=dev)
    b = torch.as_tensor(w["b"], device=dev)
    prec = {"bf16": dcg.PREC_BF16, "bf16x2": dcg.PREC_BF16X2, "fp32": dcg.PREC_FP32,
            "fp16": dcg.PREC_FP16}[args.prec]
    op = dcg.Operator(X, w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=prec)
    items = 2048
    if args.sweep_items > 0:
        items = args.sweep_items
        op.set_sweep_items(items)
    elif not args.no_tune:
        items, tms = op.tune(reps=5)
        print(f"tuned sweep plan: {items} work items, {tms:.3f} ms per sweep", file=sys.stderr,
              flush=True)
    rc = dcg.Recycle(n, w["k"], w["L"], device=dev)
    ws = dcg.SolveWorkspace(n, dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    kw = dict(tol=w["tol"], refine=args.refine, inner_tol=args.inner_tol, ws=ws, out=x,
              refresh_every=args.refresh, ritz_route=args.ritz_route,
              extraction=args.extraction, select_largest=args.select == "largest",
              check_every=8)

    for st in run_sequence(dcg, op, rc, w, b, kw, 0, args.warmup):
        print(f"warmup system {st['system']}: {st['iters']} its, {st['outer_steps']} outer, "
              f"{st['t_total_ms']:.1f} ms, res {st['rel_res_true']:.2e}", file=sys.stderr,
              flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = run_sequence(dcg, op, rc, w, b, kw, args.warmup, args.steps, profile=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    for st in stats:
        print(f"system {st['system']}: {st['iters']} its, {st['outer_steps']} outer, "
              f"{st['t_total_ms']:.1f} ms (refresh {st['t_refresh_ms']:.1f}: m {st['refresh_dim']} "
              f"rank {st['refresh_rank']} sweeps {st['refresh_sweeps']}), "
              f"res {st['rel_res_true']:.2e}, status {st['status']}", file=sys.stderr, flush=True)
    bad = [st for st in stats if st["status"] != 0 or st["rel_res_true"] > w["tol"]]
    if bad:
        print(f"bench.py: {len(bad)} solves missed the tolerance", file=sys.stderr)
        sys.exit(1)

    sweeps = sum(st["sweeps_timed"] for st in stats)
    t_sweep = sum(st["t_sweeps_ms"] for st in stats) / max(1, sweeps) * 1e-3   # s
    pairs = n * (n + 1) / 2.0
    slots = pairs * SLOTS_PER_PAIR[w["kernel"]]
    achieved = slots / t_sweep
    gflops = n * n * (2 * d + 2) / t_sweep / 1e9
    ex_n = sum(st["exact_sweeps_timed"] for st in stats)
    t_ex = sum(st["t_exact_sweeps_ms"] for st in stats) / max(1, ex_n) * 1e-3    # s
    walls = [st["wall_ms"] for st in stats]
    mean = lambda key: sum(st[key] for st in stats) / len(stats)
    t_other = mean("t_total_ms") - mean("t_init_ms") - mean("t_loop_ms") - mean("t_refresh_ms")

    out = {
        "metric": "time-to-tol per solve & matvec GFLOP/s: deflated vs plain CG, n=65536, 1 GPU",
        "value": round(ms_per_step, 2),
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "bf16x2": "split bf16", "fp16": "fp16",
                  "fp32": "fp32 points (three bf16 terms on bf16 MFMA)"}[args.prec]
                 + (" MFMA distances" if args.prec != "fp32" else "")
                 + ", f32 kernel values, f64 CG",
        "data": "synthetic",
        "config": {"workload": ("bf16_shift" + ("_literal" if args.literal else "")
                                + f": n={n} d={d} X~U[-1,1] matern52 ell={w['ell']:.4f} "
                                f"sigma2=1e-3*0.9^i (i mod 10) k={w['k']} L={w['L']} "
                                f"refine to 1e-8"),
                   "systems_timed": args.steps, "first_system": args.warmup,
                   "sequence_length": len(w["sigma2s"]),
                   "refine": args.refine, "refresh": args.refresh, "inner_tol": args.inner_tol,
                   "extraction": args.extraction, "select": args.select,
                   "sweep_items": items},
        "ms_per_solve_median": round(_median(walls), 2),
        "ms_per_solve_min": round(min(walls), 2),
        "phases_ms_per_solve": {
            "init": round(mean("t_init_ms"), 2),
            "cg_loop": round(mean("t_loop_ms"), 2),
            "refresh": round(mean("t_refresh_ms"), 2),
            "fp64_residuals_and_host": round(t_other, 2)},
        "iters_per_solve": round(mean("iters"), 1),
        "matvecs_per_solve": round(mean("matvecs"), 1),
        "exact_matvecs_per_solve": round(mean("matvecs_exact"), 1),
        "rel_res_true_max": max(st["rel_res_true"] for st in stats),
        "matvec_ms": round(t_sweep * 1e3, 4),
        "matvec_gflops": round(gflops, 1),
        "gpair_per_s": round(n * n / t_sweep / 1e9, 1),
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 2),
                     "peak": round(PEAK_VALU_SLOTS / 1e12, 2), "unit": "TOP/s",
                     "frac": round(achieved / PEAK_VALU_SLOTS, 3),
                     "traffic": sweep_traffic(args.prec, n, d, w["kernel"], items),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "kernel": "symv_kernel (symmetric pair sweep)",
                     "per_launch": f"{pairs:.4g} unique pairs x {SLOTS_PER_PAIR[w['kernel']]} "
                                   "VALU slots"},
    }
    if ex_n:
        # the FP64 pair sweep of the refinement residuals: FP64 MFMA distances
        # and FP64 kernel values share the DP issue rate (78.6 TFLOP/s = one
        # FP64 FMA per lane and clock either way)
        dp = pairs * DP_SLOTS_PER_PAIR[w["kernel"]]
        out["roofline_fp64"] = {
            "bound": "fp64", "achieved": round(dp / t_ex / 1e12, 2),
            "peak": round(PEAK_DP_SLOTS / 1e12, 2), "unit": "T DP-slots/s",
            "frac": round(dp / t_ex / PEAK_DP_SLOTS, 3), "ms": round(t_ex * 1e3, 4),
            "launches_timed": ex_n, "kernel": "symv64_kernel (FP64 pair sweep)",
            "per_launch": f"{pairs:.4g} unique pairs x {DP_SLOTS_PER_PAIR[w['kernel']]} FP64 "
                          "issue slots (MFMA FMAs and VALU instructions)"}

    if not args.no_plain:
        # the same systems by plain CG inside the same refinement
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        tp = run_sequence(dcg, op, None, w, b, kw, args.warmup, args.steps)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.steps
        out["plain_ms_per_solve"] = round(plain_ms, 2)
        out["plain_ms_per_solve_median"] = round(_median([st["wall_ms"] for st in tp]), 2)
        out["plain_matvecs_per_solve"] = round(sum(s["matvecs"] for s in tp) / args.steps, 1)
        out["plain_exact_matvecs_per_solve"] = round(
            sum(s["matvecs_exact"] for s in tp) / args.steps, 1)
        out["speedup_vs_plain"] = round(plain_ms / ms_per_step, 3)
        print(f"plain CG: {plain_ms:.1f} ms/solve, {out['plain_matvecs_per_solve']} matvecs",
              file=sys.stderr, flush=True)

    if not args.literal and not args.no_literal:
        # the configuration as written (ell = 0.5: K is close to I, CG needs a
        # few steps and deflation has nothing to remove), same points and b
        wl = workloads.bf16_shift(n=args.n, systems=10, literal=True)
        opl = dcg.Operator(X, wl["kernel"], wl["ell"], 1.0, wl["sigma2s"][0], prec=prec)
        rcl = dcg.Recycle(n, wl["k"], wl["L"], device=dev)
        run_sequence(dcg, opl, rcl, wl, b, kw, 0, 2)
        lit = run_sequence(dcg, opl, rcl, wl, b, kw, 2, 5)
        litp = run_sequence(dcg, opl, None, wl, b, kw, 2, 5)
        out["literal"] = {
            "config": f"ell=0.5 as written, systems 2-6 of the sequence",
            "ms_per_solve": round(sum(s["wall_ms"] for s in lit) / len(lit), 2),
            "plain_ms_per_solve": round(sum(s["wall_ms"] for s in litp) / len(litp), 2),
            "iters_per_solve": round(sum(s["iters"] for s in lit) / len(lit), 1),
            "plain_iters_per_solve": round(sum(s["iters"] for s in litp) / len(litp), 1),
            "outer_steps_per_solve": round(sum(s["outer_steps"] for s in lit) / len(lit), 1),
            "rel_res_true_max": max(s["rel_res_true"] for s in lit + litp)}
        del opl, rcl

    if cpu is not None:
        t_prod, procs, affinity = cpu
        out["cpu_baseline"] = cpu_baseline(t_prod, procs, affinity, n,
                                           out["matvecs_per_solve"] + out["exact_matvecs_per_solve"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
