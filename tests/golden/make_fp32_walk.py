"""Writes fp32_walk_n16384.json: the oracle's solve of the FP32 log-lengthscale
walk (n = 16384, d = 16, RBF, sigma2 = 1e-2, 20 systems, k = 32, L = 48,
tol 1e-6; the workload ``workloads.fp32_walk``) on the operator of the
FP32-rounded scaled points, the operator the library's FP32 precision
represents.

Stored per system: the step counts and the selected harmonic Ritz values of
def-CG(32, 48) with exact FP64 products (Algorithm 1 literal and with the
per-step re-projection), and the same with the per-term product error of
``tests/emulation.py`` at eta = 1e-7 for two seeds (the level of the FP32
operator's evaluation error), from which the GPU test draws its bands.

Every number comes from ``oracle/`` (the dense operator, the sequence
driver, the extraction); the emulated runs add the test suite's error model
to the oracle's own products.  Run from the repository root:

    python tests/golden/make_fp32_walk.py      (about 30 min on 8 cores)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import kernels as OK          # noqa: E402
from oracle import precision as OP        # noqa: E402
from oracle import sequence as OS         # noqa: E402
import workloads                          # noqa: E402
from emulation import noisy_product       # noqa: E402

ETA = 1e-7
SEEDS = (0, 1)


def main(out=os.path.join(HERE, "fp32_walk_n16384.json")):
    w = workloads.fp32_walk()
    X, b = w["X"], w["b"]
    kw = dict(k=w["k"], L=w["L"], tol=w["tol"])
    # every run advances one system at a time, so one dense operator (2.1 GB)
    # is held at once
    runs = {"literal": OS.Sequence(**kw), "reproject": OS.Sequence(reproject=True, **kw),
            "plain": OS.Sequence(recycle=False, **kw)}
    for seed in SEEDS:
        runs[f"emulated{seed}"] = OS.Sequence(reproject=True, **kw)
        runs[f"emulated_plain{seed}"] = OS.Sequence(recycle=False, **kw)
    rec = {name: dict(iters=[], theta=[]) for name in runs}
    t0 = time.time()
    for i, ell in enumerate(w["ells"]):
        Xr = OP.round_points(X, OP.PREC_FP32, w["kernel"], ell)
        A = OK.operator(Xr, w["kernel"], ell, w["s2"], w["sigma2"])
        for name, seq in runs.items():
            if name.startswith("emulated"):
                seed = int(name[-1])
                r = seq.step(noisy_product(A, ETA, 1000 * seed + i), b)
            else:
                r = seq.step(A, b)
            rec[name]["iters"].append(r.iters)
            rec[name]["theta"].append(None if r.theta is None else [float(v) for v in r.theta])
        del A
        print(f"system {i}: " + ", ".join(f"{k} {v['iters'][-1]}" for k, v in rec.items())
              + f"  ({time.time() - t0:.0f} s)", flush=True)
    doc = dict(workload="fp32_walk: n=16384 d=16 X~N(0,1) (FP32 values) RBF s2=1 sigma2=1e-2, "
                        "20 systems on a log-ell walk of step 0.05, b~N(0,1), k=32 L=48 tol 1e-6",
               operator="exact kernel of the FP32-rounded scaled points rnd(c x)/c, FP64",
               ells=[float(v) for v in w["ells"]], eta=ETA, runs=rec)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
