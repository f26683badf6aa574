"""The sweep-plan autotuner: every work-item target gives the oracle's
product (the plans differ only in how block offsets are grouped into work
items, so only the FP64 summation order of row partials changes), the tuner
returns one of its candidates, and tuned operators keep the batched solve
equal to one-by-one solves bit for bit."""

import numpy as np
import pytest

from oracle import kernels as OK
from oracle import precision as OP
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CANDIDATES = (256, 512, 1024, 2048, 4096, 8192)


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("items", CANDIDATES)
def test_every_plan_matches_oracle(lib, prec, items):
    n, d = 5000, 8
    g = np.random.default_rng(workloads.SEED_BASE + 90)
    X = g.standard_normal((n, d))
    ell = workloads.median_distance(X)
    op = lib.Operator(_dev(X), 2, ell, 1.1, 1e-2, prec=prec)
    op.set_sweep_items(items)
    v = g.standard_normal(n)
    y = _np(op.matvec(_dev(v)))
    A = OK.operator(OP.round_points(X, prec, 2, ell), 2, ell, 1.1, 1e-2)
    err = np.abs(y - A @ v) / (np.abs(A) @ np.abs(v))
    assert err.max() <= 2e-5
    # a solve under this plan converges to the tolerance
    b = g.standard_normal(n)
    x, st = lib.solve(op, _dev(b), tol=1e-6)
    assert st["status"] == 0
    xh = _np(x)
    # the GPU solves its own product: allow the product's deviation at x
    floor = np.linalg.norm(_np(op.matvec(x)) - A @ xh) / np.linalg.norm(b)
    assert np.linalg.norm(b - A @ xh) / np.linalg.norm(b) <= 1e-6 + 2 * floor


def test_sweep_items_range(lib):
    X = np.random.default_rng(1).standard_normal((100, 3))
    op = lib.Operator(_dev(X), 0, 1.0, 1.0, 1e-2, prec=1)
    for bad in (0, 255, 8193):
        with pytest.raises(lib.DcgError):
            op.set_sweep_items(bad)


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_tuner_returns_candidate(lib, prec):
    g = np.random.default_rng(workloads.SEED_BASE + 91)
    X = g.standard_normal((20000, 16))
    ell = workloads.median_distance(X)
    op = lib.Operator(_dev(X), 0, ell, 1.0, 1e-2, prec=prec)
    items, ms = op.tune(reps=4)
    assert items in CANDIDATES and ms > 0.0
    print(f"prec {prec}: tuned items {items}, {ms:.3f} ms per sweep", flush=True)
    # the product under the tuned plan, on sampled rows computed by the oracle
    v = g.standard_normal(20000)
    y = _np(op.matvec(_dev(v)))
    Xr = OP.round_points(X, prec, 0, ell)
    y64 = _np(op.matvec_exact(_dev(v)))    # the FP64 sweep under its tuned plan
    for i in g.choice(20000, size=32, replace=False):
        ki = OK.gram(Xr[i:i + 1], 0, ell, 1.0, Y=Xr)[0]
        ki[i] += 1e-2
        tol = 2e-5 if prec != 3 else 1e-12
        assert abs(y[i] - ki @ v) <= tol * (np.abs(ki) @ np.abs(v))
        k64 = OK.gram(X[i:i + 1], 0, ell, 1.0, Y=X)[0]
        k64[i] += 1e-2
        assert abs(y64[i] - k64 @ v) <= 1e-12 * (np.abs(k64) @ np.abs(v))


def test_tuned_batch_equals_single(lib):
    w = workloads.ragged(count=5, n_min=300, n_max=6000, systems=2)
    seqs = w["seqs"]
    stream = torch.cuda.Stream()
    opsA, opsB, rcsA, rcsB = [], [], [], []
    for q in seqs:
        for ops, rcs in ((opsA, rcsA), (opsB, rcsB)):
            ops.append(lib.Operator(_dev(q["X"]), q["kernel"], q["ells"][0], q["s2"],
                                    q["sigma2"], prec=0, stream=stream))
            rcs.append(lib.Recycle(q["X"].shape[0], 8, 12))
        items, _ = opsA[-1].tune(reps=2)
        opsB[-1].set_sweep_items(items)
    bs = [_dev(q["b"]) for q in seqs]
    for t in range(2):
        for s, q in enumerate(seqs):
            opsA[s].set_hyper(q["ells"][t], q["s2"], q["sigma2"])
            opsB[s].set_hyper(q["ells"][t], q["s2"], q["sigma2"])
        xa, sa = lib.solve_batched(opsA, bs, rcs=rcsA, tol=1e-6)
        for s in range(len(seqs)):
            x, st = lib.solve(opsB[s], bs[s], rc=rcsB[s], tol=1e-6)
            assert st["iters"] == sa[s]["iters"] and torch.equal(x, xa[s])
