"""GPU parity of the implicit extraction (extraction = "implicit"): F and G
of Eq. 7 from the scalars of the first L steps (section 2.3, as Saad et al.
formed them) and AW' from the residual recurrence, against the oracle's
``ritz.implicit_extract`` on the same sequence (tests/test_oracle_implicit.py
pins that one against the explicit F = (AZ)^T Z, G = (AZ)^T AZ)."""

import numpy as np
import pytest

from oracle import kernels as OK
from oracle import precision as OP
from oracle import ritz as ORZ
from oracle import sequence as OS
import workloads


pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec,tol,th_rtol", [(3, 1e-8, 1e-6), (0, 1e-6, 2e-3)])
def test_implicit_sequence_matches_oracle(lib, prec, tol, th_rtol):
    """The n = 1024 five-system sequence (def-CG(8, 12)) with the implicit
    extraction: iteration counts as the oracle's implicit sequence (within 2
    on the FP64 operator; within the FP32 band of the explicit sequence
    test on the FP32 operator), the selected harmonic Ritz values to 1e-6
    (FP64) / 2e-3 (FP32), and AW' from the recurrence equal to the dense
    product A W' of the same points (1e-10 / 1e-4 of (|A| |W'|)_i): the
    implied products are the operator's own."""
    w = workloads.small()
    X = w["X"]
    n = X.shape[0]
    mats = [OK.operator(OP.round_points(X, prec, w["kernel"], ell), w["kernel"], ell, 1.0,
                        w["sigma2"]) for ell in w["ells"]]
    bs = [A @ w["xstar"] + w["noise"][i] for i, A in enumerate(mats)]
    ref = OS.solve_sequence(mats, bs, k=8, L=12, tol=tol, extraction=ORZ.IMPLICIT,
                            reproject=True)
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], 1.0, w["sigma2"], prec=prec)
    rc = lib.Recycle(n, 8, 12)
    # FP64: AW' from the recurrence; FP32: the sweep's products of W'
    # (2e-5 of (|A| |p|)_i each), combined through the cleanup's U
    prod_tol = 1e-10 if prec == 3 else 1e-4
    for i, (ell, A, b) in enumerate(zip(w["ells"], mats, bs)):
        op.set_hyper(ell, 1.0, w["sigma2"])
        x, st = lib.solve(op, _dev(b), rc=rc, tol=tol, extraction="implicit")
        assert st["status"] == 0
        res = np.linalg.norm(b - A @ _np(x)) / np.linalg.norm(b)
        fl = np.linalg.norm(_np(op.matvec(x)) - A @ _np(x)) / np.linalg.norm(b)
        assert res <= tol + 2 * fl
        th = np.array(rc.theta())
        print(f"system {i}: its {st['iters']} oracle {ref[i].iters}; theta {th[:3]} "
              f"oracle {ref[i].theta[:3]}", flush=True)
        if prec == 3:
            assert abs(st["iters"] - ref[i].iters) <= 2, (i, st["iters"], ref[i].iters)
        else:
            assert ref[i].iters - 3 <= st["iters"] <= 1.15 * ref[i].iters + 2
        np.testing.assert_allclose(th, ref[i].theta, rtol=th_rtol)
        W, AW = _np(rc.get_W()), _np(rc.get_AW())
        scale = np.abs(A) @ np.abs(W)
        assert np.all(np.abs(AW - A @ W) <= prod_tol * scale), np.max(np.abs(AW - A @ W) / scale)


def test_implicit_matches_explicit_extraction_fp64(lib):
    """The same first solve extracted both ways (FP64 operator, n = 1024,
    def-CG(8, 12) from W = 0): the implicit pencil gives the explicit one's
    Ritz values to 1e-8 and the same recycled space (principal-angle cosines
    1 - 1e-8), as exact arithmetic says."""
    w = workloads.small()
    X = w["X"]
    n = X.shape[0]
    ell = w["ells"][0]
    A = OK.operator(X, w["kernel"], ell, 1.0, w["sigma2"])
    b = A @ w["xstar"] + w["noise"][0]
    op = lib.Operator(_dev(X), w["kernel"], ell, 1.0, w["sigma2"], prec=3)
    out = {}
    for kind in ("harmonic", "implicit"):
        rc = lib.Recycle(n, 8, 12)
        lib.solve(op, _dev(b), rc=rc, tol=1e-8, extraction=kind)
        out[kind] = (np.array(rc.theta()), _np(rc.get_W()))
    np.testing.assert_allclose(out["implicit"][0], out["harmonic"][0], rtol=1e-8)
    Qa, _ = np.linalg.qr(out["implicit"][1])
    Qb, _ = np.linalg.qr(out["harmonic"][1])
    s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    assert s.min() > 1 - 1e-8


def test_implicit_refinement_bf16(lib):
    """Refinement to 1e-8 with bf16 inner solves (n = 3000, Matern-5/2,
    def-CG(16, 24), refresh after the first inner solve, three systems of
    the sigma2 sequence) with the implicit extraction: every system reaches
    the tolerance in the dense FP64 residual, the recycled AW is the bf16
    operator's product of W (1e-4 of (|A| |W|)_i), and the step counts stay
    within 15% (+2) of the explicit extraction's on the same sequence."""
    w = workloads.bf16_shift(n=3000, systems=3)
    X, b, kern, ell = w["X"], w["b"], w["kernel"], w["ell"]
    K64 = OK.gram(X, kern, ell, 1.0)
    its = {}
    for kind in ("harmonic", "implicit"):
        op = lib.Operator(_dev(X), kern, ell, 1.0, w["sigma2s"][0], prec=1)
        rc = lib.Recycle(3000, 16, 24)
        its[kind] = []
        for s2 in w["sigma2s"]:
            op.set_hyper(ell, 1.0, s2)
            x, st = lib.solve(op, _dev(b), rc=rc, tol=1e-8, refine=True, inner_tol=1e-2,
                              extraction=kind)
            assert st["status"] == 0
            A64 = K64 + s2 * np.eye(3000)
            res = np.linalg.norm(b - A64 @ _np(x)) / np.linalg.norm(b)
            assert res <= 1.05e-8, (kind, res)
            its[kind].append(st["iters"])
            # the recycled AW is the bf16 operator's product of W
            W, AW = _np(rc.get_W()), _np(rc.get_AW())
            Ab = OK.operator(OP.round_points(X, 1, kern, ell), kern, ell, 1.0, s2)
            err = np.max(np.abs(AW - Ab @ W) / (np.abs(Ab) @ np.abs(W)))
            assert err <= 1e-4, (kind, err)
    print(f"steps: {its}", flush=True)
    for a, c in zip(its["implicit"], its["harmonic"]):
        assert a <= 1.15 * c + 2, its


def test_implicit_refused_where_undefined(lib):
    """The implicit pencil describes one Krylov sequence: the pooled refresh
    of refinement (directions of several inner solves) and the batched solve
    refuse it with DCG_E_ARG."""
    w = workloads.small(n=600)
    X = w["X"]
    op = lib.Operator(_dev(X), w["kernel"], w["ells"][0], 1.0, w["sigma2"], prec=0)
    rc = lib.Recycle(600, 8, 12)
    b = _dev(np.random.default_rng(1).standard_normal(600))
    with pytest.raises(lib.DcgError) as e:
        lib.solve(op, b, rc=rc, tol=1e-8, refine=True, refresh_every="accum",
                  extraction="implicit")
    assert e.value.status == -1
    with pytest.raises(lib.DcgError) as e:
        lib.solve_batched([op], [b], rcs=[rc], tol=1e-6, extraction="implicit")
    assert e.value.status == -1
    # and the handle still works
    _, st = lib.solve(op, b, rc=rc, tol=1e-6, extraction="implicit")
    assert st["status"] == 0 and st["k_next"] == 8


def test_implicit_headline_sequence(lib):
    """The implicit extraction on the first four systems of the n = 65536
    sigma2 sequence (bf16 points, Matern-5/2, def-CG(64, 96), refinement to
    1e-8 with inner solves to 2e-2, refresh after the first inner solve):
    every system meets the tolerance, and after each extraction the recycled
    AW is the operator's product of W (relative Frobenius difference 1e-4;
    the bf16 sweep's own products differ by ~1e-5).  Regression for implied
    products that, combined through a U built without the lost conjugacy,
    were off by 34% after the first recycled system (the refined solve of
    the next system then broke down)."""
    w = workloads.bf16_shift(n=65536, systems=4)
    X, b = _dev(w["X"]), _dev(w["b"])
    op = lib.Operator(X, w["kernel"], w["ell"], 1.0, w["sigma2s"][0], prec=1)
    rc = lib.Recycle(65536, w["k"], w["L"])
    for i, s2 in enumerate(w["sigma2s"]):
        op.set_hyper(w["ell"], 1.0, s2)
        _, st = lib.solve(op, b, rc=rc, tol=w["tol"], refine=True, inner_tol=2e-2,
                          extraction="implicit", max_iter=4000, refine_max=16)
        W, AW = rc.get_W(), rc.get_AW()
        rel = float(torch.linalg.norm(AW - op.matvec(W.contiguous())) / torch.linalg.norm(AW))
        print(f"system {i}: its {st['iters']} outer {st['outer_steps']} k_next {st['k_next']} "
              f"res {st['rel_res_true']:.2e} |AW - A W| / |AW| {rel:.1e}", flush=True)
        assert st["status"] == 0 and st["rel_res_true"] <= w["tol"]
        assert st["k_next"] >= w["k"] // 2
        assert rel <= 1e-4, (i, rel)
