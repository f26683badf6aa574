"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, sizes workspaces and rejects invalid arguments before any
GPU call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dcg_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_1706_00241_amd as dcg
    if not os.path.exists(dcg.LIB_PATH):
        pytest.fail("libdcg.so is not built (run python -m paper_1706_00241_amd.build)")
    return dcg.load()


def test_exports_every_declared_symbol(L):
    import paper_1706_00241_amd as dcg
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(dcg.EXPORTED)


def test_workspace_queries(L):
    assert L.dcg_operator_workspace_bytes(65536, 32, 1) > 65536 * 32 * 8
    assert L.dcg_operator_workspace_bytes(0, 32, 1) == 0
    assert L.dcg_operator_workspace_bytes(100, 65, 0) == 0       # FP32 points: d <= 64
    assert L.dcg_operator_workspace_bytes(100, 65, 3) == 0       # FP64 operator: d <= 64
    # bf16 / fp16 points beyond 64 coordinates: the LDS-staged sweep, K padded
    # to slices of 64, no FP64 operands
    assert L.dcg_operator_workspace_bytes(1000, 784, 1) >= 1024 * 832 * 2 * 2
    assert L.dcg_operator_workspace_bytes(1000, 4096, 4) > 0
    assert L.dcg_operator_workspace_bytes(1000, 4097, 1) == 0
    assert L.dcg_operator_workspace_bytes(100, 8, 7) == 0
    assert L.dcg_operator_workspace_bytes(100, 8, 4) > 0       # fp16
    # the stored operator: K0 in FP32 over the padded size, any d up to 4096
    assert L.dcg_operator_workspace_bytes(1000, 784, 5) >= 1024 * 1024 * 4
    assert L.dcg_operator_workspace_bytes(1000, 4097, 5) == 0
    assert L.dcg_operator_workspace_bytes(1000, 784, 0) == 0     # sweep operands: d <= 64
    assert L.dcg_operator_workspace_bytes(100, 8, 6) == 0
    assert L.dcg_recycle_workspace_bytes(1000, 8, 12) >= 1000 * 20 * 8 * 2
    assert L.dcg_recycle_workspace_bytes(1000, 8, 4) == 0       # L < k
    assert L.dcg_recycle_workspace_bytes(1000, 65, 100) == 0    # k too large
    assert L.dcg_solve_workspace_bytes(1000, 0, 0) > 0
    # the Newton loop: one solve's workspace plus b~, K b~ / b and z
    assert L.dcg_laplace_gpc_workspace_bytes(1000) >= \
        L.dcg_solve_workspace_bytes(1000, 0, 0) + 3 * 1000 * 8
    assert L.dcg_laplace_gpc_workspace_bytes(0) == 0
    # SLQ: the block solve's workspace, the probe solutions and 2 x max_steps
    # coefficients per probe
    assert L.dcg_slq_logdet_workspace_bytes(1000, 16, 512) >= \
        L.dcg_solve_block_workspace_bytes(1000, 16) + 1000 * 16 * 8 + 16 * 2 * 512 * 8
    assert L.dcg_slq_logdet_workspace_bytes(1000, 65, 512) == 0
    assert L.dcg_slq_logdet_workspace_bytes(1000, 16, 0) == 0
    assert L.dcg_slq_logdet_workspace_bytes(1000, 16, 4097) == 0
    assert L.dcg_laplace_evidence_workspace_bytes(1000, 16, 512) > \
        L.dcg_slq_logdet_workspace_bytes(1000, 16, 512) + 1000 * 8
    assert L.dcg_laplace_evidence_workspace_bytes(1000, 65, 512) == 0


def test_argument_validation_without_gpu(L):
    import paper_1706_00241_amd as dcg
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1024)
    # null X / bad sizes / bad kernel: rejected before any HIP call
    assert L.dcg_create_operator(None, 10, 3, 0, 1.0, 1.0, 0.1, 0, buf, 1024, None, ctypes.byref(h)) == -1
    assert L.dcg_create_operator(buf, 0, 3, 0, 1.0, 1.0, 0.1, 0, buf, 1024, None, ctypes.byref(h)) == -1
    assert L.dcg_create_operator(buf, 10, 3, 9, 1.0, 1.0, 0.1, 0, buf, 1024, None, ctypes.byref(h)) == -1
    assert L.dcg_create_operator(buf, 10, 3, 0, -1.0, 1.0, 0.1, 0, buf, 1024, None, ctypes.byref(h)) == -1
    assert L.dcg_create_operator(buf, 10, 3, 0, 1.0, 1.0, -0.1, 0, buf, 1024, None, ctypes.byref(h)) == -1
    # workspace too small
    assert L.dcg_create_operator(buf, 10, 3, 0, 1.0, 1.0, 0.1, 0, buf, 16, None, ctypes.byref(h)) == -6
    assert L.dcg_recycle_create(10, 8, 4, buf, 1024, ctypes.byref(h)) == -1
    p = dcg.Params(tol=1e-6)
    st = dcg.Stats()
    assert L.dcg_solve(None, None, None, 0, None, ctypes.byref(p), ctypes.byref(st), None, 0) == -1
    assert L.dcg_set_hyper(None, 1.0, 1.0, 1.0) == -1
    assert L.dcg_set_sweep_items(None, 2048) == -1
    assert L.dcg_tune_operator(None, 5, None, None) == -1
    assert L.dcg_matvec(None, None, None, 1) == -1
    assert L.dcg_set_diag(None, None) == -1
    steps = ctypes.c_int(7)
    assert L.dcg_laplace_gpc(None, None, None, ctypes.byref(p), 5, 1.0, None, None, None,
                             ctypes.byref(steps), None, None, 0) == -1
    assert steps.value == 0
    quad = (ctypes.c_double * 2)()
    assert L.dcg_slq_logdet(None, None, 2, ctypes.byref(p), 64, quad, None, None, None, 0) == -1
    assert L.dcg_status_string(-2).decode().startswith("operator not positive")
    assert "gfx950" in L.dcg_version().decode()


def test_batched_arguments_without_gpu(L):
    import paper_1706_00241_amd as dcg
    ns = (ctypes.c_int64 * 3)(1000, 2048, 1)
    total = L.dcg_solve_batched_workspace_bytes(3, ns)
    # every system's CG vectors (r, p, q and three more FP64 n-vectors) and the
    # device tables; batched solves do not refine, so no outer directions
    assert total >= 8 * 6 * (1000 + 2048 + 1)
    assert total < L.dcg_solve_workspace_bytes(1000, 0, 0) + L.dcg_solve_workspace_bytes(2048, 0, 0) \
        + L.dcg_solve_workspace_bytes(1, 0, 0)
    assert total > L.dcg_solve_batched_workspace_bytes(2, ns)
    assert L.dcg_solve_batched_workspace_bytes(0, ns) == 0
    assert L.dcg_solve_batched_workspace_bytes(5000, None) == 0
    bad = (ctypes.c_int64 * 2)(10, 0)
    assert L.dcg_solve_batched_workspace_bytes(2, bad) == 0
    p = dcg.Params(tol=1e-6)
    VP = ctypes.c_void_p * 2
    null2 = VP(None, None)
    st = (dcg.Stats * 2)()
    assert L.dcg_solve_batched(0, null2, null2, null2, 0, None, ctypes.byref(p), st, None, 0) == -1
    assert L.dcg_solve_batched(2, null2, null2, null2, 0, None, ctypes.byref(p), st, None, 0) == -1
    assert L.dcg_solve_batched(2, None, null2, null2, 0, None, ctypes.byref(p), st, None, 0) == -1
    pr = dcg.Params(tol=1e-6, refine=1)
    assert L.dcg_solve_batched(2, null2, null2, null2, 0, None, ctypes.byref(pr), st, None, 0) == -1


def test_extract_basis_arguments_without_gpu(L):
    import paper_1706_00241_amd as dcg
    assert L.dcg_extract_basis_workspace_bytes(1000, 160) > 2 * 160 * 160 * 8
    assert L.dcg_extract_basis_workspace_bytes(1000, 193) == 0
    assert L.dcg_extract_basis_workspace_bytes(0, 10) == 0
    buf = ctypes.create_string_buffer(4096)
    th = (ctypes.c_double * 64)()
    k, r = ctypes.c_int(0), ctypes.c_int(0)
    args = lambda **kw: dict(dict(Z=buf, AZ=buf, n=100, m=10, k=4, largest=1, kind=0, route=0,
                                  W=buf, th=th, k_out=ctypes.byref(k)), **kw)
    def call(a):
        return L.dcg_extract_basis(a["Z"], a["AZ"], a["n"], a["m"], a["k"], a["largest"],
                                   a["kind"], a["route"], a["W"], a["th"], a["k_out"],
                                   ctypes.byref(r), None, buf, 16)
    # every argument error is found before any HIP call; then the workspace
    assert call(args(Z=None)) == -1
    assert call(args(m=0)) == -1
    assert call(args(m=193)) == -1
    assert call(args(k=65)) == -1
    assert call(args(route=2)) == -1
    assert call(args(kind=2)) == -1
    assert call(args()) == -6


def test_extract_basis_noalloc_arguments_without_gpu(L):
    """The entry point without allocation: its scratch is sized for the
    largest pencil (m = 192, k = 64), and every size beyond it, like every
    other argument error, is refused before any HIP call."""
    assert L.dcg_extract_basis_noalloc_max_bytes() >= L.dcg_extract_basis_workspace_bytes(10**7, 192)
    assert L.dcg_extract_basis_noalloc_max_bytes() <= 24 * 2**20
    buf = ctypes.create_string_buffer(4096)
    th = (ctypes.c_double * 64)()
    k, r = ctypes.c_int(0), ctypes.c_int(0)

    def call(Z=buf, n=100, m=10, kk=4, kind=0, route=0, W=buf):
        return L.dcg_extract_basis_noalloc(Z, buf, n, m, kk, 1, kind, route, W, th,
                                           ctypes.byref(k), ctypes.byref(r), None)
    assert call(Z=None) == -1
    assert call(W=None) == -1
    assert call(n=0) == -1
    assert call(m=0) == -1
    assert call(m=193) == -1
    assert call(kk=65) == -1
    assert call(kind=2) == -1
    assert call(route=2) == -1
