"""The extraction entry point that allocates nothing
(dcg_extract_basis_noalloc, scratch in the library's own device array)
against dcg_extract_basis, which takes the same scratch from a caller-owned
workspace.  Both run the same kernels with the same split-K partial layout,
so W' = Z U, the kept harmonic (or Rayleigh-Ritz) values and the rank of the
metric must agree bit for bit.  Several calls in a row, each on a smaller
pencil than the one before, so that a value left in the shared array by an
earlier call could only show if the extraction read scratch it had not
written in the same call."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pencil(n, m, seed):
    """Z (n x m Gaussian) and AZ = A Z for the SPD A = B B^T / r + I, with B
    an n x r Gaussian (r = 40), formed in FP64 on the host."""
    g = np.random.default_rng(seed)
    B = g.standard_normal((n, 40))
    Z = g.standard_normal((n, m))
    AZ = B @ (B.T @ Z) / 40.0 + Z
    return torch.as_tensor(Z, device="cuda"), torch.as_tensor(AZ, device="cuda")


@pytest.mark.parametrize("order", ["large_first", "repeat"])
def test_noalloc_extraction_equals_workspace_extraction(lib, order):
    cases = [(6000, 150, 48, "harmonic", "auto"), (1500, 40, 16, "harmonic", "eigen"),
             (700, 24, 8, "rayleigh", "auto")]
    if order == "repeat":
        cases = cases + cases[:1]
    L = lib.load()
    assert L.dcg_extract_basis_noalloc_max_bytes() >= L.dcg_extract_basis_workspace_bytes(6000, 192)
    for call, (n, m, k, kind, route) in enumerate(cases):
        print(f"call {call}: n {n} m {m} k {k} {kind} {route}", flush=True)
        Z, AZ = _pencil(n, m, seed=100 + call)
        W_ref, th_ref, rank_ref = lib.extract_basis(Z, AZ, k, extraction=kind, ritz_route=route)
        W_out = torch.full((k, n), float("nan"), dtype=torch.float64, device="cuda")
        kk, th, rank = lib.extract_basis_noalloc(Z, AZ, W_out, extraction=kind,
                                                 ritz_route=route)
        torch.cuda.synchronize()
        assert kk == W_ref.shape[1] and kk > 0
        assert rank == rank_ref
        assert th == th_ref
        assert torch.equal(W_out[:kk].t(), W_ref)
