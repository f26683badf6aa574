"""Python binding of libdcg.so: deflated CG with Krylov subspace recycling on MI355X.

Argument marshalling only.  Every step of the method (distance GEMM, kernel
evaluation, CG recurrences, deflation projections, harmonic Ritz extraction,
iterative refinement) runs in the library's HIP kernels; PyTorch provides the
device memory and the stream.  The names follow the C ABI in include/dcg.h.

There is no fallback: if the library is not built, or no GPU is present,
every entry point raises.

Typical use (a sequence of related systems, section 1 of de Roos & Hennig)::

    op = Operator(X, kernel=RBF, ell=1.0, s2=1.0, sigma2=1e-2, prec=PREC_FP32)
    rc = Recycle(n, k=32, L=48)
    for ell in ells:
        op.set_hyper(ell, 1.0, 1e-2)
        x, st = solve(op, b, rc=rc, tol=1e-6)
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcg.so")

RBF, MATERN32, MATERN52 = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_BF16X2, PREC_FP64, PREC_FP16, PREC_STORED = 0, 1, 2, 3, 4, 5
STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "not SPD",
          -3: "non-finite", -4: "W rank deficient", -5: "HIP error",
          -6: "workspace"}


class DcgError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("L", ctypes.c_int), ("select_largest", ctypes.c_int),
                ("check_every", ctypes.c_int), ("refine", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("refine_max", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("true_residual", ctypes.c_int),
                ("profile", ctypes.c_int), ("refresh_every", ctypes.c_int),
                ("ritz_route", ctypes.c_int), ("extraction", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("matvecs_exact", ctypes.c_int), ("k_used", ctypes.c_int),
                ("k_next", ctypes.c_int), ("outer_steps", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("t_init_ms", ctypes.c_double),
                ("t_loop_ms", ctypes.c_double), ("t_refresh_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("sweeps_timed", ctypes.c_int),
                ("t_sweeps_ms", ctypes.c_double), ("refresh_dim", ctypes.c_int),
                ("refresh_rank", ctypes.c_int), ("refresh_sweeps", ctypes.c_int * 2),
                ("exact_sweeps_timed", ctypes.c_int), ("t_exact_sweeps_ms", ctypes.c_double)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["refresh_sweeps"] = list(self.refresh_sweeps)
        return d


_lib = None

_SIGS = {
    "dcg_operator_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]),
    "dcg_create_operator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "dcg_set_hyper": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]),
    "dcg_set_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dcg_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "dcg_matvec_exact": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64]),
    "dcg_set_sweep_items": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "dcg_tune_operator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_double)]),
    "dcg_destroy_operator": (None, [ctypes.c_void_p]),
    "dcg_recycle_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    "dcg_recycle_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "dcg_recycle_set_W": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "dcg_recycle_get_W": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int)]),
    "dcg_recycle_get_AW": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dcg_recycle_get_theta": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int)]),
    "dcg_recycle_destroy": (None, [ctypes.c_void_p]),
    "dcg_solve_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
    "dcg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.POINTER(Params), ctypes.POINTER(Stats),
                                 ctypes.c_void_p, ctypes.c_size_t]),
    "dcg_solve_block_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
    "dcg_solve_block": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(Params),
                                       ctypes.POINTER(Stats), ctypes.c_void_p, ctypes.c_size_t]),
    "dcg_solve_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int,
                                                           ctypes.POINTER(ctypes.c_int64)]),
    "dcg_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Params),
                                         ctypes.POINTER(Stats), ctypes.c_void_p, ctypes.c_size_t]),
    "dcg_mll_grad_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "dcg_mll_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                    ctypes.c_size_t]),
    "dcg_mll_value": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "dcg_extract_basis_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int]),
    "dcg_extract_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t]),
    "dcg_extract_basis_noalloc_max_bytes": (ctypes.c_size_t, []),
    "dcg_extract_basis_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                 ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_double),
                                                 ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]),
    "dcg_laplace_gpc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "dcg_laplace_gpc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(Params), ctypes.c_int, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Stats),
                                       ctypes.c_void_p, ctypes.c_size_t]),
    "dcg_slq_logdet_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64,
                                                        ctypes.c_int]),
    "dcg_slq_logdet": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(Params), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                      ctypes.c_size_t]),
    "dcg_laplace_evidence_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64,
                                                              ctypes.c_int]),
    "dcg_laplace_evidence": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.POINTER(Params), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                            ctypes.c_size_t]),
    "dcg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dcg_version": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def load(path=LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1706_00241_amd.build`")
    # torch first: the library then binds the HIP runtime torch has loaded
    # (the same soname), so device pointers and streams from torch are valid
    # in it; loaded first, it would bind the system runtime and torch a copy
    # of its own
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, where):
    if status < 0:
        raise DcgError(status, where)
    return status


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the deflated-CG library runs on an MI355X only")
    return torch


def _workspace(nbytes, device):
    torch = _torch()
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off, int(nbytes)


class _ordered:
    """Order the library's stream after the caller's current stream on entry
    and the caller's stream after the library's on exit."""

    def __init__(self, stream):
        self.stream = stream

    def __enter__(self):
        torch = _torch()
        self.cur = torch.cuda.current_stream(self.stream.device)
        self.stream.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        self.cur.wait_stream(self.stream)
        return False


def _colmajor(V):
    """(n,) or (n, m) tensor -> contiguous (m, n) FP64 buffer = n x m column-major."""
    torch = _torch()
    if V.dim() == 1:
        return V.to(torch.float64).contiguous().view(1, -1)
    return V.to(torch.float64).t().contiguous()


class Operator:
    """A = K_theta(X, X) + sigma2 I applied matrix-free on the GPU."""

    def __init__(self, X, kernel, ell, s2, sigma2, prec=PREC_FP32, stream=None):
        torch = _torch()
        lib = load()
        X = X.to(device="cuda", dtype=torch.float64).contiguous()
        self.n, self.d = X.shape
        self.device = X.device
        self.kernel, self.prec = int(kernel), int(prec)
        # a dedicated stream (default priority): the library captures its
        # iteration chunks as hipGraphs, which the legacy default stream
        # cannot do; every call orders it against the caller's stream.
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        nbytes = lib.dcg_operator_workspace_bytes(self.n, self.d, self.prec)
        if nbytes == 0:
            raise DcgError(-1, "dcg_operator_workspace_bytes")
        self._ws, ptr, size = _workspace(nbytes, self.device)
        h = ctypes.c_void_p()
        with _ordered(self.stream):
            _check(lib.dcg_create_operator(X.data_ptr(), self.n, self.d, self.kernel, float(ell),
                                           float(s2), float(sigma2), self.prec, ptr, size,
                                           self.stream.cuda_stream, ctypes.byref(h)),
                   "dcg_create_operator")
        self.handle = h
        self.ell, self.s2, self.sigma2 = float(ell), float(s2), float(sigma2)

    def set_hyper(self, ell, s2, sigma2):
        _check(load().dcg_set_hyper(self.handle, float(ell), float(s2), float(sigma2)),
               "dcg_set_hyper")
        self.ell, self.s2, self.sigma2 = float(ell), float(s2), float(sigma2)

    def set_diag(self, D=None):
        """A = D K D + sigma2 I from now on (D: (n,) nonnegative); None removes it."""
        torch = _torch()
        ptr = None
        if D is not None:
            self._dsc_src = D.to(device=self.device, dtype=torch.float64).contiguous()
            ptr = self._dsc_src.data_ptr()
        with _ordered(self.stream):
            _check(load().dcg_set_diag(self.handle, ptr), "dcg_set_diag")
        self._dsc_src = None

    def _mv(self, fn, V):
        torch = _torch()
        Vc = _colmajor(V.to(self.device))
        Y = torch.empty_like(Vc)
        with _ordered(self.stream):
            _check(fn(self.handle, Vc.data_ptr(), Y.data_ptr(), Vc.shape[0]), fn.__name__)
        return Y.view(-1) if V.dim() == 1 else Y.t()

    def matvec(self, V):
        """A V with the operator's compute precision (V: (n,) or (n, m))."""
        return self._mv(load().dcg_matvec, V)

    def matvec_exact(self, V):
        """A V with the FP64 operator on the unrounded points."""
        return self._mv(load().dcg_matvec_exact, V)

    def set_sweep_items(self, items):
        """Work-item target of the pair sweep (256..8192)."""
        _check(load().dcg_set_sweep_items(self.handle, int(items)), "dcg_set_sweep_items")

    def tune(self, reps=5):
        """Time the sweep plans and keep the fastest; returns (items, ms per sweep)."""
        items, ms = ctypes.c_int(), ctypes.c_double()
        with _ordered(self.stream):
            _check(load().dcg_tune_operator(self.handle, int(reps), ctypes.byref(items),
                                            ctypes.byref(ms)), "dcg_tune_operator")
        return items.value, ms.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            load().dcg_destroy_operator(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Recycle:
    """Recycled basis W (n x k) and the storage of the first L directions."""

    def __init__(self, n, k, L, device="cuda"):
        lib = load()
        _torch()
        self.n, self.k, self.L = int(n), int(k), int(L)
        nbytes = lib.dcg_recycle_workspace_bytes(self.n, self.k, self.L)
        if nbytes == 0:
            raise DcgError(-1, "dcg_recycle_workspace_bytes")
        self._ws, ptr, size = _workspace(nbytes, device)
        h = ctypes.c_void_p()
        _check(lib.dcg_recycle_create(self.n, self.k, self.L, ptr, size, ctypes.byref(h)),
               "dcg_recycle_create")
        self.handle = h
        self.device = device

    def set_W(self, W):
        torch = _torch()
        if W is None or W.numel() == 0:
            _check(load().dcg_recycle_set_W(self.handle, None, 0), "dcg_recycle_set_W")
            return
        Wc = _colmajor(W.to(self.device))
        torch.cuda.synchronize()
        _check(load().dcg_recycle_set_W(self.handle, Wc.data_ptr(), Wc.shape[0]),
               "dcg_recycle_set_W")

    def get_W(self):
        torch = _torch()
        k = ctypes.c_int()
        _check(load().dcg_recycle_get_W(self.handle, None, ctypes.byref(k)), "dcg_recycle_get_W")
        out = torch.empty((k.value, self.n), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize()
        if k.value:
            _check(load().dcg_recycle_get_W(self.handle, out.data_ptr(), ctypes.byref(k)),
                   "dcg_recycle_get_W")
        return out.t()

    def get_AW(self):
        """AW for the operator of the last solve (n x k_used)."""
        torch = _torch()
        k = ctypes.c_int()
        _check(load().dcg_recycle_get_W(self.handle, None, ctypes.byref(k)), "dcg_recycle_get_W")
        out = torch.empty((k.value, self.n), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize()
        if k.value:
            _check(load().dcg_recycle_get_AW(self.handle, out.data_ptr()), "dcg_recycle_get_AW")
        return out.t()

    def theta(self):
        buf = (ctypes.c_double * max(1, self.k))()
        cnt = ctypes.c_int()
        _check(load().dcg_recycle_get_theta(self.handle, buf, ctypes.byref(cnt)),
               "dcg_recycle_get_theta")
        return [buf[i] for i in range(cnt.value)]

    def close(self):
        if getattr(self, "handle", None) is not None:
            load().dcg_recycle_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SolveWorkspace:
    def __init__(self, n, device="cuda"):
        nbytes = load().dcg_solve_workspace_bytes(int(n), 0, 0)
        self._ws, self.ptr, self.size = _workspace(nbytes, device)


def _refresh_mode(mode):
    modes = {False: 0, None: 0, 0: 0, "first": 0, True: 1, 1: 1, "every": 1, 2: 2, "accum": 2}
    if mode not in modes:
        raise ValueError(f"refresh_every must be 'first', 'every' or 'accum', not {mode!r}")
    return modes[mode]


def _refine_mode(refine):
    if refine in (False, None, 0):
        return 0
    if refine in (True, 1, "ir"):
        return 1
    if refine in (2, "fcg"):
        return 2
    raise ValueError(f"refine must be False, True/'ir' or 'fcg', not {refine!r}")


def _ritz_route(route):
    if route in ("auto", 0):
        return 0
    if route in ("eigen", 1):
        return 1
    raise ValueError(f"ritz_route must be 'auto' or 'eigen', not {route!r}")


def _extraction(kind):
    if kind in ("harmonic", 0):
        return 0
    if kind in ("rayleigh", 1):
        return 1
    if kind in ("implicit", 2):
        return 2
    raise ValueError(f"extraction must be 'harmonic', 'rayleigh' or 'implicit', not {kind!r}")


def solve(op, b, x0=None, rc=None, tol=1e-6, max_iter=0, L=0, select_largest=True,
          check_every=8, refine=False, inner_tol=1e-4, refine_max=20, use_graph=True,
          true_residual=False, profile=False, refresh_every=False, ritz_route="auto",
          extraction="harmonic", ws=None, out=None):
    """Deflated CG (Algorithm 1) for A x = b; returns (x, stats dict).

    rc=None runs plain CG; with a Recycle the solve uses its W and leaves the
    next W' (harmonic Ritz vectors, Eq. 7) in it.  refine=True (or "ir") runs
    iterative refinement to ``tol`` against the FP64 operator, refine="fcg"
    flexible CG in FP64 with the inner deflated solve as preconditioner.
    ritz_route="eigen" reduces F in the harmonic Ritz problem by its
    eigendecomposition even where the Cholesky reduction is safe;
    extraction="rayleigh" extracts the next W by Rayleigh-Ritz instead.
    """
    torch = _torch()
    lib = load()
    b = b.to(device=op.device, dtype=torch.float64).contiguous()
    if out is None:
        out = torch.empty_like(b)
    x_given = 0
    if x0 is not None:
        out.copy_(x0)
        x_given = 1
    if ws is None:
        ws = SolveWorkspace(op.n, op.device)
    p = Params(tol=float(tol), max_iter=int(max_iter), L=int(L),
               select_largest=1 if select_largest else 0, check_every=int(check_every),
               refine=_refine_mode(refine), inner_tol=float(inner_tol), refine_max=int(refine_max),
               use_graph=1 if use_graph else 0, true_residual=1 if true_residual else 0,
               profile=1 if profile else 0, refresh_every=_refresh_mode(refresh_every),
               ritz_route=_ritz_route(ritz_route), extraction=_extraction(extraction))
    st = Stats()
    with _ordered(op.stream):
        status = lib.dcg_solve(op.handle, b.data_ptr(), out.data_ptr(), x_given,
                               rc.handle if rc is not None else None, ctypes.byref(p),
                               ctypes.byref(st), ws.ptr, ws.size)
    _check(status, "dcg_solve")
    return out, st.as_dict()


def version():
    return load().dcg_version().decode()


def slq_logdet(op, Z, tol=1e-6, max_iter=0, max_steps=1024, check_every=8):
    """log det A by stochastic Lanczos quadrature: one block CG solve over the
    probe columns of Z (n x P, P <= 64), each column's Lanczos tridiagonal
    from its CG coefficients.  Returns (estimate, per-probe values, steps)."""
    torch = _torch()
    lib = load()
    Zc = _colmajor(Z.to(device=op.device, dtype=torch.float64))
    P = Zc.shape[0]
    nbytes = lib.dcg_slq_logdet_workspace_bytes(op.n, P, int(max_steps))
    if nbytes == 0:
        raise DcgError(-1, "dcg_slq_logdet_workspace_bytes")
    ws, ptr, size = _workspace(nbytes, op.device)
    p = Params(tol=float(tol), max_iter=int(max_iter), check_every=int(check_every))
    quad = (ctypes.c_double * P)()
    steps = (ctypes.c_int * P)()
    est = ctypes.c_double()
    with _ordered(op.stream):
        status = lib.dcg_slq_logdet(op.handle, Zc.data_ptr(), P, ctypes.byref(p), int(max_steps),
                                    quad, steps, ctypes.byref(est), ptr, size)
    _check(status, "dcg_slq_logdet")
    del ws
    return est.value, list(quad), list(steps)


def laplace_evidence(op, y, f, a, Z, tol=1e-8, max_steps=2048, check_every=8):
    """Laplace log evidence Psi(f) - 1/2 log det(I + D K D) at the mode (f, a)
    with the determinant by SLQ over the probe columns of Z (FP64 or stored
    operator).  Returns (evidence, psi, logdet)."""
    torch = _torch()
    lib = load()
    y = y.to(device=op.device, dtype=torch.float64).contiguous()
    f = f.to(device=op.device, dtype=torch.float64).contiguous()
    a = a.to(device=op.device, dtype=torch.float64).contiguous()
    Zc = _colmajor(Z.to(device=op.device, dtype=torch.float64))
    P = Zc.shape[0]
    nbytes = lib.dcg_laplace_evidence_workspace_bytes(op.n, P, int(max_steps))
    if nbytes == 0:
        raise DcgError(-1, "dcg_laplace_evidence_workspace_bytes")
    ws, ptr, size = _workspace(nbytes, op.device)
    p = Params(tol=float(tol), check_every=int(check_every))
    ev, ps, ld = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    with _ordered(op.stream):
        status = lib.dcg_laplace_evidence(op.handle, y.data_ptr(), f.data_ptr(), a.data_ptr(),
                                          Zc.data_ptr(), P, ctypes.byref(p), int(max_steps),
                                          ctypes.byref(ev), ctypes.byref(ps), ctypes.byref(ld),
                                          ptr, size)
    _check(status, "dcg_laplace_evidence")
    del ws
    return ev.value, ps.value, ld.value


def laplace_gpc(op, y, rc=None, max_newton=50, psi_tol=1.0, tol=1e-5, max_iter=0, L=0,
                select_largest=True, check_every=8, refine=False, inner_tol=1e-4,
                refine_max=20, use_graph=True, ritz_route="auto", extraction="harmonic",
                profile=False):
    """Laplace GPC mode by Newton's method (section 3, Eqs. 8-10), each
    system A = I + D K D solved by deflated CG with W carried over through
    ``rc``.  y: (n,) labels in {-1, +1}.  With profile, each solve's stats
    hold the device time of its CG steps' sweeps (HIP events around each
    sweep launch).  Returns (f, a, psi list, list of per-solve stats dicts,
    status)."""
    torch = _torch()
    lib = load()
    y = y.to(device=op.device, dtype=torch.float64).contiguous()
    f = torch.empty(op.n, dtype=torch.float64, device=op.device)
    a = torch.empty_like(f)
    nbytes = lib.dcg_laplace_gpc_workspace_bytes(op.n)
    ws, ptr, size = _workspace(nbytes, op.device)
    p = Params(tol=float(tol), max_iter=int(max_iter), L=int(L),
               select_largest=1 if select_largest else 0, check_every=int(check_every),
               refine=_refine_mode(refine), inner_tol=float(inner_tol), refine_max=int(refine_max),
               use_graph=1 if use_graph else 0, true_residual=0, profile=1 if profile else 0,
               refresh_every=0, ritz_route=_ritz_route(ritz_route),
               extraction=_extraction(extraction))
    psi = (ctypes.c_double * (max_newton + 1))()
    stats = (Stats * max_newton)()
    steps = ctypes.c_int()
    with _ordered(op.stream):
        status = lib.dcg_laplace_gpc(op.handle, y.data_ptr(), rc.handle if rc is not None else None,
                                     ctypes.byref(p), int(max_newton), float(psi_tol),
                                     f.data_ptr(), a.data_ptr(), psi, ctypes.byref(steps), stats,
                                     ptr, size)
    _check(status, "dcg_laplace_gpc")
    del ws
    k = steps.value
    return f, a, list(psi[:k + 1]), [stats[i].as_dict() for i in range(k)], status


def solve_block(op, B, rc=None, tol=1e-6, max_iter=0, check_every=8, out=None):
    """X = A^{-1} B for the columns of B (n x m, m <= 64), each by deflated CG
    with the basis W of rc (reused, not refreshed); returns (X, stats)."""
    torch = _torch()
    lib = load()
    Bc = _colmajor(B.to(op.device))
    m = Bc.shape[0]
    X = torch.empty_like(Bc)
    nbytes = lib.dcg_solve_block_workspace_bytes(op.n, m)
    if nbytes == 0:
        raise DcgError(-1, "dcg_solve_block_workspace_bytes")
    _wsbuf, ptr, size = _workspace(nbytes, op.device)
    p = Params(tol=float(tol), max_iter=int(max_iter), check_every=int(check_every))
    st = Stats()
    with _ordered(op.stream):
        status = lib.dcg_solve_block(op.handle, Bc.data_ptr(), X.data_ptr(), m,
                                     rc.handle if rc is not None else None, ctypes.byref(p),
                                     ctypes.byref(st), ptr, size)
    _check(status, "dcg_solve_block")
    torch.cuda.current_stream(op.device).synchronize()
    return X.t(), st.as_dict()


def solve_batched(ops, bs, rcs=None, x0s=None, tol=1e-6, max_iter=0, L=0, select_largest=True,
                  check_every=8, use_graph=True, true_residual=False, ritz_route="auto",
                  extraction="harmonic", ws=None):
    """Independent systems ops[s] x_s = bs[s], each by deflated CG with the
    basis of rcs[s] (or plain CG for a None entry) and the extraction of the
    next basis, iterated in lockstep.  The operators must share one stream.
    Returns (list of x, list of stats dicts)."""
    torch = _torch()
    lib = load()
    count = len(ops)
    if len(bs) != count or (rcs is not None and len(rcs) != count):
        raise ValueError("ops, bs and rcs must have the same length")
    dev = ops[0].device
    bs = [b.to(device=dev, dtype=torch.float64).contiguous() for b in bs]
    xs = [torch.empty_like(b) for b in bs]
    x_given = 0
    if x0s is not None:
        for x, x0 in zip(xs, x0s):
            x.copy_(x0)
        x_given = 1
    VP = ctypes.c_void_p * count
    h_ops = VP(*[op.handle for op in ops])
    h_b = VP(*[b.data_ptr() for b in bs])
    h_x = VP(*[x.data_ptr() for x in xs])
    h_rc = VP(*[(rc.handle if rc is not None else None) for rc in (rcs or [None] * count)])
    ns = (ctypes.c_int64 * count)(*[op.n for op in ops])
    if ws is None:
        nbytes = lib.dcg_solve_batched_workspace_bytes(count, ns)
        if nbytes == 0:
            raise DcgError(-1, "dcg_solve_batched_workspace_bytes")
        _wsbuf, ptr, size = _workspace(nbytes, dev)
    else:
        _wsbuf, ptr, size = ws
    p = Params(tol=float(tol), max_iter=int(max_iter), L=int(L),
               select_largest=1 if select_largest else 0, check_every=int(check_every),
               use_graph=1 if use_graph else 0, true_residual=1 if true_residual else 0,
               ritz_route=_ritz_route(ritz_route), extraction=_extraction(extraction))
    st = (Stats * count)()
    with _ordered(ops[0].stream):
        status = lib.dcg_solve_batched(count, h_ops, h_b, h_x, x_given, h_rc, ctypes.byref(p),
                                       st, ptr, size)
    _check(status, "dcg_solve_batched")
    return xs, [s.as_dict() for s in st]


def mll_grad(op, alpha, U, Z):
    """Gradient of the GP log marginal likelihood w.r.t. (log ell, log s2,
    log sigma2) from alpha = A^{-1} y, probes Z (n x P) and U = A^{-1} Z."""
    torch = _torch()
    lib = load()
    a = alpha.to(device=op.device, dtype=torch.float64).contiguous()
    Uc = _colmajor(U.to(op.device))
    Zc = _colmajor(Z.to(op.device))
    nbytes = lib.dcg_mll_grad_workspace_bytes(op.n)
    _wsbuf, ptr, size = _workspace(nbytes, op.device)
    g = (ctypes.c_double * 3)()
    with _ordered(op.stream):
        _check(lib.dcg_mll_grad(op.handle, a.data_ptr(), Uc.data_ptr(), Zc.data_ptr(),
                                Uc.shape[0], g, ptr, size), "dcg_mll_grad")
    return [g[0], g[1], g[2]]


def mll_value(op, y, alpha, logdet=None):
    """-1/2 y^T alpha - n/2 log(2 pi) [- 1/2 logdet]: the GP log marginal
    likelihood from alpha = A^{-1} y (the sum is taken by the library)."""
    torch = _torch()
    lib = load()
    y = y.to(device=op.device, dtype=torch.float64).contiguous()
    a = alpha.to(device=op.device, dtype=torch.float64).contiguous()
    out = ctypes.c_double()
    ld = None if logdet is None else ctypes.byref(ctypes.c_double(float(logdet)))
    with _ordered(op.stream):
        _check(lib.dcg_mll_value(op.handle, y.data_ptr(), a.data_ptr(), ld, ctypes.byref(out)),
               "dcg_mll_value")
    return out.value


def extract_basis(Z, AZ, k, largest=True, extraction="harmonic", ritz_route="auto"):
    """The extraction of the next basis (section 2.3: harmonic Ritz, Eq. 7, or
    Rayleigh-Ritz) on given Z and AZ (n x m device tensors): returns (W' = Z U
    as an n x k_out tensor, the kept Ritz values, the number of directions of
    the metric kept).  Runs on the caller's current stream."""
    torch = _torch()
    lib = load()
    dev = Z.device
    n, m = Z.shape
    Zc = _colmajor(Z)
    AZc = _colmajor(AZ.to(dev))
    nbytes = lib.dcg_extract_basis_workspace_bytes(n, m)
    if nbytes == 0:
        raise DcgError(-1, "dcg_extract_basis_workspace_bytes")
    _wsbuf, ptr, size = _workspace(nbytes, dev)
    W = torch.zeros((k, n), dtype=torch.float64, device=dev)
    th = (ctypes.c_double * k)()
    kout, rank = ctypes.c_int(0), ctypes.c_int(0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    _check(lib.dcg_extract_basis(Zc.data_ptr(), AZc.data_ptr(), n, m, int(k), 1 if largest else 0,
                                 _extraction(extraction), _ritz_route(ritz_route), W.data_ptr(),
                                 th, ctypes.byref(kout), ctypes.byref(rank), stream, ptr, size),
           "dcg_extract_basis")
    kk = kout.value
    return W[:kk].t(), [th[i] for i in range(kk)], rank.value


def extract_basis_noalloc(Z, AZ, W_out, largest=True, extraction="harmonic", ritz_route="auto"):
    """extract_basis without any device allocation in the library: the
    scratch is the library's own device array of the current device.  W_out
    is a caller-given (k, n) FP64 tensor on Z's device (k <= 64) whose first
    k_out rows receive the columns of W' = Z U.  Returns (k_out, the kept Ritz
    values, the number of directions of the metric kept).  Runs on the
    caller's current stream; calls that overlap on one device race."""
    torch = _torch()
    lib = load()
    dev = Z.device
    n, m = Z.shape
    k = W_out.shape[0]
    if W_out.shape[1] != n or W_out.dtype != torch.float64 or not W_out.is_contiguous() \
            or W_out.device != dev:
        raise ValueError("W_out must be a contiguous (k, n) float64 tensor on Z's device")
    Zc = _colmajor(Z)
    AZc = _colmajor(AZ.to(dev))
    th = (ctypes.c_double * k)()
    kout, rank = ctypes.c_int(0), ctypes.c_int(0)
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev).cuda_stream
        _check(lib.dcg_extract_basis_noalloc(Zc.data_ptr(), AZc.data_ptr(), n, m, int(k),
                                             1 if largest else 0, _extraction(extraction),
                                             _ritz_route(ritz_route), W_out.data_ptr(), th,
                                             ctypes.byref(kout), ctypes.byref(rank), stream),
               "dcg_extract_basis_noalloc")
    kk = kout.value
    return kk, [th[i] for i in range(kk)], rank.value


class GPMarginalLikelihood:
    """torch.autograd.Function for the GP log marginal likelihood in
    theta = (log ell, log s2, log sigma2).

    forward: alpha = A^{-1} y by deflated CG with the recycled basis of `rc`
    (refreshed by every solve), value = -1/2 y^T alpha - n/2 log(2 pi)
    assembled by the library (dcg_mll_value); with
    ``GPContext(logdet=True)`` also -1/2 log|A| estimated by stochastic
    Lanczos quadrature over the context's probes (one more block solve,
    plain CG, since the quadrature needs the probes' own Krylov spaces).
    backward: the probe solves U = A^{-1} Z reuse the same recycled W (the
    adjoint of the symmetric solve is the same solve), then one fused sweep
    gives the full gradient, log-determinant term included (Hutchinson).
    The backward sets the operator back to the forward's hyperparameters
    when another forward has changed them in between.

    Use through ``GPMarginalLikelihood.apply(theta, ctx_obj)`` where ctx_obj
    is a ``GPContext`` holding the operator, y, the recycle handle and the
    probes of the current step.
    """

    _fn = None

    @classmethod
    def apply(cls, theta, gpc):
        if cls._fn is None:
            cls._fn = _make_mll_function()
        return cls._fn.apply(theta, gpc)


class GPContext:
    def __init__(self, op, y, rc, probes, tol=1e-6, probe_tol=None, logdet=False):
        self.op, self.y, self.rc, self.probes = op, y, rc, probes
        self.tol = tol
        self.logdet = bool(logdet)
        self.probe_tol = tol if probe_tol is None else probe_tol
        self.last = {}


def _make_mll_function():
    import math
    torch = _torch()

    class _MLL(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, gpc):
            th = theta.detach().double().cpu().tolist()
            op = gpc.op
            hyper = (math.exp(th[0]), math.exp(th[1]), math.exp(th[2]))
            op.set_hyper(*hyper)
            alpha, st = solve(op, gpc.y, rc=gpc.rc, tol=gpc.tol)
            alpha = alpha.clone()
            gpc.last = {"alpha_stats": st}
            ctx.gpc = gpc
            ctx.alpha = alpha
            # the hyperparameters of this forward: the backward runs its probe
            # solves and derivative sweep at them, whatever the operator holds
            # by then (another forward may have moved it, e.g. a line search)
            ctx.hyper = hyper
            logdet = None
            if gpc.logdet:
                logdet, quad, steps = slq_logdet(op, gpc.probes, tol=gpc.probe_tol)
                gpc.last["logdet"] = logdet
                gpc.last["logdet_steps"] = steps
            value = mll_value(op, gpc.y, alpha, logdet)
            return theta.new_tensor(value)

        @staticmethod
        def backward(ctx, grad_out):
            gpc = ctx.gpc
            if (gpc.op.ell, gpc.op.s2, gpc.op.sigma2) != ctx.hyper:
                gpc.op.set_hyper(*ctx.hyper)
            U, st = solve_block(gpc.op, gpc.probes, rc=gpc.rc, tol=gpc.probe_tol)
            gpc.last["probe_stats"] = st
            g = mll_grad(gpc.op, ctx.alpha, U, gpc.probes)
            gpc.last["grad"] = g
            return grad_out * grad_out.new_tensor(g), None

    return _MLL
