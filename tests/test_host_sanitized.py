"""The library's host-only arithmetic (paper_1706_00241_amd/csrc/host.cpp:
operand geometry, the work plans of the pair sweeps and their partial-sum
sizes, the tridiagonal eigenproblems and quadratures of stochastic Lanczos
quadrature) built with the host compiler under AddressSanitizer and
UndefinedBehaviorSanitizer, every finding fatal.  The driver
(tests/host/host_checks.cpp) checks the plan and geometry rules itself; the
eigenvalues and quadratures it prints are compared here with numpy's dense
eigensolver and with the exact z^T log(A) z that an n-step quadrature of an
n x n matrix gives (Gauss quadrature with as many nodes as the spectrum has
points is exact; Golub & Meurant)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import cg as OC

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    rocm_inc = "/opt/rocm/include"
    if gxx is None or not os.path.isdir(rocm_inc):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path_factory.mktemp("host") / "host_checks")
    cmd = [gxx, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-I", rocm_inc, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "host_checks.cpp"),
           os.path.join(ROOT, "paper_1706_00241_amd", "csrc", "host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, text):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout.splitlines()


def test_plans_and_geometry(driver):
    out = _run(driver, "plans\ngeometry\nwide\n")
    assert out[0].startswith("plans ok ") and int(out[0].split()[2]) > 300
    assert out[1].startswith("geometry ok ") and int(out[1].split()[2]) == 6 * 64 * 6
    assert out[2].startswith("wide ok ") and int(out[2].split()[2]) > 100


def _tridiag_cases():
    g = np.random.default_rng(7)
    cases = [(np.array([2.5]), np.array([]))]
    for m in (2, 3, 10, 57, 300):
        cases.append((g.standard_normal(m), g.standard_normal(m - 1)))
    d = g.standard_normal(40)
    e = g.standard_normal(39)
    e[[5, 6, 20]] = 0.0                            # splits into blocks
    cases.append((d, e))
    cases.append((np.full(30, 1.5), np.full(29, 1e-9)))      # near-repeated eigenvalues
    cases.append((np.logspace(-8, 8, 25), np.logspace(-8, 7, 24) * 0.1))   # graded
    cases.append((np.zeros(6), np.zeros(5)))        # already diagonal
    return cases


def test_tridiagonal_eigenproblems(driver):
    cases = _tridiag_cases()
    text = ""
    for d, e in cases:
        text += "tridiag %d %s %s\n" % (len(d), " ".join(repr(float(v)) for v in d),
                                        " ".join(repr(float(v)) for v in e))
    out = _run(driver, text)
    assert len(out) == len(cases)
    for (d, e), line in zip(cases, out):
        f = line.split()
        m = len(d)
        assert f[0] == "tridiag" and f[1] == "1"
        lam = np.array([float(v) for v in f[2:2 + m]])
        q = np.array([float(v) for v in f[2 + m:2 + 2 * m]])
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        ref, V = np.linalg.eigh(T)
        scale = max(np.max(np.abs(ref)), 1e-300)
        np.testing.assert_allclose(np.sort(lam), ref, atol=1e-12 * scale, rtol=0)
        # first components: the weights of e_1 on the eigenvectors sum to 1, and
        # the weight of each cluster of equal eigenvalues matches numpy's
        assert abs(np.sum(q * q) - 1.0) <= 1e-12
        order = np.argsort(lam)
        ls, ws = lam[order], (q * q)[order]
        wr = V[0] ** 2
        start = 0
        for i in range(1, m + 1):
            if i == m or ref[i] - ref[i - 1] > 1e-6 * scale:
                assert abs(np.sum(ws[start:i]) - np.sum(wr[start:i])) <= 1e-9, (start, i)
                start = i


def test_slq_quadrature_exact_on_full_krylov(driver):
    """m = n CG steps on an n x n SPD matrix: the quadrature equals
    z^T log(A) z (to 1e-9 relative); a non-positive alpha is DCG_E_NOT_SPD."""
    g = np.random.default_rng(3)
    lines, refs = [], []
    for n in (1, 5, 24):
        Q, _ = np.linalg.qr(g.standard_normal((n, n)))
        lam = np.exp(g.uniform(-2.0, 3.0, n))
        A = (Q * lam) @ Q.T
        z = g.choice([-1.0, 1.0], n)
        res = OC.cg(A, z, tol=1e-15, L=n, max_iter=n)
        a, b = res.alpha[:n], res.beta[:n - 1]
        m = len(a)
        lines.append("slq %d %r %s %s" % (m, float(z @ z), " ".join(repr(float(v)) for v in a),
                                          " ".join(repr(float(v)) for v in b)))
        w = Q.T @ z
        refs.append((m == n, float(np.sum(w * w * np.log(lam)))))
    assert sum(e for e, _ in refs) >= 2
    lines.append("slq 3 1.0 1.0 -2.0 1.0 0.5 0.5")
    out = _run(driver, "\n".join(lines) + "\n")
    for (exact, ref), line in zip(refs, out):
        f = line.split()
        assert f[0] == "slq" and f[1] == "0"
        if exact:
            assert abs(float(f[2]) - ref) <= 1e-9 * max(1.0, abs(ref)), (float(f[2]), ref)
    assert out[-1].split()[1] == "-2"
