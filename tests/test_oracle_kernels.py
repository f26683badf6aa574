"""Pins of the oracle's covariance functions and rounding (CPU only).

Each check compares the oracle with something other than itself: brute-force
loops, closed-form values of the kernels, an independent library
implementation (scikit-learn's RBF / Matern kernels, scipy's cdist), finite
differences, or hand-derived rounding cases.
"""

import numpy as np
import pytest
import scipy.spatial.distance as ssd
from sklearn.gaussian_process import kernels as skk

from oracle import kernels as K
from oracle import precision as P

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def test_sqdist_brute_force():
    g = np.random.default_rng(0)
    X = g.standard_normal((7, 3))
    D = K.sqdist(X)
    for i in range(7):
        for j in range(7):
            s = 0.0
            for t in range(3):
                s += (X[i, t] - X[j, t]) ** 2
            assert abs(D[i, j] - s) <= 1e-14 * max(1.0, s)
    assert np.all(np.diag(D) == 0.0)
    Y = g.standard_normal((5, 3))
    np.testing.assert_allclose(K.sqdist(X, Y), ssd.cdist(X, Y, "sqeuclidean"),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("ell,s2", [(1.0, 1.0), (0.7, 2.5), (3.3, 0.4)])
def test_kernel_closed_forms(ell, s2):
    # r = 0 gives the signal variance for every kernel
    for kern in (K.RBF, K.MATERN32, K.MATERN52):
        assert K.kernel_from_r2(0.0, kern, ell, s2) == pytest.approx(s2, rel=1e-15)
    e = np.exp(-1.0)
    # RBF at r^2 = 2 ell^2: s2 e^-1
    assert K.kernel_from_r2(2 * ell * ell, K.RBF, ell, s2) == pytest.approx(s2 * e, rel=1e-14)
    # Matern-3/2 at r = ell/sqrt3: t = 1 -> s2 (1 + 1) e^-1
    assert K.kernel_from_r2(ell * ell / 3, K.MATERN32, ell, s2) == pytest.approx(2 * s2 * e, rel=1e-14)
    # Matern-5/2 at r = ell/sqrt5: t = 1 -> s2 (1 + 1 + 1/3) e^-1
    assert K.kernel_from_r2(ell * ell / 5, K.MATERN52, ell, s2) == pytest.approx(7 / 3 * s2 * e, rel=1e-14)


@pytest.mark.parametrize("kern,sk", [
    (K.RBF, lambda ell: skk.RBF(length_scale=ell)),
    (K.MATERN32, lambda ell: skk.Matern(length_scale=ell, nu=1.5)),
    (K.MATERN52, lambda ell: skk.Matern(length_scale=ell, nu=2.5)),
])
def test_gram_matches_sklearn(kern, sk):
    g = np.random.default_rng(1)
    X = g.standard_normal((40, 5))
    ell, s2 = 1.7, 1.3
    ref = s2 * sk(ell)(X)
    np.testing.assert_allclose(K.gram(X, kern, ell, s2), ref, rtol=1e-12, atol=1e-14)


def test_operator_spd_and_blocked_matvec():
    g = np.random.default_rng(2)
    X = g.standard_normal((300, 4))
    A = K.operator(X, K.MATERN52, 1.1, 1.0, 1e-3)
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0.9e-3
    V = g.standard_normal((300, 3))
    np.testing.assert_allclose(K.matvec_blocked(X, K.MATERN52, 1.1, 1.0, 1e-3, V, block=37),
                               A @ V, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kern", [K.RBF, K.MATERN32, K.MATERN52])
def test_dgram_dlog_ell_finite_difference(kern):
    g = np.random.default_rng(3)
    X = g.standard_normal((30, 3))
    ell, s2, h = 1.4, 0.8, 1e-5
    fd = (K.gram(X, kern, ell * np.exp(h), s2) - K.gram(X, kern, ell * np.exp(-h), s2)) / (2 * h)
    np.testing.assert_allclose(K.dgram_dlog_ell(X, kern, ell, s2), fd, rtol=1e-7, atol=1e-9)


def test_round_bf16_hand_cases():
    u = 2.0 ** -7                     # bf16 spacing just above 1
    cases = [
        (1.0, 1.0),
        (1.0 + u / 2, 1.0),                     # tie -> even (1.0)
        (1.0 + 3 * u / 2, 1.0 + 2 * u),         # tie -> even (mantissa ...010)
        (1.0 + u / 2 + 2.0 ** -30, 1.0 + u),    # just above the tie: single rounding rounds up
        (-(1.0 + u / 2 + 2.0 ** -30), -(1.0 + u)),
        (3.14159265358979, 3.140625),
        (255.5, 256.0),
        (0.1, 0.10009765625),
        (1e-3, 0.00099945068359375),
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert P.round_bf16(np.array([x]))[0] == want, x


def test_round_bf16_matches_torch_on_fp32_values():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(4)
    x = g.uniform(-4, 4, 20000).astype(np.float32).astype(np.float64)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(P.round_bf16(x), ref)


def test_round_bf16x2():
    g = np.random.default_rng(6)
    x = g.uniform(-3, 3, 5000)
    y = P.round_bf16x2(x)
    # 16 significant bits: relative error below 2^-16
    assert np.all(np.abs(y - x) <= 2.0 ** -16 * np.abs(x))
    # both parts are bf16 values, and values with 16 significant bits are kept
    hi = P.round_bf16(x)
    assert np.array_equal(P.round_bf16(y - hi), y - hi)
    exact = np.ldexp(np.round(np.ldexp(x, 13)), -13)[np.abs(x) >= 0.5]
    exact = exact[np.abs(exact) < 4]
    np.testing.assert_array_equal(P.round_bf16x2(exact), exact)
    c = P.point_scale(P.RBF, 1.0)
    assert P.round_points(np.array([[0.1]]), P.PREC_BF16X2, P.RBF, 1.0)[0, 0] == \
        P.round_bf16x2(np.array([0.1 * c]))[0] / c


def test_round_fp32():
    assert P.round_fp32(np.array([0.1]))[0] == float(np.float32(0.1))
    assert P.round_points(np.array([[0.1]]), P.PREC_FP64, P.MATERN52, 0.3)[0, 0] == 0.1


def test_point_scale_gives_base2_forms_of_the_kernels():
    """With u = c r, c = point_scale(kernel, ell), the forms the low-precision
    product evaluates equal the textbook kernels: RBF 2^-(u^2), Matern-3/2
    (1 + ln2 u) 2^-u, Matern-5/2 (1 + ln2 u + ln2^2 u^2 / 3) 2^-u."""
    assert (P.RBF, P.MATERN32, P.MATERN52) == (K.RBF, K.MATERN32, K.MATERN52)
    assert P.LOG2E == np.log2(np.e)
    r = np.linspace(0.0, 6.0, 241)
    ln2 = np.log(2.0)
    for ell in (0.3, 1.0, 2.2937):
        u = P.point_scale(K.RBF, ell) * r
        np.testing.assert_allclose(2.0 ** -(u * u), K.kernel_from_r2(r * r, K.RBF, ell, 1.0),
                                   rtol=1e-13)
        u = P.point_scale(K.MATERN32, ell) * r
        np.testing.assert_allclose((1 + ln2 * u) * 2.0 ** -u,
                                   K.kernel_from_r2(r * r, K.MATERN32, ell, 1.0), rtol=1e-13)
        u = P.point_scale(K.MATERN52, ell) * r
        np.testing.assert_allclose((1 + ln2 * u + ln2 * ln2 * u * u / 3) * 2.0 ** -u,
                                   K.kernel_from_r2(r * r, K.MATERN52, ell, 1.0), rtol=1e-13)
    # the represented points: the scaled points' rounding, scaled back
    X = np.random.default_rng(9).uniform(-1, 1, (50, 4))
    for prec, rnd in ((P.PREC_FP32, P.round_fp32), (P.PREC_BF16, P.round_bf16)):
        c = P.point_scale(K.MATERN52, 0.8)
        Xr = P.round_points(X, prec, K.MATERN52, 0.8)
        np.testing.assert_allclose(Xr * c, rnd(c * X), rtol=2e-16, atol=0)
        assert np.abs(Xr - X).max() > 0


def test_sqdist_gemm_matches_difference_form():
    g = np.random.default_rng(44)
    X = 3.0 * g.standard_normal((200, 7))
    Y = g.uniform(-2, 2, (150, 7))
    ref = K.sqdist(X, Y)
    got = K.sqdist_gemm(X, Y)
    scale = np.sum(X * X, 1)[:, None] + np.sum(Y * Y, 1)[None, :]
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    # identical points: exactly zero after the clip, never negative
    Z = K.sqdist_gemm(X, X)
    assert np.all(Z >= 0.0)
    assert np.all(np.diag(Z) <= 1e-13 * 2.0 * np.sum(X * X, 1))


def test_fp32_values_are_three_exact_bf16_terms():
    """The FP32 operator's operands carry each FP32 coordinate as h + m + l
    with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m): the sum is x
    exactly, across magnitudes; |m| <= 2^-8 |x| and |l| <= 2^-17 |x|, so each
    dropped product m.l is at most 2^-25 |x|^2."""
    g = np.random.default_rng(12)
    x = np.concatenate([g.standard_normal(200_000) * s for s in (1e-3, 1.0, 7.0, 1e3)]
                       + [np.ldexp(g.uniform(1, 2, 100_000), g.integers(-90, 90, 100_000))])
    x = P.round_fp32(x)
    h = P.round_bf16(x)
    m = P.round_bf16(x - h)
    l = P.round_bf16(x - h - m)
    np.testing.assert_array_equal(h + m + l, x)
    assert np.all(np.abs(m) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(l) <= 2.0 ** -17 * np.abs(x))
    assert np.all(np.abs(m * l) <= 2.0 ** -25 * x * x)


def test_round_fp16_matches_python_half_packing():
    """binary16 rounding against Python's own half-precision packing (struct
    format 'e', round half to even from the double), over normal and
    subnormal magnitudes, exact ties and the largest finite value."""
    import struct
    g = np.random.default_rng(21)
    x = np.concatenate([g.standard_normal(20000) * s for s in (1e-6, 1e-3, 1.0, 30.0, 3000.0)]
                       + [np.ldexp(np.arange(1, 2049, dtype=np.float64) + 0.5, -11),   # ties
                          np.ldexp(np.arange(0, 1024, dtype=np.float64) + 0.5, -24),   # subnormal ties
                          np.array([65504.0, -65504.0, 2.0 ** -14, 2.0 ** -24, 0.0])])
    ref = np.array([struct.unpack("<e", struct.pack("<e", v))[0] for v in x])
    np.testing.assert_array_equal(P.round_fp16(x), ref)
    with pytest.raises(ValueError):
        P.round_fp16(np.array([65520.0]))
    c = P.point_scale(P.MATERN52, 0.7)
    np.testing.assert_allclose(P.round_points(np.array([[0.3]]), P.PREC_FP16, P.MATERN52, 0.7) * c,
                               P.round_fp16(np.array([[0.3 * c]])), rtol=2e-16)
