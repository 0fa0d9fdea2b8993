"""Pins for the oracle's filters against brute force, closed forms, library
routines and the paper's printed results. None of these compares the oracle
with itself: each expected value comes from a different route."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import coeffs as K
from oracle import filters as F
from oracle import native as C
from synth import checkerboard, edge_rich, ramp_rectangles


def _scipy_gauss(f, sigma_s):
    """Normalised truncated Gaussian via scipy, half-sample mirror."""
    g = F.spatial_kernel_1d(sigma_s)
    g = g / g.sum()
    out = ndimage.correlate1d(f, g, axis=0, mode="reflect")
    return ndimage.correlate1d(out, g, axis=1, mode="reflect")


def _brute_direct(f, sigma_s, sigma_r):
    """Eq. (1) with explicit loops and numpy.pad's symmetric extension."""
    H, Wd = f.shape
    W = F.radius(sigma_s)
    fp = np.pad(f, W, mode="symmetric")
    out = np.empty_like(f)
    for r in range(H):
        for c in range(Wd):
            num = den = 0.0
            for j1 in range(-W, W + 1):
                for j2 in range(-W, W + 1):
                    t = fp[r - j1 + W, c - j2 + W]
                    w = math.exp(-(j1 * j1 + j2 * j2) / (2 * sigma_s ** 2)) * \
                        math.exp(-(t - f[r, c]) ** 2 / (2 * sigma_r ** 2))
                    num += w * t
                    den += w
            out[r, c] = num / den
    return out


def test_mirror_matches_numpy_symmetric_pad():
    for M in (1, 2, 5, 8):
        line = np.arange(M)
        for pad in (M - 1, M, 2 * M + 3):
            ref = np.pad(line, pad, mode="symmetric")
            got = line[F.mirror_index(np.arange(-pad, M + pad), M)]
            np.testing.assert_array_equal(got, ref)


def test_radius():
    assert F.radius(3.0) == 9 and F.radius(10.0) == 30 and F.radius(5.0) == 15
    assert F.radius(2.1) == 7 and F.radius(0.2) == 1


def test_direct_matches_bruteforce_and_c():
    f = ramp_rectangles(9, 7, seed=3)
    ref = _brute_direct(f, 1.5, 20.0)
    np.testing.assert_allclose(F.direct_bf(f, 1.5, 20.0), ref, rtol=0, atol=1e-11)
    np.testing.assert_allclose(C.direct_bf(f, 1.5, 20.0), ref, rtol=0, atol=1e-11)


def test_direct_region_equals_crop():
    f = ramp_rectangles(40, 33, seed=4)
    full = C.direct_bf(f, 2.0, 30.0)
    crop = F.direct_bf(f, 2.0, 30.0, region=(5, 30, 0, 17))
    np.testing.assert_allclose(crop, full[5:30, 0:17], rtol=0, atol=1e-11)


def test_direct_constant_image():
    f = np.full((13, 10), 77.25)
    np.testing.assert_allclose(F.direct_bf(f, 2.0, 30.0), f, rtol=0, atol=1e-12)


def test_direct_large_sigma_r_is_gaussian():
    f = ramp_rectangles(31, 26, seed=5)
    np.testing.assert_allclose(C.direct_bf(f, 2.5, 1e7), _scipy_gauss(f, 2.5), rtol=0, atol=1e-7)


def test_direct_two_level_image_keeps_edges():
    """0/255 image, sigma_r = 30: the cross-edge weight is exp(-255^2/1800),
    below 1e-15, so the output equals the input to ~1e-12."""
    f = checkerboard(24, 20, cell=5)
    np.testing.assert_allclose(C.direct_bf(f, 3.0, 30.0), f, rtol=0, atol=1e-9)


@pytest.mark.parametrize("shape,sigma_s", [((17, 23), 2.0), ((6, 5), 3.0), ((1, 9), 1.3)])
def test_gauss_separable_equals_definition_and_scipy(shape, sigma_s):
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, size=shape)
    sep = F.gauss_filter_separable(X, sigma_s)
    two = F.gauss_filter_2d(X, sigma_s)
    np.testing.assert_allclose(sep, two, rtol=0, atol=1e-12)
    g = F.spatial_kernel_1d(sigma_s)
    np.testing.assert_allclose(two / g.sum() ** 2, _scipy_gauss(X, sigma_s), rtol=0, atol=1e-12)


def test_gauss_filter_is_symmetric_operator():
    """Half-sample mirroring makes the truncated filter a symmetric matrix:
    <G x, y> = <x, G y>, the property the adjoint relies on."""
    rng = np.random.default_rng(2)
    for shape, s in (((19, 11), 2.0), ((7, 9), 4.0)):
        x = rng.normal(size=shape)
        y = rng.normal(size=shape)
        lhs = np.sum(F.gauss_filter_separable(x, s) * y)
        rhs = np.sum(x * F.gauss_filter_separable(y, s))
        assert abs(lhs - rhs) < 1e-10 * (abs(lhs) + 1)


def test_gcf_constant_image():
    for val in (0.0, 40.0, 127.5, 255.0):
        f = np.full((12, 9), val)
        np.testing.assert_allclose(F.gcf(f, 2.0, 30.0, 28), f, rtol=0, atol=1e-9)


@pytest.mark.parametrize("shape,sigma_s,sigma_r,N", [
    ((14, 12), 1.5, 30.0, 28),
    ((10, 16), 2.0, 40.0, 16),
    ((9, 9), 1.0, 25.0, 40),
    ((12, 8), 1.2, 30.0, 10),
])
def test_gcf_stack_equals_pairwise(shape, sigma_s, sigma_r, N):
    """The exchange of sums in Section II (eqs. 5 -> 8, 9) is exact: the stack
    form equals the approximate kernel put straight into eq. (1)."""
    f = ramp_rectangles(*shape, seed=11)
    stack = F.gcf(f, sigma_s, sigma_r, N)
    pair = F.gcf_pairwise(f, sigma_s, sigma_r, N)
    # Both routes round in FP64; the series they sum has terms as large as
    # I_0(mu) ~ exp(mu), so their rounding grows like N * 2^-52 * I_0(mu)
    # relative to a kernel value of 1 (about 4e-12 at sigma_r = 30, 3e-5 at 25).
    _, mu = K.gcf_params(sigma_r)
    tol = max(1e-8, 255.0 * N * 2.0 ** -52 * math.exp(mu) * 10)
    np.testing.assert_allclose(stack, pair, rtol=0, atol=tol)


def test_gcf_large_sigma_r_is_gaussian():
    """mu -> 0: the range kernel is flat and the filter is the normalised
    spatial Gaussian."""
    f = ramp_rectangles(21, 18, seed=12)
    np.testing.assert_allclose(F.gcf(f, 2.0, 1e7, 4), _scipy_gauss(f, 2.0), rtol=0, atol=1e-6)


def test_gcf_python_equals_c_with_regions():
    f = edge_rich(48, 40, seed=13)
    ref = F.gcf(f, 2.5, 30.0, 28)
    np.testing.assert_allclose(C.gcf(f, 2.5, 30.0, 28), ref, rtol=0, atol=1e-10)
    crop = C.gcf(f, 2.5, 30.0, 28, region=(3, 41, 10, 40))
    np.testing.assert_allclose(crop, ref[3:41, 10:40], rtol=0, atol=1e-10)
    _, parts = F.gcf(f, 2.5, 30.0, 28, return_parts=True)
    _, P, Q = C.gcf(f, 2.5, 30.0, 28, return_pq=True)
    np.testing.assert_allclose(P, parts["P"], rtol=1e-11, atol=0)
    np.testing.assert_allclose(Q, parts["Q"], rtol=1e-11, atol=0)


def test_gcf_2d_equals_separable():
    f = ramp_rectangles(15, 13, seed=14)
    a = F.gcf(f, 1.5, 30.0, 28, separable=True)
    b = F.gcf(f, 1.5, 30.0, 28, separable=False)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)


def _weighted_kernel_error(sigma_r, N, c=None):
    t_c, mu = K.gcf_params(sigma_r)
    if c is None:
        c, _ = K.gcf_coefficients(sigma_r, N)
    y = np.linspace(-1, 1, 40001)
    import mpmath
    with mpmath.workdps(40):
        def err(v):
            p = mpmath.fsum(mpmath.mpf(cn) * (mu * v) ** n for n, cn in enumerate(c))
            return float(mpmath.exp(-mu * abs(v)) * abs(p - mpmath.exp(mu * v)))
        return max(err(v) for v in y[::20])


def test_gcf_converges_to_direct_within_a_priori_bound():
    """|B_hat - B| <= (U - L) eps S / (1 - eps S), S = sum of the spatial
    weights (w_0 = 1), eps the largest kernel error |K_hat - K| over the
    centred range; and the error falls as N grows."""
    f = edge_rich(20, 18, seed=15)
    sigma_s, sigma_r = 1.0, 30.0
    S = F.spatial_kernel_1d(sigma_s).sum() ** 2
    direct = C.direct_bf(f, sigma_s, sigma_r)
    errs = []
    for N in (28, 34, 40, 50):
        e = np.abs(C.gcf(f, sigma_s, sigma_r, N) - direct).max()
        eps = _weighted_kernel_error(sigma_r, N)
        if eps * S < 1:
            assert e <= 255.0 * eps * S / (1 - eps * S) * 1.0001 + 1e-9, (N, e, eps)
        errs.append(e)
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-8


def _mse_db(a, b):
    return 10 * math.log10(np.mean((a - b) ** 2))


@pytest.mark.slow
def test_table1_shape_on_binary_checker(golden):
    """Soft pin on Table 1 (sigma_s = 5, sigma_r = 30): on a 150 x 150 binary
    checkerboard stand-in for the Checker image, the Gauss-polynomial (Taylor)
    filter is worse than the Gauss-Chebyshev filter at every N of the table,
    and the Chebyshev error falls steeply from N = 10 to N = 16. The image
    itself is not available, so the printed dB values are not matched."""
    t1 = golden["table1"]
    f = checkerboard(150, 150, cell=15)
    direct = C.direct_bf(f, t1["sigma_s"], t1["sigma_r"])
    gcf_db, gpf_db = [], []
    for N in t1["N"]:
        c_cheb, _ = K.gcf_coefficients(t1["sigma_r"], N)
        g = C.polynomial_filter(f, t1["sigma_s"], t1["sigma_r"], c_cheb)
        p = C.polynomial_filter(f, t1["sigma_s"], t1["sigma_r"], K.taylor_coefficients(N))
        gcf_db.append(_mse_db(g, direct))
        gpf_db.append(_mse_db(p, direct) if np.all(np.isfinite(p)) else float("inf"))
    for N, a, b, pa, pb in zip(t1["N"], gcf_db, gpf_db, t1["GCF"], t1["GPF"]):
        assert a < b, (N, a, b)
        assert pa < pb
    i10, i16 = t1["N"].index(10), t1["N"].index(16)
    assert gcf_db[i10] - gcf_db[i16] > 20.0, gcf_db
