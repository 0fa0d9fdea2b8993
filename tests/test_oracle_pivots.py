"""Pins for the oracle's pivoted form (small sigma_r): one sub-range is the
plain filter; a pair-wise evaluation with the Chebyshev series (no monomial
conversion, no exchange of sums) gives the same values; every pixel meets the
a-priori bound of its own sub-range against the direct filter; the error falls
with N."""
import math

import numpy as np
import pytest

from oracle import coeffs as K
from oracle import filters as F
from oracle import native as C
from synth import edge_rich


def _kernel_error(mu, c):
    """max_y exp(-mu|y|) |p(mu y) - exp(mu y)| on a fine grid."""
    y = np.linspace(-1, 1, 8001)
    p = np.polynomial.polynomial.polyval(mu * y, np.asarray(c))
    return float(np.max(np.exp(-mu * np.abs(y)) * np.abs(p - np.exp(mu * y))))


def test_one_pivot_is_the_plain_filter():
    f = edge_rich(30, 26, seed=21)
    np.testing.assert_allclose(F.pivot_gcf(f, 2.0, 30.0, 1, 28), C.gcf(f, 2.0, 30.0, 28), rtol=0, atol=1e-9)


def test_pivot_plan_geometry():
    plan = F.pivot_plan(10.0, 4)
    assert [p[0] for p in plan] == [0.0, 63.75, 127.5, 191.25] and plan[-1][1] == 255.0
    for lo, hi, t, h, R, mu, N in plan:
        assert h == pytest.approx(255 / 8) and t == pytest.approx((lo + hi) / 2)
        assert R == pytest.approx(max(t, 255 - t)) and mu == pytest.approx(h * R / 100.0)


def test_pivot_pairwise_form():
    """Each pixel from the approximate kernel of its sub-range put straight
    into eq. 1: E_i E_j sum_l d_l T_l(y) with y = (g_i / h)(g_j / R_k), the
    Chebyshev series summed in 40-digit arithmetic (its coefficients reach
    1e15 at these mu, beyond float64 for a direct sum)."""
    import mpmath
    f = edge_rich(7, 8, seed=22).astype(np.float64)
    sigma_s, sigma_r, KK = 0.6, 12.0, 4
    W = F.radius(sigma_s)
    plan = F.pivot_plan(sigma_r, KK)
    out = np.empty_like(f)
    fp = F._gather(f, np.arange(-W, f.shape[0] + W), np.arange(-W, f.shape[1] + W))
    for r in range(f.shape[0]):
        for c in range(f.shape[1]):
            v = f[r, c]
            k = min(int(v / (255.0 / KK)), KK - 1)
            lo, hi, t, h, R, mu, N = plan[k]
            with mpmath.workdps(40):
                d = K.chebyshev_fit(mpmath.exp, mpmath.mpf(mu), N)
                num = den = mpmath.mpf(0)
                gi = mpmath.mpf(v - t)
                for j1 in range(-W, W + 1):
                    for j2 in range(-W, W + 1):
                        fj = mpmath.mpf(fp[r - j1 + W, c - j2 + W])
                        gj = fj - t
                        ws = mpmath.exp(-mpmath.mpf(j1 * j1 + j2 * j2) / (2 * sigma_s ** 2))
                        yy = (gi / h) * (gj / R)
                        series = mpmath.fsum(d[l] * mpmath.chebyt(l, yy) for l in range(N + 1))
                        kr = mpmath.exp(-(gi * gi + gj * gj) / (2 * sigma_r ** 2)) * series
                        num += ws * kr * fj
                        den += ws * kr
                out[r, c] = float(num / den)
    np.testing.assert_allclose(F.pivot_gcf(f, sigma_s, sigma_r, KK), out, rtol=0, atol=1e-8)


@pytest.mark.parametrize("sigma_r,KK", [(10.0, 8), (10.0, 16), (15.0, 4), (20.0, 4)])
def test_pivots_meet_the_a_priori_bound(sigma_r, KK):
    """|B_hat - B| <= (U - L) eps_k S / (1 - eps_k S) for every pixel in
    sub-range k, eps_k the kernel error of that sub-range's polynomial at
    mu_k; the single expansion at sigma_r = 10 is far outside it."""
    f = edge_rich(40, 44, seed=23).astype(np.float64)
    sigma_s = 1.5
    S = F.spatial_kernel_1d(sigma_s).sum() ** 2
    direct = C.direct_bf(f, sigma_s, sigma_r)
    y = F.pivot_gcf(f, sigma_s, sigma_r, KK)
    for k, (lo, hi, t, h, R, mu, N) in enumerate(F.pivot_plan(sigma_r, KK)):
        mask = (f >= lo) & ((f < hi) if k < KK - 1 else (f <= hi))
        if not mask.any():
            continue
        eps = _kernel_error(mu, K.chebyshev_coefficients_mu(mu, N))
        assert eps * S < 1
        bound = 255.0 * eps * S / (1 - eps * S)
        assert np.abs(y - direct)[mask].max() <= bound * 1.0001 + 1e-9, (k, mu, N)


def test_pivot_error_falls_with_degree():
    f = edge_rich(24, 28, seed=24).astype(np.float64)
    direct = C.direct_bf(f, 1.0, 10.0)
    errs = [np.abs(F.pivot_gcf(f, 1.0, 10.0, 8, N) - direct).max() for N in (40, 50, 60, 70)]
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6


@pytest.mark.parametrize("sigma_r,KK,region", [(10.0, 8, None), (12.0, 32, (5, 30, 3, 40)), (15.0, 4, (0, 1, 0, 44))])
def test_native_pivots_equal_the_numpy_pivots(sigma_r, KK, region):
    """The C binding of the pivoted filter (used for large crops) takes the
    same steps as the numpy one: the same values to rounding."""
    f = edge_rich(34, 44, seed=26).astype(np.float64)
    a = C.pivot_gcf(f, 2.0, sigma_r, KK, region=region)
    b = F.pivot_gcf(f, 2.0, sigma_r, KK, region=region)
    assert np.isfinite(a).all()
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-9)
