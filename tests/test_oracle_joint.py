"""Pins for the oracle's joint (cross) bilateral filter: reductions to the
plain filter and to the normalised Gaussian, a library route, and convergence
to the direct joint filter within the a-priori bound."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import coeffs as K
from oracle import filters as F
from oracle import native as C
from synth import edge_rich, ramp_rectangles


def _scipy_gauss(f, sigma_s):
    g = F.spatial_kernel_1d(sigma_s)
    g = g / g.sum()
    out = ndimage.correlate1d(f, g, axis=0, mode="reflect")
    return ndimage.correlate1d(out, g, axis=1, mode="reflect")


def test_direct_joint_with_guide_f_is_the_plain_direct_filter():
    f = edge_rich(23, 19, seed=3)
    np.testing.assert_allclose(F.direct_joint_bf(f, f, 2.0, 30.0), C.direct_bf(f, 2.0, 30.0), rtol=0, atol=1e-10)


def test_joint_gcf_with_guide_f_is_the_plain_gcf():
    f = edge_rich(26, 31, seed=4)
    np.testing.assert_allclose(F.joint_gcf(f, f, 2.0, 30.0, 28), C.gcf(f, 2.0, 30.0, 28), rtol=0, atol=1e-8)


@pytest.mark.parametrize("N", [4, 28])
def test_constant_guide_gives_the_normalised_gaussian(N):
    """A constant guide makes every range weight equal (exactly, for any
    polynomial): the output is the normalised truncated Gaussian of f."""
    f = ramp_rectangles(29, 24, seed=6)
    g = np.full_like(f, 77.0)
    want = _scipy_gauss(f, 2.5)
    np.testing.assert_allclose(F.direct_joint_bf(f, g, 2.5, 30.0), want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(F.joint_gcf(f, g, 2.5, 30.0, N), want, rtol=0, atol=1e-9)


def test_joint_region_equals_crop():
    f = edge_rich(30, 28, seed=8)
    g = ramp_rectangles(30, 28, seed=9)
    full = F.joint_gcf(f, g, 1.5, 40.0, 16)
    crop = F.joint_gcf(f, g, 1.5, 40.0, 16, region=(5, 20, 3, 17))
    np.testing.assert_allclose(crop, full[5:20, 3:17], rtol=0, atol=1e-12)


def test_joint_gcf_converges_to_direct_within_a_priori_bound():
    """|P/Q - B| <= (max f - min f) eps S / (1 - eps S): the approximate weights
    differ from the exact ones by at most eps times the peak, and the output
    is a weighted mean of f in both cases."""
    f = ramp_rectangles(20, 22, seed=10)
    g = edge_rich(20, 22, seed=11)
    sigma_s, sigma_r = 1.0, 30.0
    S = F.spatial_kernel_1d(sigma_s).sum() ** 2
    direct = F.direct_joint_bf(f, g, sigma_s, sigma_r)
    errs = []
    for N in (28, 34, 40, 50):
        e = np.abs(F.joint_gcf(f, g, sigma_s, sigma_r, N) - direct).max()
        _, mu = K.gcf_params(sigma_r)
        c, _ = K.gcf_coefficients(sigma_r, N)
        y = np.linspace(-1, 1, 4001)
        p = np.polynomial.polynomial.polyval(mu * y, np.asarray(c))
        eps = np.max(np.exp(-mu * np.abs(y)) * np.abs(p - np.exp(mu * y)))
        if eps * S < 1:
            assert e <= (f.max() - f.min()) * eps * S / (1 - eps * S) * 1.0001 + 1e-9, (N, e, eps)
        errs.append(e)
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-8
