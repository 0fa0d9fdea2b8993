"""Pins for the oracle's recursive (IIR) Gaussian: the recursion against the
closed-form impulse response it realises, the sampled Gaussian it
approximates (Deriche's published accuracy), unit DC gain, the boundary rule
against a direct convolution over an explicitly mirrored line, and the flat
range limit of the filter built on it."""
import numpy as np
import pytest

from oracle import filters as F
from oracle import recursive as R
from synth import edge_rich, ramp_rectangles


@pytest.mark.parametrize("sigma", [1.5, 5.0, 12.0])
def test_recursion_realises_the_closed_form(sigma):
    x = np.zeros(1201)
    x[600] = 1.0
    y = R.recursive_gauss_1d(x, sigma)
    _, _, _, k = R.recursion_coefficients(sigma)
    np.testing.assert_allclose(y, k * R.impulse_response(np.arange(1201) - 600, sigma), rtol=0, atol=1e-14)


@pytest.mark.parametrize("sigma", [2.0, 5.0, 10.0, 20.0])
def test_close_to_the_sampled_gaussian(sigma):
    n = np.arange(-int(40 * sigma), int(40 * sigma) + 1)
    h = R.impulse_response(n, sigma)
    h /= h.sum()
    g = np.exp(-n * n / (2 * sigma * sigma))
    g /= g.sum()
    assert np.abs(h - g).max() <= 5e-4 * g.max()


def test_unit_dc_gain():
    """Constant lines stay constant, up to the zero start over 14 sigma
    (relative 1e-10)."""
    X = np.full((5, 77), 42.0)
    np.testing.assert_allclose(R.recursive_gauss_1d(X, 6.0, axis=1), X, rtol=1e-10, atol=0)
    np.testing.assert_allclose(R.recursive_gauss_2d(np.full((33, 21), 3.0), 4.0), 3.0, rtol=1e-10, atol=0)


@pytest.mark.parametrize("M,sigma", [(50, 3.0), (7, 4.0), (200, 1.2)])
def test_boundary_rule_is_a_convolution_over_the_mirrored_line(M, sigma):
    """Both recursions start from zero at the ends of a 14-sigma mirrored
    extension; that equals the convolution of the normalised impulse response
    with the mirror-extended line (taken over 40 sigma) to the response's
    decay over 14 sigma."""
    rng = np.random.default_rng(M)
    x = rng.uniform(0, 255, size=M)
    y = R.recursive_gauss_1d(x, sigma)
    Pw = int(40 * sigma)
    n = np.arange(-Pw, Pw + 1)
    _, _, _, k = R.recursion_coefficients(sigma)
    h = k * R.impulse_response(n, sigma)
    ref = np.array([np.sum(h * x[F.mirror_index(i - n, M)]) for i in range(M)])
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-7)


def test_recursive_filter_flat_range_is_the_recursive_gaussian():
    f = ramp_rectangles(30, 26, seed=41)
    np.testing.assert_allclose(R.recursive_gcf(f, 2.0, 1e7, 28), R.recursive_gauss_2d(f, 2.0), rtol=0, atol=1e-7)


def test_recursive_filter_is_near_the_truncated_one():
    """The recursive Gaussian extends past 3 sigma_s and deviates from the
    truncated one by up to ~0.5% of its mass, so the two filters differ by a
    grey level or so at strong edges, not by rounding."""
    from oracle import native as C
    f = edge_rich(40, 36, seed=42)
    d = np.abs(R.recursive_gcf(f, 2.0, 30.0, 28) - C.gcf(f, 2.0, 30.0, 28)).max()
    assert 1e-3 < d < 3.0
