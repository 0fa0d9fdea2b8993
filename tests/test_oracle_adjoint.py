"""Pins for the FP64 gradient oracle: finite differences of the independent
numpy/C forward oracle, torch.autograd.gradcheck, and closed forms at a
constant image and in the flat-range limit."""
import math

import mpmath
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import coeffs as K
from oracle import filters as F
from oracle import native as C
from synth import edge_rich, ramp_rectangles


def test_coefficient_derivative_matches_central_difference():
    for sr, N in ((30.0, 28), (40.0, 16), (25.0, 40)):
        c, dc = K.gcf_coefficients_with_derivative(sr, N)
        h = 1e-6
        cp, _ = K.gcf_coefficients(sr + h, N, dps=60)
        cm, _ = K.gcf_coefficients(sr - h, N, dps=60)
        _, mu = K.gcf_params(sr)
        # compare at kernel level: exp(-mu|x|/mu...) weighted sum_n dc_n x^n over the range
        xs = np.linspace(-mu, mu, 9)
        scale = max(math.exp(-abs(x)) * sum(abs(v * x ** n) for n, v in enumerate(dc)) for x in xs)
        for x in xs:
            d_an = sum(v * x ** n for n, v in enumerate(dc))
            d_fd = sum((a - b) / (2 * h) * x ** n for n, (a, b) in enumerate(zip(cp, cm)))
            assert math.exp(-abs(x)) * abs(d_an - d_fd) <= 1e-6 * scale, (sr, N, x)


def test_torch_forward_equals_numpy_oracle():
    f = edge_rich(17, 23, seed=30)
    y = A.gcf_torch(torch.tensor(f), 2.0, torch.tensor(30.0, dtype=torch.float64), 28).numpy()
    np.testing.assert_allclose(y, F.gcf(f, 2.0, 30.0, 28), rtol=0, atol=1e-9)


def test_gradients_match_central_differences_of_the_numpy_oracle():
    f = ramp_rectangles(14, 12, seed=31)
    rng = np.random.default_rng(32)
    ybar = rng.uniform(-1, 1, size=f.shape)
    ss, sr, N = 1.5, 30.0, 28
    gf, gs = A.gcf_grad(f, ss, sr, N, ybar)
    h = 1e-4
    for (i, j) in ((0, 0), (3, 7), (13, 11), (6, 0), (9, 5)):
        fp, fm = f.copy(), f.copy()
        fp[i, j] += h
        fm[i, j] -= h
        fd = (np.sum(ybar * F.gcf(fp, ss, sr, N)) - np.sum(ybar * F.gcf(fm, ss, sr, N))) / (2 * h)
        assert abs(gf[i, j] - fd) <= 1e-6 * (abs(fd) + 1e-3), (i, j, gf[i, j], fd)
    hs = 1e-4
    fd = (np.sum(ybar * F.gcf(f, ss, sr + hs, N)) - np.sum(ybar * F.gcf(f, ss, sr - hs, N))) / (2 * hs)
    assert abs(gs - fd) <= 1e-6 * abs(fd), (gs, fd)


def test_gradcheck_small():
    f = torch.tensor(ramp_rectangles(6, 5, seed=33), requires_grad=True)
    sr = torch.tensor(40.0, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: A.gcf_torch(a, 1.0, b, 16), (f, sr), eps=1e-5, atol=1e-6)


def test_constant_image_closed_forms():
    """At a constant image every output equals the constant for any sigma_r,
    so dL/dsigma_r = 0; with an accurate fit the range weights are flat to
    first order, so dL/df is the normalised Gaussian filter applied to ybar
    (the filter is symmetric, so it is its own adjoint)."""
    f = np.full((11, 13), 90.0)
    rng = np.random.default_rng(34)
    ybar = rng.uniform(-1, 1, size=f.shape)
    gf, gs = A.gcf_grad(f, 2.0, 30.0, 50, ybar)
    assert abs(gs) <= 1e-9
    g = F.spatial_kernel_1d(2.0)
    expect = F.gauss_filter_separable(ybar, 2.0) / g.sum() ** 2
    np.testing.assert_allclose(gf, expect, rtol=0, atol=1e-8)


def test_flat_range_limit_is_gaussian_adjoint():
    f = ramp_rectangles(9, 10, seed=35)
    rng = np.random.default_rng(36)
    ybar = rng.uniform(-1, 1, size=f.shape)
    gf, _ = A.gcf_grad(f, 1.5, 1e5, 6, ybar)
    g = F.spatial_kernel_1d(1.5)
    np.testing.assert_allclose(gf, F.gauss_filter_separable(ybar, 1.5) / g.sum() ** 2, rtol=0, atol=1e-4)
