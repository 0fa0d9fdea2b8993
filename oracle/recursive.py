"""Recursive (IIR) Gaussian and the Gauss-Chebyshev filter built on it (oracle;
test infrastructure only).

Section I names recursion as the O(1) way to apply the Gaussian of eq. 7 and
cites Deriche's recursive Gaussian. This is that filter, in FP64:

  impulse response (one dimension, scale sigma, n integer)
    h(n) = [a0 cos(w0 n/s) + a1 sin(w0 n/s)] e^{-b0 |n|/s}
         + [c0 cos(w1 n/s) + c1 sin(w1 n/s)] e^{-b1 |n|/s}
  with Deriche's constants for the Gaussian (a0, a1, b0, b1, w0, w1, c0, c1)
  = (1.680, 3.735, 1.783, 1.723, 0.6318, 1.997, -0.6803, -0.2598),
  normalised to unit sum;

  realised as a causal 4th-order recursion over n >= 0 plus an anticausal one
  over n <= -1, whose coefficients come from the z-transform of each damped
  cosine section,
    sum_{n>=0} r^n (A cos(t n) + B sin(t n)) z^-n
        = (A + r (B sin t - A cos t) z^-1) / (1 - 2 r cos t z^-1 + r^2 z^-2),
  r = e^{-b/s}, t = w/s, added over the two sections.

Boundary: each line is extended by P = ceil(14 sigma) samples per side through
the symmetric extension (half-sample mirror, period 2M); both recursions start
from a zero state at the far end of the extension (the response has decayed
below 1e-10 over 14 sigma) and the middle M samples are kept.

This filter approximates the untruncated Gaussian (max deviation 4.6e-4 of the
peak), so it is not the truncated convolution of the other oracles: the GPU's
recursive variant is held to this module.
"""
from __future__ import annotations

import math

import numpy as np

from .coeffs import DEFAULT_L, DEFAULT_U, gcf_coefficients
from .filters import mirror_index

__all__ = ["DERICHE", "impulse_response", "recursion_coefficients", "padding", "recursive_gauss_1d",
           "recursive_gauss_2d", "recursive_polynomial_filter", "recursive_gcf"]

DERICHE = {"a0": 1.680, "a1": 3.735, "b0": 1.783, "b1": 1.723, "w0": 0.6318, "w1": 1.997,
           "c0": -0.6803, "c1": -0.2598}


def impulse_response(n, sigma: float) -> np.ndarray:
    """h(n) of the closed form above (not normalised)."""
    D = DERICHE
    n = np.abs(np.asarray(n, dtype=np.float64))
    return ((D["a0"] * np.cos(D["w0"] * n / sigma) + D["a1"] * np.sin(D["w0"] * n / sigma)) *
            np.exp(-D["b0"] * n / sigma) +
            (D["c0"] * np.cos(D["w1"] * n / sigma) + D["c1"] * np.sin(D["w1"] * n / sigma)) *
            np.exp(-D["b1"] * n / sigma))


def recursion_coefficients(sigma: float):
    """(n[0..3], m[1..4], d[1..4], k): causal numerator, anticausal numerator,
    common denominator 1 + sum d_i z^-i, and the unit-sum factor k."""
    D = DERICHE
    sections = [(D["a0"], D["a1"], D["b0"], D["w0"]), (D["c0"], D["c1"], D["b1"], D["w1"])]
    nums, dens = [], []
    for A, B, b, w in sections:
        r, t = math.exp(-b / sigma), w / sigma
        nums.append(np.array([A, r * (B * math.sin(t) - A * math.cos(t))]))
        dens.append(np.array([1.0, -2.0 * r * math.cos(t), r * r]))
    den = np.convolve(dens[0], dens[1])                       # 1, d1..d4
    num = np.convolve(nums[0], dens[1]) + np.convolve(nums[1], dens[0])   # degree 3
    n = num[:4]
    d = den[1:5]
    m = np.array([n[1] - n[0] * d[0], n[2] - n[0] * d[1], n[3] - n[0] * d[2], -n[0] * d[3]])
    total = (2.0 * n.sum() - n[0] * den.sum()) / den.sum()     # sum over all n of h(n)
    return n, m, d, 1.0 / total


def padding(sigma: float) -> int:
    return int(math.ceil(14.0 * sigma))


def recursive_gauss_1d(X: np.ndarray, sigma: float, axis: int = -1) -> np.ndarray:
    """The recursive Gaussian along `axis` of X (FP64), per the module
    docstring."""
    X = np.moveaxis(np.asarray(X, dtype=np.float64), axis, -1)
    M = X.shape[-1]
    P = padding(sigma)
    ext = X[..., mirror_index(np.arange(-P, M + P), M)]
    n, m, d, k = recursion_coefficients(sigma)
    L = ext.shape[-1]
    yp = np.zeros_like(ext)
    for i in range(L):                                          # causal
        acc = n[0] * ext[..., i]
        for j in range(1, 4):
            if i - j >= 0:
                acc = acc + n[j] * ext[..., i - j]
        for j in range(1, 5):
            if i - j >= 0:
                acc = acc - d[j - 1] * yp[..., i - j]
        yp[..., i] = acc
    ym = np.zeros_like(ext)
    for i in range(L - 1, -1, -1):                              # anticausal
        acc = np.zeros(ext.shape[:-1])
        for j in range(1, 5):
            if i + j < L:
                acc = acc + m[j - 1] * ext[..., i + j] - d[j - 1] * ym[..., i + j]
        ym[..., i] = acc
    out = k * (yp + ym)[..., P:P + M]
    return np.moveaxis(out, -1, axis)


def recursive_gauss_2d(X: np.ndarray, sigma: float) -> np.ndarray:
    """Columns, then rows (the GPU's order)."""
    return recursive_gauss_1d(recursive_gauss_1d(X, sigma, axis=0), sigma, axis=1)


def recursive_polynomial_filter(f: np.ndarray, sigma_s: float, sigma_r: float, c,
                                L: float = DEFAULT_L, U: float = DEFAULT_U) -> np.ndarray:
    """The fast algorithm of Section II (eqs. 6, 8-10, centred as in
    Section III-B) with the recursive Gaussian in place of eq. 7."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    N = c.size - 1
    t_c = 0.5 * (L + U)
    g = f - t_c
    u = g / sigma_r
    E = np.exp(-g * g / (2.0 * sigma_r * sigma_r))
    P = np.zeros_like(g)
    Q = np.zeros_like(g)
    for n in range(N + 2):
        Fbar = recursive_gauss_2d(E * u ** n, sigma_s)
        if n <= N:
            Q += c[n] * u ** n * Fbar
        if n >= 1:
            P += sigma_r * c[n - 1] * u ** (n - 1) * Fbar
    return P / Q + t_c


def recursive_gcf(f: np.ndarray, sigma_s: float, sigma_r: float, N: int,
                  L: float = DEFAULT_L, U: float = DEFAULT_U) -> np.ndarray:
    c, _ = gcf_coefficients(sigma_r, N, L, U)
    return recursive_polynomial_filter(f, sigma_s, sigma_r, c, L, U)
