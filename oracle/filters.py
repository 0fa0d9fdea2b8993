"""FP64 numpy oracle for the bilateral filter and its Gauss-Chebyshev
approximation (test infrastructure only; see the package docstring).

Notation follows the paper: image f on a rectangle I, extended outside I by
symmetry (Section I); spatial kernel g_s(j) = exp(-|j|^2 / 2 sigma_s^2) on
Omega = [-W, W]^2 with W = 3 sigma_s (Section I); range kernel
g_r(t) = exp(-t^2 / 2 sigma_r^2).

Readings where the paper is silent:
* symmetric extension is the half-sample mirror (... c b a | a b c ...),
  periodic with period 2M for offsets beyond one image side;
* W = ceil(3 sigma_s) when 3 sigma_s is not an integer; the taps use the real
  sigma_s;
* [L, U] = [0, 255] (the 8-bit example of Section II), so t_c = 127.5.
"""
from __future__ import annotations

import math

import numpy as np

from .coeffs import DEFAULT_L, DEFAULT_U, gcf_coefficients, gcf_params

__all__ = [
    "mirror_index",
    "radius",
    "spatial_kernel_1d",
    "direct_bf",
    "gauss_filter_2d",
    "gauss_filter_separable",
    "gcf",
    "gcf_pairwise",
    "polynomial_filter",
    "pivot_plan",
    "pivot_gcf",
    "direct_joint_bf",
    "joint_polynomial_filter",
    "joint_gcf",
]


def mirror_index(i, M: int):
    """Index into [0, M) of position i of the symmetric extension of a
    length-M line: half-sample mirror, period 2M."""
    i = np.asarray(i)
    p = np.mod(i, 2 * M)
    return np.where(p >= M, 2 * M - 1 - p, p)


def radius(sigma_s: float) -> int:
    """W = 3 sigma_s (Section I), rounded up to an integer."""
    return int(math.ceil(3.0 * sigma_s - 1e-12))


def spatial_kernel_1d(sigma_s: float) -> np.ndarray:
    """exp(-k^2 / 2 sigma_s^2) for k = -W..W. The 2-D spatial kernel on
    Omega is the outer product of this vector with itself."""
    W = radius(sigma_s)
    k = np.arange(-W, W + 1, dtype=np.float64)
    return np.exp(-k * k / (2.0 * sigma_s * sigma_s))


def _gather(f: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    H, Wd = f.shape
    return f[np.ix_(mirror_index(rows, H), mirror_index(cols, Wd))]


def _region(f: np.ndarray, region):
    H, Wd = f.shape
    if region is None:
        return 0, H, 0, Wd
    r0, r1, c0, c1 = region
    if not (0 <= r0 <= r1 <= H and 0 <= c0 <= c1 <= Wd):
        raise ValueError("region out of bounds")
    return r0, r1, c0, c1


def direct_bf(f: np.ndarray, sigma_s: float, sigma_r: float, region=None) -> np.ndarray:
    """Gaussian bilateral filter, eq. (1), by brute force over Omega.

    For each offset j in Omega the shifted image f(i - j) is gathered once
    through the symmetric extension; numerator and denominator accumulate
    g_s(j) g_r(f(i-j) - f(i)) f(i-j) and g_s(j) g_r(f(i-j) - f(i)).
    `region` = (r0, r1, c0, c1) restricts the output to a crop of I."""
    f = np.asarray(f, dtype=np.float64)
    r0, r1, c0, c1 = _region(f, region)
    W = radius(sigma_s)
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    center = f[r0:r1, c0:c1]
    num = np.zeros_like(center)
    den = np.zeros_like(center)
    for j1 in range(-W, W + 1):
        for j2 in range(-W, W + 1):
            gs = math.exp(-(j1 * j1 + j2 * j2) / (2.0 * sigma_s * sigma_s))
            t = _gather(f, rows - j1, cols - j2)
            d = t - center
            w = gs * np.exp(-d * d / (2.0 * sigma_r * sigma_r))
            num += w * t
            den += w
    return num / den


def gauss_filter_2d(F: np.ndarray, sigma_s: float, region=None) -> np.ndarray:
    """Eq. (7) by its definition: sum over the square Omega of
    g_s(j) F(i - j), with F extended by symmetry. Works on (H, W) or on a
    stack (P, H, W) of images filtered independently."""
    F = np.asarray(F, dtype=np.float64)
    stack = F if F.ndim == 3 else F[None]
    H, Wd = stack.shape[1:]
    r0, r1, c0, c1 = _region(stack[0], region)
    W = radius(sigma_s)
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    out = np.zeros((stack.shape[0], r1 - r0, c1 - c0))
    for j1 in range(-W, W + 1):
        ri = mirror_index(rows - j1, H)
        for j2 in range(-W, W + 1):
            gs = math.exp(-(j1 * j1 + j2 * j2) / (2.0 * sigma_s * sigma_s))
            ci = mirror_index(cols - j2, Wd)
            out += gs * stack[:, ri[:, None], ci[None, :]]
    return out if F.ndim == 3 else out[0]


def gauss_filter_separable(F: np.ndarray, sigma_s: float, region=None) -> np.ndarray:
    """Eq. (7) computed through separability of g_s on the square Omega
    (Section I; the separable route named in Section I): a 1-D filter along
    rows, then along columns, each over k = -W..W with the symmetric
    extension. Equal to `gauss_filter_2d` up to rounding."""
    F = np.asarray(F, dtype=np.float64)
    stack = F if F.ndim == 3 else F[None]
    H, Wd = stack.shape[1:]
    r0, r1, c0, c1 = _region(stack[0], region)
    W = radius(sigma_s)
    g = spatial_kernel_1d(sigma_s)
    # Rows r0-W .. r1+W are needed by the column pass.
    rows_ext = mirror_index(np.arange(r0 - W, r1 + W), H)
    cols = np.arange(c0, c1)
    tmp = np.zeros((stack.shape[0], rows_ext.size, c1 - c0))
    for k in range(-W, W + 1):
        tmp += g[k + W] * stack[:, rows_ext[:, None], mirror_index(cols - k, Wd)[None, :]]
    out = np.zeros((stack.shape[0], r1 - r0, c1 - c0))
    for k in range(-W, W + 1):
        out += g[k + W] * tmp[:, W - k: W - k + (r1 - r0), :]
    return out if F.ndim == 3 else out[0]


def polynomial_filter(f: np.ndarray, sigma_s: float, sigma_r: float, c,
                      L: float = DEFAULT_L, U: float = DEFAULT_U, region=None,
                      separable: bool = True, return_parts: bool = False, t_c: float | None = None):
    """The fast algorithm of Section II for a given polynomial
    exp(x) ~ sum_n c_n x^n (eq. 3), applied to the centred image (eq. 17),
    with the centring undone at the end (Section III-B).

    Steps, in the paper's notation (g is the centred image):
      G_n = (g / sigma_r)^n,  F_n = exp(-g^2 / 2 sigma_r^2) G_n    (eq. 6)
      F_bar_n = Gaussian filter of F_n over Omega,  n = 0..N+1      (eq. 7)
      P = sigma_r sum_{n=0}^{N} c_n G_n F_bar_{n+1}                  (eq. 8)
      Q = sum_{n=0}^{N} c_n G_n F_bar_n                              (eq. 9)
      B_hat[g] = P / Q                                               (eq. 10)
      B_hat[f] = B_hat[g] + t_c

    With return_parts, also returns a dict holding P, Q and the stacks F
    (n = 0..N+1, on the output region) and F_bar. t_c overrides the centre
    (L + U)/2 (the pivoted form below)."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    N = c.size - 1
    t_c = 0.5 * (L + U) if t_c is None else float(t_c)
    r0, r1, c0, c1 = _region(f, region)
    W = radius(sigma_s)
    H, Wd = f.shape
    # Pixels that feed the region: the region grown by W, through the
    # symmetric extension.
    rows = np.arange(r0 - W, r1 + W)
    cols = np.arange(c0 - W, c1 + W)
    g_ext = _gather(f, rows, cols) - t_c                         # eq. (17)
    g_ctr = g_ext[W:W + (r1 - r0), W:W + (c1 - c0)]
    E_ext = np.exp(-g_ext * g_ext / (2.0 * sigma_r * sigma_r))
    u_ext = g_ext / sigma_r
    u_ctr = g_ctr / sigma_r
    filt = gauss_filter_separable if separable else gauss_filter_2d
    inner = (W, W + (r1 - r0), W, W + (c1 - c0))
    P = np.zeros_like(g_ctr)
    Q = np.zeros_like(g_ctr)
    F_stack, Fbar_stack = [], []
    for n in range(N + 2):
        F_n = E_ext * u_ext ** n                                   # eq. (6)
        Fbar_n = filt(F_n, sigma_s, region=inner)                  # eq. (7)
        if n <= N:
            Q += c[n] * u_ctr ** n * Fbar_n                        # eq. (9)
        if n >= 1:
            P += sigma_r * c[n - 1] * u_ctr ** (n - 1) * Fbar_n    # eq. (8)
        if return_parts:
            F_stack.append(F_n[W:W + (r1 - r0), W:W + (c1 - c0)])
            Fbar_stack.append(Fbar_n)
    out = P / Q + t_c                                              # eq. (10)
    if return_parts:
        return out, {"P": P, "Q": Q, "F": np.stack(F_stack), "F_bar": np.stack(Fbar_stack)}
    return out


def gcf(f: np.ndarray, sigma_s: float, sigma_r: float, N: int,
        L: float = DEFAULT_L, U: float = DEFAULT_U, region=None,
        separable: bool = True, return_parts: bool = False):
    """Gauss-Chebyshev filter (Section III-B summary): `polynomial_filter`
    with the coefficients c_n of eq. (19)."""
    c, _ = gcf_coefficients(sigma_r, N, L, U)
    return polynomial_filter(f, sigma_s, sigma_r, c, L, U, region, separable, return_parts)


def gcf_pairwise(f: np.ndarray, sigma_s: float, sigma_r: float, N: int,
                 L: float = DEFAULT_L, U: float = DEFAULT_U, region=None) -> np.ndarray:
    """The Gauss-Chebyshev filter without the exchange of sums of Section II:
    the approximate range kernel (eq. 4 with the expansion eq. 18 for the
    cross term) is evaluated for every pair (i, i-j) and put straight into
    eq. (1) on the centred image. The cross term uses the Chebyshev series
    sum_l d_l T_l(x / mu), evaluated by numpy's Chebyshev routine, not the
    monomial coefficients. O(|Omega|) per pixel: tiny images only."""
    from numpy.polynomial import chebyshev as npcheb

    f = np.asarray(f, dtype=np.float64)
    _, d = gcf_coefficients(sigma_r, N, L, U)
    t_c, mu = gcf_params(sigma_r, L, U)
    r0, r1, c0, c1 = _region(f, region)
    W = radius(sigma_s)
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    tau = f[r0:r1, c0:c1] - t_c
    num = np.zeros_like(tau)
    den = np.zeros_like(tau)
    s2 = 2.0 * sigma_r * sigma_r
    for j1 in range(-W, W + 1):
        for j2 in range(-W, W + 1):
            gs = math.exp(-(j1 * j1 + j2 * j2) / (2.0 * sigma_s * sigma_s))
            t = _gather(f, rows - j1, cols - j2) - t_c
            x = tau * t / (sigma_r * sigma_r)
            k = np.exp(-tau * tau / s2) * np.exp(-t * t / s2) * npcheb.chebval(x / mu, d)
            num += gs * k * t
            den += gs * k
    return num / den + t_c


# ---------------------------------------------------------------------------
# Joint (cross) bilateral filter: the range kernel is taken on a guide image g
# while f is averaged (the application the conclusion points to, e.g.
# aggregation of matching costs). Not a formula of the paper; its fast form is
# the paper's Section II expansion with the range variable taken from g.
# ---------------------------------------------------------------------------

def direct_joint_bf(f: np.ndarray, g: np.ndarray, sigma_s: float, sigma_r: float, region=None) -> np.ndarray:
    """sum_j g_s(j) g_r(g(i-j) - g(i)) f(i-j) / sum_j g_s(j) g_r(g(i-j) - g(i))
    by brute force over Omega, both images through the symmetric extension."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if f.shape != g.shape:
        raise ValueError("f and g must have the same shape")
    r0, r1, c0, c1 = _region(f, region)
    W = radius(sigma_s)
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    gc = g[r0:r1, c0:c1]
    num = np.zeros_like(gc)
    den = np.zeros_like(gc)
    for j1 in range(-W, W + 1):
        for j2 in range(-W, W + 1):
            gs = math.exp(-(j1 * j1 + j2 * j2) / (2.0 * sigma_s * sigma_s))
            d = _gather(g, rows - j1, cols - j2) - gc
            w = gs * np.exp(-d * d / (2.0 * sigma_r * sigma_r))
            num += w * _gather(f, rows - j1, cols - j2)
            den += w
    return num / den


def joint_polynomial_filter(f: np.ndarray, g: np.ndarray, sigma_s: float, sigma_r: float, c,
                            L: float = DEFAULT_L, U: float = DEFAULT_U, region=None):
    """The Section II expansion with the range variable from the guide:
      h = g - t_c (eq. 17 on the guide),  G_n = (h / sigma_r)^n,
      F_n = exp(-h^2 / 2 sigma_r^2) G_n                         (eq. 6 on g)
      Q = sum_{n=0}^{N} c_n G_n Gauss[F_n]                      (eq. 9)
      P = sum_{n=0}^{N} c_n G_n Gauss[F_n f]                    (eq. 8, f in place of g)
      output P / Q                                              (eq. 10)
    With g = f, F_n f = F_n (h + t_c) = sigma_r F_{n+1} + t_c F_n, which gives
    back the plain filter."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    N = c.size - 1
    t_c = 0.5 * (L + U)
    r0, r1, c0, c1 = _region(f, region)
    W = radius(sigma_s)
    rows = np.arange(r0 - W, r1 + W)
    cols = np.arange(c0 - W, c1 + W)
    h_ext = _gather(g, rows, cols) - t_c
    f_ext = _gather(f, rows, cols)
    u_ext = h_ext / sigma_r
    u_ctr = u_ext[W:W + (r1 - r0), W:W + (c1 - c0)]
    E_ext = np.exp(-h_ext * h_ext / (2.0 * sigma_r * sigma_r))
    inner = (W, W + (r1 - r0), W, W + (c1 - c0))
    P = np.zeros_like(u_ctr)
    Q = np.zeros_like(u_ctr)
    for n in range(N + 1):
        F_n = E_ext * u_ext ** n
        Q += c[n] * u_ctr ** n * gauss_filter_separable(F_n, sigma_s, region=inner)
        P += c[n] * u_ctr ** n * gauss_filter_separable(F_n * f_ext, sigma_s, region=inner)
    return P / Q


def joint_gcf(f: np.ndarray, g: np.ndarray, sigma_s: float, sigma_r: float, N: int,
              L: float = DEFAULT_L, U: float = DEFAULT_U, region=None):
    """Joint filter with the Gauss-Chebyshev coefficients of eq. (19)."""
    c, _ = gcf_coefficients(sigma_r, N, L, U)
    return joint_polynomial_filter(f, g, sigma_s, sigma_r, c, L, U, region)


# ---------------------------------------------------------------------------
# Pivoted form for small sigma_r (not in the paper). The single expansion of
# Section III-B centres every pixel at t_c = (L+U)/2, so the cross term
# exp(g_i g_j / sigma_r^2) spans [-mu, mu], mu = (U-L)^2 / (4 sigma_r^2), which
# grows as 1/sigma_r^2 and makes the monomial sums ill-conditioned. Splitting
# [L, U] into K equal sub-ranges and centring each at its midpoint t_k bounds
# the centre pixel's offset by h = (U-L)/(2K), so the cross term spans
# [-mu_k, mu_k] with mu_k = h R_k / sigma_r^2, R_k = max(t_k - L, U - t_k) the
# largest neighbour offset. A pixel takes the output of the sub-range its own
# value lies in (the last sub-range includes U).
# ---------------------------------------------------------------------------

def pivot_plan(sigma_r: float, K: int, N=None, L: float = DEFAULT_L, U: float = DEFAULT_U):
    """Per sub-range k: (lo_k, hi_k, t_k, h, R_k, mu_k, N_k); N_k from the
    degree rule at mu_k when N is None."""
    from .coeffs import degree_rule_mu
    out = []
    h = (U - L) / (2.0 * K)
    for k in range(K):
        lo = L + (U - L) * k / K
        hi = L + (U - L) * (k + 1) / K
        t = 0.5 * (lo + hi)
        R = max(t - L, U - t)
        mu = h * R / (sigma_r * sigma_r)
        out.append((lo, hi, t, h, R, mu, degree_rule_mu(mu, L, U) if N is None else int(N)))
    return out


def pivot_gcf(f: np.ndarray, sigma_s: float, sigma_r: float, K: int, N=None,
              L: float = DEFAULT_L, U: float = DEFAULT_U, region=None):
    """Pivoted Gauss-Chebyshev filter: for each sub-range, the fast algorithm
    of Section II centred at t_k with the eq. 19 coefficients of exp on
    [-mu_k, mu_k]; each output pixel from the sub-range of its own value."""
    from .coeffs import chebyshev_coefficients_mu
    f = np.asarray(f, dtype=np.float64)
    r0, r1, c0, c1 = _region(f, region)
    ctr = f[r0:r1, c0:c1]
    out = np.full(ctr.shape, np.nan)
    for k, (lo, hi, t, h, R, mu, Nk) in enumerate(pivot_plan(sigma_r, K, N, L, U)):
        mask = (ctr >= lo) & ((ctr < hi) if k < K - 1 else (ctr <= hi))
        if not mask.any():
            continue
        c = chebyshev_coefficients_mu(mu, Nk)
        y = polynomial_filter(f, sigma_s, sigma_r, c, L, U, region=(r0, r1, c0, c1), t_c=t)
        out[mask] = y[mask]
    return out
