"""ctypes binding of the plain-C FP64 oracle in c/oracle.c (test
infrastructure only). Loads oracle/_liboracle.so, building it first if it is
not there."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .coeffs import DEFAULT_L, DEFAULT_U, gcf_coefficients
from . import build as _build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.oracle_direct_bf.restype = ctypes.c_int
        lib.oracle_direct_bf.argtypes = [
            _dp, ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_long]
        lib.oracle_polynomial_filter.restype = ctypes.c_int
        lib.oracle_polynomial_filter.argtypes = [
            _dp, ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, _dp, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_long, _dp, _dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _prep(f, region):
    f = np.ascontiguousarray(f, dtype=np.float64)
    H, Wd = f.shape
    r0, r1, c0, c1 = (0, H, 0, Wd) if region is None else region
    return f, H, Wd, r0, r1, c0, c1


def direct_bf(f, sigma_s, sigma_r, region=None):
    """Eq. (1) in C; same contract as oracle.filters.direct_bf."""
    f, H, Wd, r0, r1, c0, c1 = _prep(f, region)
    out = np.empty((r1 - r0, c1 - c0))
    rc = _load().oracle_direct_bf(_ptr(f), H, Wd, Wd, float(sigma_s), float(sigma_r),
                                  r0, r1, c0, c1, _ptr(out), max(1, c1 - c0))
    if rc != 0:
        raise ValueError(f"oracle_direct_bf failed ({rc})")
    return out


def polynomial_filter(f, sigma_s, sigma_r, c, L=DEFAULT_L, U=DEFAULT_U, region=None,
                      return_pq=False, t_c=None):
    """Section II fast algorithm in C; same contract as
    oracle.filters.polynomial_filter (without the plane stacks). t_c overrides
    the centre (L + U)/2."""
    f, H, Wd, r0, r1, c0, c1 = _prep(f, region)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.empty((r1 - r0, c1 - c0))
    P = np.empty_like(out)
    Q = np.empty_like(out)
    rc = _load().oracle_polynomial_filter(
        _ptr(f), H, Wd, Wd, float(sigma_s), float(sigma_r), c.size - 1, _ptr(c),
        0.5 * (L + U) if t_c is None else float(t_c), r0, r1, c0, c1, _ptr(out), max(1, c1 - c0), _ptr(P),
        _ptr(Q))
    if rc != 0:
        raise ValueError(f"oracle_polynomial_filter failed ({rc})")
    return (out, P, Q) if return_pq else out


def gcf(f, sigma_s, sigma_r, N, L=DEFAULT_L, U=DEFAULT_U, region=None, return_pq=False):
    """Gauss-Chebyshev filter in C with the coefficients of eq. (19)."""
    c, _ = gcf_coefficients(sigma_r, N, L, U)
    return polynomial_filter(f, sigma_s, sigma_r, c, L, U, region, return_pq)


def pivot_gcf(f, sigma_s, sigma_r, K, N=None, L=DEFAULT_L, U=DEFAULT_U, region=None):
    """Pivoted Gauss-Chebyshev filter with the C polynomial filter; same
    contract and steps as oracle.filters.pivot_gcf (per sub-range, the fast
    algorithm centred at t_k with the coefficients of exp on [-mu_k, mu_k];
    each output pixel from the sub-range of its own value)."""
    from .coeffs import chebyshev_coefficients_mu
    from .filters import pivot_plan
    f, H, Wd, r0, r1, c0, c1 = _prep(f, region)
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
