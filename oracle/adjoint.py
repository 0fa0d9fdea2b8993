"""FP64 gradients of the Gauss-Chebyshev filter (oracle; test infrastructure
only). The paper has no backward pass; these are the exact derivatives of the
forward algorithm of Section II with the coefficients of eq. (19).

The forward is transcribed into torch FP64 CPU operations in the paper's order
and notation (centring eq. 17, G_n and F_n of eq. 6, the truncated Gaussian of
eq. 7 through the symmetric extension, P and Q of eqs. 8-9, P/Q of eq. 10) and
differentiated by autograd. The coefficients c_n(sigma_r) enter through a small
autograd function whose values and derivatives dc_n/dsigma_r come from mpmath
(`coeffs.gcf_coefficients_with_derivative`; for the minimax polynomial,
`coeffs.minimax_coefficients_with_derivative`).
"""
from __future__ import annotations

import numpy as np
import torch

from .coeffs import DEFAULT_L, DEFAULT_U, gcf_coefficients_with_derivative, minimax_coefficients_with_derivative
from .filters import mirror_index, radius

__all__ = ["gcf_torch", "gcf_grad"]


class _Coefficients(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma_r, N, L, U, kind):
        fn = minimax_coefficients_with_derivative if kind == "minimax" else gcf_coefficients_with_derivative
        c, dc = fn(float(sigma_r.item()), int(N), L, U)
        ctx.save_for_backward(torch.tensor(dc, dtype=torch.float64))
        return torch.tensor(c, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_c):
        (dc,) = ctx.saved_tensors
        return (grad_c * dc).sum().reshape(()), None, None, None, None


def _gauss_2d(F: torch.Tensor, sigma_s: float) -> torch.Tensor:
    """Eq. (7) through separability (Section I) on an already extended array:
    F has W extra rows and columns on every side; returns the interior."""
    W = radius(sigma_s)
    k = torch.arange(-W, W + 1, dtype=torch.float64)
    g = torch.exp(-k * k / (2.0 * sigma_s * sigma_s))
    h = F.shape[0] - 2 * W
    w = F.shape[1] - 2 * W
    rows = sum(g[t] * F[:, t:t + w] for t in range(2 * W + 1))            # along rows
    return sum(g[t] * rows[t:t + h, :] for t in range(2 * W + 1))          # along columns


def gcf_torch(f: torch.Tensor, sigma_s: float, sigma_r: torch.Tensor, N: int,
              L: float = DEFAULT_L, U: float = DEFAULT_U, kind: str = "chebyshev") -> torch.Tensor:
    """Gauss-Chebyshev filter of a 2-D FP64 CPU tensor, differentiable in f and
    sigma_r (a 0-d FP64 tensor); kind "minimax" takes the minimax polynomial's
    coefficients instead of eq. 19's."""
    H, Wd = f.shape
    W = radius(sigma_s)
    t_c = 0.5 * (L + U)
    ri = torch.as_tensor(mirror_index(np.arange(-W, H + W), H))
    ci = torch.as_tensor(mirror_index(np.arange(-W, Wd + W), Wd))
    g = f[ri][:, ci] - t_c                                                 # eq. (17), extended
    g_ctr = g[W:W + H, W:W + Wd]
    c = _Coefficients.apply(sigma_r, N, L, U, kind)
    E = torch.exp(-g * g / (2.0 * sigma_r * sigma_r))
    u = g / sigma_r
    u_ctr = g_ctr / sigma_r
    P = torch.zeros_like(g_ctr)
    Q = torch.zeros_like(g_ctr)
    for n in range(N + 2):
        F_n = E * u ** n                                                   # eq. (6)
        Fbar = _gauss_2d(F_n, sigma_s)                                     # eq. (7)
        if n <= N:
            Q = Q + c[n] * u_ctr ** n * Fbar                               # eq. (9)
        if n >= 1:
            P = P + sigma_r * c[n - 1] * u_ctr ** (n - 1) * Fbar           # eq. (8)
    return P / Q + t_c                                                     # eq. (10)


def gcf_grad(f, sigma_s: float, sigma_r: float, N: int, ybar, L: float = DEFAULT_L,
             U: float = DEFAULT_U, kind: str = "chebyshev"):
    """Gradients of sum(ybar * y) with y the Gauss-Chebyshev filter of f:
    returns (dL/df as a numpy array, dL/dsigma_r as a float)."""
    ft = torch.tensor(np.asarray(f, dtype=np.float64), requires_grad=True)
    sr = torch.tensor(float(sigma_r), dtype=torch.float64, requires_grad=True)
    y = gcf_torch(ft, sigma_s, sr, N, L, U, kind)
    loss = (y * torch.as_tensor(np.asarray(ybar, dtype=np.float64))).sum()
    loss.backward()
    return ft.grad.numpy(), float(sr.grad.item())
