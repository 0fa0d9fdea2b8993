"""Precision form: the 4096^2 edge-rich image (seed 3) at sigma_s in {5, 10, 20}
x sigma_r in {10, 30, 50}, with FP32, FP16 and BF16 stacks (FP32 or FP64
accumulation as each path has it), against the FP64 oracle on the 512^2 centre
crop: max-abs error and PSNR (peak 255), stated per configuration.

sigma_r = 30 and 50 run the single expansion at the degree rule's N (28 and
11). BF16 at sigma_r = 30 lies outside the conditioning domain the library
accepts by default (kappa u_bf16 = 0.06 > 1e-2); it runs with the allow flag
and is held to a bound of the same kappa u t_h kind as the others. sigma_r =
10 is where the single expansion is hopeless (kappa ~ 1e59 at the rule's
N = 245): it runs the pivoted form with the smallest sub-range count whose
conditioning holds for the stack (FP32: 8, FP16 and BF16: 32), against the
oracle's pivoted filter.

Bars: FP32 1e-3 (measured at most 1.8e-4); the 16-bit stacks per cell, about
three times the measured max-abs error (in the table below). PSNR is
reported, not held."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CROP = (1792, 2304, 1792, 2304)
GRID = [(ss, sr) for ss in (5.0, 10.0, 20.0) for sr in (10.0, 30.0, 50.0)]
FP32_TOL = 1e-3
# (stack, sigma_s, sigma_r): bar (measured max-abs on the 512^2 centre crop)
BOUND = {
    ("f16", 5.0, 10.0): 0.013, ("f16", 5.0, 30.0): 3.6, ("f16", 5.0, 50.0): 0.09,          # 4.2e-3, 1.18, 2.9e-2
    ("f16", 10.0, 10.0): 0.012, ("f16", 10.0, 30.0): 1.4, ("f16", 10.0, 50.0): 0.04,       # 3.8e-3, 0.44, 1.3e-2
    ("f16", 20.0, 10.0): 0.013, ("f16", 20.0, 30.0): 0.75, ("f16", 20.0, 50.0): 0.023,     # 4.2e-3, 0.25, 7.5e-3
    ("bf16", 5.0, 10.0): 0.12, ("bf16", 5.0, 30.0): 23.0, ("bf16", 5.0, 50.0): 0.43,       # 4.0e-2, 7.7, 0.14
    ("bf16", 10.0, 10.0): 0.1, ("bf16", 10.0, 30.0): 8.8, ("bf16", 10.0, 50.0): 0.43,      # 3.3e-2, 2.9, 0.14
    ("bf16", 20.0, 10.0): 0.085, ("bf16", 20.0, 30.0): 6.7, ("bf16", 20.0, 50.0): 0.25,    # 2.8e-2, 2.2, 8.1e-2
}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def image():
    from synth import edge_rich
    return edge_rich(4096, 4096, seed=3).astype(np.float32).astype(np.float64)


def _log(msg):
    print(msg, flush=True)


def _psnr(err):
    mse = float(np.mean(err * err))
    return math.inf if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


@pytest.mark.parametrize("sigma_s,sigma_r", GRID)
def test_precision_grid(torch_cuda, image, sigma_s, sigma_r):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    torch = torch_cuda
    f = torch.tensor(image, dtype=torch.float32, device="cuda:0")
    r0, r1, c0, c1 = CROP
    refs = {}
    for dtype in ("f32", "f16", "bf16"):
        if sigma_r >= 30.0:
            N = bf.degree_rule(sigma_r)
            _, kappa = bf.query(sigma_r, N)
            if "single" not in refs:
                refs["single"] = C.gcf(image, sigma_s, sigma_r, N, region=CROP)
            ref = refs["single"]
            y = bf.gc_filter(f, sigma_s, sigma_r, N, stack_dtype=dtype, allow_ill_conditioned=True)
            form = f"N={N}"
        else:
            K = bf.pivot_count(sigma_r, dtype)
            assert K > 0
            kappa = max(k for _, _, k in bf.pivot_plan(sigma_r, K))
            if K not in refs:
                refs[K] = C.pivot_gcf(image, sigma_s, sigma_r, K, region=CROP)
            ref = refs[K]
            y = bf.gc_filter_pivots(f, sigma_s, sigma_r, K, stack_dtype=dtype)
            form = f"K={K} sub-ranges"
        err = y[r0:r1, c0:c1].cpu().double().numpy() - ref
        mx = float(np.abs(err).max())
        bound = FP32_TOL if dtype == "f32" else BOUND[(dtype, sigma_s, sigma_r)]
        _log(f"grid sigma_s={sigma_s:g} sigma_r={sigma_r:g} {dtype} ({form}, kappa {kappa:.3g}): "
             f"max-abs {mx:.3e}, PSNR {_psnr(err):.1f} dB (bound {bound:.3g})")
        assert np.isfinite(mx) and mx <= bound
