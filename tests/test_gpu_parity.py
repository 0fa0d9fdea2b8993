"""GPU parity: the HIP library against the FP64 CPU oracle, element by element
on the same seeded inputs, through the C ABI.

Bar for the FP32 stack: max |gpu - oracle| <= 1e-3 on the 0-255 scale. FP32
rounding of the stored planes reaches the output amplified by the
conditioning kappa = max_y e^{-mu|y|} sum |b_n| |y|^n (about kappa 2^-24 t_h),
so the bar holds where kappa 2^-24 <= 1e-5 (sigma_r >= 25 at the rule's
degree). The cases outside it are numbered exceptions with bars of their own,
about three times the measured error:
  E1  W = 1, sigma_r = 25, N = 40 (kappa 150), staged: measured 1.5e-3, bar 5e-3;
  E2  the degree sweep at N = 4, 8, 12, 16 (kappa 2e5, 1.3e5, 2.5e4, 2e3),
      bars in SWEEP_Y (test_degree_sweep_edge_rich).
Reduced-precision stacks are held to bars per configuration, about three
times the measured error."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-3


# numbered exception E1 (module docstring): (shape, sigma_s, sigma_r, N) -> bar
FP32_EXCEPTIONS = {((64, 65), 0.3, 25.0, 40): 5e-3}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def _np(t):
    return t.detach().cpu().double().numpy()


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("staged", [False, True])
def test_c1_ramp_rectangles(torch_cuda, staged):
    """256x256 ramp + 12 rectangles + N(0,10^2), sigma_s = 3, sigma_r = 30, N = 28."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import ramp_rectangles
    f = ramp_rectangles(256, 256, seed=1)
    f32 = f.astype(np.float32).astype(np.float64)       # what the GPU sees
    y = _np(bf.gc_filter(_gpu(torch_cuda, f32), 3.0, 30.0, 28, staged=staged))
    ref = C.gcf(f32, 3.0, 30.0, 28)
    err = np.abs(y - ref).max()
    direct = C.direct_bf(f32, 3.0, 30.0)
    _log(f"C1 staged={staged}: max|gpu-gc oracle| = {err:.3e}; max|gpu-direct| = {np.abs(y - direct).max():.3e}")
    assert err <= FP32_TOL


SHAPES = [
    ((97, 131), 2.5, 30.0, 28),    # ragged in both directions
    ((1, 50), 2.0, 30.0, 28),      # single row: column pass sees only mirrors
    ((50, 1), 2.0, 30.0, 28),
    ((1, 1), 1.0, 30.0, 28),
    ((7, 300), 7.0, 30.0, 28),     # W = 21 >= height: repeated reflection
    ((300, 7), 7.0, 30.0, 28),
    ((65, 64), 1.0, 40.0, 16),
    ((64, 65), 0.3, 25.0, 40),     # W = 1
    ((130, 70), 5.0, 50.0, 11),
]


@pytest.mark.parametrize("shape,sigma_s,sigma_r,N", SHAPES)
@pytest.mark.parametrize("staged", [False, True])
def test_ragged_and_degenerate_shapes(torch_cuda, shape, sigma_s, sigma_r, N, staged):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(*shape, seed=sum(shape) + 7).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), sigma_s, sigma_r, N, staged=staged))
    ref = C.gcf(f, sigma_s, sigma_r, N)
    err = np.abs(y - ref).max()
    tol = FP32_EXCEPTIONS.get((shape, sigma_s, sigma_r, N), FP32_TOL)
    _log(f"{shape} ss={sigma_s} sr={sigma_r} N={N} staged={staged}: {err:.3e} (tol {tol:.2e})")
    assert err <= tol


def test_row_stride_larger_than_width(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    big = edge_rich(90, 120, seed=3).astype(np.float32)
    t = _gpu(torch, big)[:, 10:87]                      # ld = 120, width = 77
    out = torch.full((90, 120), -1.0, device="cuda:0")[:, 10:87]
    bf.gc_filter(t, 2.0, 30.0, 28, out=out)
    ref = C.gcf(big[:, 10:87].astype(np.float64), 2.0, 30.0, 28)
    assert np.abs(_np(out) - ref).max() <= FP32_TOL


def test_constant_and_two_level_images(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import checkerboard
    for v in (0.0, 31.0, 127.5, 255.0):
        f = np.full((70, 90), v)
        y = _np(bf.gc_filter(_gpu(torch_cuda, f), 4.0, 30.0, 28))
        assert np.abs(y - v).max() <= FP32_TOL, v
    # a 0/255 image stays put to within the kernel error at the edges
    f = checkerboard(96, 96, cell=16)
    from oracle import native as C
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), 3.0, 30.0, 28))
    assert np.abs(y - C.gcf(f, 3.0, 30.0, 28)).max() <= FP32_TOL


def test_stage_parity(torch_cuda):
    """Each stage against the oracle's own intermediate arrays:
    planes H_n = mu^{-n/2} F_n (eq. 6), filtered planes Hbar_n = mu^{-n/2}
    F_bar_n / S (eq. 7, S = sum of the unnormalised weights), P' = P/(t_h S)
    and Q' = Q/S (eqs. 8-9), and y (eq. 10)."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from synth import edge_rich
    torch = torch_cuda
    ss, sr, N = 2.0, 30.0, 28
    f = edge_rich(61, 83, seed=5).astype(np.float32).astype(np.float64)
    ref, parts = F.gcf(f, ss, sr, N, return_parts=True)
    mu = (127.5 / sr) ** 2
    S = F.spatial_kernel_1d(ss).sum() ** 2
    scale = mu ** (-0.5 * np.arange(N + 2))[:, None, None]
    ft = _gpu(torch, f)
    st = bf.stack_build(ft, sr, N)
    planes = st.view().double().cpu().numpy()
    assert np.abs(planes - parts["F"] * scale).max() <= 2e-7
    bf.gauss_planes(st, ss)
    fplanes = st.view().double().cpu().numpy()
    assert np.abs(fplanes - parts["F_bar"] * scale / S).max() <= 4e-7
    y, P, Q = bf.combine(ft, st, sr, want_pq=True)
    Pr, Qr = parts["P"] / (127.5 * S), parts["Q"] / S
    assert np.max(np.abs(_np(P) - Pr) / (np.abs(Pr) + np.abs(Qr))) <= 1e-5
    assert np.max(np.abs(_np(Q) - Qr) / np.abs(Qr)) <= 1e-5
    assert np.abs(_np(y) - ref).max() <= FP32_TOL


def test_fp16_plane_scaling_in_stack(torch_cuda):
    """FP16 planes hold 2^k_n H_n with every plane's largest value near 2^14."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from synth import ramp_rectangles
    torch = torch_cuda
    sr, N = 30.0, 28
    f = ramp_rectangles(40, 52, seed=9).astype(np.float32).astype(np.float64)
    _, parts = F.gcf(f, 2.0, sr, N, return_parts=True)
    mu = (127.5 / sr) ** 2
    k = np.array(bf.plane_scales(sr, N, "f16"))
    st = bf.stack_build(_gpu(torch, f), sr, N, stack_dtype="f16")
    planes = st.view().double().cpu().numpy()
    want = parts["F"] * (mu ** (-0.5 * np.arange(N + 2)) * 2.0 ** k)[:, None, None]
    rel = np.abs(planes - want) / np.maximum(np.abs(want), 2.0 ** -14)
    assert rel.max() <= 2.0 ** -11 * 1.01
    assert np.abs(planes).max() <= 2 ** 15


# Bars for the reduced-precision stacks on the three-kernel tiles (FP64
# accumulation and combine), about three times the larger of the fused and
# staged errors measured: 0.49, 0.040, 0.35. FP16 at sigma_r = 30 carries
# kappa 2^-11 ~ 7e-3 of kernel error.
REDUCED = [
    ("f16", 30.0, 28, 1.5),
    ("f16", 50.0, 11, 0.12),
    ("bf16", 50.0, 11, 1.05),
]


@pytest.mark.parametrize("dtype,sigma_r,N,bound", REDUCED)
def test_reduced_precision_stated_bounds(torch_cuda, dtype, sigma_r, N, bound):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(200, 180, seed=21).astype(np.float32).astype(np.float64)
    ref = C.gcf(f, 3.0, sigma_r, N)
    for staged in (False, True):
        y = _np(bf.gc_filter(_gpu(torch_cuda, f), 3.0, sigma_r, N, stack_dtype=dtype, staged=staged))
        err = np.abs(y - ref).max()
        _log(f"{dtype} sr={sigma_r} N={N} staged={staged}: max err {err:.3e} (bound {bound})")
        assert err <= bound


def test_range_flag_and_determinism(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import ramp_rectangles
    torch = torch_cuda
    f = _gpu(torch, ramp_rectangles(64, 64, seed=2))
    ws = torch.empty(bf.workspace_bytes(64, 64, 2.0, 28), dtype=torch.uint8, device="cuda:0")
    a = bf.gc_filter(f, 2.0, 30.0, 28, workspace=ws)
    assert bf.read_flags(ws) == 0
    b = bf.gc_filter(f, 2.0, 30.0, 28, workspace=ws)
    assert torch.equal(a, b)
    g = f.clone()
    g[5, 7] = 300.0
    bf.gc_filter(g, 2.0, 30.0, 28, workspace=ws)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE
    g[5, 7] = float("nan")
    bf.gc_filter(g, 2.0, 30.0, 28, workspace=ws)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE
    bf.gc_filter(f, 2.0, 30.0, 28, workspace=ws)
    assert bf.read_flags(ws) == 0


def test_empty_image(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.empty((0, 17), device="cuda:0")
    y = bf.gc_filter(f, 2.0, 30.0, 28)
    assert y.shape == (0, 17)


def test_ill_conditioned_refused(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.zeros((16, 16), device="cuda:0")
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 2.0, 12.0, 170)
    assert e.value.status == 3


# Degree sweep bars on y (max-abs, 0-255 scale), about three times the measured
# error; N <= 16 is exception E2 (kappa >= 2e3 puts FP32's rounding above
# 1e-3): measured 0.83, 0.088, 0.36, 0.025, 3.1e-4, 1.1e-4, 2.7e-5, 8.1e-6.
SWEEP_Y = {4: 2.5, 8: 0.27, 12: 1.1, 16: 0.075, 20: FP32_TOL, 24: FP32_TOL, 28: FP32_TOL, 34: FP32_TOL}
# Bars on P' and Q' (eqs. 8-9) at every pixel, relative to the crop's largest
# |Q'|, about three times the measured 7.6e-8, 1.1e-7, 8.1e-7, 5.1e-6, 4.3e-6,
# 1.5e-6, 3.3e-7, 8.9e-8.
SWEEP_PQ = {4: 2.5e-7, 8: 3.5e-7, 12: 2.5e-6, 16: 1.6e-5, 20: 1.3e-5, 24: 4.5e-6, 28: 1e-6, 34: 2.7e-7}


@pytest.mark.parametrize("N", [4, 8, 12, 16, 20, 24, 28, 34])
def test_degree_sweep_edge_rich(torch_cuda, N):
    """1024^2 edge-rich image, sigma_s = 5, sigma_r = 30, on a 256^2 crop,
    against the approximation oracle (held) and the direct filter (reported:
    below N ~ 24 the polynomial's kernel error exceeds 1 and the filter is far
    from the direct one, as the paper's choice of N = 28 implies). For N < 28
    kappa grows (kappa(20) ~ 2e2, kappa(4) ~ 2e5), and so does the FP32
    rounding the filter carries. Every pixel's P' and Q' (eqs. 8-9, from the
    staged kernels) is held to the oracle's, relative to the crop's scale of
    Q'. At low N the polynomial can make Q cancel, and y = t_c + t_h P'/Q'
    there is conditioned by the cancellation, not by kappa: y is held at the
    pixels whose oracle Q' is at least 1% of the crop's median (every pixel
    for N >= 24), and reported at the others. N = 4 (kappa ~ 2e5) is outside
    the domain the library accepts and is refused without the allow flag."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    f = edge_rich(1024, 1024, seed=2).astype(np.float32).astype(np.float64)
    _, kappa = bf.query(30.0, N)
    in_domain = kappa * 2.0 ** -24 <= 1e-2
    if not in_domain:
        with pytest.raises(bf.BFError) as e:
            bf.gc_filter(_gpu(torch, f[:64, :64]), 5.0, 30.0, N)
        assert e.value.status == 3
    ft = _gpu(torch, f)
    y = _np(bf.gc_filter(ft, 5.0, 30.0, N, allow_ill_conditioned=True))
    st = bf.gauss_planes(bf.stack_build(ft, 30.0, N), 5.0)
    _, Pg, Qg = bf.combine(ft, st, 30.0, want_pq=True)
    reg = (384, 640, 384, 640)
    ref, P, Q = C.gcf(f, 5.0, 30.0, N, region=reg, return_pq=True)
    S = F.spatial_kernel_1d(5.0).sum() ** 2
    Pr, Qr = P / (127.5 * S), Q / S
    scale = np.abs(Qr).max()
    ePQ = max(np.abs(_np(Pg)[384:640, 384:640] - Pr).max(), np.abs(_np(Qg)[384:640, 384:640] - Qr).max()) / scale
    direct = C.direct_bf(f, 5.0, 30.0, region=reg)
    ok = Q >= 1e-2 * np.median(Q[Q > 0])
    if N >= 24:
        assert ok.all()
    yc = y[384:640, 384:640]
    err = np.abs(yc - ref)[ok].max()
    ed = np.abs(yc - direct)[ok].max()
    e_rest = float(np.abs(yc - ref)[~ok].max()) if (~ok).any() else 0.0
    _log(f"sweep N={N}: max err {err:.3e} against the approximation oracle, {ed:.3e} against the direct "
         f"filter, P'/Q' {ePQ:.3e} of max|Q'|, kappa {kappa:.3g}, pixels with cancelled Q {int((~ok).sum())} "
         f"(y there {e_rest:.3e}){'' if in_domain else ' (outside the domain)'}")
    assert ePQ <= SWEEP_PQ[N]
    assert err <= SWEEP_Y[N]


def test_headline_size_sampled(torch_cuda):
    """4096^2 edge-rich, sigma_s = 10, sigma_r = 30, N = 28, FP32 stack, in the
    launch configuration the benchmark times: the oracle on a 512^2 centre
    crop and two 96^2 corner crops (all borders of the image included)."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(4096, 4096, seed=3).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), 10.0, 30.0, 28))
    for reg in ((1792, 2304, 1792, 2304), (0, 96, 0, 96), (4000, 4096, 4000, 4096), (0, 96, 4000, 4096)):
        ref = C.gcf(f, 10.0, 30.0, 28, region=reg)
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - ref).max()
        _log(f"4096^2 crop {reg}: {err:.3e}")
        assert err <= FP32_TOL
