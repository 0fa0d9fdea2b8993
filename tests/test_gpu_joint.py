"""GPU parity of the joint (cross) bilateral filter (bf_gc_joint_forward)
against the FP64 oracle's joint filter, through the C ABI. Bars on the 0-255
scale: the FP32 stack 1e-3 (measured at most 1.8e-4); the 16-bit stacks about
three times the largest error measured per configuration (in the comments)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _pair(shape, seed):
    from synth import edge_rich, ramp_rectangles
    f = ramp_rectangles(*shape, seed=seed).astype(np.float32).astype(np.float64)
    g = edge_rich(*shape, seed=seed + 1).astype(np.float32).astype(np.float64)
    return f, g


FP32_TOL = 1e-3


SHAPES = [((150, 170), 3.0), ((65, 129), 10.0), ((1, 77), 2.0), ((129, 5), 2.0), ((7, 300), 5.0),
          ((300, 7), 5.0), ((1, 1), 1.0), ((97, 131), 0.3)]


@pytest.mark.parametrize("shape,sigma_s", SHAPES)
def test_joint_fp32_parity(torch_cuda, shape, sigma_s):
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    f, g = _pair(shape, sum(shape))
    y = _np(bf.gc_joint_filter(_gpu(torch_cuda, f), _gpu(torch_cuda, g), sigma_s, 30.0, 28))
    err = np.abs(y - F.joint_gcf(f, g, sigma_s, 30.0, 28)).max()
    _log(f"joint f32 {shape} ss={sigma_s}: {err:.3e}")
    assert err <= FP32_TOL


def test_joint_reductions(torch_cuda):
    """guide = f gives the plain filter; a constant guide gives the normalised
    Gaussian of f."""
    import paper_1605_02178_amd as bf
    from scipy import ndimage
    from oracle import filters as F
    torch = torch_cuda
    f, _ = _pair((120, 140), 5)
    ft = _gpu(torch, f)
    same = _np(bf.gc_joint_filter(ft, ft.clone(), 3.0, 30.0, 28))
    assert np.abs(same - _np(bf.gc_filter(ft, 3.0, 30.0, 28))).max() <= 1e-3
    y = _np(bf.gc_joint_filter(ft, torch.full_like(ft, 200.0), 3.0, 30.0, 28))
    w = F.spatial_kernel_1d(3.0)
    w = w / w.sum()
    ref = ndimage.correlate1d(ndimage.correlate1d(f, w, axis=0, mode="reflect"), w, axis=1, mode="reflect")
    assert np.abs(y - ref).max() <= 1e-3


# three-kernel tiles: measured 0.156, 0.0218, 0.23
@pytest.mark.parametrize("dtype,sigma_r,N,bound", [("f16", 30.0, 28, 0.5), ("f16", 50.0, 11, 0.07),
                                                   ("bf16", 50.0, 11, 0.7)])
def test_joint_reduced_precision_bounds(torch_cuda, dtype, sigma_r, N, bound):
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    f, g = _pair((140, 150), 7)
    y = _np(bf.gc_joint_filter(_gpu(torch_cuda, f), _gpu(torch_cuda, g), 4.0, sigma_r, N, stack_dtype=dtype))
    err = np.abs(y - F.joint_gcf(f, g, 4.0, sigma_r, N)).max()
    _log(f"joint {dtype} sr={sigma_r} N={N}: {err:.3e} (bound {bound})")
    assert err <= bound


@pytest.mark.parametrize("coeffs", ["taylor", "minimax"])
def test_joint_other_coefficients(torch_cuda, coeffs):
    import paper_1605_02178_amd as bf
    from oracle import coeffs as K
    from oracle import filters as F
    f, g = _pair((90, 110), 9)
    sr, N = 50.0, 11
    c = K.taylor_coefficients(N) if coeffs == "taylor" else K.minimax_coefficients(sr, N)
    y = _np(bf.gc_joint_filter(_gpu(torch_cuda, f), _gpu(torch_cuda, g), 2.0, sr, N, coeffs=coeffs))
    err = np.abs(y - F.joint_polynomial_filter(f, g, 2.0, sr, c)).max()
    _log(f"joint {coeffs}: {err:.3e}")
    assert err <= 1e-3


def test_joint_flags_and_errors(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f, g = _pair((64, 70), 11)
    ft, gt = _gpu(torch, f), _gpu(torch, g)
    ws = torch.empty(bf.joint_workspace_bytes(64, 70, 2.0, 28), dtype=torch.uint8, device="cuda:0")
    bf.gc_joint_filter(ft, gt, 2.0, 30.0, 28, workspace=ws)
    assert bf.read_flags(ws) == 0
    for which in ("f", "g"):
        a, b = ft.clone(), gt.clone()
        (a if which == "f" else b)[10, 20] = 300.0
        bf.gc_joint_filter(a, b, 2.0, 30.0, 28, workspace=ws)
        assert bf.read_flags(ws) & bf.DEVFLAG_RANGE, which
    with pytest.raises(bf.BFError) as e:
        bf.gc_joint_filter(ft, gt, 2.0, 30.0, 28, out=gt)
    assert e.value.status == 1
    with pytest.raises(bf.BFError) as e:
        bf.gc_joint_filter(ft, gt, 17.0, 30.0, 28, stack_dtype="f16", tile_config=bf.TILE_FUSED)   # W = 51 > 48
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_joint_filter(ft, gt, 2.0, 30.0, 28, stack_dtype="f32", tile_config=bf.TILE_FUSED)
    assert e.value.status == 2
    with pytest.raises(ValueError):
        bf.gc_joint_filter(ft, gt[:, :60], 2.0, 30.0, 28)
    empty = torch.empty((0, 9), device="cuda:0")
    assert bf.gc_joint_filter(empty, empty.clone(), 2.0, 30.0, 28).shape == (0, 9)


def test_joint_1024_crops(torch_cuda):
    """1024^2: f ramp + rectangles, guide edge-rich, sigma_s = 5, sigma_r = 30,
    N = 28, FP32: the oracle on a 160^2 centre crop and a corner crop."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    f, g = _pair((1024, 1024), 13)
    y = _np(bf.gc_joint_filter(_gpu(torch_cuda, f), _gpu(torch_cuda, g), 5.0, 30.0, 28))
    for reg in ((432, 592, 432, 592), (0, 64, 960, 1024)):
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - F.joint_gcf(f, g, 5.0, 30.0, 28, region=reg)).max()
        _log(f"joint 1024^2 crop {reg}: {err:.3e}")
        assert err <= 1e-3


@pytest.mark.parametrize("shape,sigma_s", [((150, 170), 2.0), ((150, 170), 5.0), ((65, 129), 10.0), ((1, 77), 2.0),
                                           ((129, 5), 2.0), ((300, 7), 3.0), ((150, 170), 12.0), ((97, 140), 13.0),
                                           ((140, 190), 15.0)])
# fused tile: measured at most 0.80 (FP16) and 0.91 (BF16), both on 65 x 129 at sigma_s = 10
@pytest.mark.parametrize("dtype,sigma_r,N,bound", [("f16", 30.0, 28, 2.4), ("bf16", 50.0, 11, 2.7)])
def test_joint_fused_parity(torch_cuda, shape, sigma_s, dtype, sigma_r, N, bound):
    """The fused matrix-core joint kernel (all three geometries: W <= 16 and
    W <= 32 on 64-column tiles, W = 36, 39, 45 on 32-column tiles; ragged
    tiles) against the oracle's joint filter at the stated bounds."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    f, g = _pair(shape, sum(shape) + 3)
    y = _np(bf.gc_joint_filter(_gpu(torch_cuda, f), _gpu(torch_cuda, g), sigma_s, sigma_r, N, stack_dtype=dtype,
                               tile_config=bf.TILE_FUSED))
    err = np.abs(y - F.joint_gcf(f, g, sigma_s, sigma_r, N)).max()
    _log(f"joint fused {dtype} {shape} ss={sigma_s}: {err:.3e}")
    assert np.isfinite(y).all() and err <= bound


def test_joint_fused_guide_f_matches_plain_fused(torch_cuda):
    """With g = f the joint expansion is the plain one (B_n = A_{n+1}); the
    fused joint kernel and the plain fused kernel round differently but stay
    within the FP16 bound of each other."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f, _ = _pair((128, 160), 17)
    ft = _gpu(torch, f)
    a = _np(bf.gc_joint_filter(ft, ft.clone(), 4.0, 30.0, 28, stack_dtype="f16"))
    b = _np(bf.gc_filter(ft, 4.0, 30.0, 28, stack_dtype="f16"))
    _log(f"joint fused with g = f against the plain fused kernel: {np.abs(a - b).max():.3e}")
    assert np.abs(a - b).max() <= 2.4
    assert np.array_equal(a, _np(bf.gc_joint_filter(ft, ft.clone(), 4.0, 30.0, 28, stack_dtype="f16")))
