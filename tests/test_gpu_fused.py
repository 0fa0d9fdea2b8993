"""GPU parity of the fused FP16/BF16 kernel (tile configuration TILE_FUSED:
planes made in registers, both passes of eq. 7 as banded Toeplitz products on
the matrix cores with FP32 accumulation, eqs. 8-10 folded in) against the FP64
oracle, element by element, through the C ABI.

Bars (max |gpu - oracle| on the 0-255 scale) per (stack, sigma_r, N), about
three times the largest error measured over every test that uses the
configuration (in the comments). Storage rounding of the planes dominates:
FP16 at sigma_r = 30, N = 28 carries kappa 2^-11 ~ 7e-3 of kernel error,
which falls with N as kappa does (15 at N = 28, 1.6 at N = 34).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BOUND = {
    ("f16", 30.0, 28): 2.4,     # measured 0.78 (65 x 129, sigma_s = 10); 0.44 on the 4096^2 centre crop
    ("f16", 30.0, 30): 0.7,     # measured 0.23 (4096^2 centre crop)
    ("f16", 30.0, 31): 0.35,    # measured 0.105 (4096^2 centre crop, the benchmark's FP16 configuration)
    ("f16", 30.0, 32): 0.35,    # measured 0.097 (4096^2 centre crop)
    ("f16", 50.0, 11): 0.05,    # measured 0.0156
    ("bf16", 50.0, 11): 1.0,    # measured 0.34 (1100 x 2050 corner)
}


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


# (shape, sigma_s): W = 3, 9, 15, 30, 45, 50-64 covers the FP16 geometries
# (64 x 128 tiles up to W = 32, 64 x 64 up to 48, 32 x 128 up to 64, all on
# 16 waves); ragged tails in both directions, single rows and columns, W
# above a side.
SHAPES = [
    ((130, 200), 1.0), ((130, 200), 3.0), ((130, 200), 5.0), ((130, 200), 10.0), ((130, 200), 15.0),
    ((64, 64), 10.0), ((65, 129), 10.0), ((1, 77), 2.0), ((129, 5), 2.0), ((7, 300), 5.0), ((300, 7), 5.0),
    ((2, 2), 3.0), ((1, 1), 1.0),
    # FP16 radii 49-64 (32 x 128 tiles on 16 waves): ragged, taller and wider than the radius, and not
    ((150, 290), 16.5), ((200, 300), 20.0), ((97, 131), 21.0), ((1, 77), 20.0), ((300, 40), 17.0), ((33, 260), 21.3),
]


@pytest.mark.parametrize("shape,sigma_s", SHAPES)
def test_fused_f16_parity(torch_cuda, shape, sigma_s):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    _log(f"fused f16 {shape} ss={sigma_s}")
    f = edge_rich(*shape, seed=sum(shape) + 7).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), sigma_s, 30.0, 28, stack_dtype="f16", tile_config=bf.TILE_FUSED))
    ref = C.gcf(f, sigma_s, 30.0, 28)
    err = np.abs(y - ref).max()
    _log(f"fused f16 {shape} ss={sigma_s}: max err {err:.3e}")
    assert np.isfinite(y).all()
    assert err <= BOUND[("f16", 30.0, 28)]


@pytest.mark.parametrize("dtype,sigma_r,N", [("f16", 50.0, 11), ("bf16", 50.0, 11), ("f16", 30.0, 30)])
@pytest.mark.parametrize("sigma_s", [3.0, 10.0, 14.0])
def test_fused_stated_bounds(torch_cuda, dtype, sigma_r, N, sigma_s):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(200, 180, seed=21).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), sigma_s, sigma_r, N, stack_dtype=dtype))
    err = np.abs(y - C.gcf(f, sigma_s, sigma_r, N)).max()
    _log(f"fused {dtype} ss={sigma_s} sr={sigma_r} N={N}: max err {err:.3e} (bound {BOUND[(dtype, sigma_r, N)]})")
    assert err <= BOUND[(dtype, sigma_r, N)]


def test_fused_is_default_deterministic_and_strided(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    f = _gpu(torch, edge_rich(150, 170, seed=5))
    a = bf.gc_filter(f, 4.0, 30.0, 28, stack_dtype="f16")
    b = bf.gc_filter(f, 4.0, 30.0, 28, stack_dtype="f16", tile_config=bf.TILE_FUSED)
    assert torch.equal(a, b)
    assert torch.equal(a, bf.gc_filter(f, 4.0, 30.0, 28, stack_dtype="f16"))
    big = torch.full((150, 200), -1.0, device="cuda:0")
    big[:, :170] = f
    view = big[:, :170]
    out = torch.full((150, 200), -5.0, device="cuda:0")
    bf.gc_filter(view, 4.0, 30.0, 28, stack_dtype="f16", out=out[:, :170])
    assert torch.equal(out[:, :170], a)
    assert bool((out[:, 170:] == -5.0).all())


def test_fused_argument_errors_and_fallback(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    f64 = edge_rich(160, 150, seed=8).astype(np.float32).astype(np.float64)
    f = _gpu(torch, f64)
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 4.0, 30.0, 28, stack_dtype="f32", tile_config=bf.TILE_FUSED)
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 22.0, 30.0, 28, stack_dtype="f16", tile_config=bf.TILE_FUSED)   # W = 66 > 64
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 17.0, 50.0, 11, stack_dtype="bf16", tile_config=bf.TILE_FUSED)  # W = 51 > 48 for BF16
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 4.0, 30.0, 28, stack_dtype="f16", tile_config=bf.TILE_FUSED, staged=True)
    assert e.value.status == 1
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter_batched([f], [4.0], [30.0], [28], stack_dtype="f32", tile_config=bf.TILE_FUSED)
    assert e.value.status == 2
    # W = 66 (FP16) and W = 51 (BF16) without a tile flag take the three-kernel path
    y = _np(bf.gc_filter(f, 22.0, 30.0, 28, stack_dtype="f16"))
    assert np.abs(y - C.gcf(f64, 22.0, 30.0, 28)).max() <= BOUND[("f16", 30.0, 28)]
    y = _np(bf.gc_filter(f, 17.0, 50.0, 11, stack_dtype="bf16"))
    assert np.abs(y - C.gcf(f64, 17.0, 50.0, 11)).max() <= BOUND[("bf16", 50.0, 11)]


def test_fused_range_flag(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import ramp_rectangles
    torch = torch_cuda
    f = _gpu(torch, ramp_rectangles(100, 140, seed=2))
    ws = torch.empty(bf.workspace_bytes(100, 140, 5.0, 28, "f16"), dtype=torch.uint8, device="cuda:0")
    bf.gc_filter(f, 5.0, 30.0, 28, stack_dtype="f16", workspace=ws)
    assert bf.read_flags(ws) == 0
    for r, c in ((99, 139), (0, 0), (70, 3)):
        g = f.clone()
        g[r, c] = 256.0
        bf.gc_filter(g, 5.0, 30.0, 28, stack_dtype="f16", workspace=ws)
        assert bf.read_flags(ws) & bf.DEVFLAG_RANGE, (r, c)
    g = f.clone()
    g[40, 77] = float("nan")
    bf.gc_filter(g, 5.0, 30.0, 28, stack_dtype="f16", workspace=ws)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE


def test_fused_range_flag_follows_the_last_call(torch_cuda):
    """The fused kernel reports the range per block (nothing to clear first);
    the flag read always describes the workspace's last call, whichever path
    or image size it took."""
    import paper_1605_02178_amd as bf
    from synth import ramp_rectangles
    torch = torch_cuda
    f = _gpu(torch, ramp_rectangles(200, 260, seed=3))
    bad = f.clone()
    bad[150, 250] = -1.0
    small = f[:70, :90].contiguous()
    ws = torch.empty(bf.workspace_bytes(200, 260, 5.0, 28, "f16"), dtype=torch.uint8, device="cuda:0")
    steps = [(bad, bf.TILE_FUSED, True), (f, bf.TILE_FUSED, False), (bad, 0, True), (f, bf.TILE_FUSED, False),
             (bad, bf.TILE_FUSED, True), (f, 0, False), (bad, bf.TILE_FUSED, True), (small, bf.TILE_FUSED, False)]
    for k, (img, cfg, flagged) in enumerate(steps):
        bf.gc_filter(img, 5.0, 30.0, 28, stack_dtype="f16", workspace=ws, tile_config=cfg)
        got = bf.read_flags(ws) & bf.DEVFLAG_RANGE
        assert bool(got) == flagged, (k, cfg, flagged)


@pytest.mark.parametrize("N", [28, 30, 31, 32])
def test_fused_headline_size_sampled(torch_cuda, N):
    """4096^2 edge-rich, sigma_s = 10, sigma_r = 30, FP16 stack, fused tile (the
    configuration the benchmark times for the FP16 stack): the oracle on a
    512^2 centre crop and three 96^2 corner crops."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(4096, 4096, seed=3).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), 10.0, 30.0, N, stack_dtype="f16", tile_config=bf.TILE_FUSED))
    for reg in ((1792, 2304, 1792, 2304), (0, 96, 0, 96), (4000, 4096, 4000, 4096), (0, 96, 4000, 4096)):
        ref = C.gcf(f, 10.0, 30.0, N, region=reg)
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - ref).max()
        _log(f"fused f16 N={N} 4096^2 crop {reg}: {err:.3e}")
        assert err <= BOUND[("f16", 30.0, N)]


@pytest.mark.parametrize("dtype,sigma_r,N", [("f16", 30.0, 30), ("bf16", 50.0, 11)])
@pytest.mark.parametrize("sigma_s", [10.0, 15.0])
def test_fused_persistent_ragged_sampled(torch_cuda, dtype, sigma_r, N, sigma_s):
    """A ragged 1100 x 2050 image with more tiles than resident blocks (W = 30:
    594 tiles of 64 x 64; W = 45: 1170 of 64 x 32), in both launch forms:
    FP16, one block per tile with two blocks per CU; BF16, persistent blocks
    that run several tiles each with the next one's halo in flight. The
    oracle on crops at the four corners (ragged ones included), the centre
    and a tile seam."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(1100, 2050, seed=41).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), sigma_s, sigma_r, N, stack_dtype=dtype, tile_config=bf.TILE_FUSED))
    assert np.isfinite(y).all()
    for reg in ((0, 70, 0, 70), (0, 70, 1980, 2050), (1030, 1100, 0, 70), (1030, 1100, 1980, 2050),
                (500, 580, 990, 1070), (630, 650, 0, 2050)):
        ref = C.gcf(f, sigma_s, sigma_r, N, region=reg)
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - ref).max()
        _log(f"fused {dtype} 1100x2050 sigma_s={sigma_s} crop {reg}: {err:.3e}")
        assert err <= BOUND[(dtype, sigma_r, N)]


@pytest.mark.parametrize("shape,seed", [((4096, 4096), 3), ((1100, 2050), 41)])
def test_fused_f16_wide_radius_sampled(torch_cuda, shape, seed):
    """FP16 at sigma_s = 20 (W = 60: 32 x 128 tiles on 16 waves, the fused
    tile's widest geometry) at N = 32: the 4096^2 headline image and a ragged
    1100 x 2050 image against the oracle on crops at the corners, the centre
    and a tile seam."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    H, Wd = shape
    f = edge_rich(H, Wd, seed=seed).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), 20.0, 30.0, 32, stack_dtype="f16", tile_config=bf.TILE_FUSED))
    assert np.isfinite(y).all()
    for reg in ((0, 70, 0, 70), (0, 70, Wd - 70, Wd), (H - 70, H, 0, 70), (H - 70, H, Wd - 70, Wd),
                (H // 2 - 40, H // 2 + 40, Wd // 2 - 40, Wd // 2 + 40), (30, 34, 0, Wd)):
        ref = C.gcf(f, 20.0, 30.0, 32, region=reg)
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - ref).max()
        _log(f"fused f16 W=60 {shape} crop {reg}: {err:.3e}")
        assert err <= BOUND[("f16", 30.0, 32)]


# Images with many more 64-row tiles than CUs: the single-image FP16 kernel
# then runs strips of several tiles per block (each tile after a strip's
# first reuses two halo chunks of the tile above and loads the other two
# during that tile's planes). (shape, sigma_s): Q = 4 (W = 30) and Q = 3
# (W = 12), ragged in both directions.
STRIP_SHAPES = [((4096, 2048), 10.0), ((4000, 2100), 10.0), ((4030, 2000), 4.0)]


@pytest.mark.parametrize("shape,sigma_s", STRIP_SHAPES)
def test_fused_strips_equal_one_block_per_tile_bitwise(torch_cuda, shape, sigma_s):
    """The strip kernel against the batched fused kernel (one block per tile,
    every tile's halo loaded whole) on the same image: bit for bit, also with
    a row stride; the oracle on crops at the first and last tile rows and
    across a strip seam."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    H, Wd = shape
    f64 = edge_rich(H, Wd, seed=H + Wd).astype(np.float32).astype(np.float64)
    f = _gpu(torch, f64)
    y = bf.gc_filter(f, sigma_s, 30.0, 30, stack_dtype="f16", tile_config=bf.TILE_FUSED)
    outs, status = bf.gc_filter_batched([f], [sigma_s], [30.0], [30], stack_dtype="f16", graph=False,
                                        tile_config=bf.TILE_FUSED)
    assert status == [0]
    diff = float((outs[0] - y).abs().max())
    _log(f"strips {shape} sigma_s={sigma_s}: against one block per tile {diff:.3e}")
    assert torch.equal(outs[0], y)
    big = torch.full((H, Wd + 40), -1.0, device="cuda:0")
    big[:, :Wd] = f
    out = torch.full((H, Wd + 40), -5.0, device="cuda:0")
    bf.gc_filter(big[:, :Wd], sigma_s, 30.0, 30, stack_dtype="f16", tile_config=bf.TILE_FUSED, out=out[:, :Wd])
    assert torch.equal(out[:, :Wd], y)
    assert bool((out[:, Wd:] == -5.0).all())
    yn = _np(y)
    for reg in ((0, 40, 0, 60), (H - 40, H, Wd - 60, Wd), (H // 2 - 70, H // 2 + 70, 100, 140),
                (1000, 1100, Wd // 2 - 20, Wd // 2 + 20)):
        ref = C.gcf(f64, sigma_s, 30.0, 30, region=reg)
        err = np.abs(yn[reg[0]:reg[1], reg[2]:reg[3]] - ref).max()
        _log(f"strips {shape} sigma_s={sigma_s} crop {reg}: {err:.3e}")
        assert err <= BOUND[("f16", 30.0, 30)]


def test_fused_strips_range_flag_in_later_tiles(torch_cuda):
    """Out-of-range pixels in the second and the last tile of a strip raise
    the range flag; a clean image after them clears it."""
    import paper_1605_02178_amd as bf
    from synth import ramp_rectangles
    torch = torch_cuda
    f = _gpu(torch, ramp_rectangles(4096, 1024, seed=6))
    ws = torch.empty(bf.workspace_bytes(4096, 1024, 10.0, 30, "f16"), dtype=torch.uint8, device="cuda:0")
    bf.gc_filter(f, 10.0, 30.0, 30, stack_dtype="f16", workspace=ws, tile_config=bf.TILE_FUSED)
    assert bf.read_flags(ws) == 0
    for r, c in ((70, 5), (4095, 1023), (2100, 600)):
        g = f.clone()
        g[r, c] = -0.5
        bf.gc_filter(g, 10.0, 30.0, 30, stack_dtype="f16", workspace=ws, tile_config=bf.TILE_FUSED)
        assert bf.read_flags(ws) & bf.DEVFLAG_RANGE, (r, c)
    bf.gc_filter(f, 10.0, 30.0, 30, stack_dtype="f16", workspace=ws, tile_config=bf.TILE_FUSED)
    assert bf.read_flags(ws) == 0


def test_fused_centre_value_pixels(torch_cuda):
    """Pixels equal to t_c = 127.5 have s = 0 (up to the rounding of s), where
    P = (s P)/s would be 0/0; the kernel takes s = 2^-64 there: a constant
    127.5 image stays 127.5, and an image with many such pixels matches the
    oracle."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    for dtype, sr, N in (("f16", 30.0, 28), ("bf16", 50.0, 11)):
        y = bf.gc_filter(torch.full((70, 90), 127.5, device="cuda:0"), 4.0, sr, N, stack_dtype=dtype)
        assert float((y - 127.5).abs().max()) <= 1e-3, dtype
        f = edge_rich(96, 130, seed=31).astype(np.float32)
        rng = np.random.default_rng(31)
        f[rng.random(f.shape) < 0.2] = 127.5
        f64 = f.astype(np.float64)
        out = _np(bf.gc_filter(_gpu(torch, f64), 4.0, sr, N, stack_dtype=dtype))
        err = np.abs(out - C.gcf(f64, 4.0, sr, N)).max()
        _log(f"fused {dtype} with s = 0 pixels: max err {err:.3e}")
        assert np.isfinite(out).all() and err <= BOUND[(dtype, sr, N)]
