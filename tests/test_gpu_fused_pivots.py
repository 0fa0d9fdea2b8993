"""GPU parity of the pivoted form on the fused matrix-core tile
(bf_gc_forward_pivots with BF_TILE_FUSED, the default for 16-bit stacks with
radius <= 48) against the FP64 oracle's pivoted filter, through the C ABI.

Each 64-row tile runs only the sub-ranges its own output pixels fall in, so
the cases include tiles that hold one sub-range, tiles that hold all of them,
pixels on every sub-range boundary, every geometry class of the fused tile
(W = 6, 12, 21, 30, 36, 45), ragged tails and images narrower or shorter than
the radius. Bars on the 0-255 scale, about three times the largest error
measured over these tests: FP16 0.02 (measured 6.95e-3), BF16 0.12 (measured
3.95e-2); every sub-range has kappa near 1, so its rounding stays near the
stack's own unit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BAR = {"f16": 0.02, "bf16": 0.12}


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


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("shape,sigma_s,sigma_r", [((150, 200), 2.0, 10.0), ((131, 97), 4.0, 12.0),
                                                   ((140, 190), 7.0, 10.0), ((150, 170), 10.0, 15.0),
                                                   ((133, 120), 12.0, 10.0), ((160, 110), 15.0, 20.0)])
def test_fused_pivots_parity(torch_cuda, dtype, shape, sigma_s, sigma_r):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(*shape, seed=sum(shape) + int(sigma_s)).astype(np.float32).astype(np.float64)
    K = bf.pivot_count(sigma_r, dtype)
    _log(f"fused pivots {dtype} {shape} ss={sigma_s} sr={sigma_r} K={K}")
    y = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), sigma_s, sigma_r, K, stack_dtype=dtype,
                                tile_config=bf.TILE_FUSED))
    err = np.abs(y - C.pivot_gcf(f, sigma_s, sigma_r, K)).max()
    _log(f"  max-abs vs oracle {err:.3e} (bar {BAR[dtype]})")
    assert np.isfinite(err) and err <= BAR[dtype]


def test_fused_pivots_match_three_kernel_tiles(torch_cuda):
    """The same sub-ranges through the three-kernel tiles (per-plane scales)
    and the fused tile (one geometric scale): both within the bar of the
    oracle, and of each other."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(200, 230, seed=41).astype(np.float32).astype(np.float64)
    K = bf.pivot_count(10.0, "f16")
    ft = _gpu(torch_cuda, f)
    a = _np(bf.gc_filter_pivots(ft, 5.0, 10.0, K, stack_dtype="f16", tile_config=bf.TILE_FUSED))
    b = _np(bf.gc_filter_pivots(ft, 5.0, 10.0, K, stack_dtype="f16", tile_config=0))
    ref = C.pivot_gcf(f, 5.0, 10.0, K)
    ea, eb, eab = (float(np.abs(x).max()) for x in (a - ref, b - ref, a - b))
    _log(f"fused pivots K={K}: fused {ea:.3e}, three-kernel {eb:.3e}, between {eab:.3e}")
    assert ea <= BAR["f16"] and eb <= BAR["f16"] and eab <= BAR["f16"]


def test_fused_pivots_tiles_with_one_and_all_subranges(torch_cuda):
    """Tile-aligned blocks: constant blocks at values on and between the
    sub-range ends (each tile holds one sub-range; the output of a constant
    block's interior is the constant), and blocks holding a ramp over
    0..255 (each tile holds every sub-range)."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    K = 32
    H, Wd = 192, 256
    f = np.zeros((H, Wd), np.float64)
    vals = [255.0 * k / K for k in range(K + 1)] + [3.3, 100.7, 254.9]
    for by in range(3):
        for bx in range(4):
            blk = f[64 * by:64 * by + 64, 64 * bx:64 * bx + 64]
            if (by + bx) % 2 == 0:
                blk[:] = vals[(5 * by + 7 * bx) % len(vals)]
            else:
                r, c = np.mgrid[0:64, 0:64]
                blk[:] = np.round(((r * 64 + c) * 255.0 / 4095.0) * 4) / 4
    out = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), 2.0, 10.0, K, stack_dtype="f16",
                                  tile_config=bf.TILE_FUSED))
    ref = C.pivot_gcf(f, 2.0, 10.0, K)
    err = np.abs(out - ref).max()
    _log(f"fused pivots one/all sub-ranges per tile: {err:.3e}")
    assert err <= BAR["f16"]
    for by in range(3):
        for bx in range(4):
            if (by + bx) % 2 == 0:
                v = vals[(5 * by + 7 * bx) % len(vals)]
                inner = out[64 * by + 8:64 * by + 56, 64 * bx + 8:64 * bx + 56]
                assert np.abs(inner - v).max() <= 0.25, (by, bx, v)


@pytest.mark.parametrize("shape,sigma_s", [((1, 77), 2.0), ((129, 5), 1.0), ((33, 40), 15.0), ((70, 64), 10.0)])
def test_fused_pivots_small_and_ragged(torch_cuda, shape, sigma_s):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(*shape, seed=43 + shape[0]).astype(np.float32).astype(np.float64)
    K = bf.pivot_count(10.0, "f16")
    y = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), sigma_s, 10.0, K, stack_dtype="f16",
                                tile_config=bf.TILE_FUSED))
    err = np.abs(y - C.pivot_gcf(f, sigma_s, 10.0, K)).max()
    _log(f"fused pivots {shape} ss={sigma_s}: {err:.3e}")
    assert err <= BAR["f16"]


def test_fused_pivots_boundaries_flags_and_every_output(torch_cuda):
    """Pixels on every sub-range end match the oracle; values below 0, above
    255 and NaN raise the range flag, every output is written, and a clean
    call on the same workspace clears it."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    K = 32
    f = edge_rich(96, 150, seed=45).astype(np.float32)
    f[5, :K + 1] = [255.0 * k / K for k in range(K + 1)]
    clean = f.astype(np.float64)
    ft = _gpu(torch, clean)
    ws = torch.empty(bf.pivots_workspace_bytes(96, 150, 3.0, 10.0, K, None, "f16"), dtype=torch.uint8,
                     device="cuda:0")
    bad = ft.clone()
    bad[10, 10], bad[20, 130], bad[70, 50] = -3.0, 300.0, float("nan")
    out = torch.full_like(ft, -7.0)
    bf.gc_filter_pivots(bad, 3.0, 10.0, K, stack_dtype="f16", tile_config=bf.TILE_FUSED, out=out, workspace=ws)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE
    assert not bool((out == -7.0).any())
    out = torch.full_like(ft, -7.0)
    bf.gc_filter_pivots(ft, 3.0, 10.0, K, stack_dtype="f16", tile_config=bf.TILE_FUSED, out=out, workspace=ws)
    assert bf.read_flags(ws) == 0
    y = _np(out)
    err = np.abs(y - C.pivot_gcf(clean, 3.0, 10.0, K)).max()
    _log(f"fused pivots boundaries: {err:.3e}")
    assert err <= BAR["f16"]


def test_fused_pivots_errors_and_fallback(torch_cuda):
    import ctypes
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    f = _gpu(torch, edge_rich(80, 90, seed=47))
    with pytest.raises(bf.BFError) as e:          # radius 51 > 48
        bf.gc_filter_pivots(f, 17.0, 10.0, 32, stack_dtype="f16", tile_config=bf.TILE_FUSED)
    assert e.value.status == 2
    a = bf.gc_filter_pivots(f, 17.0, 10.0, 32, stack_dtype="f16")            # default: three-kernel tiles
    b = bf.gc_filter_pivots(f, 17.0, 10.0, 32, stack_dtype="f16", tile_config=0)
    assert torch.equal(a, b)
    a = bf.gc_filter_pivots(f, 3.0, 10.0, 32, stack_dtype="f16")             # default: the fused tile
    b = bf.gc_filter_pivots(f, 3.0, 10.0, 32, stack_dtype="f16", tile_config=bf.TILE_FUSED)
    assert torch.equal(a, b)
    lib = bf._lib.load()
    need = bf.pivots_workspace_bytes(80, 90, 3.0, 10.0, 32, None, "f16")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    out = torch.empty_like(f)
    st = lib.bf_gc_forward_pivots(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), 80, 90, 90, 3.0,
                                  10.0, 32, 0, 1, bf.flag_tile(bf.TILE_FUSED), ctypes.c_void_p(ws.data_ptr()),
                                  need - 256, None)
    assert st == 4                                 # BF_ERR_WORKSPACE


def test_fused_pivots_4096_sampled(torch_cuda):
    """4096^2 edge-rich, sigma_s = 10, sigma_r = 10, FP16, K = 32 (the
    small-sigma_r workload timed by the benchmark): the oracle on a centre
    crop and two corner crops."""
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(4096, 4096, seed=3).astype(np.float32).astype(np.float64)
    K = bf.pivot_count(10.0, "f16")
    y = bf.gc_filter_pivots(_gpu(torch_cuda, f), 10.0, 10.0, K, stack_dtype="f16")
    for reg in ((1984, 2112, 1984, 2112), (0, 96, 0, 96), (4000, 4096, 4020, 4096)):
        err = np.abs(_np(y[reg[0]:reg[1], reg[2]:reg[3]]) - C.pivot_gcf(f, 10.0, 10.0, K, region=reg)).max()
        _log(f"fused pivots 4096^2 crop {reg}: {err:.3e}")
        assert err <= BAR["f16"]
