"""GPU parity of the pivoted form for small sigma_r (bf_gc_forward_pivots)
against the FP64 oracle's pivoted filter, through the C ABI. Bars on the 0-255
scale: FP32 1e-3 (measured at most 7.8e-6, the output's own rounding); FP16
0.02 (measured 5.8e-3)."""
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


def _tol(sigma_r, K):
    import paper_1605_02178_amd as bf
    kappa = max(k for _, _, k in bf.pivot_plan(sigma_r, K))
    return 1e-3, kappa


@pytest.mark.parametrize("shape,sigma_s,sigma_r,K", [((120, 150), 3.0, 10.0, 8), ((120, 150), 3.0, 10.0, 16),
                                                     ((97, 131), 5.0, 15.0, 4), ((65, 129), 2.0, 12.0, 8),
                                                     ((1, 77), 2.0, 10.0, 8), ((129, 5), 1.0, 15.0, 4)])
def test_pivots_fp32_parity(torch_cuda, shape, sigma_s, sigma_r, K):
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from synth import edge_rich
    f = edge_rich(*shape, seed=sum(shape) + K).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), sigma_s, sigma_r, K))
    ref = F.pivot_gcf(f, sigma_s, sigma_r, K)
    err = np.abs(y - ref).max()
    tol, kappa = _tol(sigma_r, K)
    _log(f"pivots f32 {shape} ss={sigma_s} sr={sigma_r} K={K}: {err:.3e} (kappa {kappa:.3g}, tol {tol:.3g})")
    assert err <= tol


def test_one_pivot_is_the_plain_forward(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    f = _gpu(torch_cuda, edge_rich(90, 100, seed=31))
    a = _np(bf.gc_filter_pivots(f, 3.0, 30.0, 1, 28))
    b = _np(bf.gc_filter(f, 3.0, 30.0, 28))
    assert np.abs(a - b).max() <= 1e-5


def test_pivots_every_output_written_boundaries_and_flags(torch_cuda):
    """Values on every sub-range boundary, below 0, above 255 and NaN: every
    output is written exactly by one sub-range (no sentinel survives), the
    in-range ones match the oracle, and the device flag is raised."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from synth import edge_rich
    torch = torch_cuda
    K = 8
    f = edge_rich(64, 80, seed=33).astype(np.float32)
    edges = [255.0 * k / K for k in range(K + 1)]
    f[3, :K + 1] = edges
    clean = f.astype(np.float64)
    ft = _gpu(torch, clean)
    ws = torch.empty(bf.pivots_workspace_bytes(64, 80, 2.0, 10.0, K), dtype=torch.uint8, device="cuda:0")
    out = torch.full_like(ft, -7.0)
    bf.gc_filter_pivots(ft, 2.0, 10.0, K, out=out, workspace=ws)
    assert bf.read_flags(ws) == 0
    y = _np(out)
    assert not (y == -7.0).any()
    tol, _ = _tol(10.0, K)
    assert np.abs(y - F.pivot_gcf(clean, 2.0, 10.0, K)).max() <= tol
    bad = ft.clone()
    bad[10, 10], bad[20, 30], bad[40, 50] = -3.0, 300.0, float("nan")
    out = torch.full_like(ft, -7.0)
    bf.gc_filter_pivots(bad, 2.0, 10.0, K, out=out, workspace=ws)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE
    assert not bool((out == -7.0).any())


def test_pivots_fp16(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from synth import edge_rich
    K = bf.pivot_count(15.0, "f16")
    f = edge_rich(100, 110, seed=35).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), 3.0, 15.0, K, stack_dtype="f16", tile_config=0))
    err = np.abs(y - F.pivot_gcf(f, 3.0, 15.0, K)).max()
    _log(f"pivots f16 (three-kernel tiles) sr=15 K={K}: {err:.3e}")
    assert err <= 0.02


def test_pivot_argument_errors(torch_cuda):
    import ctypes
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.zeros((16, 16), device="cuda:0")
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter_pivots(f, 2.0, 10.0, 8, stack_dtype="f32", tile_config=bf.TILE_FUSED)
    assert e.value.status == 2                          # the fused tile takes 16-bit stacks
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter_pivots(f, 2.0, 10.0, 1)            # the single expansion at sigma_r = 10
    assert e.value.status == 3
    lib = bf._lib.load()
    ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda:0")
    out = torch.empty_like(f)
    args = (ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), 16, 16, 16, 2.0, 10.0)
    tail = (ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert lib.bf_gc_forward_pivots(*args, 0, 0, 0, 0, *tail) == 1       # K = 0
    assert lib.bf_gc_forward_pivots(*args, 65, 0, 0, 0, *tail) == 1      # K > 64
    assert lib.bf_gc_forward_pivots(*args, 8, 0, 0, 0x8, *tail) == 1     # Taylor
    assert bf.pivot_count(10.0, "f32") == 8 and bf.pivot_count(30.0, "f32") == 1


def test_pivots_1024_crops_and_direct_filter(torch_cuda):
    """1024^2 edge-rich, sigma_s = 5, sigma_r = 10 (C3's small-sigma_r column),
    K = 8, FP32: the oracle on a 128^2 centre crop and a corner crop; the
    error against the direct filter (64^2 crop) is at the degree rule's
    level, where the single expansion is refused."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    from oracle import native as C
    from synth import edge_rich
    f = edge_rich(1024, 1024, seed=37).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter_pivots(_gpu(torch_cuda, f), 5.0, 10.0, 8))
    tol, _ = _tol(10.0, 8)
    for reg in ((448, 576, 448, 576), (0, 64, 0, 64)):
        err = np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - F.pivot_gcf(f, 5.0, 10.0, 8, region=reg)).max()
        _log(f"pivots 1024^2 crop {reg}: {err:.3e}")
        assert err <= tol
    d = C.direct_bf(f, 5.0, 10.0, region=(480, 544, 480, 544))
    ed = np.abs(y[480:544, 480:544] - d).max()
    _log(f"pivots 1024^2 vs direct (64^2): {ed:.3e}")
    assert ed <= 0.1
