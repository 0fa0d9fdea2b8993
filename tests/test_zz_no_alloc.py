"""bf_gc_forward_noalloc, the entry point for callers that cannot allocate
device memory, called through the C ABI (ctypes), against bf_gc_forward on
the same inputs: bit for bit (the same fused kernel; the only difference is
where the range words live), on two calls in a row with the second on a
smaller image, in FP16 and BF16 and on each geometry of the fused tile; the
range flag it writes; its refusals."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _call(torch, lib, f, out, sigma_s, sigma_r, N, dtype, flag=None):
    H, Wd = f.shape
    code = {"f16": 1, "bf16": 2}[dtype]
    return lib.bf_gc_forward_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), H, Wd,
                                     f.stride(0) if H > 1 else Wd, float(sigma_s), float(sigma_r), int(N), code, 0,
                                     ctypes.c_void_p(flag.data_ptr() if flag is not None else 0),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("dtype,sigma_r,N", [("f16", 30.0, 32), ("bf16", 50.0, 11)])
@pytest.mark.parametrize("sigma_s", [3.0, 10.0, 14.0])
def test_noalloc_equals_forward_two_calls(torch_cuda, dtype, sigma_r, N, sigma_s):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    lib = bf._lib.load()
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
    for shape in ((700, 530), (130, 97)):          # the second call on a smaller image
        print(f"noalloc {dtype} ss={sigma_s} {shape}", flush=True)
        f = torch.tensor(edge_rich(*shape, seed=sum(shape)).astype(np.float32), device="cuda:0")
        out = torch.full_like(f, -1.0)
        assert _call(torch, lib, f, out, sigma_s, sigma_r, N, dtype, flag) == 0
        ref = bf.gc_filter(f, sigma_s, sigma_r, N, stack_dtype=dtype, tile_config=bf.TILE_FUSED)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
        assert int(flag.item()) == 0


def test_noalloc_range_flag_and_binding(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    f = torch.tensor(edge_rich(200, 260, seed=9).astype(np.float32), device="cuda:0")
    bad = f.clone()
    bad[150, 250] = 300.0
    flag = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    y = bf.gc_filter_noalloc(bad, 5.0, 30.0, 32, "f16", range_flag=flag)
    assert int(flag.item()) & bf.DEVFLAG_RANGE
    small = f[:70, :90].contiguous()
    y2 = bf.gc_filter_noalloc(small, 5.0, 30.0, 32, "f16", range_flag=flag)
    assert int(flag.item()) == 0
    assert torch.equal(y2, bf.gc_filter(small, 5.0, 30.0, 32, stack_dtype="f16"))
    assert torch.equal(torch.nan_to_num(y), torch.nan_to_num(bf.gc_filter(bad, 5.0, 30.0, 32, stack_dtype="f16")))


def test_noalloc_refusals(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    lib = bf._lib.load()
    f = torch.zeros((64, 64), device="cuda:0")
    out = torch.empty_like(f)
    code = lambda ss, sr, N, dt, flags=0: lib.bf_gc_forward_noalloc(  # noqa: E731
        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), 64, 64, 64, ss, sr, N, dt, flags, None,
        None)
    assert code(3.0, 30.0, 28, 0) == 2               # FP32 stack: not on the fused tile
    assert code(22.0, 30.0, 28, 1) == 2              # FP16 radius 66 > 64
    assert code(17.0, 50.0, 11, 2) == 2              # BF16 radius 51 > 48
    assert code(3.0, 30.0, 28, 1, 0x2) == 1          # staged flag
    assert code(3.0, 30.0, 28, 1, (0 + 1) << 8) == 1  # a three-kernel tile
    assert code(3.0, 12.0, 170, 1) == 3              # ill-conditioned
    # a 32768^2 image needs 8 MiB of range words: refused by size before any pointer is used
    big = 1 << 15
    assert lib.bf_gc_forward_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), big, big,
                                     big, 3.0, 30.0, 28, 1, 0, None, None) == 2
