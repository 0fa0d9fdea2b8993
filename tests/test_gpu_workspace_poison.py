"""Every path on a workspace filled with 0xFF bytes (NaN in FP16, FP32 and
FP64) against the same call on a zeroed workspace: outputs equal bit for bit,
and the range flag of a clean input reads 0. So no path reads workspace
memory it has not written in the same call (flag words, parameter blocks,
stacks, range words, sub-range tables and masks, queue counters, batch
blobs, adjoint planes and partial sums)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _two(torch, nbytes):
    poisoned = torch.full((max(nbytes, 256),), 255, dtype=torch.uint8, device="cuda:0")
    zeroed = torch.zeros((max(nbytes, 256),), dtype=torch.uint8, device="cuda:0")
    return poisoned, zeroed


def _image(shape, seed):
    from synth import edge_rich
    return edge_rich(*shape, seed=seed).astype(np.float32)


CASES = [
    ("three-kernel f32", dict(stack_dtype="f32")),
    ("staged f32", dict(stack_dtype="f32", staged=True)),
    ("three-kernel f16", dict(stack_dtype="f16", tile_config=0)),
    ("fused f16", dict(stack_dtype="f16")),
    ("fused bf16", dict(stack_dtype="bf16")),
    ("recursive f32", dict(stack_dtype="f32", recursive=True)),
]


@pytest.mark.parametrize("name,kw", CASES)
def test_forward_paths(torch_cuda, name, kw):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.tensor(_image((150, 170), 1), device="cuda:0")
    sr, N = (30.0, 32) if kw["stack_dtype"] == "f16" else (50.0, 11) if kw["stack_dtype"] == "bf16" else (30.0, 28)
    ws_p, ws_z = _two(torch, bf.workspace_bytes(150, 170, 4.0, N, kw["stack_dtype"]))
    a = bf.gc_filter(f, 4.0, sr, N, workspace=ws_p, **kw)
    fa = bf.read_flags(ws_p)
    b = bf.gc_filter(f, 4.0, sr, N, workspace=ws_z, **kw)
    assert torch.equal(a, b), name
    assert fa == 0 and bf.read_flags(ws_z) == 0


@pytest.mark.parametrize("dtype,cfg", [("f32", None), ("f16", None), ("bf16", None), ("f16", 0)])
def test_pivots(torch_cuda, dtype, cfg):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.tensor(_image((140, 200), 2), device="cuda:0")
    K = bf.pivot_count(12.0, dtype)
    ws_p, ws_z = _two(torch, bf.pivots_workspace_bytes(140, 200, 5.0, 12.0, K, None, dtype))
    a = bf.gc_filter_pivots(f, 5.0, 12.0, K, stack_dtype=dtype, workspace=ws_p, tile_config=cfg)
    fa = bf.read_flags(ws_p)
    b = bf.gc_filter_pivots(f, 5.0, 12.0, K, stack_dtype=dtype, workspace=ws_z, tile_config=cfg)
    assert torch.equal(a, b) and fa == 0


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_joint(torch_cuda, dtype):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.tensor(_image((120, 160), 3), device="cuda:0")
    g = torch.tensor(_image((120, 160), 4), device="cuda:0")
    sr, N = (50.0, 11) if dtype == "bf16" else (30.0, 28)
    ws_p, ws_z = _two(torch, bf.joint_workspace_bytes(120, 160, 3.0, N, dtype))
    a = bf.gc_joint_filter(f, g, 3.0, sr, N, stack_dtype=dtype, workspace=ws_p)
    fa = bf.read_flags(ws_p)
    b = bf.gc_joint_filter(f, g, 3.0, sr, N, stack_dtype=dtype, workspace=ws_z)
    assert torch.equal(a, b) and fa == 0


@pytest.mark.parametrize("dtype,cfg", [("f32", None), ("f16", None), ("bf16", None), ("f16", 3)])
def test_batched(torch_cuda, dtype, cfg):
    """Plain and routed images (sigma_r 12 and 20 are outside every stack's
    accuracy domain here), with and without the graph."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    shapes = [(90, 130), (1, 50), (200, 64), (64, 200), (77, 77)]
    fs = [torch.tensor(_image(s, 10 + k), device="cuda:0") for k, s in enumerate(shapes)]
    ss = [2.0, 1.0, 7.0, 12.0, 4.0]
    sr = [30.0, 50.0, 12.0, 20.0, 45.0]
    deg = [bf.degree_rule(x) for x in sr]
    need = bf.batched_workspace_bytes(shapes, ss, deg, dtype, sigmas_r=sr)
    for graph in (False, True):
        ws_p, ws_z = _two(torch, need)
        a, sa = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype=dtype, graph=graph, tile_config=cfg,
                                     workspace=ws_p)
        fa = bf.read_flags(ws_p)
        b, sb = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype=dtype, graph=graph, tile_config=cfg,
                                     workspace=ws_z)
        assert sa == sb == [0] * len(fs)
        assert all(torch.equal(x, y) for x, y in zip(a, b)) and fa == 0


def test_backward(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.tensor(_image((96, 110), 5), device="cuda:0")
    g = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (96, 110)).astype(np.float32), device="cuda:0")
    ws_p, ws_z = _two(torch, bf.workspace_bytes(96, 110, 3.0, 28, for_backward=True))
    ga, sa = bf.gc_backward(f, g, 3.0, 30.0, 28, workspace=ws_p)
    gb, sb = bf.gc_backward(f, g, 3.0, 30.0, 28, workspace=ws_z)
    assert torch.equal(ga, gb) and torch.equal(sa, sb)


def test_saving_pair(torch_cuda):
    """The saving forward and its backward (flag word, parameters, per-tile
    partial sums in the workspace) on a 0xFF workspace and a zeroed one."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    x = torch.tensor(np.stack([_image((70, 90), 7 + b) for b in range(2)]), device="cuda:0")
    g = torch.tensor(np.random.default_rng(7).uniform(-1, 1, (2, 70, 90)).astype(np.float32), device="cuda:0")
    ws_p, ws_z = _two(torch, bf.saving_workspace_bytes(2, 70, 90, 3.0, 28))
    ya, sva = bf.gc_forward_saving(x, 3.0, 30.0, 28, workspace=ws_p)
    yb, svb = bf.gc_forward_saving(x, 3.0, 30.0, 28, workspace=ws_z)
    assert torch.equal(ya, yb) and torch.equal(sva, svb)
    assert bf.read_flags(ws_p) == 0
    ga, sa = bf.gc_backward_saving(x, g, sva, 3.0, 30.0, 28, workspace=ws_p)
    gb, sb = bf.gc_backward_saving(x, g, svb, 3.0, 30.0, 28, workspace=ws_z)
    assert torch.equal(ga, gb) and torch.equal(sa, sb)
