"""Calls on a side stream (stream=...) while torch's current stream keeps
allocating and writing. Every tensor the binding allocates for such a call
(workspace, outputs, contiguous copies) belongs to the side stream, so the
caching allocator cannot hand a workspace that the call's kernels still use
to work on the current stream. Each output is checked bit for bit against the
same call on the current stream, and a crop against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _scribble(torch, nbytes, rounds=4):
    """Allocations of the workspace's size on the current stream, filled with
    a non-finite pattern: a freed side-stream workspace handed out here would
    be overwritten while the side stream still reads it."""
    keep = []
    for _ in range(rounds):
        t = torch.empty(nbytes // 4 + 1024, dtype=torch.float32, device="cuda:0")
        t.fill_(float("nan"))
        keep.append(t)
    return keep


def test_forward_on_side_stream(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    from synth import edge_rich
    torch = torch_cuda
    f64 = edge_rich(1024, 1024, seed=77).astype(np.float32).astype(np.float64)
    f = torch.tensor(f64, dtype=torch.float32, device="cuda:0")
    ref = bf.gc_filter(f, 5.0, 30.0, 28)              # three-kernel FP32 path: stacks in the workspace
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    nbytes = bf.workspace_bytes(1024, 1024, 5.0, 28)
    for _ in range(3):
        outs.append(bf.gc_filter(f, 5.0, 30.0, 28, stream=side))
        junk = _scribble(torch, nbytes)
        del junk
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for y in outs:
        assert torch.equal(y, ref)
    reg = (448, 576, 448, 576)
    err = np.abs(outs[-1].cpu().double().numpy()[448:576, 448:576] - C.gcf(f64, 5.0, 30.0, 28, region=reg)).max()
    assert err <= 1e-3


def test_batched_and_pivots_on_side_stream(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    imgs = [edge_rich(300 + 40 * k, 400 - 30 * k, seed=90 + k).astype(np.float32) for k in range(4)]
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    ss, sr = [3.0, 5.0, 7.0, 2.0], [30.0, 12.0, 45.0, 20.0]
    deg = [bf.degree_rule(x) for x in sr]
    ref, st = bf.gc_filter_batched(fs, ss, sr, deg, graph=False)
    ref_p = bf.gc_filter_pivots(fs[1], 5.0, 12.0, stack_dtype="f16")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    nbytes = bf.batched_workspace_bytes([a.shape for a in imgs], ss, deg)
    for graph in (False, True):
        outs, st2 = bf.gc_filter_batched(fs, ss, sr, deg, graph=graph, stream=side)
        yp = bf.gc_filter_pivots(fs[1], 5.0, 12.0, stack_dtype="f16", stream=side)
        junk = _scribble(torch, nbytes)
        del junk
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        assert st2 == st == [0, 0, 0, 0]
        for a, b in zip(outs, ref):
            assert torch.equal(a, b)
        assert torch.equal(yp, ref_p)


def test_backward_on_side_stream(torch_cuda):
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    f = torch.tensor(edge_rich(256, 320, seed=5).astype(np.float32), device="cuda:0")
    g = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (256, 320)).astype(np.float32), device="cuda:0")
    rf, rs = bf.gc_backward(f, g, 3.0, 30.0, 28)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    gf, gs = bf.gc_backward(f, g, 3.0, 30.0, 28, stream=side)
    junk = _scribble(torch, bf.workspace_bytes(256, 320, 3.0, 28, for_backward=True))
    del junk
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(gf, rf) and torch.equal(gs, rs)
