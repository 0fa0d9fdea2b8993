"""GPU batched form (bf_gc_batched): one graph of three persistent phase
kernels over images of uneven sizes and parameters. Checked bit for bit against the single-image
forward under the same tile configuration, against the FP64 oracle, for the
per-image status of skipped images, and across hipGraph replays with
changing descriptors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _log(msg):
    print(msg, flush=True)


def _batch(seed, n=6):
    from synth import edge_rich
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(20, 300)), int(rng.integers(20, 300))) for _ in range(n)]
    shapes[0] = (1, 77)
    shapes[1] = (129, 5)
    imgs = [edge_rich(h, w, seed=seed + k).astype(np.float32) for k, (h, w) in enumerate(shapes)]
    ss = [float(rng.uniform(0.5, 6.0)) for _ in range(n)]
    sr = [float(rng.uniform(30.0, 60.0)) for _ in range(n)]
    return imgs, ss, sr


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("cfg", [0, 3])
def test_batched_equals_single_image_bitwise(torch_cuda, dtype, graph, cfg):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    imgs, ss, sr = _batch(100 + cfg)
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    degrees = [bf.degree_rule(x) for x in sr]
    outs, status = bf.gc_filter_batched(fs, ss, sr, degrees, stack_dtype=dtype, graph=graph, tile_config=cfg)
    assert status == [0] * len(fs)
    for k, f in enumerate(fs):
        ref = bf.gc_filter(f, ss[k], sr[k], degrees[k], stack_dtype=dtype, tile_config=cfg)
        assert torch.equal(outs[k], ref), (k, f.shape, float((outs[k] - ref).abs().max()))


def test_batched_parity_with_oracle(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    torch = torch_cuda
    imgs, ss, sr = _batch(200, n=5)
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    degrees = [bf.degree_rule(x) for x in sr]
    outs, status = bf.gc_filter_batched(fs, ss, sr, degrees)
    for k in range(len(fs)):
        ref = C.gcf(imgs[k].astype(np.float64), ss[k], sr[k], degrees[k])
        err = np.abs(outs[k].cpu().double().numpy() - ref).max()
        _log(f"batched image {k} {imgs[k].shape} ss={ss[k]:.2f} sr={sr[k]:.1f} N={degrees[k]}: {err:.3e}")
        assert err <= 1e-3


def test_batched_statuses_and_skips(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    imgs, ss, sr = _batch(300, n=4)
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    degrees = [bf.degree_rule(x) for x in sr]
    sr[1], degrees[1] = 12.0, 170          # ill-conditioned in FP32
    ss[2] = -1.0                           # invalid
    outs = [torch.full_like(f, -7.0) for f in fs]
    outs, status = bf.gc_filter_batched(fs, ss, sr, degrees, outs=outs)
    assert status[0] == 0 and status[1] == 3 and status[2] == 1 and status[3] == 0
    assert bool((outs[1] == -7.0).all()) and bool((outs[2] == -7.0).all())
    for k in (0, 3):
        assert torch.equal(outs[k], bf.gc_filter(fs[k], ss[k], sr[k], degrees[k]))
    outs2, status2 = bf.gc_filter_batched(fs, ss, sr, degrees, allow_ill_conditioned=True)
    assert status2[1] == 0 and status2[2] == 1


def test_graph_replays_with_new_descriptors(torch_cuda):
    """The same cached graph is replayed with three different batches of the
    same capacity, with eager work and synchronisation between the replays;
    every replay matches the single-image forward."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    ws = None
    for rep in range(3):
        imgs, ss, sr = _batch(400 + rep, n=5)
        fs = [torch.tensor(a, device="cuda:0") for a in imgs]
        degrees = [bf.degree_rule(x) for x in sr]
        if ws is None:
            need = max(bf.batched_workspace_bytes([a.shape for a in imgs], ss, degrees) for _ in range(1))
            ws = torch.empty(4 * need + (1 << 24), dtype=torch.uint8, device="cuda:0")
        outs, status = bf.gc_filter_batched(fs, ss, sr, degrees, graph=True, workspace=ws)
        junk = torch.randn(1 << 20, device="cuda:0").sum()          # eager work between replays
        torch.cuda.synchronize()
        for k, f in enumerate(fs):
            assert torch.equal(outs[k], bf.gc_filter(f, ss[k], sr[k], degrees[k])), (rep, k)
        assert bf.read_flags(ws) == 0
        del junk


def test_empty_batch_and_single(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    outs, status = bf.gc_filter_batched([], [], [], [])
    assert outs == [] and status == []
    f = torch.tensor(np.full((33, 47), 40.0, dtype=np.float32), device="cuda:0")
    outs, status = bf.gc_filter_batched([f], [2.0], [30.0], [28])
    assert status == [0] and float((outs[0] - 40.0).abs().max()) <= 1e-3
