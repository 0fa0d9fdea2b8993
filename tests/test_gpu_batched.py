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


@pytest.mark.parametrize("form", ["many", "wide"])
def test_persistent_three_kernel_batch_equals_single_image_bitwise(torch_cuda, form):
    """The persistent column and row phases (more than 256 descriptors, or an
    item table plus the staged tile of the widest radius above 64 KiB) against
    the single-image kernels (LDS-staged), bit for bit."""
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    rng = np.random.default_rng(77 if form == "many" else 78)
    if form == "many":
        shapes = [(int(rng.integers(4, 40)), int(rng.integers(4, 40))) for _ in range(300)]
        ss = [float(rng.uniform(0.5, 3.0)) for _ in shapes]
    else:
        shapes = [(70, 90), (130, 40), (33, 200)]
        ss = [32.0, 2.0, 5.0]                      # W = 96: (64 + 192) x 64 x 4 B of tile alone
    fs = [torch.tensor(edge_rich(h, w, seed=k).astype(np.float32), device="cuda:0") for k, (h, w) in enumerate(shapes)]
    sr = [float(rng.uniform(30.0, 60.0)) for _ in shapes]
    degrees = [bf.degree_rule(x) for x in sr]
    outs, status = bf.gc_filter_batched(fs, ss, sr, degrees, stack_dtype="f32", tile_config=0)
    assert status == [0] * len(fs)
    for k, f in enumerate(fs):
        ref = bf.gc_filter(f, ss[k], sr[k], degrees[k], stack_dtype="f32", tile_config=0)
        assert torch.equal(outs[k], ref), (k, f.shape)


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
    sr[1], degrees[1] = 2.0, 100           # ill-conditioned in FP32, and no sub-range count helps
    ss[2] = -1.0                           # invalid
    assert bf.batched_route(2.0, 100, "f32") == 0
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


# sigma_s per geometry class of the fused form: W = 6, 12, 21, 30, 36, 45
FUSED_CLASS_SIGMAS = [2.0, 4.0, 7.0, 10.0, 12.0, 15.0]


def _fused_batch(seed):
    from synth import edge_rich
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(40, 260)), int(rng.integers(40, 260))) for _ in FUSED_CLASS_SIGMAS]
    shapes += [(1, 70), (97, 3), (300, 70)]
    ss = FUSED_CLASS_SIGMAS + [2.0, 1.0, 15.0]
    imgs = [edge_rich(h, w, seed=seed + k).astype(np.float32) for k, (h, w) in enumerate(shapes)]
    return imgs, ss


@pytest.mark.parametrize("dtype,sr,N", [("f16", 30.0, 28), ("bf16", 50.0, 11)])
@pytest.mark.parametrize("graph", [False, True])
def test_fused_batched_equals_single_image_bitwise(torch_cuda, dtype, sr, N, graph):
    """Every geometry class of the fused form in one call; each image equals
    its single-image fused forward bit for bit."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    imgs, ss = _fused_batch(700 + N)
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    outs, status = bf.gc_filter_batched(fs, ss, [sr] * len(fs), [N] * len(fs), stack_dtype=dtype, graph=graph)
    assert status == [0] * len(fs)
    for k, f in enumerate(fs):
        ref = bf.gc_filter(f, ss[k], sr, N, stack_dtype=dtype, tile_config=bf.TILE_FUSED)
        assert torch.equal(outs[k], ref), (k, f.shape, ss[k], float((outs[k] - ref).abs().max()))


def test_fused_batched_parity_statuses_and_fallback(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import native as C
    torch = torch_cuda
    imgs, ss = _fused_batch(800)
    imgs, ss = imgs[:4], ss[:4]
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    sr = [30.0, 30.0, 50.0, 30.0]
    deg = [28, 28, 11, 30]
    outs, status = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype="f16")
    assert status == [0, 0, 0, 0]
    for k in range(4):
        err = np.abs(outs[k].cpu().double().numpy() - C.gcf(imgs[k].astype(np.float64), ss[k], sr[k], deg[k])).max()
        _log(f"fused batched image {k} {imgs[k].shape} ss={ss[k]} sr={sr[k]} N={deg[k]}: {err:.3e}")
        assert err <= (0.5 if sr[k] == 50.0 else 2.5)
    # an image with radius above 48: explicit fused tile skips it, the default
    # runs the whole batch through the three-kernel form
    big = torch.tensor(imgs[0], device="cuda:0")
    fs2 = fs[:2] + [big]
    ss2 = ss[:2] + [17.0]
    pre = [torch.full_like(x, -3.0) for x in fs2]
    outs2, st2 = bf.gc_filter_batched(fs2, ss2, [30.0] * 3, [28] * 3, stack_dtype="f16",
                                      tile_config=bf.TILE_FUSED, outs=pre)
    assert st2 == [0, 0, 2] and bool((outs2[2] == -3.0).all())
    outs3, st3 = bf.gc_filter_batched(fs2, ss2, [30.0] * 3, [28] * 3, stack_dtype="f16")
    assert st3 == [0, 0, 0]
    for k in range(3):
        assert torch.equal(outs3[k], bf.gc_filter(fs2[k], ss2[k], 30.0, 28, stack_dtype="f16", tile_config=0))


def test_fused_batched_graph_replays(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    ws = None
    for rep in range(3):
        imgs, ss = _fused_batch(900 + rep)
        fs = [torch.tensor(a, device="cuda:0") for a in imgs]
        if ws is None:
            ws = torch.empty(4 * bf.batched_workspace_bytes([a.shape for a in imgs], ss, [28] * len(fs), "f16")
                             + (1 << 24), dtype=torch.uint8, device="cuda:0")
        outs, status = bf.gc_filter_batched(fs, ss, [30.0] * len(fs), [28] * len(fs), stack_dtype="f16",
                                            graph=True, workspace=ws)
        junk = torch.randn(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert status == [0] * len(fs)
        for k, f in enumerate(fs):
            assert torch.equal(outs[k], bf.gc_filter(f, ss[k], 30.0, 28, stack_dtype="f16")), (rep, k)
        assert bf.read_flags(ws) == 0
        del junk


# Images routed to the pivoted form: sigma_r below the stack type's domain,
# one per geometry class of the fused tile, plus ragged and degenerate shapes.
ROUTED_SIGMAS = [(2.0, 12.0), (4.0, 15.0), (7.0, 20.0), (10.0, 12.0), (12.0, 25.0), (15.0, 10.0),
                 (2.0, 20.0), (1.0, 15.0), (15.0, 12.0)]


def _routed_batch(seed):
    from synth import edge_rich
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(40, 260)), int(rng.integers(40, 260))) for _ in range(6)]
    shapes += [(1, 70), (97, 3), (300, 70)]
    imgs = [edge_rich(h, w, seed=seed + k).astype(np.float32) for k, (h, w) in enumerate(shapes)]
    ss = [a for a, _ in ROUTED_SIGMAS]
    sr = [b for _, b in ROUTED_SIGMAS]
    return imgs, ss, sr


@pytest.mark.parametrize("dtype,cfg", [("f16", None), ("bf16", None), ("f32", 0), ("f32", 3), ("f16", 0)])
@pytest.mark.parametrize("graph", [False, True])
def test_routed_images_equal_pivoted_forward_bitwise(torch_cuda, dtype, cfg, graph):
    """Images whose own expansion is ill-conditioned for the stack type run
    the pivoted form inside the batch, next to plain images; each equals
    bf_gc_forward_pivots with the route's sub-range count (rule degrees) bit
    for bit under the same tile configuration (fused tile for the 16-bit
    stacks by default, three-kernel tiles with cfg)."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    imgs, ss, sr = _routed_batch(1100)
    # two plain images in the same call
    imgs += [imgs[0].copy(), imgs[3].copy()]
    ss += [3.0, 9.0]
    sr += [50.0, 60.0]
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    deg = [bf.degree_rule(x) for x in sr]
    routes = [bf.batched_route(sr[k], deg[k], dtype) for k in range(len(fs))]
    _log(f"routes {dtype}: {routes}")
    assert all(r >= 2 for r in routes[:-2]) and routes[-2:] == [1, 1]
    outs, status = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype=dtype, graph=graph, tile_config=cfg)
    assert status == [0] * len(fs)
    for k, f in enumerate(fs):
        if routes[k] == 1:
            ref = bf.gc_filter(f, ss[k], sr[k], deg[k], stack_dtype=dtype, tile_config=cfg)
        else:
            ref = bf.gc_filter_pivots(f, ss[k], sr[k], K=routes[k], stack_dtype=dtype, tile_config=cfg)
        assert torch.equal(outs[k], ref), (k, f.shape, ss[k], sr[k], float((outs[k] - ref).abs().max()))


def test_routed_images_graph_replays_and_flags(torch_cuda):
    """One cached graph replayed over three routed batches (eager work between
    replays), each replay against the pivoted forward; then a batch with an
    out-of-range pixel in a routed image raises the range flag."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    ws = None
    for rep in range(3):
        imgs, ss, sr = _routed_batch(1200 + rep)
        fs = [torch.tensor(a, device="cuda:0") for a in imgs]
        deg = [bf.degree_rule(x) for x in sr]
        if ws is None:
            ws = torch.empty(4 * bf.batched_workspace_bytes([a.shape for a in imgs], ss, deg, "f16", sigmas_r=sr)
                             + (1 << 24),
                             dtype=torch.uint8, device="cuda:0")
        outs, status = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype="f16", graph=True, workspace=ws)
        junk = torch.randn(1 << 20, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert status == [0] * len(fs)
        for k, f in enumerate(fs):
            K = bf.batched_route(sr[k], deg[k], "f16")
            assert torch.equal(outs[k], bf.gc_filter_pivots(f, ss[k], sr[k], K=K, stack_dtype="f16")), (rep, k)
        assert bf.read_flags(ws) == 0
        del junk
    imgs, ss, sr = _routed_batch(1300)
    imgs[3][5, 7] = 300.0
    fs = [torch.tensor(a, device="cuda:0") for a in imgs]
    deg = [bf.degree_rule(x) for x in sr]
    outs, status = bf.gc_filter_batched(fs, ss, sr, deg, stack_dtype="f16", graph=True, workspace=ws)
    assert status == [0] * len(fs)
    assert bf.read_flags(ws) & bf.DEVFLAG_RANGE
    K = bf.batched_route(sr[3], deg[3], "f16")
    ref = bf.gc_filter_pivots(fs[3], ss[3], sr[3], K=K, stack_dtype="f16")
    assert torch.equal(torch.nan_to_num(outs[3]), torch.nan_to_num(ref))
