"""GPU backward (bf_gc_backward, GaussChebyshevBF) against the FP64 gradient
oracle (torch autograd of the paper's algorithm) and against central finite
differences of the FP64 C oracle.

Also the saving forward and the backward from its sums (gc_forward_saving,
gc_backward_saving), and that pair against the recomputing backward.

Stated bounds (stack recomputed in FP64, FP64 adjoint planes, FP64 sums):
  dL/df       max |gpu - oracle| <= 1e-6 * max |oracle|
  dL/dsigma_r |gpu - oracle| <= 1e-6 * |oracle| + 1e-9 * sum |ybar|
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda:0")


def _log(msg):
    print(msg, flush=True)


CASES = [
    ((48, 40), 2.0, 30.0, 28),
    ((37, 53), 1.5, 40.0, 16),
    ((9, 70), 4.0, 30.0, 28),      # W = 12 > height
    ((1, 33), 1.0, 30.0, 28),
    ((64, 64), 0.3, 25.0, 40),
    # radii above 16: the staged passes over FP64 plane stacks (LDS-staged up to
    # W = 32, unstaged above)
    ((40, 58), 6.0, 30.0, 20),     # W = 18
    ((75, 36), 11.0, 30.0, 16),    # W = 33 > width
]


@pytest.mark.parametrize("shape,sigma_s,sigma_r,N", CASES)
def test_backward_matches_fp64_oracle(torch_cuda, shape, sigma_s, sigma_r, N):
    import paper_1605_02178_amd as bf
    from oracle import adjoint as A
    from synth import edge_rich
    torch = torch_cuda
    f = edge_rich(*shape, seed=sum(shape) + 40).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(sum(shape))
    ybar = rng.uniform(-1, 1, size=shape).astype(np.float32).astype(np.float64)
    gf, gs = bf.gc_backward(_gpu(torch, f), _gpu(torch, ybar), sigma_s, sigma_r, N)
    rf, rs = A.gcf_grad(f, sigma_s, sigma_r, N, ybar)
    ef = np.abs(gf.cpu().double().numpy() - rf).max()
    es = abs(float(gs.item()) - rs)
    _log(f"{shape} ss={sigma_s} sr={sigma_r} N={N}: |dL/df| err {ef:.3e} (max {np.abs(rf).max():.3e}); "
         f"dL/dsr gpu {float(gs.item()):.6e} oracle {rs:.6e}")
    assert ef <= REL * np.abs(rf).max()
    assert es <= REL * abs(rs) + 1e-9 * np.abs(ybar).sum()


def test_autograd_function_batch(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import adjoint as A
    from synth import edge_rich
    torch = torch_cuda
    imgs = np.stack([edge_rich(40, 36, seed=60 + b) for b in range(2)]).astype(np.float32)
    tgt = np.random.default_rng(61).uniform(0, 255, size=imgs.shape).astype(np.float32)
    f = _gpu(torch, imgs[:, None]).requires_grad_(True)
    sr = torch.tensor(30.0, dtype=torch.float64, device="cuda:0", requires_grad=True)
    y = bf.gc_filter_autograd(f, sr, 2.0, 28)
    loss = ((y - _gpu(torch, tgt[:, None])) ** 2).mean()
    loss.backward()
    ybar = (2.0 * (y.detach() - _gpu(torch, tgt[:, None])) / y.numel()).cpu().double().numpy()
    gsum = 0.0
    for b in range(2):
        rf, rs = A.gcf_grad(imgs[b].astype(np.float64), 2.0, 30.0, 28, ybar[b, 0])
        assert np.abs(f.grad[b, 0].cpu().double().numpy() - rf).max() <= REL * np.abs(rf).max() + 1e-9
        gsum += rs
    assert abs(float(sr.grad.item()) - gsum) <= REL * abs(gsum) + 1e-9


def test_autograd_sigma_r_without_device_sync(torch_cuda):
    """sigma_r as a CPU tensor, or its value passed as sigma_r_host, gives the
    same outputs and gradients as a device sigma_r; a 16-bit forward gets the
    FP64-recomputed gradient (documented), the same as the FP32 one."""
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    imgs = np.stack([edge_rich(50, 44, seed=70 + b) for b in range(3)]).astype(np.float32)
    res = []
    for mode in ("device", "cpu", "host", "f16"):
        f = _gpu(torch, imgs).requires_grad_(True)
        dev = "cpu" if mode == "cpu" else "cuda:0"
        sr = torch.tensor(30.0, dtype=torch.float64, device=dev, requires_grad=True)
        y = bf.gc_filter_autograd(f, sr, 2.0, 28, stack_dtype="f16" if mode == "f16" else "f32",
                                  sigma_r_host=30.0 if mode == "host" else None)
        (y * y).sum().backward()
        res.append((y.detach(), f.grad, sr.grad.to("cuda:0")))
    for y, gf, gs in res[1:3]:
        assert torch.equal(y, res[0][0]) and torch.equal(gf, res[0][1]) and torch.equal(gs, res[0][2])
    # the 16-bit forward differs in y (rounding) but the gradient formula is the same
    assert float((res[3][0] - res[0][0]).abs().max()) <= 2.5
    with pytest.raises(ValueError):
        bf.gc_filter_autograd(_gpu(torch, imgs), torch.tensor(12.0, dtype=torch.float64), 2.0, 170)


def test_differentiation_workload_finite_differences(torch_cuda):
    """Batch 8 x 1 x 1024 x 1024 edge-rich, sigma_s = 5, sigma_r = 30, N = 28,
    L = mean((y - target)^2), target i.i.d. U[0,255]; forward and backward
    through GaussChebyshevBF. dL/df at 32 seeded pixels against central
    differences (h = 1e-3) of the FP64 C oracle; dL/dsigma_r per image for
    two images against central differences (h = 1e-3) of the same oracle;
    and a 64 x 64 crop run as a standalone image against the FP64 adjoint."""
    import paper_1605_02178_amd as bf
    from oracle import adjoint as A
    from oracle import native as C
    from synth import diff_batch
    torch = torch_cuda
    ss, sr, N = 5.0, 30.0, 28
    W = bf.radius(ss)
    imgs, tgts = diff_batch(8, 1024, 1024)
    imgs = imgs.astype(np.float32).astype(np.float64)
    tgts = tgts.astype(np.float32).astype(np.float64)
    f = _gpu(torch, imgs[:, None]).requires_grad_(True)
    srt = torch.tensor(sr, dtype=torch.float64, device="cuda:0", requires_grad=True)
    y = bf.gc_filter_autograd(f, srt, ss, N)
    nall = y.numel()
    loss = ((y - _gpu(torch, tgts[:, None])) ** 2).mean()
    loss.backward()
    gf = f.grad[:, 0].cpu().double().numpy()
    _log(f"C5 forward+backward done, loss {float(loss.item()):.4f}")

    rng = np.random.default_rng(5200)
    h = 1e-3
    worst = 0.0
    for k in range(32):
        b = int(rng.integers(0, 8))
        i, j = int(rng.integers(0, 1024)), int(rng.integers(0, 1024))
        reg = (max(0, i - W), min(1024, i + W + 1), max(0, j - W), min(1024, j + W + 1))
        t = tgts[b, reg[0]:reg[1], reg[2]:reg[3]]
        vals = []
        for sgn in (1.0, -1.0):
            g = imgs[b].copy()
            g[i, j] += sgn * h
            yy = C.gcf(g, ss, sr, N, region=reg)
            vals.append(np.sum((yy - t) ** 2) / nall)
        fd = (vals[0] - vals[1]) / (2 * h)
        err = abs(gf[b, i, j] - fd)
        worst = max(worst, err / (abs(fd) + 1e-9))
        assert err <= 1e-5 * abs(fd) + 1e-12, (b, i, j, gf[b, i, j], fd)
    _log(f"C5 dL/df vs FD on 32 pixels: worst relative {worst:.3e}")

    for b in range(2):
        ybar = (2.0 * (y.detach()[b, 0] - _gpu(torch, tgts[b])) / nall)
        _, gsb = bf.gc_backward(_gpu(torch, imgs[b]), ybar.float().contiguous(), ss, sr, N)
        vals = []
        for sgn in (1.0, -1.0):
            yy = C.gcf(imgs[b], ss, sr + sgn * h, N)
            vals.append(np.sum((yy - tgts[b]) ** 2) / nall)
        fd = (vals[0] - vals[1]) / (2 * h)
        _log(f"C5 image {b}: dL/dsigma_r gpu {float(gsb.item()):.6e} fd {fd:.6e}")
        assert abs(float(gsb.item()) - fd) <= 1e-5 * abs(fd) + 1e-12

    crop = imgs[0, 480:544, 480:544]
    tcrop = tgts[0, 480:544, 480:544]
    fc = _gpu(torch, crop).requires_grad_(True)
    sc = torch.tensor(sr, dtype=torch.float64, device="cuda:0", requires_grad=True)
    yc = bf.gc_filter_autograd(fc, sc, ss, N)
    lc = ((yc - _gpu(torch, tcrop)) ** 2).mean()
    lc.backward()
    ybar = (2.0 * (yc.detach() - _gpu(torch, tcrop)) / yc.numel()).cpu().double().numpy()
    rf, rs = A.gcf_grad(crop, ss, sr, N, ybar)
    assert np.abs(fc.grad.cpu().double().numpy() - rf).max() <= REL * np.abs(rf).max() + 1e-9
    assert abs(float(sc.grad.item()) - rs) <= REL * abs(rs) + 1e-9


def test_backward_argument_errors(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.zeros((8, 8), device="cuda:0")
    with pytest.raises(bf.BFError):
        bf.gc_backward(f, f.clone(), 2.0, 12.0, 170)          # ill-conditioned
    e = torch.empty((0, 5), device="cuda:0")
    gf, gs = bf.gc_backward(e, e.clone(), 2.0, 30.0, 28)
    assert gf.shape == (0, 5) and float(gs.item()) == 0.0


# Forward with saved sums and the backward from them (count images in one
# launch each). Shapes: several 64 x 32 tiles with ragged edges, one row, one
# column band, radii 1..16 (sigma_s = 5.3: W = 16, the largest).
SAVING_CASES = [
    ((130, 70), 2.0, 30.0, 28),
    ((65, 33), 5.0, 40.0, 16),
    ((1, 40), 1.0, 30.0, 28),
    ((7, 200), 5.3, 30.0, 28),
    ((200, 9), 0.3, 25.0, 40),
]


def _batch(shape, count, seed):
    from synth import edge_rich
    return np.stack([edge_rich(*shape, seed=seed + b) for b in range(count)]).astype(np.float32)


@pytest.mark.parametrize("shape,sigma_s,sigma_r,N", SAVING_CASES)
def test_forward_saving_matches_oracle(torch_cuda, shape, sigma_s, sigma_r, N):
    """y within 1e-5 of the FP64 oracle (the FP32 rounding of a value below
    256 is at most 7.6e-6); the saved Q and t_h P' against the oracle's Q and
    P (eqs. 8-9 in the paper's unscaled form: the scaled coefficients are
    b_n = c_n (t_h / sigma_r)^{2n}, so these sums agree term by term; the
    oracle's Gaussian of eq. 7 is not normalised, the library's taps sum to
    1 along each axis, hence the factor (sum of the 1-D weights)^2) to 1e-11
    of their largest magnitude."""
    import paper_1605_02178_amd as bf
    from oracle import filters as F
    torch = torch_cuda
    imgs = _batch(shape, 3, sum(shape) + 90)
    y, saved = bf.gc_forward_saving(_gpu(torch, imgs), sigma_s, sigma_r, N)
    y = y.cpu().double().numpy()
    saved = saved.cpu().numpy()
    norm = F.spatial_kernel_1d(sigma_s).sum() ** 2
    for b in range(3):
        ref, parts = F.gcf(imgs[b].astype(np.float64), sigma_s, sigma_r, N, return_parts=True)
        ey = np.abs(y[b] - ref).max()
        eq = np.abs(norm * saved[b, 1] - parts["Q"]).max() / np.abs(parts["Q"]).max()
        ep = np.abs(norm * 127.5 * saved[b, 0] - parts["P"]).max() / np.abs(parts["P"]).max()
        _log(f"saving {shape} ss={sigma_s} image {b}: y {ey:.3e}, Q rel {eq:.3e}, P rel {ep:.3e}")
        assert ey <= 1e-5 and eq <= 1e-11 and ep <= 1e-11


@pytest.mark.parametrize("shape,sigma_s,sigma_r,N", SAVING_CASES)
def test_backward_saving_matches_fp64_oracle(torch_cuda, shape, sigma_s, sigma_r, N):
    """Three images in one launch: dL/df per image against the FP64 autograd
    oracle, dL/dsigma_r against the sum of the per-image oracle values."""
    import paper_1605_02178_amd as bf
    from oracle import adjoint as A
    torch = torch_cuda
    imgs = _batch(shape, 3, sum(shape) + 95)
    ybar = np.random.default_rng(sum(shape) + 5).uniform(-1, 1, size=imgs.shape).astype(np.float32)
    x = _gpu(torch, imgs)
    _, saved = bf.gc_forward_saving(x, sigma_s, sigma_r, N)
    gf, gs = bf.gc_backward_saving(x, _gpu(torch, ybar), saved, sigma_s, sigma_r, N)
    gf = gf.cpu().double().numpy()
    rsum = 0.0
    for b in range(3):
        rf, rs = A.gcf_grad(imgs[b].astype(np.float64), sigma_s, sigma_r, N, ybar[b].astype(np.float64))
        ef = np.abs(gf[b] - rf).max()
        assert ef <= REL * np.abs(rf).max(), (b, ef)
        rsum += rs
    _log(f"saving backward {shape} ss={sigma_s}: dL/dsr gpu {float(gs.item()):.6e} oracle {rsum:.6e}")
    assert abs(float(gs.item()) - rsum) <= REL * abs(rsum) + 1e-9 * np.abs(ybar).sum()


def test_saving_pair_equals_recompute_backward(torch_cuda):
    """bf_gc_backward recomputes the same six sums with the same tile kernel,
    so on one image the two backward forms agree bit for bit."""
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    imgs = _batch((150, 100), 1, 123)
    ybar = np.random.default_rng(124).uniform(-1, 1, size=imgs.shape).astype(np.float32)
    x, g = _gpu(torch, imgs), _gpu(torch, ybar)
    _, saved = bf.gc_forward_saving(x, 4.0, 30.0, 28)
    gf, gs = bf.gc_backward_saving(x, g, saved, 4.0, 30.0, 28)
    rf, rs = bf.gc_backward(x[0], g[0], 4.0, 30.0, 28)
    assert torch.equal(gf[0], rf) and torch.equal(gs.reshape(()), rs.reshape(()))


def test_saving_errors_and_empty(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    x = _gpu(torch, _batch((40, 40), 2, 130))
    with pytest.raises(bf.BFError) as e:
        bf.gc_forward_saving(x, 5.4, 30.0, 28)             # W = 17 > 16
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_forward_saving(x, 2.0, 12.0, 170)            # ill-conditioned
    assert e.value.status == 3
    empty = torch.empty((0, 40, 40), device="cuda:0")
    y, saved = bf.gc_forward_saving(empty, 2.0, 30.0, 28)
    assert y.shape == (0, 40, 40) and saved.shape == (0, 6, 40, 40)
    gf, gs = bf.gc_backward_saving(empty, empty.clone(), saved, 2.0, 30.0, 28)
    assert gf.shape == (0, 40, 40) and float(gs.item()) == 0.0
    # the autograd function's f64 form refuses radii above 16, like the call
    with pytest.raises(ValueError):
        bf.gc_filter_autograd(x, torch.tensor(30.0, dtype=torch.float64), 5.4, 28, stack_dtype="f64")


def test_autograd_keep_sums_false_recomputes_identically(torch_cuda):
    """The f64 form with keep_sums=False keeps only f and sigma_r and
    recomputes the sums in the backward with the same kernel: outputs and
    gradients equal the default's bit for bit."""
    import paper_1605_02178_amd as bf
    from synth import edge_rich
    torch = torch_cuda
    imgs = np.stack([edge_rich(70, 90, seed=140 + b) for b in range(3)]).astype(np.float32)
    res = []
    for keep in (True, False):
        f = _gpu(torch, imgs[:, None]).requires_grad_(True)
        sr = torch.tensor(30.0, dtype=torch.float64, device="cuda:0", requires_grad=True)
        y = bf.gc_filter_autograd(f, sr, 3.0, 28, sigma_r_host=30.0, keep_sums=keep)
        (y * y).sum().backward()
        res.append((y.detach(), f.grad, sr.grad))
    assert all(torch.equal(a, b) for a, b in zip(res[0], res[1]))


def test_saving_pair_row_stride_and_image_stride(torch_cuda):
    """Through the C ABI with ld > width and an image stride beyond one image:
    the same outputs, sums and gradients as the contiguous batch, bit for bit;
    the padding columns are left untouched."""
    import ctypes
    import paper_1605_02178_amd as bf
    from paper_1605_02178_amd import _lib
    torch = torch_cuda
    B, H, Wd, ld, gap = 3, 70, 45, 53, 4 * 53
    stride = H * ld + gap
    imgs = _batch((H, Wd), B, 160)
    ybar = np.random.default_rng(161).uniform(-1, 1, size=imgs.shape).astype(np.float32)
    x, g = _gpu(torch, imgs), _gpu(torch, ybar)
    y_ref, saved_ref = bf.gc_forward_saving(x, 4.0, 30.0, 28)
    gf_ref, gs_ref = bf.gc_backward_saving(x, g, saved_ref, 4.0, 30.0, 28)

    def strided(a, fill):
        buf = torch.full((B * stride,), fill, dtype=torch.float32, device="cuda:0")
        view = torch.as_strided(buf, (B, H, Wd), (stride, ld, 1))
        if a is not None:
            view.copy_(a)
        return buf, view

    fbuf, _ = strided(x, 7.0)
    gbuf, _ = strided(g, 0.0)
    ybuf, yv = strided(None, -5.0)
    gfbuf, gfv = strided(None, -6.0)
    saved = torch.empty((B, 6, H, Wd), dtype=torch.float64, device="cuda:0")
    gs = torch.empty((), dtype=torch.float64, device="cuda:0")
    nbytes = bf.saving_workspace_bytes(B, H, Wd, 4.0, 28)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    lib = _lib.load()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.bf_gc_forward_saving(vp(fbuf), vp(ybuf), vp(saved), B, stride, H, Wd, ld, 4.0, 30.0, 28, 0, vp(ws),
                                    nbytes, stream) == 0
    assert lib.bf_gc_backward_saving(vp(fbuf), vp(gbuf), vp(saved), vp(gfbuf), vp(gs), B, stride, H, Wd, ld, 4.0,
                                     30.0, 28, 0, vp(ws), nbytes, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(yv, y_ref) and torch.equal(saved, saved_ref)
    assert torch.equal(gfv, gf_ref) and torch.equal(gs.reshape(()), gs_ref.reshape(()))
    pad = torch.ones(B * stride, dtype=torch.bool, device="cuda:0")
    pad[torch.as_strided(torch.arange(B * stride, device="cuda:0"), (B, H, Wd), (stride, ld, 1)).reshape(-1)] = False
    assert bool((ybuf[pad] == -5.0).all()) and bool((gfbuf[pad] == -6.0).all())
    # an image stride smaller than one image ((H - 1) ld + W elements) is refused
    assert lib.bf_gc_forward_saving(vp(fbuf), vp(ybuf), vp(saved), B, (H - 1) * ld + Wd - 1, H, Wd, ld, 4.0, 30.0,
                                    28, 0, vp(ws), nbytes, stream) == 1
