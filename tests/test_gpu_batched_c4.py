"""The uneven batch of the batched workload through bf_gc_batched, with no
allow flag: 64 edge-rich images (seeds 4000-4063), long side uniform over
{256, 384, ..., 2048}, square or 2:1, sigma_s ~ U[2, 16], sigma_r ~ U[10, 60],
degree from the rule. Images whose own expansion fails the conditioning check
for the stack type (Section III-B: mu = t_h^2/sigma_r^2 grows as 1/sigma_r^2)
run the pivoted form. Every image is held, on two 128 x 128 crops (the
top-left corner, with the symmetric extension, and the centre), to the FP64
oracle: its fast filter of eqs. 6-10 at the image's degree, or, for a routed
image, its pivoted filter with the same sub-range count. Bars per stack and
route are about three times the largest error measured over the batch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# max-abs bars on the 0-255 scale, per (stack, routed), about three times the
# largest error measured over the 64 images x 2 crops (in the comments). FP32
# keeps its 1e-3 claim: images outside its accuracy domain (kappa u > 1e-5)
# are routed. The 16-bit stacks' own expansions keep the conditioning check's
# domain (kappa u <= 1e-2), where their rounding reaches about one grey level
# at sigma_r = 30, N = 28; their routed images run sub-ranges with kappa near 1.
BARS = {
    ("f32", False): 1e-3,      # measured 2.2e-4
    ("f32", True): 3e-5,       # measured 7.9e-6
    ("f16", False): 3.5,       # measured 1.17 (sigma_r = 30.15, N = 28)
    ("f16", True): 0.05,       # measured 1.65e-2
    ("bf16", False): 3.3,      # measured 1.08
    ("bf16", True): 0.6,       # measured 0.19
}
CROP = 128


def _crops(H, Wd):
    c = min(CROP, H), min(CROP, Wd)
    r0, c0 = (H - c[0]) // 2, (Wd - c[1]) // 2
    return [(0, c[0], 0, c[1]), (r0, r0 + c[0], c0, c0 + c[1])]


@pytest.fixture(scope="module")
def batch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1605_02178_amd as bf
    from synth import batch_specs
    specs = batch_specs()
    imgs = [sp.image() for sp in specs]
    fs = [torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in imgs]
    deg = [bf.degree_rule(sp.sigma_r) for sp in specs]
    return specs, imgs, fs, deg


_oracle_cache = {}


def _oracle(k, sp, img, N, K, reg):
    from oracle import native as C
    key = (k, N, K, reg)
    if key not in _oracle_cache:
        f64 = img.astype(np.float32).astype(np.float64)
        if K == 1:
            _oracle_cache[key] = C.gcf(f64, sp.sigma_s, sp.sigma_r, N, region=reg)
        else:
            _oracle_cache[key] = C.pivot_gcf(f64, sp.sigma_s, sp.sigma_r, K, region=reg)
    return _oracle_cache[key]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_uneven_batch_against_oracle(batch, dtype):
    import paper_1605_02178_amd as bf
    specs, imgs, fs, deg = batch
    routes = [bf.batched_route(sp.sigma_r, deg[k], dtype) for k, sp in enumerate(specs)]
    assert all(r >= 1 for r in routes), routes
    print(f"{dtype}: {sum(r > 1 for r in routes)} of {len(routes)} images routed, counts {sorted(set(routes))}",
          flush=True)
    outs, status = bf.gc_filter_batched(fs, [sp.sigma_s for sp in specs], [sp.sigma_r for sp in specs], deg,
                                        stack_dtype=dtype, graph=True)
    assert status == [0] * len(fs)
    worst = {}
    fails = []
    for k, sp in enumerate(specs):
        y = outs[k].cpu().double().numpy()
        for reg in _crops(sp.height, sp.width):
            ref = _oracle(k, sp, imgs[k], deg[k], routes[k], reg)
            err = float(np.abs(y[reg[0]:reg[1], reg[2]:reg[3]] - ref).max())
            grp = (dtype, routes[k] > 1)
            worst[grp] = max(worst.get(grp, 0.0), err)
            print(f"{dtype} image {k} {sp.height}x{sp.width} ss={sp.sigma_s:.2f} sr={sp.sigma_r:.2f} "
                  f"N={deg[k]} K={routes[k]} crop {reg}: {err:.3e}", flush=True)
            if not err <= BARS[grp]:
                fails.append((k, reg, err))
    print(f"{dtype}: worst per route {worst}", flush=True)
    assert not fails, fails
