"""GPU parity of the recursive variant (BF_FLAG_RECURSIVE: Deriche's
recursive Gaussian in place of the truncated convolution of eq. 7) against the
oracle's recursive filter, through the C ABI.

Bar: 1.5e-3 on the 0-255 scale. Each plane value is rounded to FP32 five
times (the build, the causal half parked in the plane and the result, for the
column and the row pass) instead of twice in the truncated path; each
rounding of a plane value reaches the output amplified by at most
kappa * t_h * 2^-24 ~ 1.1e-4 at sigma_r = 30 (kappa = 15), so about 6e-4 in
the worst alignment, with a margin."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BAR = 1.5e-3


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


# the 14 sigma_s extension exceeds the side in several of these (repeated
# reflection), and 65 / 129 / 300 leave ragged tiles
SHAPES = [((120, 140), 3.0), ((65, 129), 10.0), ((1, 77), 2.0), ((129, 5), 2.0), ((7, 300), 5.0),
          ((300, 7), 1.0), ((1, 1), 1.0), ((256, 256), 4.0)]


@pytest.mark.parametrize("shape,sigma_s", SHAPES)
def test_recursive_parity(torch_cuda, shape, sigma_s):
    import paper_1605_02178_amd as bf
    from oracle import recursive as R
    from synth import edge_rich
    f = edge_rich(*shape, seed=sum(shape) + 51).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch_cuda, f), sigma_s, 30.0, 28, recursive=True))
    err = np.abs(y - R.recursive_gcf(f, sigma_s, 30.0, 28)).max()
    _log(f"recursive {shape} ss={sigma_s}: {err:.3e}")
    assert err <= BAR


def test_recursive_flat_range_and_distance_to_truncated(torch_cuda):
    import paper_1605_02178_amd as bf
    from oracle import recursive as R
    from synth import edge_rich, ramp_rectangles
    torch = torch_cuda
    f = ramp_rectangles(90, 110, seed=52).astype(np.float32).astype(np.float64)
    y = _np(bf.gc_filter(_gpu(torch, f), 3.0, 1e7, 8, recursive=True, allow_ill_conditioned=True))
    assert np.abs(y - R.recursive_gauss_2d(f, 3.0)).max() <= BAR
    g = _gpu(torch, edge_rich(128, 128, seed=53))
    d = np.abs(_np(bf.gc_filter(g, 5.0, 30.0, 28, recursive=True)) - _np(bf.gc_filter(g, 5.0, 30.0, 28))).max()
    _log(f"recursive vs truncated at sigma_s = 5: max {d:.3f}")
    assert d < 3.0


def test_recursive_argument_errors(torch_cuda):
    import paper_1605_02178_amd as bf
    torch = torch_cuda
    f = torch.zeros((16, 16), device="cuda:0")
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 2.0, 30.0, 28, stack_dtype="f16", recursive=True)
    assert e.value.status == 2
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 2.0, 30.0, 28, recursive=True, tile_config=1)
    assert e.value.status == 1
    with pytest.raises(bf.BFError) as e:
        bf.gc_filter(f, 2.0, 30.0, 28, recursive=True, staged=True)
    assert e.value.status == 1
