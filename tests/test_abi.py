"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, its planner agrees with the oracle, and
argument errors come back as status codes before anything touches a device."""
import ctypes
import math
import os
import re

import mpmath
import numpy as np
import pytest

from oracle import coeffs as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfgc.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1605_02178_amd import _lib
    return _lib.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_1605_02178_amd._lib import SIGNATURES
    assert set(SIGNATURES) == set(names)


def test_degree_rule_matches_oracle(lib):
    for sr in (10.0, 15.0, 20.0, 25.0, 29.8, 30.0, 30.2, 40.0, 50.0, 60.0, 120.0):
        assert lib.bf_gc_degree_rule(sr) == K.degree_rule(sr), sr
    assert lib.bf_gc_degree_rule(-1.0) == -1
    assert lib.bf_gc_degree_rule(float("nan")) == -1


@pytest.mark.parametrize("sigma_r,N", [(30.0, 28), (30.0, 10), (40.0, 16), (50.0, 11), (25.0, 40), (20.0, 62)])
def test_planner_coefficients_match_oracle_at_kernel_level(sigma_r, N):
    """The monomial coefficients are ill-conditioned individually; what the
    filter uses is the polynomial, so compare exp(-mu|y|) p(mu y) over y."""
    import paper_1605_02178_amd as bf
    b, mu = bf.coefficients(sigma_r, N)
    c, _ = K.gcf_coefficients(sigma_r, N)
    assert mu == pytest.approx(K.gcf_params(sigma_r)[1], rel=1e-15)
    with mpmath.workdps(50):
        worst = 0.0
        for y in np.linspace(-1, 1, 401):
            pb = mpmath.fsum(mpmath.mpf(v) * mpmath.mpf(y) ** n for n, v in enumerate(b))
            pc = mpmath.fsum(mpmath.mpf(v) * (mu * mpmath.mpf(y)) ** n for n, v in enumerate(c))
            worst = max(worst, float(abs(pb - pc) * mpmath.exp(-mu * abs(y))))
    assert worst < 1e-11, worst


def test_query_values(lib):
    import paper_1605_02178_amd as bf
    err, kappa = bf.query(30.0, 28)
    assert 4e-3 < err < 9e-3          # weighted kernel error at the paper's operating point
    assert 5 < kappa < 40
    e2, _ = bf.query(30.0, 34)
    assert e2 < err / 100


def test_plane_scales():
    import paper_1605_02178_amd as bf
    assert bf.plane_scales(30.0, 28, "f32") == [0] * 30
    k = bf.plane_scales(30.0, 28, "f16")
    mu = K.gcf_params(30.0)[1]
    for n, kn in enumerate(k):
        m = 1.0 if n == 0 else ((n / (math.e * mu)) ** (n / 2) if n <= mu else math.exp(-mu / 2))
        assert 2 ** 13 <= m * 2 ** kn <= 2 ** 15


def test_workspace_bytes():
    import paper_1605_02178_amd as bf
    a = bf.workspace_bytes(4096, 4096, 10.0, 28, "f32")
    b = bf.workspace_bytes(4096, 4096, 10.0, 28, "f16")
    assert a >= 2 * 30 * 4096 * 4096 * 4
    assert b < a * 0.6
    assert bf.workspace_bytes(10, 10, -1.0, 28) == 0
    assert bf.workspace_bytes(10, 10, 1000.0, 28) == 0


def _fwd(lib, f=1 << 20, out=1 << 24, H=8, Wd=8, ld=8, ss=2.0, sr=30.0, N=28, dt=0, flags=0, ws=256 * 1024, wsb=1 << 30):
    return lib.bf_gc_forward(ctypes.c_void_p(f), ctypes.c_void_p(out), H, Wd, ld, ss, sr, N, dt, flags,
                             ctypes.c_void_p(ws), wsb, None)


def test_forward_argument_errors_need_no_device(lib):
    big = 1 << 40
    assert _fwd(lib, f=0) == 1                       # null f
    assert _fwd(lib, H=-1) == 1
    assert _fwd(lib, ld=4) == 1                      # ld < width
    assert _fwd(lib, ss=0.0) == 1
    assert _fwd(lib, sr=float("inf")) == 1
    assert _fwd(lib, N=0) == 1 and _fwd(lib, N=400) == 1
    assert _fwd(lib, dt=7) == 1
    assert _fwd(lib, f=big, out=big + 16) == 1      # out overlaps f
    assert _fwd(lib, ss=40.0) == 2                   # W = 120 > BF_MAX_RADIUS
    assert _fwd(lib, H=3000000, ld=16) == 2          # side above BF_MAX_SIDE
    assert _fwd(lib, sr=12.0, N=170) == 3            # ill-conditioned in FP32
    assert _fwd(lib, sr=30.0, N=28, dt=2) == 3       # BF16 at sigma_r = 30
    assert _fwd(lib, ws=0) == 4
    assert _fwd(lib, wsb=100) == 4
    assert _fwd(lib, ws=256 * 1024 + 8) == 4         # misaligned
    assert _fwd(lib, H=0, f=0, out=0) == 0           # empty image: nothing to do
    assert lib.bf_status_string(3) == b"BF_ERR_ILL_CONDITIONED"
    _fwd(lib, ss=-1.0)
    assert b"sigma_s" in lib.bf_last_error()


def test_stage_argument_errors(lib):
    vp = ctypes.c_void_p
    assert lib.bf_gc_stack_build(vp(1), 8, 8, 8, 30.0, 28, 0, vp(0), 64 * 8, 64, vp(0), vp(1), None) == 1
    assert lib.bf_gc_gauss_planes(vp(1 << 20), vp(0), 1 << 20, 30, 8, 8, 64 * 8, 64, 2.0, 0, vp(1), None) == 4
    assert lib.bf_gc_gauss_planes(vp(1 << 20), vp(1 << 24), 1 << 20, 30, 8, 8, 64 * 8 + 1, 64, 2.0, 0, vp(1), None) == 1
    assert lib.bf_gc_gauss_planes(vp(0), vp(1), 1 << 20, 30, 8, 8, 64 * 8, 64, 2.0, 0, vp(1), None) == 1
    assert lib.bf_gc_combine(vp(1), vp(1), 8, 8, 8, 8 * 8, 4, 30.0, 28, 0, vp(1), vp(0), vp(0), vp(1), None) == 1


def test_autotune_keys_and_cache(tmp_path, monkeypatch):
    from paper_1605_02178_amd import autotune
    monkeypatch.setenv("BFGC_AUTOTUNE_CACHE", str(tmp_path / "t.json"))
    autotune.clear_memory()
    k1 = autotune.forward_key(4096, 4096, 10.0, 28, 0, arch="gfx950")
    k2 = autotune.forward_key(4000, 4096, 10.0, 28, 0, arch="gfx950")
    k3 = autotune.forward_key(4096, 4096, 3.0, 28, 0, arch="gfx950")
    assert k1 == k2 and k1 != k3
    assert autotune.lookup(k1) is None
    autotune._store(k1, 2, [1.0, 0.5, 0.4, 0.9])
    autotune.clear_memory()
    assert autotune.lookup(k1) == 2
    (tmp_path / "t.json").write_text("not json")
    autotune.clear_memory()
    assert autotune.lookup(k1) is None
    autotune.clear_memory()


def test_taylor_flag_conditioning(lib):
    # the Taylor polynomial's kappa is at most 1: accepted in BF16 where the
    # Chebyshev interpolant at the same degree is refused
    assert _fwd(lib, sr=30.0, N=28, dt=2) == 3
    assert _fwd(lib, sr=30.0, N=28, dt=2, flags=0x8, ws=0) == 4


@pytest.mark.parametrize("sigma_r,N", [(30.0, 28), (50.0, 11), (25.0, 40), (60.0, 8)])
def test_planner_minimax_matches_oracle_at_kernel_level(sigma_r, N):
    """The binary128 Remez of the planner against the oracle's 60-digit one,
    compared as polynomials weighted by exp(-mu|y|), as for eq. 19."""
    import paper_1605_02178_amd as bf
    F = bf.fit(sigma_r, N, "minimax")
    c = K.minimax_coefficients(sigma_r, N)
    mu = F["mu"]
    with mpmath.workdps(50):
        worst = 0.0
        for y in np.linspace(-1, 1, 401):
            pb = mpmath.fsum(mpmath.mpf(v) * mpmath.mpf(y) ** n for n, v in enumerate(F["b"]))
            pc = mpmath.fsum(mpmath.mpf(v) * (mu * mpmath.mpf(y)) ** n for n, v in enumerate(c))
            worst = max(worst, float(abs(pb - pc) * mpmath.exp(-mu * abs(y))))
    assert worst < 1e-11, worst


def test_planner_minimax_derivative_matches_oracle():
    """db_n/dmu of the planner (implicit form) against the oracle's central
    difference of dc_n/dsigma_r, as polynomials."""
    import paper_1605_02178_amd as bf
    sr, N = 50.0, 11
    F = bf.fit(sr, N, "minimax")
    _, dc = K.minimax_coefficients_with_derivative(sr, N)
    mu = F["mu"]
    dmu = -2.0 * mu / sr
    # d/dsigma_r of b_n y^n with b_n = c_n mu^n: (dc_n mu^n + c_n n mu^{n-1} dmu) y^n
    c = K.minimax_coefficients(sr, N)
    for y in np.linspace(-1, 1, 81):
        got = sum(db * dmu * y ** n for n, db in enumerate(F["db"]))
        want = sum((dc[n] * mu ** n + c[n] * n * mu ** (n - 1) * dmu) * y ** n for n in range(N + 1))
        assert abs(got - want) <= 1e-9 * math.exp(mu * abs(y)) * mu
    T = bf.fit(sr, N, "taylor")
    assert T["b"] == pytest.approx([mu ** n / math.factorial(n) for n in range(N + 1)], rel=1e-14)


def test_minimax_flag_errors(lib):
    assert _fwd(lib, flags=0x8 | 0x10) == 1          # Taylor and minimax together
    assert _fwd(lib, sr=30.0, N=101, flags=0x10) == 2
    assert _fwd(lib, sr=30.0, N=28, flags=0x10, ws=0) == 4   # accepted up to the workspace check
    assert lib.bf_gc_fit(30.0, 28, 0x18, (ctypes.c_double * 29)(), None, None, None, None) == 1
    assert lib.bf_gc_fit(30.0, 101, 0x10, (ctypes.c_double * 102)(), None, None, None, None) == 2
