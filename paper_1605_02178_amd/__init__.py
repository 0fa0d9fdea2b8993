"""Gauss-Chebyshev bilateral filter (Ghosh & Chaudhury, 2016) on AMD MI355X.

Thin torch-facing layer over the C ABI in include/bfgc.h (libbfgc.so, HIP
kernels for gfx950). torch provides device memory and the current HIP stream;
all arithmetic of the filter runs in the library.

    y = gc_filter(f, sigma_s=10.0, sigma_r=30.0)               # N from the degree rule
    y = gc_filter(f, 10.0, 30.0, degree=28, stack_dtype="f16")

The module imports without a GPU; the functions need the built library and a
CUDA (HIP) device tensor.
"""
from __future__ import annotations

import ctypes
import math

from . import _lib
from ._lib import BFError

__all__ = [
    "BFError", "STACK_DTYPES", "FLAG_ALLOW_ILL_CONDITIONED", "FLAG_STAGED", "DEVFLAG_RANGE",
    "degree_rule", "coefficients", "query", "plane_scales", "workspace_bytes", "param_bytes",
    "gc_filter", "gc_backward", "GaussChebyshevBF", "gc_filter_autograd", "stack_build", "gauss_planes",
    "combine", "read_flags", "radius", "StackLayout", "gc_filter_batched", "batched_workspace_bytes",
    "TILE_CONFIGS", "TILE_FUSED", "FUSED_MAX_RADIUS", "FUSED_F16_MAX_RADIUS", "flag_tile", "tile_configs_for", "COEFFS", "fit",
    "gc_joint_filter", "joint_workspace_bytes", "gc_filter_pivots", "pivot_count", "pivot_plan",
    "pivots_workspace_bytes", "batched_route", "gc_filter_noalloc", "NOALLOC_SCRATCH_BYTES",
    "gc_forward_saving", "gc_backward_saving", "saving_workspace_bytes", "ADJ_MAX_RADIUS",
]

STACK_DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
FLAG_ALLOW_ILL_CONDITIONED = 0x1
FLAG_STAGED = 0x2
FLAG_GRAPH = 0x4
FLAG_TAYLOR = 0x8
FLAG_MINIMAX = 0x10
FLAG_RECURSIVE = 0x20
MINIMAX_MAX_DEGREE = 100
# coefficient kinds: the Chebyshev interpolant (Section III), the Taylor
# polynomial (Section II), the minimax polynomial (Remez)
COEFFS = {"chebyshev": 0, "taylor": FLAG_TAYLOR, "minimax": FLAG_MINIMAX}
DEVFLAG_RANGE = 0x1
# Tile configurations: 0-3 are the three-kernel path, (column-pass rows,
# row-pass columns) per lane; TILE_FUSED is the fused matrix-core kernel for
# FP16/BF16 stacks with radius <= FUSED_MAX_RADIUS (the single-image forward:
# FP16 up to FUSED_F16_MAX_RADIUS).
TILE_CONFIGS = ((16, 8), (8, 8), (16, 4), (8, 4), "fused")
TILE_FUSED = 4
FUSED_MAX_RADIUS = 48
FUSED_F16_MAX_RADIUS = 64


def flag_tile(c: int) -> int:
    """Flag bits selecting tile configuration c (an index into TILE_CONFIGS)."""
    return (int(c) + 1) << 8


def tile_configs_for(stack_dtype, sigma_s) -> list:
    """Tile configurations bf_gc_forward accepts for this stack type and sigma_s."""
    code = _dtype_code(stack_dtype)
    cfgs = [0, 1, 2, 3]
    if radius(sigma_s) <= {0: -1, 1: FUSED_F16_MAX_RADIUS, 2: FUSED_MAX_RADIUS}[code]:
        cfgs.append(TILE_FUSED)
    return cfgs
MAX_DEGREE = 320
MAX_RADIUS = 96
# storage rounding unit of each stack type (FP32, FP16, BF16)
_UNIT_ROUNDOFF = {0: 2.0 ** -24, 1: 2.0 ** -11, 2: 2.0 ** -8}


def _dtype_code(stack_dtype) -> int:
    if isinstance(stack_dtype, int):
        return stack_dtype
    import torch
    table = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}
    if stack_dtype in table:
        return table[stack_dtype]
    return STACK_DTYPES[str(stack_dtype)]


def radius(sigma_s: float) -> int:
    """W = ceil(3 sigma_s), the half-width of the spatial window."""
    return int(math.ceil(3.0 * sigma_s - 1e-12))


def degree_rule(sigma_r: float) -> int:
    n = _lib.load().bf_gc_degree_rule(float(sigma_r))
    if n < 0:
        raise ValueError(f"no degree for sigma_r={sigma_r}")
    return n


def coefficients(sigma_r: float, N: int):
    """(b_n list, mu) as the library's planner computes them."""
    b = (ctypes.c_double * (N + 1))()
    mu = ctypes.c_double()
    _lib.check(_lib.load().bf_gc_coefficients(float(sigma_r), int(N), b, ctypes.byref(mu)), "bf_gc_coefficients")
    return list(b), mu.value


def _coeff_flags(coeffs, taylor=False) -> int:
    if taylor:
        if coeffs not in (None, "taylor"):
            raise ValueError("taylor=True with coeffs=%r" % (coeffs,))
        coeffs = "taylor"
    return COEFFS[coeffs or "chebyshev"]


def fit(sigma_r: float, N: int, coeffs="chebyshev"):
    """The library's polynomial for (sigma_r, N) and the coefficient kind:
    dict with b (b_n), db (db_n/dmu), mu, kernel_err, kappa."""
    b = (ctypes.c_double * (N + 1))()
    db = (ctypes.c_double * (N + 1))()
    mu, ke, ka = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().bf_gc_fit(float(sigma_r), int(N), _coeff_flags(coeffs), b, db, ctypes.byref(mu),
                                      ctypes.byref(ke), ctypes.byref(ka)), "bf_gc_fit")
    return {"b": list(b), "db": list(db), "mu": mu.value, "kernel_err": ke.value, "kappa": ka.value}


def query(sigma_r: float, N: int, stack_dtype="f32"):
    """(kernel_err, kappa) for (sigma_r, N)."""
    e, k = ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().bf_gc_query(float(sigma_r), int(N), _dtype_code(stack_dtype), ctypes.byref(e),
                                        ctypes.byref(k)), "bf_gc_query")
    return e.value, k.value


def plane_scales(sigma_r: float, N: int, stack_dtype="f32"):
    k = (ctypes.c_int * (N + 2))()
    _lib.check(_lib.load().bf_gc_plane_scales(float(sigma_r), int(N), _dtype_code(stack_dtype), k),
               "bf_gc_plane_scales")
    return list(k)


def workspace_bytes(height, width, sigma_s, N, stack_dtype="f32", for_backward=False) -> int:
    return int(_lib.load().bf_gc_workspace_bytes(int(height), int(width), float(sigma_s), int(N),
                                                 _dtype_code(stack_dtype), int(bool(for_backward))))


def param_bytes(sigma_s, N) -> int:
    return int(_lib.load().bf_gc_param_bytes(float(sigma_s), int(N)))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Runs the wrapped call with `stream` (if given) as torch's current
    stream, so that every tensor the call allocates (outputs, workspaces,
    contiguous copies) and every copy it makes belong to the stream the
    library launches on. The caching allocator then hands a freed workspace
    only to later work on that stream, which runs after the kernels that use
    it. Inputs must be ready on `stream` (the caller orders them), as for
    any torch operation on a side stream."""
    import functools

    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kw):
        if stream is None:
            return fn(*args, stream=None, **kw)
        import torch
        with torch.cuda.stream(stream):
            return fn(*args, stream=stream, **kw)
    return wrapper


def _check_image(f, name="f"):
    import torch
    if not isinstance(f, torch.Tensor) or not f.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if f.dtype != torch.float32 or f.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 tensor")
    if f.numel() and f.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")


@_on_stream
def gc_filter(f, sigma_s: float, sigma_r: float, degree: int | None = None, stack_dtype="f32",
              staged: bool = False, allow_ill_conditioned: bool = False, out=None, workspace=None,
              stream=None, tile_config: int | None = None, taylor: bool = False, coeffs=None,
              recursive: bool = False):
    """Gauss-Chebyshev bilateral filter of a 2-D float32 image in [0, 255]
    (Section III-B). Returns a new tensor (or writes `out`). coeffs: the
    polynomial for the cross term, "chebyshev" (default), "taylor" (the
    Gauss-polynomial filter of Section II; also taylor=True) or "minimax".
    tile_config: an index into TILE_CONFIGS, "auto" (autotuned), or None.
    recursive=True applies the Gaussian of eq. 7 by Deriche's recursion
    instead of the truncated convolution (FP32 stack)."""
    import torch
    _check_image(f)
    H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    code = _dtype_code(stack_dtype)
    if out is None:
        out = torch.empty_like(f, memory_format=torch.contiguous_format)
    _check_image(out, "out")
    if out.stride(0) != f.stride(0) and H > 1:
        raise ValueError("out must have the row stride of f")
    ld = f.stride(0) if H > 1 else Wd
    need = workspace_bytes(H, Wd, sigma_s, N, code)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = (FLAG_STAGED if staged else 0) | (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0)
    flags |= _coeff_flags(coeffs, taylor)
    flags |= FLAG_RECURSIVE if recursive else 0
    if tile_config == "auto":
        from . import autotune
        tile_config = autotune.lookup(autotune.forward_key(H, Wd, sigma_s, N, code))
        if tile_config is None:
            tile_config, _ = autotune.tune_forward(f, sigma_s, sigma_r, N, code, out=out, workspace=workspace)
    if tile_config is not None:
        flags |= flag_tile(tile_config)
    st = _lib.load().bf_gc_forward(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), H, Wd,
                                   max(ld, Wd), float(sigma_s), float(sigma_r), N, code, flags,
                                   ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   _stream_ptr(stream))
    _lib.check(st, "bf_gc_forward")
    return out


NOALLOC_SCRATCH_BYTES = 4 << 20


@_on_stream
def gc_filter_noalloc(f, sigma_s: float, sigma_r: float, degree: int | None = None, stack_dtype="f16", out=None,
                      range_flag=None, stream=None):
    """bf_gc_forward_noalloc: the fused-tile forward (FP16 stacks with radius
    <= FUSED_F16_MAX_RADIUS, BF16 with radius <= FUSED_MAX_RADIUS) with no
    workspace; the library's own device
    scratch holds the range words. `out` must be given where nothing may be
    allocated; range_flag: optional int32/uint32 device tensor of one element
    that receives DEVFLAG_RANGE or 0."""
    import torch
    _check_image(f)
    H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    if out is None:
        out = torch.empty_like(f, memory_format=torch.contiguous_format)
    _check_image(out, "out")
    if out.stride(0) != f.stride(0) and H > 1:
        raise ValueError("out must have the row stride of f")
    if range_flag is not None and (not range_flag.is_cuda or range_flag.numel() != 1 or range_flag.element_size() != 4):
        raise ValueError("range_flag must be one 4-byte device element")
    ld = f.stride(0) if H > 1 else Wd
    st = _lib.load().bf_gc_forward_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), H, Wd,
                                           max(ld, Wd), float(sigma_s), float(sigma_r), N, _dtype_code(stack_dtype),
                                           0, ctypes.c_void_p(range_flag.data_ptr() if range_flag is not None else 0),
                                           _stream_ptr(stream))
    _lib.check(st, "bf_gc_forward_noalloc")
    return out


def pivot_count(sigma_r: float, stack_dtype="f32") -> int:
    """Smallest number of sub-ranges (a power of two) whose pivoted expansions
    pass the conditioning check for the stack type; -1 if none up to 64."""
    return int(_lib.load().bf_gc_pivot_count(float(sigma_r), _dtype_code(stack_dtype)))


def pivot_plan(sigma_r: float, K: int, degree: int | None = None):
    """[(N_k, mu_k, kappa_k)] of the pivoted form."""
    n = (ctypes.c_int * K)()
    mu = (ctypes.c_double * K)()
    ka = (ctypes.c_double * K)()
    _lib.check(_lib.load().bf_gc_pivot_plan(float(sigma_r), int(K), int(degree or 0), n, mu, ka),
               "bf_gc_pivot_plan")
    return [(n[k], mu[k], ka[k]) for k in range(K)]


def pivots_workspace_bytes(height, width, sigma_s, sigma_r, K, degree=None, stack_dtype="f32") -> int:
    return int(_lib.load().bf_gc_pivots_workspace_bytes(int(height), int(width), float(sigma_s), float(sigma_r),
                                                        int(K), int(degree or 0), _dtype_code(stack_dtype)))


@_on_stream
def gc_filter_pivots(f, sigma_s: float, sigma_r: float, K: int | None = None, degree: int | None = None,
                     stack_dtype="f32", allow_ill_conditioned: bool = False, out=None, workspace=None,
                     stream=None, tile_config: int | None = None):
    """Pivoted Gauss-Chebyshev filter for small sigma_r: K sub-ranges of
    [0, 255], each expanded around its midpoint (K=None: the smallest count
    that is well conditioned for the stack type); degree None: the rule per
    sub-range."""
    import torch
    _check_image(f)
    H, Wd = f.shape
    code = _dtype_code(stack_dtype)
    if K is None:
        K = pivot_count(sigma_r, code)
        if K < 1:
            raise ValueError(f"no sub-range count up to 64 is well conditioned at sigma_r={sigma_r}")
    if out is None:
        out = torch.empty_like(f, memory_format=torch.contiguous_format)
    _check_image(out, "out")
    if out.stride(0) != f.stride(0) and H > 1:
        raise ValueError("out must have the row stride of f")
    ld = f.stride(0) if H > 1 else Wd
    need = pivots_workspace_bytes(H, Wd, sigma_s, sigma_r, K, degree, code)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0
    if tile_config is not None:
        flags |= flag_tile(tile_config)
    st = _lib.load().bf_gc_forward_pivots(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), H, Wd,
                                          max(ld, Wd), float(sigma_s), float(sigma_r), int(K), int(degree or 0),
                                          code, flags, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                          _stream_ptr(stream))
    _lib.check(st, "bf_gc_forward_pivots")
    return out


def joint_workspace_bytes(height, width, sigma_s, N, stack_dtype="f32") -> int:
    return int(_lib.load().bf_gc_joint_workspace_bytes(int(height), int(width), float(sigma_s), int(N),
                                                       _dtype_code(stack_dtype)))


@_on_stream
def gc_joint_filter(f, guide, sigma_s: float, sigma_r: float, degree: int | None = None, stack_dtype="f32",
                    allow_ill_conditioned: bool = False, out=None, workspace=None, stream=None,
                    tile_config: int | None = None, coeffs=None):
    """Joint (cross) bilateral filter of f with the range kernel on `guide`
    (both 2-D float32 in [0, 255], same shape and row stride)."""
    import torch
    _check_image(f)
    _check_image(guide, "guide")
    if tuple(guide.shape) != tuple(f.shape) or (f.shape[0] > 1 and guide.stride(0) != f.stride(0)):
        raise ValueError("guide must have the shape and row stride of f")
    H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    code = _dtype_code(stack_dtype)
    if out is None:
        out = torch.empty_like(f, memory_format=torch.contiguous_format)
    _check_image(out, "out")
    if out.stride(0) != f.stride(0) and H > 1:
        raise ValueError("out must have the row stride of f")
    ld = f.stride(0) if H > 1 else Wd
    need = joint_workspace_bytes(H, Wd, sigma_s, N, code)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0) | _coeff_flags(coeffs)
    if tile_config is not None:
        flags |= flag_tile(tile_config)
    st = _lib.load().bf_gc_joint_forward(ctypes.c_void_p(guide.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), H, Wd, max(ld, Wd), float(sigma_s),
                                         float(sigma_r), N, code, flags, ctypes.c_void_p(workspace.data_ptr()),
                                         workspace.numel(), _stream_ptr(stream))
    _lib.check(st, "bf_gc_joint_forward")
    return out


@_on_stream
def gc_backward(f, grad_out, sigma_s: float, sigma_r: float, degree: int | None = None,
                allow_ill_conditioned: bool = False, workspace=None, stream=None, coeffs=None, grad_f=None,
                grad_sigma_r=None):
    """(dL/df, dL/dsigma_r) for L = sum(grad_out * gc_filter(f, ...)), the
    filter recomputed in FP64. Returns a float32 tensor like f and a 0-d
    float64 tensor (or writes grad_f, contiguous like f, and grad_sigma_r, a
    float64 device element)."""
    import torch
    _check_image(f)
    _check_image(grad_out, "grad_out")
    H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    f = f.contiguous()
    grad_out = grad_out.contiguous()
    if grad_f is None:
        grad_f = torch.empty_like(f)
    elif tuple(grad_f.shape) != (H, Wd) or grad_f.dtype != torch.float32 or not grad_f.is_contiguous():
        raise ValueError("grad_f must be a contiguous float32 tensor shaped like f")
    if grad_sigma_r is None:
        grad_sr = torch.empty((), dtype=torch.float64, device=f.device)
    elif grad_sigma_r.numel() != 1 or grad_sigma_r.dtype != torch.float64 or not grad_sigma_r.is_cuda:
        raise ValueError("grad_sigma_r must be one float64 device element")
    else:
        grad_sr = grad_sigma_r
    ld = f.stride(0) if H > 1 else Wd
    need = workspace_bytes(H, Wd, sigma_s, N, 0, for_backward=True)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0) | _coeff_flags(coeffs)
    st = _lib.load().bf_gc_backward(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(grad_out.data_ptr()),
                                    ctypes.c_void_p(grad_f.data_ptr()), ctypes.c_void_p(grad_sr.data_ptr()), H, Wd,
                                    max(ld, Wd), float(sigma_s), float(sigma_r), N, 0, flags,
                                    ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(stream))
    _lib.check(st, "bf_gc_backward")
    return grad_f, grad_sr


ADJ_MAX_RADIUS = 16   # BF_ADJ_MAX_RADIUS: largest radius of the saving forward / backward pair


def saving_workspace_bytes(count, height, width, sigma_s, N) -> int:
    return int(_lib.load().bf_gc_saving_workspace_bytes(int(count), int(height), int(width), float(sigma_s),
                                                        int(N)))


def _check_batch(x, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32 or x.dim() != 3 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous (count, H, W) float32 tensor")


@_on_stream
def gc_forward_saving(f, sigma_s: float, sigma_r: float, degree: int | None = None, allow_ill_conditioned=False,
                      coeffs=None, out=None, saved=None, keep_sums=True, want_y=True, workspace=None, stream=None):
    """bf_gc_forward_saving on a contiguous (count, H, W) float32 batch: the
    filter with FP64 planes (radius <= ADJ_MAX_RADIUS). Returns (y, saved):
    y like f (None without want_y), saved the (count, 6, H, W) float64 sums
    that gc_backward_saving takes (None without keep_sums)."""
    import torch
    _check_batch(f, "f")
    if not (keep_sums or want_y):
        raise ValueError("gc_forward_saving: nothing to compute (keep_sums and want_y both off)")
    B, H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    if not want_y:
        out = None
    elif out is None:
        out = torch.empty_like(f)
    else:
        _check_batch(out, "out")
    if not keep_sums:
        saved = None
    elif saved is None:
        saved = torch.empty((B, 6, H, Wd), dtype=torch.float64, device=f.device)
    elif saved.dtype != torch.float64 or tuple(saved.shape) != (B, 6, H, Wd) or not saved.is_contiguous():
        raise ValueError("saved must be a contiguous (count, 6, H, W) float64 tensor")
    need = saving_workspace_bytes(B, H, Wd, sigma_s, N)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0) | _coeff_flags(coeffs)
    st = _lib.load().bf_gc_forward_saving(ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr() if out is not None else None),
                                          ctypes.c_void_p(saved.data_ptr() if saved is not None else None), B, H * Wd,
                                          H, Wd, Wd, float(sigma_s),
                                          float(sigma_r), N, flags, ctypes.c_void_p(workspace.data_ptr()),
                                          workspace.numel(), _stream_ptr(stream))
    _lib.check(st, "bf_gc_forward_saving")
    return out, saved


@_on_stream
def gc_backward_saving(f, grad_out, saved, sigma_s: float, sigma_r: float, degree: int | None = None,
                       allow_ill_conditioned=False, coeffs=None, grad_f=None, grad_sigma_r=None, workspace=None,
                       stream=None):
    """bf_gc_backward_saving: (dL/df, dL/dsigma_r summed over the batch) for
    L = sum(grad_out * y), y = gc_forward_saving(f, ...), from its saved sums."""
    import torch
    _check_batch(f, "f")
    _check_batch(grad_out, "grad_out")
    B, H, Wd = f.shape
    N = degree_rule(sigma_r) if degree is None else int(degree)
    if tuple(grad_out.shape) != (B, H, Wd):
        raise ValueError("grad_out must be shaped like f")
    if saved.dtype != torch.float64 or tuple(saved.shape) != (B, 6, H, Wd) or not saved.is_contiguous():
        raise ValueError("saved must be the contiguous (count, 6, H, W) float64 sums of gc_forward_saving")
    if grad_f is None:
        grad_f = torch.empty_like(f)
    else:
        _check_batch(grad_f, "grad_f")
    if grad_sigma_r is None:
        grad_sigma_r = torch.empty((), dtype=torch.float64, device=f.device)
    elif grad_sigma_r.numel() != 1 or grad_sigma_r.dtype != torch.float64 or not grad_sigma_r.is_cuda:
        raise ValueError("grad_sigma_r must be one float64 device element")
    need = saving_workspace_bytes(B, H, Wd, sigma_s, N)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    flags = (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0) | _coeff_flags(coeffs)
    st = _lib.load().bf_gc_backward_saving(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(grad_out.data_ptr()),
                                           ctypes.c_void_p(saved.data_ptr()), ctypes.c_void_p(grad_f.data_ptr()),
                                           ctypes.c_void_p(grad_sigma_r.data_ptr()), B, H * Wd, H, Wd, Wd,
                                           float(sigma_s), float(sigma_r), N, flags,
                                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                           _stream_ptr(stream))
    _lib.check(st, "bf_gc_backward_saving")
    return grad_f, grad_sigma_r


def _autograd_class():
    import torch

    class GaussChebyshevBF(torch.autograd.Function):
        """y = GaussChebyshevBF.apply(f, sigma_r, sigma_s, degree, stack_dtype, coeffs, sigma_r_host)

        f: float32 CUDA tensor (H, W) or (..., H, W); sigma_r: 0-d tensor
        (differentiable); sigma_s, degree: constants; sigma_r_host: the value
        of sigma_r as a Python float, if the caller has it (else it is read
        from the tensor, a device sync when sigma_r lives on the GPU; a CPU
        tensor is read without one).

        stack_dtype "f64" (the default up to radius ADJ_MAX_RADIUS): the whole
        batch in one bf_gc_forward_saving launch, FP64 planes, the six sums
        per pixel (48 B) kept for the backward, which is one
        bf_gc_backward_saving launch. With keep_sums=False the forward keeps
        only f and sigma_r and the backward recomputes the sums first (one
        more launch of the forward tile kernel). "f32", "f16", "bf16" (the default above that radius): the
        batch in one bf_gc_batched launch with that stack, only f and sigma_r
        kept; the backward recomputes the filter in FP64 per image
        (bf_gc_backward), so the gradient is that of the Gauss-Chebyshev
        filter itself, whatever stack type the forward used: for an FP16/BF16
        forward it is the gradient of the function the 16-bit stack
        approximates."""

        @staticmethod
        def forward(ctx, f, sigma_r, sigma_s, degree=None, stack_dtype=None, coeffs=None, sigma_r_host=None,
                    keep_sums=True):
            sr = float(sigma_r_host) if sigma_r_host is not None else float(sigma_r)
            N = degree_rule(sr) if degree is None else int(degree)
            if stack_dtype is None:
                stack_dtype = "f64" if radius(sigma_s) <= ADJ_MAX_RADIUS else "f32"
            shape = f.shape
            x = f.reshape(-1, shape[-2], shape[-1])
            if not x.is_contiguous():
                x = x.contiguous()
            ctx.sigma_s, ctx.sigma_r, ctx.N, ctx.coeffs = float(sigma_s), sr, N, coeffs
            ctx.saving = stack_dtype == "f64"
            # the conditioning check of the single-image forward (the FP32 stack's
            # for the f64 form, as its C call; the batch would route such an
            # image to the pivoted form, whose gradient the backward does not
            # compute)
            kappa = fit(sr, N, coeffs)["kappa"]
            if not kappa * _UNIT_ROUNDOFF[_dtype_code("f32" if ctx.saving else stack_dtype)] <= 1e-2:
                raise ValueError(f"GaussChebyshevBF: ill-conditioned at sigma_r={sr}, N={N} for the "
                                 f"{stack_dtype} stack (kappa={kappa:.3g})")
            if ctx.saving:
                if radius(sigma_s) > ADJ_MAX_RADIUS:
                    raise ValueError(f"GaussChebyshevBF: the f64 form takes radius <= {ADJ_MAX_RADIUS}")
                ctx.keep_sums = bool(keep_sums)
                y, saved = gc_forward_saving(x, sigma_s, sr, N, coeffs=coeffs, keep_sums=ctx.keep_sums)
                if ctx.keep_sums:
                    ctx.save_for_backward(f, sigma_r, saved)
                else:
                    ctx.save_for_backward(f, sigma_r)
                return y.reshape(shape)
            y = torch.empty_like(x)
            B = x.shape[0]
            _, status = gc_filter_batched([x[b] for b in range(B)], [sigma_s] * B, [sr] * B, [N] * B,
                                          stack_dtype=stack_dtype, graph=False, outs=[y[b] for b in range(B)],
                                          coeffs=coeffs, allow_ill_conditioned=True)
            if any(status):
                raise BFError(next(v for v in status if v), "GaussChebyshevBF forward")
            ctx.save_for_backward(f, sigma_r)
            return y.reshape(shape)

        @staticmethod
        def backward(ctx, grad_y):
            f, sigma_r = ctx.saved_tensors[:2]
            shape = f.shape
            x = f.reshape(-1, shape[-2], shape[-1])
            g = grad_y.reshape(-1, shape[-2], shape[-1]).contiguous()
            if ctx.saving:
                xc = x.contiguous()
                if ctx.keep_sums:
                    saved = ctx.saved_tensors[2]
                else:
                    _, saved = gc_forward_saving(xc, ctx.sigma_s, ctx.sigma_r, ctx.N, coeffs=ctx.coeffs, want_y=False)
                gf, gs = gc_backward_saving(xc, g, saved, ctx.sigma_s, ctx.sigma_r, ctx.N, coeffs=ctx.coeffs)
                gs = gs.to(device=sigma_r.device, dtype=sigma_r.dtype).reshape(sigma_r.shape)
                return gf.reshape(shape), gs, None, None, None, None, None, None
            B = x.shape[0]
            gf = torch.empty_like(x)
            gsr = torch.empty(B, dtype=torch.float64, device=f.device)
            ws = torch.empty(max(workspace_bytes(shape[-2], shape[-1], ctx.sigma_s, ctx.N, 0, True), 256),
                             dtype=torch.uint8, device=f.device)
            for b in range(B):
                gc_backward(x[b].contiguous(), g[b], ctx.sigma_s, ctx.sigma_r, ctx.N, workspace=ws,
                            coeffs=ctx.coeffs, grad_f=gf[b], grad_sigma_r=gsr[b])
            gs = gsr.sum().to(device=sigma_r.device, dtype=sigma_r.dtype).reshape(sigma_r.shape)
            return gf.reshape(shape), gs, None, None, None, None, None, None

    return GaussChebyshevBF
_GCBF = None


def __getattr__(name):
    global _GCBF
    if name == "GaussChebyshevBF":
        if _GCBF is None:
            _GCBF = _autograd_class()
        return _GCBF
    raise AttributeError(name)


def gc_filter_autograd(f, sigma_r, sigma_s, degree=None, stack_dtype=None, coeffs=None, sigma_r_host=None,
                       keep_sums=True):
    """Differentiable forward: GaussChebyshevBF.apply with sigma_r a tensor
    (sigma_r_host: its value as a float, which spares a device sync);
    stack_dtype None = "f64" up to radius ADJ_MAX_RADIUS, else "f32";
    keep_sums=False: the f64 form keeps only f and sigma_r."""
    return __getattr__("GaussChebyshevBF").apply(f, sigma_r, sigma_s, degree, stack_dtype, coeffs, sigma_r_host,
                                                 keep_sums)


def _descs(images, outs, sigmas_s, sigmas_r, degrees):
    n = len(images)
    arr = (_lib.ImageDesc * max(n, 1))()
    for i, (f, o) in enumerate(zip(images, outs)):
        H, Wd = f.shape
        arr[i].f = f.data_ptr() if f.numel() else None
        arr[i].out = o.data_ptr() if o.numel() else None
        arr[i].height, arr[i].width = H, Wd
        arr[i].ld = max(f.stride(0) if H > 1 else Wd, Wd)
        arr[i].sigma_s, arr[i].sigma_r, arr[i].N = float(sigmas_s[i]), float(sigmas_r[i]), int(degrees[i])
    return arr


def batched_route(sigma_r: float, degree: int, stack_dtype="f32", allow_ill_conditioned: bool = False,
                  coeffs=None) -> int:
    """How gc_filter_batched runs an image with these parameters: 1 = its own
    expansion, K >= 2 = the pivoted form with K sub-ranges (its own expansion
    is ill-conditioned for the stack type), 0 = skipped."""
    flags = (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0) | _coeff_flags(coeffs)
    return int(_lib.load().bf_gc_batched_route(float(sigma_r), int(degree), _dtype_code(stack_dtype), flags))


def batched_workspace_bytes(shapes, sigmas_s, degrees, stack_dtype="f32", sigmas_r=None) -> int:
    """Workspace bytes for gc_filter_batched on images of these shapes and
    parameters. sigmas_r decides which images run the pivoted form; without
    it every image is sized at sigma_r = 30 (its own expansion only)."""
    arr = (_lib.ImageDesc * max(len(shapes), 1))()
    for i, (H, Wd) in enumerate(shapes):
        arr[i].height, arr[i].width, arr[i].ld = H, Wd, Wd
        sr = 30.0 if sigmas_r is None else float(sigmas_r[i])
        arr[i].sigma_s, arr[i].sigma_r, arr[i].N = float(sigmas_s[i]), sr, int(degrees[i])
    return int(_lib.load().bf_gc_batched_workspace_bytes(arr, len(shapes), _dtype_code(stack_dtype)))


@_on_stream
def gc_filter_batched(images, sigmas_s, sigmas_r, degrees=None, stack_dtype="f32", graph: bool = True,
                      tile_config: int | None = None, allow_ill_conditioned: bool = False, outs=None,
                      workspace=None, stream=None, coeffs=None):
    """Filters a list of 2-D float32 images (uneven sizes, one sigma_s,
    sigma_r and degree each) in one persistent launch. Returns (outs,
    statuses): statuses[i] is the bf_status of image i (non-zero: skipped)."""
    import torch
    n = len(images)
    for f in images:
        _check_image(f)
    if degrees is None:
        degrees = [degree_rule(sr) for sr in sigmas_r]
    images = [f if f.stride(-1) == 1 else f.contiguous() for f in images]
    if outs is None:
        outs = [torch.empty_like(f, memory_format=torch.contiguous_format) for f in images]
    arr = _descs(images, outs, sigmas_s, sigmas_r, degrees)
    code = _dtype_code(stack_dtype)
    lib = _lib.load()
    if workspace is None:
        # (a caller's workspace is checked by the library: BF_ERR_WORKSPACE if too small)
        need = int(lib.bf_gc_batched_workspace_bytes(arr, n, code))
        dev = images[0].device if n else "cuda"
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    status = (ctypes.c_int * max(n, 1))()
    flags = (FLAG_GRAPH if graph else 0) | (FLAG_ALLOW_ILL_CONDITIONED if allow_ill_conditioned else 0)
    flags |= _coeff_flags(coeffs)
    if tile_config == "auto":
        from . import autotune
        tile_config = autotune.lookup(autotune.batched_key([tuple(x.shape) for x in images], sigmas_s, degrees,
                                                           code))
        if tile_config is None:
            tile_config, _ = autotune.tune_batched(images, sigmas_s, sigmas_r, degrees, code, graph=graph,
                                                   allow_ill_conditioned=allow_ill_conditioned,
                                                   workspace=workspace)
    if tile_config is not None:
        flags |= flag_tile(tile_config)
    st = lib.bf_gc_batched(arr, n, code, flags, status, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                           _stream_ptr(stream))
    _lib.check(st, "bf_gc_batched")
    return outs, list(status)[:n]


class StackLayout:
    """Device stack of N+2 planes as the stage functions use it."""

    def __init__(self, height, width, N, stack_dtype="f32", device="cuda"):
        import torch
        self.height, self.width, self.N = int(height), int(width), int(N)
        self.code = _dtype_code(stack_dtype)
        self.lds = (self.width + 63) // 64 * 64
        self.planes = self.N + 2
        self.plane_stride = self.height * self.lds
        tdtype = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}[self.code]
        self.data = torch.empty((self.planes, self.height, self.lds), dtype=tdtype, device=device)

    def view(self):
        """(N+2, height, width) view of the planes."""
        return self.data[:, :, : self.width]


@_on_stream
def stack_build(f, sigma_r, N, stack_dtype="f32", stack: StackLayout | None = None, prm=None, devflag=None,
                stream=None) -> StackLayout:
    import torch
    _check_image(f)
    H, Wd = f.shape
    stack = stack or StackLayout(H, Wd, N, stack_dtype, f.device)
    prm = prm if prm is not None else torch.empty(param_bytes(1.0, N) + 8 * 64, dtype=torch.uint8, device=f.device)
    st = _lib.load().bf_gc_stack_build(ctypes.c_void_p(f.data_ptr()), H, Wd, max(f.stride(0), Wd), float(sigma_r),
                                       int(N), stack.code, ctypes.c_void_p(stack.data.data_ptr()),
                                       stack.plane_stride, stack.lds,
                                       ctypes.c_void_p(devflag.data_ptr() if devflag is not None else 0),
                                       ctypes.c_void_p(prm.data_ptr()), _stream_ptr(stream))
    _lib.check(st, "bf_gc_stack_build")
    stack._prm = prm
    return stack


@_on_stream
def gauss_planes(stack: StackLayout, sigma_s, tmp=None, prm=None, stream=None):
    """Filters every plane of `stack` in place (eq. 7). `tmp`: optional uint8
    device scratch of at least bf_gc_gauss_tmp_bytes bytes."""
    import torch
    lib = _lib.load()
    need = int(lib.bf_gc_gauss_tmp_bytes(stack.planes, stack.height, stack.width, stack.code))
    if tmp is None:
        tmp = torch.empty(max(need, 16), dtype=torch.uint8, device=stack.data.device)
    prm = prm if prm is not None else torch.empty(param_bytes(sigma_s, 1) + 8 * 64, dtype=torch.uint8,
                                                  device=stack.data.device)
    st = lib.bf_gc_gauss_planes(ctypes.c_void_p(stack.data.data_ptr()), ctypes.c_void_p(tmp.data_ptr()),
                                tmp.numel() * tmp.element_size(), stack.planes, stack.height, stack.width,
                                stack.plane_stride, stack.lds, float(sigma_s), stack.code,
                                ctypes.c_void_p(prm.data_ptr()), _stream_ptr(stream))
    _lib.check(st, "bf_gc_gauss_planes")
    stack._tmp, stack._prm2 = tmp, prm
    return stack


@_on_stream
def combine(f, stack: StackLayout, sigma_r, out=None, want_pq=False, prm=None, stream=None):
    """Returns y, or (y, P', Q') with want_pq."""
    import torch
    _check_image(f)
    H, Wd = f.shape
    out = out if out is not None else torch.empty_like(f)
    P = torch.empty_like(f) if want_pq else None
    Q = torch.empty_like(f) if want_pq else None
    prm = prm if prm is not None else torch.empty(param_bytes(1.0, stack.N) + 8 * 64, dtype=torch.uint8,
                                                  device=f.device)
    st = _lib.load().bf_gc_combine(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(stack.data.data_ptr()), H, Wd,
                                   max(f.stride(0), Wd), stack.plane_stride, stack.lds, float(sigma_r), stack.N,
                                   stack.code, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(P.data_ptr() if want_pq else 0),
                                   ctypes.c_void_p(Q.data_ptr() if want_pq else 0),
                                   ctypes.c_void_p(prm.data_ptr()), _stream_ptr(stream))
    _lib.check(st, "bf_gc_combine")
    out._prm = prm
    return (out, P, Q) if want_pq else out


def read_flags(workspace, stream=None) -> int:
    v = ctypes.c_uint()
    _lib.check(_lib.load().bf_gc_read_flags(ctypes.c_void_p(workspace.data_ptr()), ctypes.byref(v),
                                            _stream_ptr(stream)), "bf_gc_read_flags")
    return v.value
