"""ctypes loader for libbfgc.so (the HIP library). Argument marshalling only:
every step of the filter runs in the library's kernels. Raises ImportError
with a clear message when the library has not been built."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfgc.so")

_c_int, _c_uint, _c_double, _c_size_t = ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
_c_ll, _vp = ctypes.c_longlong, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_up = ctypes.POINTER(ctypes.c_uint)

# name -> (restype, argtypes); mirrors include/bfgc.h
SIGNATURES = {
    "bf_gc_degree_rule": (_c_int, [_c_double]),
    "bf_gc_coefficients": (_c_int, [_c_double, _c_int, _dp, _dp]),
    "bf_gc_query": (_c_int, [_c_double, _c_int, _c_int, _dp, _dp]),
    "bf_gc_fit": (_c_int, [_c_double, _c_int, _c_uint, _dp, _dp, _dp, _dp, _dp]),
    "bf_gc_workspace_bytes": (_c_size_t, [_c_int, _c_int, _c_double, _c_int, _c_int, _c_int]),
    "bf_gc_forward": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _c_double, _c_double, _c_int, _c_int,
                               _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_backward": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _c_int, _c_int, _c_double, _c_double, _c_int,
                                _c_int, _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_forward_noalloc": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _c_double, _c_double, _c_int, _c_int,
                                       _c_uint, _vp, _vp]),
    "bf_gc_saving_workspace_bytes": (_c_size_t, [_c_int, _c_int, _c_int, _c_double, _c_int]),
    "bf_gc_forward_saving": (_c_int, [_vp, _vp, _vp, _c_int, _c_ll, _c_int, _c_int, _c_int, _c_double,
                                      _c_double, _c_int, _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_backward_saving": (_c_int, [_vp, _vp, _vp, _vp, _vp, _c_int, _c_ll, _c_int, _c_int, _c_int,
                                       _c_double, _c_double, _c_int, _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_pivot_count": (_c_int, [_c_double, _c_int]),
    "bf_gc_batched_route": (_c_int, [_c_double, _c_int, _c_int, _c_uint]),
    "bf_gc_pivot_plan": (_c_int, [_c_double, _c_int, _c_int, _ip, _dp, _dp]),
    "bf_gc_pivots_workspace_bytes": (_c_size_t, [_c_int, _c_int, _c_double, _c_double, _c_int, _c_int, _c_int]),
    "bf_gc_forward_pivots": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _c_double, _c_double, _c_int, _c_int,
                                      _c_int, _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_joint_workspace_bytes": (_c_size_t, [_c_int, _c_int, _c_double, _c_int, _c_int]),
    "bf_gc_joint_forward": (_c_int, [_vp, _vp, _vp, _c_int, _c_int, _c_int, _c_double, _c_double, _c_int, _c_int,
                                     _c_uint, _vp, _c_size_t, _vp]),
    "bf_gc_param_bytes": (_c_size_t, [_c_double, _c_int]),
    "bf_gc_plane_scales": (_c_int, [_c_double, _c_int, _c_int, _ip]),
    "bf_gc_stack_build": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_double, _c_int, _c_int, _vp, _c_ll,
                                   _c_int, _vp, _vp, _vp]),
    "bf_gc_gauss_tmp_bytes": (_c_size_t, [_c_int, _c_int, _c_int, _c_int]),
    "bf_gc_gauss_planes": (_c_int, [_vp, _vp, _c_size_t, _c_int, _c_int, _c_int, _c_ll, _c_int, _c_double,
                                    _c_int, _vp, _vp]),
    "bf_gc_combine": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _c_ll, _c_int, _c_double, _c_int, _c_int,
                               _vp, _vp, _vp, _vp, _vp]),
    "bf_gc_read_flags": (_c_int, [_vp, _up, _vp]),
    "bf_profile_start": (_c_int, []),
    "bf_profile_stop": (_c_int, [_vp]),
    "bf_profile_count": (_c_int, []),
    "bf_profile_entry": (_c_int, [_c_int, ctypes.c_char_p, _c_int, ctypes.POINTER(_c_ll), _dp]),
    "bf_status_string": (ctypes.c_char_p, [_c_int]),
    "bf_last_error": (ctypes.c_char_p, []),
}

class ImageDesc(ctypes.Structure):
    """bf_image_desc of include/bfgc.h."""
    _fields_ = [("f", _vp), ("out", _vp), ("height", _c_int), ("width", _c_int), ("ld", _c_int),
                ("sigma_s", _c_double), ("sigma_r", _c_double), ("N", _c_int)]


_descp = ctypes.POINTER(ImageDesc)
SIGNATURES["bf_gc_batched_workspace_bytes"] = (_c_size_t, [_descp, _c_int, _c_int])
SIGNATURES["bf_gc_batched"] = (_c_int, [_descp, _c_int, _c_int, _c_uint, _ip, _vp, _c_size_t, _vp])

_lib = None


def load() -> ctypes.CDLL:
    """Load the library (once) and attach the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libbfgc.so not found at {LIB_PATH}; build it first "
                          "(python -c 'import __graft_entry__ as g; g.build()' or "
                          "python paper_1605_02178_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class BFError(RuntimeError):
    """A non-zero bf_status from the library."""

    def __init__(self, status: int, where: str):
        lib = load()
        self.status = status
        msg = f"{where}: {lib.bf_status_string(status).decode()}: {lib.bf_last_error().decode()}"
        super().__init__(msg)


def check(status: int, where: str) -> None:
    if status != 0:
        raise BFError(status, where)
