"""Seeded synthetic inputs for the Gauss-Chebyshev bilateral filter.

This package only draws pixels. It holds none of the filter's arithmetic, so
both the GPU library's tests and the CPU oracle can take the same inputs from it.
"""
from .images import (  # noqa: F401
    ramp_rectangles,
    edge_rich,
    checkerboard,
    batch_specs,
    diff_batch,
    ImageSpec,
)
