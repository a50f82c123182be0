"""MI355X-native interior-point discarding for 2D convex hulls.

The method is G. Mei's preprocessing (arXiv:1405.3454): extremes of the point
set along the axes of the original and three rotated copies, their convex
polygon, a strict-inside discard, and the hull of the survivors.  The C ABI
is include/hull.h (libhullgpu.so, HIP for gfx950); ``Hull`` in ``api`` wraps
it for torch tensors.  ``inputs`` draws the seeded synthetic point sets.
"""

__all__ = ["Hull", "as_u32", "inputs"]


def __getattr__(name):
    if name in ("Hull", "as_u32", "split_csr", "HULL_DIRS_PAPER", "HULL_DIRS_CUMULATIVE"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
