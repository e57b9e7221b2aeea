"""GIFT search stage (arXiv 1604.01879) on AMD MI355X.

The compute path is libgift.so (HIP kernels for gfx950) behind the C ABI in
include/gift.h; ``paper_1604_01879_amd._lib`` is its ctypes binding.  Build
with ``python -m paper_1604_01879_amd.build``.
"""
__all__ = ["lib"]


def lib():
    """Imports and returns the binding module (raises if not built)."""
    from . import _lib
    return _lib
