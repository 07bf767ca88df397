"""MI355X-native seam carving (arXiv 2410.21207): HIP kernels behind the C ABI of include/sc.h.

The package imports nothing heavy at import time; the library is loaded on first use and
its absence is an error (there is no CPU fallback).
"""
__all__ = ["energy", "dp_seam", "remove_seam", "transpose", "carve", "carve_hv", "BatchCarver", "variants",
           "read_status", "workspace"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
