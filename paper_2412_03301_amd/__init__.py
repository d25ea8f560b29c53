"""MI355X-native hot path of bio-inspired vector-set search.

FlyHash encoding, per-set count/binary Bloom sketches, Bloom-filter
candidate scoring with top-T selection and exact Hausdorff re-ranking,
implemented as HIP kernels for gfx950 behind the C ABI in include/bvs.h.

`paper_2412_03301_amd.bvs` is the thin Python binding (ctypes; PyTorch only
supplies device memory and streams).  Submodules are imported on demand so
that the synthetic-data module works on machines without the built library.
"""
import importlib

__all__ = ["bvs", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
