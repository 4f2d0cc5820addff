"""MI355X-native hot path of anonymized network sensing (arXiv 2510.14050).

Windows of (source, destination) IPv4 pairs become hypersparse 2^32 x 2^32
traffic matrices (sorted COO, uint64 counts) and are reduced to the eight
network quantities on the GPU. The compute lives in hand-written HIP kernels
behind the C ABI of ``libns.so`` (``include/ns.h``); ``ns`` is its thin ctypes
binding. Submodules load lazily so that the input generator can be imported on
hosts without a GPU.
"""
__all__ = ["ns", "synth", "serve", "tune"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
