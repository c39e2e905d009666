"""MI355X-native AIR reconstruction path (arXiv 1310.1434).

The compute lives in ``libair.so`` (hand-written HIP kernels for gfx950 behind
the C ABI of ``include/air.h``); ``air`` is its ctypes binding.  Importing
``paper_1310_1434_amd.air`` fails loudly if the library is not built.
"""
__all__ = ["air", "build"]
