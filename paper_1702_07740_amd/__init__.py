"""MI355X-native syndrome-form sum-product decoder for QC multi-edge LDPC codes.

The decoder runs as hand-written HIP kernels for gfx950 behind the C-ABI
library ``libldpc.so`` (declared in ``include/ldpc.h``); ``ldpc`` is the thin
ctypes binding over it.  ``synth`` draws seeded synthetic inputs.
"""
__all__ = ["ldpc", "synth"]
