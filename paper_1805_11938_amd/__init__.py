"""MI355X-native SpMV over five storage formats (CSR, CSR5, ELL, SELL-C-sigma, HYB).

The compute lives in ``libspmv.so`` (hand-written HIP for gfx950) behind the
C-ABI of ``include/spmv.h``; ``paper_1805_11938_amd.spmv`` is the thin ctypes
binding.  PyTorch is used only for device memory and streams.
"""
__all__ = ["spmv", "synth"]
