"""MI355X-native NUFFT Lomb-Scargle periodograms (nifty-ls method, hand-written HIP).

The compute path lives in ``libmils.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/mils.h``); ``paper_2409_08090_amd.mils`` is the thin ctypes
binding that marshals torch device tensors into it.  Importing this package does
not load the library; the binding does, and fails loudly when it is missing.
"""
__all__ = ["mils", "workloads"]
