"""MI355X (gfx950) communication-manager data path of the HiCR model.

``paper_2509_01425_amd.hicr`` is the ctypes binding of ``libhicr.so``: slots,
fused batched memcpy, per-slot counters, fences and channels, all executed by
the library's own HIP kernels.  Build the library with
``python -m paper_2509_01425_amd.build``.
"""
