"""Memory-safe GPU co-scheduler for one MI355X (gfx950).

The compute path is the HIP library ``libsched.so`` (sources in ``csrc/``,
C ABI in ``include/cosched.h``); ``cosched`` is its Python binding.  Nothing
is loaded at import time.
"""
__all__ = ["cosched"]
