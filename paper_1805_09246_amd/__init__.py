"""Sliding super point sketches (SRE / SLE arrays) on MI355X, hand-written HIP for gfx950.

The library is ``libsps.so`` (C ABI in include/sps.h); ``sps`` is its ctypes binding.
Importing this package does not load the library; the first call into ``sps`` does, and
fails loudly when it has not been built.
"""
