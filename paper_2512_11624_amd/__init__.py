"""MI355X-native hot path of Gaussian-primitive slice-to-volume reconstruction.

The compute lives in ``libsvr.so`` (hand-written HIP for gfx950 behind a C ABI,
declared in ``include/svr.h``).  ``paper_2512_11624_amd.svr`` is the thin ctypes
binding; ``synth`` draws seeded synthetic inputs.  Importing the package does
not load the library: ``svr.load()`` does, and fails loudly if it is missing.
"""
__all__ = ["synth", "svr"]
