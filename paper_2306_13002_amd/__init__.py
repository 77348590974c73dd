"""MI355X stencil sweeps in plain and saturated forms (HIP, gfx950).

The compute lives in ``libstencil.so`` (C ABI, ``include/stencil.h``); the
Python side only marshals arguments.  Importing this package does not load
the library; ``paper_2306_13002_amd.stencil`` does, and raises if it is not
built.
"""
__all__ = ["stencil", "synth"]
