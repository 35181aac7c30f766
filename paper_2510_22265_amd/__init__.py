"""EBCC on MI355X: two-layer error-bounded compression of 2-D float32 fields.

The compute path lives in ``libebcc.so`` (hand-written HIP for gfx950, C ABI
declared in ``include/ebcc.h``).  ``paper_2510_22265_amd.ebcc`` is the thin
ctypes binding; ``paper_2510_22265_amd.synth`` holds the seeded synthetic
field generators.  Importing the package does not load the GPU library.
"""
__all__ = ["ebcc", "synth"]
