"""MI355X-native fast level set evolution (arXiv 1409.7474).

The compute path is the HIP library ``liblse.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/lse.h``; ``paper_1409_7474_amd.lse`` is the thin
ctypes binding with the same names.  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["lse", "synth"]
