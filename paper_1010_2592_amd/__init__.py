"""MI355X multi-shift BiCGstab(l): single-pass and double-pass f(A) b.

The compute path is the HIP library libmsb.so (C-ABI in include/msb.h); the
Python modules here only marshal arguments to it.
"""
__version__ = "0.1.0"
