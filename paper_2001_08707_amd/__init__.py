"""MI355X-native shifted Krylov solver for (z_k I - H) x^(k) = b.

The compute path lives in the HIP library libkomega_hip.so (sources under
csrc/, C interface in include/komega_hip.h).  This package is a thin ctypes
binding over it plus seeded input generators.  Importing the package does not
load the native library; `paper_2001_08707_amd.komega` does, and fails loudly
if it has not been built.
"""
__all__ = ["inputs"]
