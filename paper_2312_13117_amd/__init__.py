"""MI355X-native contour-integral eigensolver (pmCIMb quadrature sweep).

The compute path is the HIP library ``libnep.so`` (kernels + C ABI declared in
include/nep.h).  ``paper_2312_13117_amd.nep`` is a thin ctypes binding with the same
entry-point names; it only marshals arguments.  Importing the binding on a machine
without the built library raises immediately: there is no fallback path.
"""
__all__ = ["nep", "build"]
