"""MI355X (gfx950) DSMC collision step: NTC selection, VHS / ab initio
quadrature / neural scattering rules and cell-wise moment matching, as
hand-written HIP kernels behind the C-ABI in include/dsmc.h.

The compiled library (libdsmc.so) is required: importing the API without it
raises ``LibraryMissing`` when a kernel is first called.  There is no CPU
fallback.
"""
from ._lib import LibraryMissing, DsmcError, load as load_library  # noqa: F401

__all__ = ["LibraryMissing", "DsmcError", "load_library"]
