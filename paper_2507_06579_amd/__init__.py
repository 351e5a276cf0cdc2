"""MI355X (gfx950) search for Eisenstein discriminants (Breuer & Punch).

The work runs in ``libeis.so`` (hand-written HIP kernels behind the C ABI of
``include/eis.h``); this package is a thin ctypes binding with the same
names.  Importing the package does not load the library; the first call that
needs it does, and raises if it was not built.
"""
from ._lib import (  # noqa: F401
    EIS_MAX_D,
    EIS_FLAG_NO_GRAPHS,
    EIS_FLAG_KERNEL_TIMES,
    EIS_FLAG_NO_CONJUGATE_LOOKUPS,
    EIS_FLAG_NO_SMALL_NORM_PRODUCT,
    EIS_SET_SQUAREFREE,
    EIS_SET_PRIME,
    KERNELS,
    ABI_VERSION,
    EisError,
    Context,
    Status,
    Method,
    lib,
    lib_path,
    eis_num_candidates,
    eis_first_candidate,
    eis_strerror,
    eis_abi_version,
    EXPORTED_SYMBOLS,
    NOALLOC_MAX_CANDIDATES,
)
