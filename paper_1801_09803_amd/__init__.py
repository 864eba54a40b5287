"""MI355X line-by-line molecular cross sections (HIP/CDNA4), after the ExoCross paper.

The compute path is libxsec.so (hand-written HIP kernels behind a C ABI, see
include/xsec.h); this package only marshals arguments to it.  There is no CPU
fallback: importing the binding fails loudly if the library is missing.
"""
from .binding import (  # noqa: F401
    Plan, Graph, Stream, XsecError, lib_path, load_library, PROFILES, PRECISIONS, BROADENING, abi_version,
)
