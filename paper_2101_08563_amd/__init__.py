"""MI355X-native FastFCA: the IP+EM iteration and multichannel Wiener filter of
Ito et al., "A Joint Diagonalization Based Efficient Approach to Underdetermined
Blind Audio Source Separation Using the Multichannel Wiener Filter"
(arXiv 2101.08563), as hand-written HIP kernels for gfx950 behind a C ABI
(include/fastfca.h). This package is the thin Python binding.
"""
from .fastfca import FastFCA, FastFCAError, load_library, LIB_PATH  # noqa: F401

__all__ = ["FastFCA", "FastFCAError", "load_library", "LIB_PATH"]
