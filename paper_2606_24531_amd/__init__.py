"""aceseek: gfx950 two-layer decoder for absolute-offset LZ77 + interleaved
rANS archives (paper: unified position-invariant random access through two
compression layers via absolute-offset coordinates).

The compute path is the C-ABI library libaceseek.so (HIP kernels); this
package only marshals arguments.  Import fails loudly if the library has not
been built.
"""
from .aceseek import (Archive, AceError, EncodeParams, OutOfCoreArchive, Tuning, encode,
                      encode_bound, library_path)

__all__ = ["Archive", "AceError", "EncodeParams", "OutOfCoreArchive", "Tuning", "encode",
           "encode_bound", "library_path"]
