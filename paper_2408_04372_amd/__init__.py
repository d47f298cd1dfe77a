"""MI355X space-time multigrid (STMG) hot path: C-ABI library libstmg.so plus a thin binding.

The compute path is libstmg.so (HIP for gfx950); this package only marshals
arguments (see _lib.Handle).
"""
from ._lib import Handle, StmgError, load, exported_symbols, LIB_PATH  # noqa: F401
