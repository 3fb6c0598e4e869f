"""MI355X-native block-preconditioned FSI Jacobian solver.

The hot path (FGMRES + block-LDU preconditioner with AMG V-cycles, block
SpMV and Gram-Schmidt) runs in ``libfsi.so``, hand-written HIP for gfx950
behind the C ABI in ``include/fsi.h``.  ``fsi`` is the Python binding.
"""
from .fsi import FsiError, FsiSolver, HIERARCHIES, load  # noqa: F401
