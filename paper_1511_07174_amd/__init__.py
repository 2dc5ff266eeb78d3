"""Dense direct solvers of arXiv 1511.07174 (Sec. 2: A = LU with partial pivoting
or A = L L^T, then Ly = b and Ux = y) for one AMD MI355X (gfx950).

The compute path is the HIP library libcds.so (C-ABI in include/cds.h); this
package is its Python binding.  Importing the package does not load the
library; the first call does, and raises if it has not been built.
"""
from .cds import (CdsError, Handle, IrParams, IrResult, colmajor, default_params, handle, lib,  # noqa: F401
                  EXPORTED, LIB_PATH)
from .solvers import (getrf, getrs, potrf, potrs, solve, solve_vbatched, SolveFn, solve_ad,  # noqa: F401
                      krylov_solve, solve_gmres_ir)

__all__ = ["getrf", "getrs", "potrf", "potrs", "solve", "solve_vbatched", "SolveFn", "solve_ad", "Handle",
           "krylov_solve", "solve_gmres_ir",
           "IrParams", "default_params", "colmajor", "handle", "lib", "CdsError"]
