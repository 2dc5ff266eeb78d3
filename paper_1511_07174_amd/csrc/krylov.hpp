// Internal interface of the Krylov solvers (krylov.hip).
#pragma once
#include "kernels.hpp"

namespace cds {

// Workspace of krylov_run; precond_nb > 0 adds the triangular-solve region of a preconditioner.
size_t krylov_ws_bytes(int method, int n, int restart, int precond_nb);

// One Krylov solve.  LUlo / perm (GMRES only, may be null): FP32 LU factors and the row order of
// their pivots, applied as a left preconditioner.
cds_status_t krylov_run(Ctx& c, int method, int n, const double* A, int64_t lda, const double* b, double* x,
                        const cds_krylov_params_t& p, cds_krylov_result_t* res, const float* LUlo,
                        const int32_t* perm);

}  // namespace cds
