// Internal interface of the persistent batched SPD solver.
#pragma once
#include "kernels.hpp"

namespace cds {

int vbatched_grid();
size_t vbatched_ws_bytes(int batch, int nmax, int nrhs);
cds_status_t vbatched_run(Ctx& c, int batch, int nmax, const int32_t* n, const double* const* A, const int64_t* lda,
                          const double* const* B, const int64_t* ldb, double* const* X, const int64_t* ldx, int nrhs,
                          const int32_t* order, const cds_ir_params_t& prm, cds_ir_result_t* res, uint64_t* t_start,
                          uint64_t* t_end, int jw32_max_n);

}  // namespace cds
