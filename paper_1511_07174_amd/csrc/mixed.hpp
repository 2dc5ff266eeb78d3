// Internal interface of the mixed-precision refinement drivers.
#pragma once
#include "kernels.hpp"

namespace cds {

template <typename T>
// perm_out (optional, n per matrix): the row order of the factorization (perm[i] = original row at
// position i), built alongside the interchanges
cds_status_t getrf_run_mode(Ctx& c, int n, T* A, int64_t lda, int64_t strideA, int32_t* ipiv, int64_t strideP,
                            int32_t* info, int batch, int nb, int mode, float* scale_part, int32_t* perm_out = nullptr);
template <typename T>
cds_status_t potrf_run_mode(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb, int mode, float* scale_part);

size_t ir_ws_bytes(int n, int nrhs, int batch, int nb, int chol, int fallback);

cds_status_t gesv_mixed_run(Ctx& c, int prec, int n, int nrhs, const double* A, int64_t lda, int64_t strideA,
                            const double* B, int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                            float* LU, int64_t strideLU, int32_t* ipiv, int64_t strideP, const cds_ir_params_t& prm,
                            cds_ir_result_t* res, int batch, int nb);
cds_status_t getrs_mixed_run(Ctx& c, int trans, int n, int nrhs, const double* A, int64_t lda, int64_t strideA,
                             const float* LU, int64_t strideLU, const int32_t* ipiv, int64_t strideP, const double* B,
                             int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                             const cds_ir_params_t& prm, cds_ir_result_t* res, int batch);
cds_status_t posv_mixed_run(Ctx& c, int prec, int n, int nrhs, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* X, int64_t ldx, float* L, const cds_ir_params_t& prm,
                            cds_ir_result_t* res, int nb);

size_t gmres_ir_ws_bytes(int n, int nb, int restart);
cds_status_t gesv_gmres_ir_run(Ctx& c, int prec, int n, const double* A, int64_t lda, const double* b, double* x,
                               float* LU, int32_t* ipiv, const cds_ir_params_t& prm, const cds_krylov_params_t& kp,
                               cds_ir_result_t* res, int nb);

// kScaleParts partial maxima of |B| (rows x cols, column-major) per matrix into part[b * kScaleParts + p]
hipError_t launch_maxabs_part(const float* B, int64_t ldb, int64_t strideB, int rows, int cols, float* part, int batch,
                              hipStream_t s);
hipError_t launch_outer(int m, int n, int k, double alpha, const double* X, int64_t ldx, int64_t strideX,
                        const double* Y, int64_t ldy, int64_t strideY, double* C, int64_t ldc, int64_t strideC,
                        int batch, hipStream_t s);

}  // namespace cds
