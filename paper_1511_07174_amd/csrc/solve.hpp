// Internal interface of the triangular-solve driver shared by getrs/potrs and
// the refinement loops.
#pragma once
#include "kernels.hpp"

namespace cds {

// Solve op(M) X = B for the factors of getrf (chol = 0) or potrf (chol = 1).
// T: factor / working precision; S: precision of B and X.
// The solution overwrites X (accumulate = 0) or is added to it (accumulate = 1).
// perm (optional): precomputed row order of ipiv; active (optional): per-matrix
// flag, matrices with active[b] == 0 are skipped by every kernel.
template <typename T, typename S>
struct GetrsCore {
  int trans, chol, n, nrhs, batch;
  const T* M; int64_t lda; int64_t strideA;
  const int32_t* ipiv; int64_t strideP;
  const int32_t* perm; int64_t strideQ;
  const S* B; int64_t ldb; int64_t strideB;
  S* X; int64_t ldx; int64_t strideX;
  int accumulate;
  const int* active;
  void* ws; size_t ws_bytes;
  // optional (FP32 factors, op N, one right-hand side): launch_binv_prep's output for M, which
  // switches the two triangular solves to the block-inverse kernel
  const float* binv;
};

template <typename T, typename S>
cds_status_t getrs_core(Ctx& c, const GetrsCore<T, S>& g);

size_t trsv_slot_bytes(int n, int nrhs, int batch, size_t elem);
// Diagonal-block inverses and chain products of the LU factors for the block-inverse solve:
// binv_elems(n) floats per matrix, filled by launch_binv_prep from the factors of getrf.
size_t binv_elems(int n);
hipError_t launch_binv_prep(const float* LU, int64_t lda, int64_t strideA, int n, float* out, int64_t strideO,
                            int batch, hipStream_t s);
// Row order of LAPACK interchanges (perm[i] = original row at position i).  gmap: scratch of
// perm_moves_ints(n) ints per matrix for the chunked method, or null for the per-position trace.
size_t perm_moves_ints(int n);
hipError_t launch_perm(const int32_t* ipiv, int64_t strideP, int n, int32_t* perm, int64_t strideQ, int32_t* gmap,
                       int batch, hipStream_t s);

}  // namespace cds
