// Internal launch interfaces of the gfx950 kernels (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <type_traits>
#include <vector>
#include "../../include/cds.h"

namespace cds {

// C += alpha * A * op(B); A m x k, op(B) k x n, all column-major.  The native-precision
// kernel applies alpha to A (exact for the alpha = -1 of every caller).
// transB = 1: op(B) = B^T with B stored n x k (ldb).
// lower = 1 (m >= n): only C(i, j) with i >= j is computed and written.
// For the FP16 operand mode, op(B) is multiplied before rounding by the power of
// two 2^e that brings max|op(B)| to [2^13, 2^14) (|e| <= 100), and the product by
// 2^-e; max|op(B)| comes as kScaleParts partial maxima per matrix (scale_part,
// written by launch_maxabs_part; one wave reduces them, so there are 64).  With
// scaleA the A operand is multiplied by 2^e too (|e| <= 50) and the product by 2^-2e.
constexpr int kScaleParts = 64;

template <typename T>
struct GemmArgs {
  int m, n, k;
  const T* A; int64_t lda; int64_t strideA;
  const T* B; int64_t ldb; int64_t strideB;
  T* C; int64_t ldc; int64_t strideC;
  T alpha;
  int transB;
  int lower;
  const float* scale_part;   // mode 2: kScaleParts partial maxima of |op(B)| per matrix, or null (no scaling)
  int scaleA;                // mode 2: A takes the same power of two as op(B) (the two are one block, as in SYRK)
  const int32_t* guard;   // optional: the launch does nothing when *guard != 0
};
// mode: 0 native MFMA of T, 1 bf16 operands (T = float), 2 fp16 operands (T = float)
template <typename T>
hipError_t launch_gemm(const GemmArgs<T>& g, int batch, int mode, hipStream_t s);

// Optional per-launch timing (events around launches of a kernel class).
struct KTimer {
  struct Rec { int kc; hipEvent_t a, b; double flops, bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t next();
  void reset();
  ~KTimer();
};

// RAII scope: records an event before and after the launches made inside it.
struct KScope {
  KTimer* t;
  hipStream_t s;
  size_t idx;
  KScope(KTimer* timer, int kc, hipStream_t stream, double flops, double bytes);
  ~KScope();
};

// Execution context shared by the drivers.
struct Ctx {
  hipStream_t s0;          // caller's stream
  hipStream_t s1;          // internal look-ahead stream
  hipEvent_t ev[4];        // fork/join events
  void* ws;                // workspace base (device)
  size_t ws_bytes;
  int* err;                // device error word (at the workspace base)
  int nb_override;
  int lookahead;
  int leaf;
  KTimer* timer;           // null unless kernel timing is on
};

// Sizes of the workspace regions (bytes), shared by bufferSize queries and drivers.
constexpr size_t kErrRegion = 256;
// Blocked triangular solve X = L^{-1} B (jb x jb lower L, unit or not) on MFMA tiles, from the
// FP64 inverses of L's 16 x 16 diagonal blocks (launch_diag_inv16, trsm16_inv_elems(jb) doubles
// per matrix).  trans = 1: B element (r, c) stored at B[c + r * ldb].  guard: skip when *guard != 0.
// Calls with at most narrow_cols columns in all take 16-column slices (staging L11 in LDS).
size_t trsm16_inv_elems(int jb);
template <typename T>
hipError_t launch_diag_inv16(const T* L, int64_t lda, int64_t strideA, int jb, int unit, double* Linv,
                             int64_t strideI, int batch, hipStream_t s);
template <typename T>
hipError_t launch_trsm16(const T* L, int64_t lda, int64_t strideA, const double* Linv, int64_t strideI, T* B,
                         int64_t ldb, int64_t strideB, int jb, int ncols, int trans, int batch, const int32_t* guard,
                         hipStream_t s, int narrow_cols = 1024);
size_t getrf_ws_bytes(int n, int nb, int leaf, int batch, size_t elem);
size_t getrs_ws_bytes(int n, int nrhs, int batch, size_t elem);
size_t potrf_ws_bytes(int n, int nb, size_t elem);

template <typename T>
cds_status_t getrf_run(Ctx& c, int n, T* A, int64_t lda, int64_t strideA, int32_t* ipiv, int64_t strideP,
                       int32_t* info, int batch, int nb);
template <typename T>
cds_status_t getrs_run(Ctx& c, int trans, int n, int nrhs, const T* LU, int64_t lda, int64_t strideA,
                       const int32_t* ipiv, int64_t strideP, T* B, int64_t ldb, int64_t strideB, int batch,
                       void* ws, size_t ws_bytes);
template <typename T>
cds_status_t potrf_run(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb);
template <typename T>
cds_status_t potrs_run(Ctx& c, int n, int nrhs, const T* L, int64_t lda, T* B, int64_t ldb, void* ws, size_t ws_bytes);

// small utility kernels
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s);

}  // namespace cds
