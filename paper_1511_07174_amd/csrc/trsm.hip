// Triangular solve with many right-hand sides against a jb x jb lower triangle
// (the U12 = L11^{-1} A12 step of the blocked LU, and L21 = A21 L11^{-T} of the
// blocked Cholesky, Sec. 2: the rank-k "delayed update" needs these blocks).
//
//   diag_inv16_kernel  inverts the 16 x 16 diagonal blocks of L11 (unit or not)
//                      by substitution, one column of an inverse per thread.
//   trsm16_kernel      X = L11^{-1} B on MFMA tiles.  A workgroup holds 32
//                      columns of B (all jb rows) in LDS; for each 16-row block
//                      it forms X_b = inv(L_bb) X_b (one 16x16x16 product per
//                      column tile) and updates the rows below with
//                      -L(below, b) X_b, the L operand prefetched into
//                      registers one block ahead.  Only 16 x 16 diagonal blocks
//                      are inverted: their inverses and products stay exact on
//                      small dyadic data (denominators below 2^30), where a
//                      larger explicit inverse would not.  The inverses and the
//                      diagonal-block product are FP64 for both precisions (an
//                      FP32 inverse would round those 30-bit denominators).
// trans = 1 stores B transposed (element (r, c) at B[c + r * ldb]), which turns
// the Cholesky row solve into the same column solve.
#include "common.hpp"
#include "kernels.hpp"
#include <algorithm>

namespace cds {

namespace {


template <typename T, bool UNIT>
__global__ void __launch_bounds__(256) diag_inv16_kernel(const T* L0, int64_t lda, int64_t strideA, int jb,
                                                         double* Linv0, int64_t strideI) {
  const int b = blockIdx.y;
  const T* L = L0 + (size_t)b * strideA;
  double* Linv = Linv0 + (size_t)b * strideI;
  const int nblk = (jb + 15) / 16;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nblk * 16; t += gridDim.x * 256)
    diag_inv16_column<T, UNIT>(L, lda, jb, t >> 4, t & 15, Linv);
}

// QG: 16-row groups per wave (4 waves x QG x 16 >= jb); TCW: columns of B per workgroup (16 or 32)
template <typename T, bool TRANS, int QG, int TCW>
__global__ void __launch_bounds__(256) trsm16_kernel(const T* L0, int64_t lda, int64_t strideA, const double* Linv0,
                                                     int64_t strideI, T* B0, int64_t ldb, int64_t strideB, int jb,
                                                     int ncols, const int32_t* guard) {
  if (guard != nullptr && *guard != 0) return;
  constexpr bool F64 = std::is_same<T, double>::value;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  constexpr int PX = TCW + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);   // [nblk * 16][PX]
  __shared__ double Li[16][17];
  const int b = blockIdx.y;
  const T* L = L0 + (size_t)b * strideA;
  const double* Linv = Linv0 + (size_t)b * strideI;
  T* Bm = B0 + (size_t)b * strideB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (jb + 15) / 16, jbp = nblk * 16;
  const int ncb = (ncols + TCW - 1) / TCW;
  // a bounded grid walks the column blocks (room for a concurrent panel launch)
  for (int cbk = blockIdx.x; cbk < ncb; cbk += gridDim.x) {
  const int c0 = cbk * TCW, cw = min(TCW, ncols - c0);
  __syncthreads();   // the previous column block's stores from LDS are done
  if (TRANS) {
    for (int idx = tid; idx < jbp * TCW; idx += 256) {
      const int c = idx % TCW, r = idx / TCW;
      X[r * PX + c] = (r < jb && c < cw) ? Bm[(c0 + c) + (size_t)r * ldb] : (T)0;
    }
  } else {
    for (int idx = tid; idx < jbp * TCW; idx += 256) {
      const int r = idx % jbp, c = idx / jbp;
      X[r * PX + c] = (r < jb && c < cw) ? Bm[r + (size_t)(c0 + c) * ldb] : (T)0;
    }
  }
  // -L(rows of group g, columns of block blk); wave w owns the 16-row groups g = w + 4q
  T pre[QG][4];
  auto prefetch = [&](int blk) {
#pragma unroll
    for (int q = 0; q < QG; ++q) {
      const int g = wave + 4 * q;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int rr = 16 * g + (lane & 15), kk = 16 * blk + 4 * kc + (lane >> 4);
        pre[q][kc] = (g > blk && g < nblk && rr < jb && kk < jb) ? -L[rr + (size_t)kk * lda] : (T)0;
      }
    }
  };
  prefetch(0);
  // the diagonal-block inverses are read one block ahead too, off the dependency chain
  double li_next = Linv[tid];
  for (int blk = 0; blk < nblk; ++blk) {
    const int r0 = 16 * blk;
    const double li_cur = li_next;
    if (blk + 1 < nblk) li_next = Linv[(size_t)(blk + 1) * 256 + tid];
    __syncthreads();   // X loaded / the previous block's update done; Li free
    Li[tid >> 4][tid & 15] = li_cur;
    __syncthreads();
    // X_b <- inv(L_bb) X_b: waves 0 .. TCW / 16 - 1 each own a 16-column tile
    if (wave < TCW / 16) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double a = Li[lane & 15][4 * kc + (lane >> 4)];
        const double bb = (double)X[(r0 + 4 * kc + (lane >> 4)) * PX + wave * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(r0 + (lane >> 4) + 4 * v) * PX + wave * 16 + (lane & 15)] = (T)acc[v];
    }
    __syncthreads();
    // rows below: X_g -= L_gb X_b
    T cur[QG][4];
#pragma unroll
    for (int q = 0; q < QG; ++q)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) cur[q][kc] = pre[q][kc];
    if (blk + 1 < nblk) prefetch(blk + 1);
#pragma unroll
    for (int q = 0; q < QG; ++q) {
      const int g = wave + 4 * q;
      if (g > blk && g < nblk) {
#pragma unroll
        for (int ct = 0; ct < TCW / 16; ++ct) {
          acc_t acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = F64 ? ((lane >> 4) + 4 * v) : (4 * (lane >> 4) + v);
            acc[v] = X[(16 * g + i) * PX + ct * 16 + (lane & 15)];
          }
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const T bb = X[(r0 + 4 * kc + (lane >> 4)) * PX + ct * 16 + (lane & 15)];
            if constexpr (F64)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[q][kc], bb, acc, 0, 0, 0);
            else
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[q][kc], bb, acc, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = F64 ? ((lane >> 4) + 4 * v) : (4 * (lane >> 4) + v);
            X[(16 * g + i) * PX + ct * 16 + (lane & 15)] = acc[v];
          }
        }
      }
    }
  }
  __syncthreads();
  if (TRANS) {
    for (int idx = tid; idx < jb * TCW; idx += 256) {
      const int c = idx % TCW, r = idx / TCW;
      if (c < cw) Bm[(c0 + c) + (size_t)r * ldb] = X[r * PX + c];
    }
  } else {
    for (int idx = tid; idx < jb * TCW; idx += 256) {
      const int r = idx % jb, c = idx / jb;
      if (c < cw) Bm[r + (size_t)(c0 + c) * ldb] = X[r * PX + c];
    }
  }
  }
}

}  // namespace

size_t trsm16_inv_elems(int jb) { return (size_t)((jb + 15) / 16) * 256; }

template <typename T>
hipError_t launch_diag_inv16(const T* L, int64_t lda, int64_t strideA, int jb, int unit, double* Linv,
                             int64_t strideI, int batch, hipStream_t s) {
  if (jb <= 0 || batch <= 0) return hipSuccess;
  const int nblk = (jb + 15) / 16;
  const dim3 grid((nblk * 16 + 255) / 256, batch);
  if (unit)
    hipLaunchKernelGGL((diag_inv16_kernel<T, true>), grid, dim3(256), 0, s, L, lda, strideA, jb, Linv, strideI);
  else
    hipLaunchKernelGGL((diag_inv16_kernel<T, false>), grid, dim3(256), 0, s, L, lda, strideA, jb, Linv, strideI);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trsm16(const T* L, int64_t lda, int64_t strideA, const double* Linv, int64_t strideI, T* B,
                         int64_t ldb, int64_t strideB, int jb, int ncols, int trans, int batch, const int32_t* guard,
                         hipStream_t s) {
  if (jb <= 0 || ncols <= 0 || batch <= 0) return hipSuccess;
  const int nblk = (jb + 15) / 16;
  // at most 512 rows: 4 waves x 8 groups of 16
  if (jb > 512) return hipErrorInvalidValue;
  // narrow calls (a look-ahead's next panel) take 16-column slices: twice the workgroups on a
  // dependency chain whose length does not shrink with the width
  const bool narrow = (int64_t)batch * ncols <= 1024;
  auto go = [&](auto kern, int tcw) {
    const size_t sm = (size_t)nblk * 16 * (tcw + 1) * sizeof(T);
    const dim3 grid((ncols + tcw - 1) / tcw, batch);
    hipLaunchKernelGGL(kern, grid, dim3(256), sm, s, L, lda, strideA, Linv, strideI, B, ldb, strideB, jb, ncols, guard);
  };
  if (jb <= 256) {
    if (narrow) {
      if (trans) go(trsm16_kernel<T, true, 4, 16>, 16); else go(trsm16_kernel<T, false, 4, 16>, 16);
    } else {
      if (trans) go(trsm16_kernel<T, true, 4, 32>, 32); else go(trsm16_kernel<T, false, 4, 32>, 32);
    }
  } else {
    if (trans) go(trsm16_kernel<T, true, 8, 32>, 32); else go(trsm16_kernel<T, false, 8, 32>, 32);
  }
  return hipGetLastError();
}

template hipError_t launch_diag_inv16<double>(const double*, int64_t, int64_t, int, int, double*, int64_t, int,
                                              hipStream_t);
template hipError_t launch_diag_inv16<float>(const float*, int64_t, int64_t, int, int, double*, int64_t, int,
                                             hipStream_t);
template hipError_t launch_trsm16<double>(const double*, int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                          int64_t, int, int, int, int, const int32_t*, hipStream_t);
template hipError_t launch_trsm16<float>(const float*, int64_t, int64_t, const double*, int64_t, float*, int64_t,
                                         int64_t, int, int, int, int, const int32_t*, hipStream_t);

}  // namespace cds
