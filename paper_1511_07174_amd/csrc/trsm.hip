// Triangular solve with many right-hand sides against a jb x jb lower triangle
// (the U12 = L11^{-1} A12 step of the blocked LU, and L21 = A21 L11^{-T} of the
// blocked Cholesky, Sec. 2: the delayed rank-k update needs these blocks).
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

// LDS bytes of the staged variant: X, the negated 16 x 16 tiles of L11 below the diagonal
// (tile (g, blk), g > blk, at index g (g - 1) / 2 + blk, stored column by column) and the
// diagonal-block inverses
__host__ __device__ inline size_t trsm16_stage_bytes(int nblk, int tcw, size_t elem) {
  return (size_t)nblk * 16 * (tcw + 1) * elem + (size_t)nblk * (nblk - 1) / 2 * 256 * elem + 16 +
         (size_t)nblk * 256 * 8;   // + 16: the inverses start 16-byte aligned
}

// QG: 16-row groups per wave (4 waves x QG x 16 >= jb); TCW: columns of B per workgroup (16 or 32).
// STAGE: L11's tiles below the diagonal and the diagonal-block inverses are copied to LDS once,
// before the first column block, so that the block chain reads no global memory; otherwise they
// are read from memory one block ahead.
template <typename T, bool TRANS, int QG, int TCW, bool STAGE>
__global__ void __launch_bounds__(256) trsm16_kernel(const T* L0, int64_t lda, int64_t strideA, const double* Linv0,
                                                     int64_t strideI, T* B0, int64_t ldb, int64_t strideB, int jb,
                                                     int ncols, const int32_t* guard) {
  if (guard != nullptr && *guard != 0) return;
  constexpr bool F64 = std::is_same<T, double>::value;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  constexpr int PX = TCW + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);   // [nblk * 16][PX]
  __shared__ double Li[STAGE ? 1 : 16][17];
  const int b = blockIdx.y;
  const T* L = L0 + (size_t)b * strideA;
  const double* Linv = Linv0 + (size_t)b * strideI;
  T* Bm = B0 + (size_t)b * strideB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (jb + 15) / 16, jbp = nblk * 16;
  const int ncb = (ncols + TCW - 1) / TCW;
  const int ntile = nblk * (nblk - 1) / 2;
  T* Ls = X + (size_t)jbp * PX;
  double* Lis = reinterpret_cast<double*>(smem_raw + (((size_t)jbp * PX + (size_t)ntile * 256) * sizeof(T) + 15) / 16 * 16);
  if constexpr (STAGE) {
    // element (i, j) of tile (g, blk) is L(16 g + i, 16 blk + j), at j * 16 + i (negated where read)
    if (sizeof(T) == 4 && jb % 16 == 0) {
      // direct global -> LDS loads, none of which waits for another: wave w fills elements
      // [64 w, 64 w + 64) of every tile, lane l element 64 w + l = (i, j) = (l & 15, 4 w + l / 16)
      const int i = lane & 15, j = 4 * wave + (lane >> 4);
      int tt = 0;
      for (int g = 1; g < nblk; ++g)
        for (int bl = 0; bl < g; ++bl, ++tt)
          __builtin_amdgcn_global_load_lds((const void*)(L + (16 * g + i) + (size_t)(16 * bl + j) * lda),
                                           (void*)(Ls + (size_t)tt * 256 + 64 * wave), 4, 0, 0);
    } else {
      // eight loads in flight per thread before their LDS stores; element j * 16 + i = tid
      const int i = tid & 15, j = tid >> 4;
      int g = 1, bl = 0;
      for (int t0 = 0; t0 < ntile; t0 += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = 16 * g + i, kk = 16 * bl + j;
          v[u] = (t0 + u < ntile && rr < jb && kk < jb) ? L[rr + (size_t)kk * lda] : (T)0;
          if (++bl == g) {
            ++g;
            bl = 0;
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (t0 + u < ntile) Ls[(size_t)(t0 + u) * 256 + tid] = v[u];
      }
    }
    // the inverses (16-byte aligned on both sides), 16 bytes per lane
    for (int e0 = wave * 128; e0 < nblk * 256; e0 += 512)
      __builtin_amdgcn_global_load_lds((const void*)(Linv + e0 + 2 * lane), (void*)(Lis + e0), 16, 0, 0);
  }
  // a bounded grid walks the column blocks (room for a concurrent panel launch)
  for (int cbk = blockIdx.x; cbk < ncb; cbk += gridDim.x) {
  const int c0 = cbk * TCW, cw = min(TCW, ncols - c0);
  __syncthreads();   // the previous column block's stores from LDS are done
  // B's block to LDS, eight loads in flight per thread before their stores
  for (int base = 0; base < jbp * TCW; base += 256 * 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * 256 + tid;
      int r, c;
      if (TRANS) { c = idx % TCW; r = idx / TCW; } else { r = idx % jbp; c = idx / jbp; }
      const bool ok = idx < jbp * TCW && r < jb && c < cw;
      v[u] = ok ? (TRANS ? Bm[(c0 + c) + (size_t)r * ldb] : Bm[r + (size_t)(c0 + c) * ldb]) : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * 256 + tid;
      int r, c;
      if (TRANS) { c = idx % TCW; r = idx / TCW; } else { r = idx % jbp; c = idx / jbp; }
      if (idx < jbp * TCW) X[r * PX + c] = v[u];
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
  if constexpr (!STAGE) prefetch(0);
  // the diagonal-block inverses are read one block ahead too, off the dependency chain
  double li_next = STAGE ? 0.0 : Linv[tid];
  for (int blk = 0; blk < nblk; ++blk) {
    const int r0 = 16 * blk;
    if constexpr (!STAGE) {
      const double li_cur = li_next;
      if (blk + 1 < nblk) li_next = Linv[(size_t)(blk + 1) * 256 + tid];
      __syncthreads();   // X loaded / the previous block's update done; Li free
      Li[tid >> 4][tid & 15] = li_cur;
    }
    // (staged) the direct loads into LDS have landed: they count as vector memory loads
    if constexpr (STAGE)
      if (blk == 0) __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();   // (staged) X loaded / the previous block's update done
    // X_b <- inv(L_bb) X_b: waves 0 .. TCW / 16 - 1 each own a 16-column tile
    if (wave < TCW / 16) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double a = STAGE ? Lis[(size_t)blk * 256 + (lane & 15) * 16 + 4 * kc + (lane >> 4)]
                               : Li[(lane & 15) % (STAGE ? 1 : 16)][4 * kc + (lane >> 4)];
        const double bb = (double)X[(r0 + 4 * kc + (lane >> 4)) * PX + wave * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(r0 + (lane >> 4) + 4 * v) * PX + wave * 16 + (lane & 15)] = (T)acc[v];
    }
    __syncthreads();
    // rows below: X_g -= L_gb X_b
    T cur[QG][4];
    if constexpr (STAGE) {
#pragma unroll
      for (int q = 0; q < QG; ++q) {
        const int g = wave + 4 * q;
        const bool on = g > blk && g < nblk;
        const size_t tb = on ? ((size_t)(g * (g - 1) / 2 + blk) * 256) : 0;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) cur[q][kc] = on ? -Ls[tb + 64 * kc + lane] : (T)0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < QG; ++q)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) cur[q][kc] = pre[q][kc];
      if (blk + 1 < nblk) prefetch(blk + 1);
    }
    if constexpr (QG <= 4) {
      // every LDS read of the step (block b's rows, then each group's rows) before the MFMAs, every
      // write after them; the groups' rows are disjoint and block b's rows are only read here
      T bbv[TCW / 16][4];
  #pragma unroll
      for (int ct = 0; ct < TCW / 16; ++ct)
  #pragma unroll
        for (int kc = 0; kc < 4; ++kc) bbv[ct][kc] = X[(r0 + 4 * kc + (lane >> 4)) * PX + ct * 16 + (lane & 15)];
      acc_t accs[QG][TCW / 16];
  #pragma unroll
      for (int q = 0; q < QG; ++q) {
        const int g = wave + 4 * q;
        if (g > blk && g < nblk) {
  #pragma unroll
          for (int ct = 0; ct < TCW / 16; ++ct)
  #pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = F64 ? ((lane >> 4) + 4 * v) : (4 * (lane >> 4) + v);
              accs[q][ct][v] = X[(16 * g + i) * PX + ct * 16 + (lane & 15)];
            }
        }
      }
  #pragma unroll
      for (int q = 0; q < QG; ++q) {
        const int g = wave + 4 * q;
        if (g > blk && g < nblk) {
  #pragma unroll
          for (int ct = 0; ct < TCW / 16; ++ct)
  #pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
              if constexpr (F64)
                accs[q][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[q][kc], bbv[ct][kc], accs[q][ct], 0, 0, 0);
              else
                accs[q][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[q][kc], bbv[ct][kc], accs[q][ct], 0, 0, 0);
            }
        }
      }
  #pragma unroll
      for (int q = 0; q < QG; ++q) {
        const int g = wave + 4 * q;
        if (g > blk && g < nblk) {
  #pragma unroll
          for (int ct = 0; ct < TCW / 16; ++ct)
  #pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = F64 ? ((lane >> 4) + 4 * v) : (4 * (lane >> 4) + v);
              X[(16 * g + i) * PX + ct * 16 + (lane & 15)] = accs[q][ct][v];
            }
        }
      }
    } else {
      // eight groups: one group at a time (the batched form would not fit in registers)
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
                         hipStream_t s, int narrow_cols) {
  if (jb <= 0 || ncols <= 0 || batch <= 0) return hipSuccess;
  const int nblk = (jb + 15) / 16;
  // at most 512 rows: 4 waves x 8 groups of 16
  if (jb > 512) return hipErrorInvalidValue;
  // narrow calls (a look-ahead's next panel) take 16-column slices: twice the workgroups on a
  // dependency chain whose length does not shrink with the width
  const bool narrow = (int64_t)batch * ncols <= narrow_cols;
  auto go = [&](auto kern, int tcw, bool stage) {
    const size_t sm = stage ? trsm16_stage_bytes(nblk, tcw, sizeof(T)) : (size_t)nblk * 16 * (tcw + 1) * sizeof(T);
    const dim3 grid((ncols + tcw - 1) / tcw, batch);
    hipLaunchKernelGGL(kern, grid, dim3(256), sm, s, L, lda, strideA, Linv, strideI, B, ldb, strideB, jb, ncols, guard);
  };
  // the narrow calls sit on the critical path between panels: they stage L11 in LDS when it fits
  const bool stage = narrow && jb <= 256 && trsm16_stage_bytes(nblk, 16, sizeof(T)) <= (size_t)150 * 1024;
  if (jb <= 256) {
    if (narrow) {
      if (stage) {
        if (trans) go(trsm16_kernel<T, true, 4, 16, true>, 16, true); else go(trsm16_kernel<T, false, 4, 16, true>, 16, true);
      } else {
        if (trans) go(trsm16_kernel<T, true, 4, 16, false>, 16, false); else go(trsm16_kernel<T, false, 4, 16, false>, 16, false);
      }
    } else {
      if (trans) go(trsm16_kernel<T, true, 4, 32, false>, 32, false); else go(trsm16_kernel<T, false, 4, 32, false>, 32, false);
    }
  } else {
    if (trans) go(trsm16_kernel<T, true, 8, 32, false>, 32, false); else go(trsm16_kernel<T, false, 8, 32, false>, 32, false);
  }
  return hipGetLastError();
}

template hipError_t launch_diag_inv16<double>(const double*, int64_t, int64_t, int, int, double*, int64_t, int,
                                              hipStream_t);
template hipError_t launch_diag_inv16<float>(const float*, int64_t, int64_t, int, int, double*, int64_t, int,
                                             hipStream_t);
template hipError_t launch_trsm16<double>(const double*, int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                          int64_t, int, int, int, int, const int32_t*, hipStream_t, int);
template hipError_t launch_trsm16<float>(const float*, int64_t, int64_t, const double*, int64_t, float*, int64_t,
                                         int64_t, int, int, int, int, const int32_t*, hipStream_t, int);

}  // namespace cds
