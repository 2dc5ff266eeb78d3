// Blocked right-looking Cholesky A = L L^T of an SPD matrix (Sec. 2), lower
// triangle only.
//   potf2_lds_kernel / potf2_kernel   one workgroup factors the jb x jb
//                  diagonal block in 32-wide sub-blocks (held in LDS for jb <= 128);
//                  the first non-positive (or NaN) pivot records info and stops the
//                  factorization (every later kernel of the call sees info != 0 and
//                  returns).
// L21 = A21 L11^{-T} is the MFMA triangular solve of trsm.hip on the transposed
// rows; the trailing update A22 -= L21 L21^T is the MFMA GEMM in lower-tile mode.
#include "common.hpp"
#include "kernels.hpp"
#include "mixed.hpp"
#include <algorithm>

namespace cds {

namespace {

constexpr int SB = 32;

template <typename T>
__device__ __forceinline__ T sqrt_t(T x) { return sqrt(x); }

// Factor the diagonal block D = A[k:k+jb, k:k+jb] in place (lower part).
// 32-wide sub-blocks: (a) one wave factors the sub-block's diagonal in LDS,
// (b) the rows below it in the block are solved against it (one row per thread)
// and kept in LDS, (c) the rest of the block gets the symmetric update from LDS.
template <typename T>
__global__ void __launch_bounds__(256) potf2_kernel(T* A, int64_t lda, int k, int jb, int32_t* info) {
  if (*info != 0) return;
  T* D = A + k + (size_t)k * lda;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T (*S)[SB + 1] = reinterpret_cast<T (*)[SB + 1]>(smem_raw);                      // [SB][SB+1]
  T (*Pn)[SB + 1] = reinterpret_cast<T (*)[SB + 1]>(smem_raw + sizeof(T) * SB * (SB + 1));  // [jb][SB+1]
  __shared__ int s_fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_fail = 0;
  for (int s0 = 0; s0 < jb; s0 += SB) {
    const int sw = min(SB, jb - s0);
    for (int idx = tid; idx < sw * sw; idx += 256) {
      const int r = idx % sw, c = idx / sw;
      if (r >= c) S[r][c] = D[(s0 + r) + (size_t)(s0 + c) * lda];
    }
    __syncthreads();
    if (wave == 0) {
      int fail = 0;
      for (int j = 0; j < sw; ++j) {
        const T d = S[j][j];   // a_jj minus the updates of the previous columns
        if (!(d > (T)0)) { fail = j + 1; break; }
        const T ljj = sqrt_t(d);
        wave_fence();
        if (lane == j) S[j][j] = ljj;
        if (lane > j && lane < sw) S[lane][j] = S[lane][j] / ljj;
        wave_fence();
        if (lane > j && lane < sw) {
          const T lrj = S[lane][j];
          for (int c = j + 1; c <= lane; ++c) S[lane][c] -= lrj * S[c][j];
        }
        wave_fence();
      }
      if (lane == 0 && fail) {
        s_fail = 1;
        atomicCAS(info, 0, k + s0 + fail);
      }
    }
    __syncthreads();
    if (s_fail) return;
    for (int idx = tid; idx < sw * sw; idx += 256) {
      const int r = idx % sw, c = idx / sw;
      if (r >= c) D[(s0 + r) + (size_t)(s0 + c) * lda] = S[r][c];
    }
    const int rem = jb - s0 - sw;
    for (int r = tid; r < rem; r += 256) {
      T x[SB];
      const int gr = s0 + sw + r;
#pragma unroll
      for (int c = 0; c < SB; ++c) x[c] = (c < sw) ? D[gr + (size_t)(s0 + c) * lda] : (T)0;
#pragma unroll
      for (int c = 0; c < SB; ++c) {
        if (c < sw) {
          T v = x[c];
#pragma unroll
          for (int t = 0; t < c; ++t) v -= x[t] * S[c][t];
          x[c] = v / S[c][c];
        }
      }
#pragma unroll
      for (int c = 0; c < SB; ++c)
        if (c < sw) {
          D[gr + (size_t)(s0 + c) * lda] = x[c];
          Pn[r][c] = x[c];
        }
    }
    __syncthreads();
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int r = idx % rem, c = idx / rem;
      if (r < c) continue;
      const int gr = s0 + sw + r, gc = s0 + sw + c;
      T v = D[gr + (size_t)gc * lda];
      for (int t = 0; t < sw; ++t) v -= Pn[r][t] * Pn[c][t];
      D[gr + (size_t)gc * lda] = v;
    }
    __syncthreads();
  }
}


template <typename T>
__device__ __forceinline__ T lane_get(T v, int l) {
  if constexpr (std::is_same<T, double>::value) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l), hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  }
}

// Column c of the inverse of the lower-triangular 16 x 16 block at (r0, r0) of the LDS block
// (leading dimension LD), in FP64, by forward substitution: the same operations as diag_inv16_column, as
// straight-line code (the terms q < c multiply y[q] = 0 and leave the sum as it is).  EDGE: rows
// at or beyond jb act as the identity (they read row jb - 1, and the result is replaced).
template <typename T, bool EDGE, int LD>
__device__ __forceinline__ void inv16_column_ld(const T* Ds, int r0, int jb, int c, double (&y)[16]) {
  // row i of the block is read while row i - 1 is being solved
  T row[2][16];
  auto load_row = [&](T (&dst)[16], int i) {
    const int ri = EDGE ? min(r0 + i, jb - 1) : r0 + i;
#pragma unroll
    for (int q = 0; q <= i; ++q) dst[q] = Ds[(r0 + q) * LD + ri];
  };
  load_row(row[0], 0);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i + 1 < 16) load_row(row[(i + 1) & 1], i + 1);
    const T(&Lr)[16] = row[i & 1];
    double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < i; ++q) s -= (double)Lr[q] * y[q];
    const double yi = s / (double)Lr[i];
    y[i] = (EDGE && r0 + i >= jb) ? ((i == c) ? 1.0 : 0.0) : (i < c ? 0.0 : yi);
  }
}

// jb <= 128 (FP64) or 192 (FP32): the whole diagonal block lives in LDS (column-major,
// ld jb_max + 2 for FP64 and + 4 for FP32, so that every column starts on 16 bytes) for the
// duration of the kernel; its columns arrive by direct global-to-LDS loads (the upper triangle comes
// along and is never read) and the lower triangle is written back once.  Per 32-wide sub-block:
//   (a) one wave factors the sub-block's diagonal with row r in lane r (registers).
//       The entries of column j that the later columns need come from the other
//       lanes by readlane, the next column's first, so that a column's dependent
//       chain is its square root, one division (by L(j,j), which keeps exact data
//       exact) and one update.  The same wave then inverts the sub-block's two
//       16 x 16 diagonal blocks in FP64, column by column;
//   (b) the rows below it in the block, X = A_below L^{-T}, by 16 x 16 blocks on
//       MFMA tiles: X0 = B0 inv(L00)^T, B1 -= X0 L10^T, X1 = B1 inv(L11)^T;
//   (c) the rest of the block gets the symmetric rank-32 update on MFMA tiles.
// The 16 x 16 inverses are also the ones the TRSM below the block uses.
// the largest diagonal block held in LDS
template <typename T> constexpr int pjb() { return sizeof(T) == 8 ? 128 : 192; }

template <typename T>
__global__ void __launch_bounds__(256) potf2_lds_kernel(T* A, int64_t lda, int k, int jb, int32_t* info,
                                                        double* linv) {
  constexpr bool F64 = std::is_same<T, double>::value;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  constexpr int PJB = pjb<T>();
  constexpr int PLD = PJB + (F64 ? 2 : 4);
  __shared__ __align__(16) T Ds[PJB * PLD];   // (r, c) at Ds[c * PLD + r]
  __shared__ double Iv[2][16][17];   // inverses of the sub-block's 16 x 16 diagonal blocks, (i, c) at Iv[b][i][c]
  __shared__ int s_fail;
  if (*info != 0) return;
  T* D = A + k + (size_t)k * lda;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // wave w loads columns w, w + 4, ...: a column in 16-byte pieces, one per lane, where its bytes
  // are a multiple of 16 and start on 16 bytes; else as 4-byte words, 64 per instruction
  {
    const bool v16 = (jb * (int)sizeof(T)) % 16 == 0 && (uintptr_t)D % 16 == 0 && (lda * (int64_t)sizeof(T)) % 16 == 0;
    if (v16) {
      const int nq = jb * (int)sizeof(T) / 16;
      for (int c = wave; c < jb; c += 4)
        if (lane < nq)
          __builtin_amdgcn_global_load_lds((const void*)(reinterpret_cast<const char*>(D + (size_t)c * lda) + 16 * lane),
                                           (void*)(Ds + c * PLD), 16, 0, 0);
    } else {
      const int nw = jb * (int)(sizeof(T) / 4);
      for (int c = wave; c < jb; c += 4) {
        const char* src = reinterpret_cast<const char*>(D + (size_t)c * lda);
        char* dst = reinterpret_cast<char*>(Ds + c * PLD);
        for (int w0 = 0; w0 < nw; w0 += 64)
          if (w0 + lane < nw)
            __builtin_amdgcn_global_load_lds((const void*)(src + 4 * (w0 + lane)), (void*)(dst + 4 * w0), 4, 0, 0);
      }
    }
    // the direct loads into LDS count as vector memory loads
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();
  // MFMA operand and accumulator positions (16 x 16 x 4 tiles): at k-step s, lane l supplies k index
  // kidx(s, l / 16); accumulator v of lane l is element (kidx(v, l / 16), l % 16) of the result, so a
  // product's accumulators are the next product's B operand as they stand
  const int li = lane & 15, kl = lane >> 4;
  auto kidx = [&](int s) { return F64 ? 4 * s + kl : 4 * kl + s; };
  for (int s0 = 0; s0 < jb; s0 += SB) {
    const int sw = min(SB, jb - s0);
    // (a) the sub-block's diagonal
    if (wave == 0) {
      const int r = lane;
      // rows sw .. SB-1 of a short last sub-block are padded with the identity, so every
      // step runs (straight-line code; after a failed pivot the rest is not used)
      T v[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c)
        v[c] = r < sw ? (c <= r && c < sw ? Ds[(s0 + c) * PLD + s0 + r] : (T)0) : (c == r ? (T)1 : (T)0);
      // column j: its pivot d = a_jj minus the updates of the previous columns, L(j,j) = sqrt(d)
      // and the rows below divided by it; the source order puts the next column's pivot chain ahead
      // of the rest of the current column's update (each v[c] still takes the columns in order)
      int fail = 0;
      T lj;
      {
        const T d = lane_get(v[0], 0);
        if (!(d > (T)0)) fail = 1;
        const T ljj = sqrt_t(d);
        lj = (r == 0) ? ljj : (r > 0 ? v[0] / ljj : (T)0);
        v[0] = lj;
      }
#pragma unroll
      for (int j = 0; j + 1 < SB; ++j) {
        v[j + 1] -= lj * lane_get(lj, j + 1);
        const T d = lane_get(v[j + 1], j + 1);
        if (fail == 0 && !(d > (T)0)) fail = j + 2;
        const T ljj = sqrt_t(d);
        const T ln = (r == j + 1) ? ljj : (r > j + 1 ? v[j + 1] / ljj : (T)0);
        // entries above the diagonal (c > r) take junk here; they are zeroed at step c and never stored
#pragma unroll
        for (int c = j + 2; c < SB; ++c) v[c] -= lj * lane_get(lj, c);
        v[j + 1] = ln;
        lj = ln;
      }
      if (fail) {
        if (lane == 0) {
          s_fail = 1;
          atomicCAS(info, 0, k + s0 + fail);
        }
      } else {
        if (r < sw) {
#pragma unroll
          for (int c = 0; c < SB; ++c)
            if (c <= r) Ds[(s0 + c) * PLD + s0 + r] = v[c];
        }
        wave_fence();   // the inverses read entries stored by other lanes of this wave
        // lane c: column c % 16 of the inverse of diagonal block c / 16; rows at or beyond jb act as
        // the identity
        if (lane < 32) {
          const int bb = lane >> 4, cc = lane & 15, r0 = s0 + 16 * bb;
          double y[16];
          if (s0 + SB <= jb) inv16_column_ld<T, false, PLD>(Ds, r0, jb, cc, y);
          else inv16_column_ld<T, true, PLD>(Ds, r0, jb, cc, y);
#pragma unroll
          for (int i = 0; i < 16; ++i) Iv[bb][i][cc] = y[i];
          if (linv != nullptr && r0 < jb) {
#pragma unroll
            for (int i = 0; i < 16; ++i) linv[(size_t)(r0 / 16) * 256 + i * 16 + cc] = y[i];
          }
        }
      }
    }
    __syncthreads();
    if (s_fail) break;
    const int rem = jb - s0 - sw;   // rem > 0 only below a full sub-block
    // (b) rows below the sub-block, one 16-row tile per wave at a time
    for (int ti = wave; 16 * ti < rem; ti += 4) {
      const int R = s0 + SB + 16 * ti;   // first row of the tile
      const bool rin = R + li < jb;
      acc_t x0, b1, x1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x0[v] = (T)0;
        x1[v] = (T)0;
        b1[v] = rin ? Ds[(s0 + 16 + kidx(v)) * PLD + R + li] : (T)0;
      }
      // X0 = B0 inv(L00)^T (element (j, i) of the product is X0(i, j))
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T p = (T)Iv[0][li][kidx(s)];
        const T q = rin ? Ds[(s0 + kidx(s)) * PLD + R + li] : (T)0;
        if constexpr (F64) x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(p, q, x0, 0, 0, 0);
        else x0 = __builtin_amdgcn_mfma_f32_16x16x4f32(p, q, x0, 0, 0, 0);
      }
      // B1 -= X0 L10^T
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T p = -Ds[(s0 + kidx(s)) * PLD + s0 + 16 + li];
        if constexpr (F64) b1 = __builtin_amdgcn_mfma_f64_16x16x4f64(p, x0[s], b1, 0, 0, 0);
        else b1 = __builtin_amdgcn_mfma_f32_16x16x4f32(p, x0[s], b1, 0, 0, 0);
      }
      // X1 = B1 inv(L11)^T
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const T p = (T)Iv[1][li][kidx(s)];
        if constexpr (F64) x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(p, b1[s], x1, 0, 0, 0);
        else x1 = __builtin_amdgcn_mfma_f32_16x16x4f32(p, b1[s], x1, 0, 0, 0);
      }
      if (rin) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Ds[(s0 + kidx(v)) * PLD + R + li] = x0[v];
          Ds[(s0 + 16 + kidx(v)) * PLD + R + li] = x1[v];
        }
      }
    }
    __syncthreads();
    // (c) trailing part of the block on MFMA: 16 x 16 tiles (ti >= tc) of the lower triangle,
    // D = P_rows P_cols^T with P = the sub-block's columns below it
    {
      const int b0 = s0 + sw, nt = (rem + 15) / 16, ntiles = nt * (nt + 1) / 2;
      const int lg = kl;
      auto coords = [&](int tile, int& i0, int& c0) {
        int ti = (int)((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
        while (ti * (ti + 1) / 2 > tile) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        i0 = b0 + 16 * ti;
        c0 = b0 + 16 * (tile - ti * (ti + 1) / 2);
      };
      auto finish = [&](const acc_t& acc, int i0, int c0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + (F64 ? (lg + 4 * v) : (4 * lg + v)), c = c0 + li;
          if (i < jb && c <= i) Ds[c * PLD + i] -= acc[v];
        }
      };
      // two tiles per wave at a time, so that two independent MFMA chains share the k-loop
      for (int t0 = wave; t0 < ntiles; t0 += 8) {
        const bool two = t0 + 4 < ntiles;
        int i0a, c0a, i0b, c0b;
        coords(t0, i0a, c0a);
        coords(two ? t0 + 4 : t0, i0b, c0b);
        acc_t acc0, acc1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc0[v] = (T)0;
          acc1[v] = (T)0;
        }
#pragma unroll
        for (int k4 = 0; k4 < SB; k4 += 4) {
          const int kk = k4 + lg;
          const T a0 = (kk < sw && i0a + li < jb) ? Ds[(s0 + kk) * PLD + i0a + li] : (T)0;
          const T b0v = (kk < sw && c0a + li < jb) ? Ds[(s0 + kk) * PLD + c0a + li] : (T)0;
          const T a1 = (kk < sw && i0b + li < jb) ? Ds[(s0 + kk) * PLD + i0b + li] : (T)0;
          const T b1v = (kk < sw && c0b + li < jb) ? Ds[(s0 + kk) * PLD + c0b + li] : (T)0;
          if constexpr (F64) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0v, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1v, acc1, 0, 0, 0);
          } else {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0v, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1v, acc1, 0, 0, 0);
          }
        }
        finish(acc0, i0a, c0a);
        if (two) finish(acc1, i0b, c0b);
      }
    }
    __syncthreads();
  }
  // the factored (or, after a failed pivot, partially factored) lower triangle back to A
#pragma unroll 4
  for (int c = wave; c < jb; c += 4) {
#pragma unroll
    for (int q = 0; q < PJB / 64; ++q) {
      const int r = 64 * q + lane;
      if (r >= c && r < jb) D[r + (size_t)c * lda] = Ds[c * PLD + r];
    }
  }
}

}  // namespace

size_t potrf_ws_bytes(int n, int nb, size_t elem) {
  (void)n; (void)nb;
  // the diagonal-block inverses of L11 for the TRSM, sized for the largest block (512)
  (void)elem;
  return kErrRegion + ((trsm16_inv_elems(512) * sizeof(double) + 255) & ~(size_t)255);
}

template <typename T>
cds_status_t potrf_run_mode(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb, int mode, float* scale_part) {
  hipStream_t s = c.s0;
  if (launch_fill_i32(info, 1, 0, s) != hipSuccess) return CDS_HIP_ERROR;
  if (n == 0) return CDS_SUCCESS;
  if (nb <= 0) nb = n <= 2048 ? 128 : 256;
  nb = std::min(512, std::max(SB, (nb / SB) * SB));
  double* linv = (double*)((char*)c.ws + kErrRegion);
  // the diagonal block of block column k, L21 below it, and (mode 2) the operand scale
  auto panel = [&](int k, int jb, int par, hipStream_t st) -> cds_status_t {
    {
      KScope ks(c.timer, CDS_KC_PANEL, st, (double)jb * jb * jb / 3.0, (double)jb * jb * sizeof(T));
      if (jb <= pjb<T>()) {
        hipLaunchKernelGGL((potf2_lds_kernel<T>), dim3(1), dim3(256), 0, st, A, lda, k, jb, info,
                           n - k - jb > 0 ? linv : nullptr);
      } else {
        const size_t psm = sizeof(T) * (size_t)(SB + 1) * (SB + jb);
        hipLaunchKernelGGL((potf2_kernel<T>), dim3(1), dim3(256), psm, st, A, lda, k, jb, info);
      }
    }
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    const int rem = n - k - jb;
    if (rem <= 0) return CDS_SUCCESS;
    {
      // L21 = A21 L11^{-T}: the transposed column solve L11 L21^T = A21^T on MFMA tiles
      KScope ks(c.timer, CDS_KC_TRSM, st, (double)jb * jb * rem, 0.0);
      if (jb > pjb<T>() && launch_diag_inv16<T>(A + k + (size_t)k * lda, lda, 0, jb, 0, linv, 0, 1, st) != hipSuccess)
        return CDS_HIP_ERROR;
      // the staged 16-column slices (L11 and its inverses in LDS) for every size: shorter here than
      // 32-column slices that read L11 from memory, both at the end (on the critical path) and beside
      // a large rest update
      if (launch_trsm16<T>(A + k + (size_t)k * lda, lda, 0, linv, 0, A + (k + jb) + (size_t)k * lda, lda, 0, jb, rem,
                           1, 1, info, st, 1 << 30) != hipSuccess)
        return CDS_HIP_ERROR;
    }
    if (mode == 2 && scale_part != nullptr) {
      if constexpr (std::is_same<T, float>::value) {
        if (launch_maxabs_part(A + (k + jb) + (size_t)k * lda, lda, 0, rem, jb, scale_part + (size_t)par * kScaleParts, 1,
                               st) != hipSuccess)
          return CDS_HIP_ERROR;
      }
    }
    return CDS_SUCCESS;
  };
  // A[r0:r1, c0:c1] -= L21(r0:r1) L21(c0:c1)^T with L21 = A[k+jb:n, k:k+jb]; lower: only the entries on
  // or below the diagonal (r0 == c0, r1 >= c1).  par: the operand-scale region of block column k.
  auto syrk = [&](int k, int jb, int r0, int r1, int c0, int c1, bool lower, int par,
                  hipStream_t st) -> cds_status_t {
    const int m = r1 - r0, nn = c1 - c0;
    if (m <= 0 || nn <= 0) return CDS_SUCCESS;
    GemmArgs<T> g;
    g.m = m; g.n = nn; g.k = jb;
    g.A = A + r0 + (size_t)k * lda; g.lda = lda; g.strideA = 0;
    g.B = A + c0 + (size_t)k * lda; g.ldb = lda; g.strideB = 0;
    g.C = A + r0 + (size_t)c0 * lda; g.ldc = lda; g.strideC = 0;
    g.alpha = (T)-1; g.transB = 1; g.lower = lower ? 1 : 0; g.scale_part = nullptr; g.scaleA = 0;
    g.guard = info;
    if (mode == 2 && scale_part != nullptr) {
      g.scale_part = scale_part + (size_t)par * kScaleParts;
      g.scaleA = 1;   // A and B are both L21
    }
    KScope ks(c.timer, CDS_KC_UPDATE, st, lower ? (double)m * nn * jb * 2.0 - (double)nn * nn * jb : 2.0 * m * nn * jb,
              (double)sizeof(T) * ((double)m * nn + (double)(m + nn) * jb));
    return launch_gemm<T>(g, 1, mode, st) == hipSuccess ? CDS_SUCCESS : CDS_HIP_ERROR;
  };
  const bool la = c.lookahead && n > nb;
  if (!la) {
    // right-looking, in stream order
    for (int k = 0, step = 0; k < n; k += nb, ++step) {
      const int jb = std::min(nb, n - k);
      cds_status_t st = panel(k, jb, step & 1, s);
      if (st != CDS_SUCCESS) return st;
      if (n - k - jb <= 0) break;
      st = syrk(k, jb, k + jb, n, k + jb, n, true, step & 1, s);
      if (st != CDS_SUCCESS) return st;
    }
    return CDS_SUCCESS;
  }
  // Look-ahead, as in getrf: the first stream updates the next block column (its diagonal block
  // and the rows below it), then factors it (diagonal block, TRSM); the second stream updates the
  // rest of the trailing matrix meanwhile.  The next block column's update waits for the previous
  // rest update, which reached its columns.
  hipStream_t s1 = c.s1;
  hipEvent_t evL = c.ev[1], evR = c.ev[2];
  if (hipEventRecord(c.ev[0], s) != hipSuccess) return CDS_HIP_ERROR;
  if (hipStreamWaitEvent(s1, c.ev[0], 0) != hipSuccess) return CDS_HIP_ERROR;
  cds_status_t st = panel(0, std::min(nb, n), 0, s);
  if (st != CDS_SUCCESS) return st;
  bool have_rest = false;
  for (int k = 0, step = 0; k < n; k += nb, ++step) {
    const int jb = std::min(nb, n - k), par = step & 1;
    const int kn = k + jb, jbn = std::min(nb, n - kn);
    if (jbn > 0) {
      if (have_rest && hipStreamWaitEvent(s, evR, 0) != hipSuccess) return CDS_HIP_ERROR;
      st = syrk(k, jb, kn, n, kn, kn + jbn, true, par, s);   // the next diagonal block and the rows below it
      if (st != CDS_SUCCESS) return st;
    }
    if (hipEventRecord(evL, s) != hipSuccess) return CDS_HIP_ERROR;
    if (jbn > 0) {
      st = panel(kn, jbn, par ^ 1, s);
      if (st != CDS_SUCCESS) return st;
    }
    if (hipStreamWaitEvent(s1, evL, 0) != hipSuccess) return CDS_HIP_ERROR;
    if (jbn > 0) {
      st = syrk(k, jb, kn + jbn, n, kn + jbn, n, true, par, s1);
      if (st != CDS_SUCCESS) return st;
    }
    if (hipEventRecord(evR, s1) != hipSuccess) return CDS_HIP_ERROR;
    have_rest = true;
  }
  if (hipStreamWaitEvent(s, evR, 0) != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

template <typename T>
cds_status_t potrf_run(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb) {
  return potrf_run_mode<T>(c, n, A, lda, info, nb, 0, nullptr);
}

template cds_status_t potrf_run<double>(Ctx&, int, double*, int64_t, int32_t*, int);
template cds_status_t potrf_run<float>(Ctx&, int, float*, int64_t, int32_t*, int);
template cds_status_t potrf_run_mode<float>(Ctx&, int, float*, int64_t, int32_t*, int, int, float*);

}  // namespace cds
