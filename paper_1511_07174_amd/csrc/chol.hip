// Blocked right-looking Cholesky A = L L^T (Sec. 2: "In the case of SPD
// matrices, we have A = LL^t"), lower triangle only.
//   potf2_kernel   one workgroup factors the jb x jb diagonal block in 32-wide
//                  sub-blocks; the first non-positive (or NaN) pivot records
//                  info and stops the factorization (every later kernel of the
//                  call sees info != 0 and returns).
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

}  // namespace

size_t potrf_ws_bytes(int n, int nb, size_t elem) {
  (void)n; (void)nb;
  // the diagonal-block inverses of L11 for the TRSM, sized for the largest block (512)
  (void)elem;
  return kErrRegion + ((trsm16_inv_elems(512) * sizeof(double) + 255) & ~(size_t)255);
}

template <typename T>
cds_status_t potrf_run_mode(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb, int mode, int* scale_exp) {
  hipStream_t s = c.s0;
  if (launch_fill_i32(info, 1, 0, s) != hipSuccess) return CDS_HIP_ERROR;
  if (n == 0) return CDS_SUCCESS;
  if (nb <= 0) nb = n <= 2048 ? 128 : 256;
  nb = std::min(512, std::max(SB, (nb / SB) * SB));
  for (int k = 0; k < n; k += nb) {
    const int jb = std::min(nb, n - k);
    size_t psm = sizeof(T) * (size_t)(SB + 1) * (SB + jb);
    {
      KScope ks(c.timer, CDS_KC_PANEL, s, (double)jb * jb * jb / 3.0, (double)jb * jb * sizeof(T));
      hipLaunchKernelGGL((potf2_kernel<T>), dim3(1), dim3(256), psm, s, A, lda, k, jb, info);
    }
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    const int rem = n - k - jb;
    if (rem <= 0) break;
    {
      // L21 = A21 L11^{-T}: the transposed column solve L11 L21^T = A21^T on MFMA tiles
      KScope ks(c.timer, CDS_KC_TRSM, s, (double)jb * jb * rem, 0.0);
      double* linv = (double*)((char*)c.ws + kErrRegion);
      if (launch_diag_inv16<T>(A + k + (size_t)k * lda, lda, 0, jb, 0, linv, 0, 1, s) != hipSuccess)
        return CDS_HIP_ERROR;
      if (launch_trsm16<T>(A + k + (size_t)k * lda, lda, 0, linv, 0, A + (k + jb) + (size_t)k * lda, lda, 0, jb, rem,
                           1, 1, info, s) != hipSuccess)
        return CDS_HIP_ERROR;
    }
    GemmArgs<T> g;
    g.m = rem; g.n = rem; g.k = jb;
    g.A = A + (k + jb) + (size_t)k * lda; g.lda = lda; g.strideA = 0;
    g.B = A + (k + jb) + (size_t)k * lda; g.ldb = lda; g.strideB = 0;
    g.C = A + (k + jb) + (size_t)(k + jb) * lda; g.ldc = lda; g.strideC = 0;
    g.alpha = (T)-1; g.transB = 1; g.lower = 1; g.scale_exp = nullptr;
    g.guard = info;
    if (mode == 2 && scale_exp != nullptr) {
      if constexpr (std::is_same<T, float>::value) {
        if (launch_maxabs_exp(A + (k + jb) + (size_t)k * lda, lda, 0, rem, jb, scale_exp, 1, s) != hipSuccess)
          return CDS_HIP_ERROR;
      }
      g.scale_exp = scale_exp;
    }
    KScope ks(c.timer, CDS_KC_UPDATE, s, (double)rem * (rem + 1) * jb, (double)sizeof(T) * ((double)rem * (rem + 1) + (double)rem * jb));
    if (launch_gemm<T>(g, 1, mode, s) != hipSuccess) return CDS_HIP_ERROR;
  }
  return CDS_SUCCESS;
}

template <typename T>
cds_status_t potrf_run(Ctx& c, int n, T* A, int64_t lda, int32_t* info, int nb) {
  return potrf_run_mode<T>(c, n, A, lda, info, nb, 0, nullptr);
}

template cds_status_t potrf_run<double>(Ctx&, int, double*, int64_t, int32_t*, int);
template cds_status_t potrf_run<float>(Ctx&, int, float*, int64_t, int32_t*, int);
template cds_status_t potrf_run_mode<float>(Ctx&, int, float*, int64_t, int32_t*, int, int, int*);

}  // namespace cds
