// Blocked right-looking Cholesky A = L L^T (Sec. 2: "In the case of SPD
// matrices, we have A = LL^t"), lower triangle only.
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

// jb <= 128: the whole diagonal block lives in LDS (column-major, ld 129) for the
// duration of the kernel; it is read from and written to global memory once.  Per
// 32-wide sub-block: (a) one wave factors the sub-block's diagonal with row r in
// lane r (registers), column j broadcast through LDS, division by L(j,j) so that
// exact data stays exact; (b) the rows below in the block are solved against it,
// one row per thread, with the reciprocal of the diagonal; (c) the rest of the
// block gets the symmetric rank-32 update on MFMA tiles.
constexpr int PJB = 128, PLD = PJB + 1;

template <typename T>
__global__ void __launch_bounds__(256) potf2_lds_kernel(T* A, int64_t lda, int k, int jb, int32_t* info,
                                                        double* linv) {
  __shared__ T Ds[PJB * PLD];   // (r, c) at Ds[c * PLD + r]
  __shared__ T colb[64];
  __shared__ T rdiag[SB];
  __shared__ int s_fail;
  if (*info != 0) return;
  T* D = A + k + (size_t)k * lda;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // 16 loads in flight per thread (the block is jb x jb, at most 64 elements per thread)
  for (int base = 0; base < jb * jb; base += 16 * 256) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * 256 + tid, r = idx % jb, c = idx / jb;
      v[u] = (idx < jb * jb && r >= c) ? D[r + (size_t)c * lda] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * 256 + tid;
      if (idx < jb * jb) Ds[(idx / jb) * PLD + idx % jb] = v[u];
    }
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();
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
      int fail = 0;
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        const T d = lane_get(v[j], j);   // a_jj minus the updates of the previous columns
        if (fail == 0 && !(d > (T)0)) fail = j + 1;
        const T ljj = sqrt_t(d);
        v[j] = (r == j) ? ljj : (r > j ? v[j] / ljj : (T)0);
        colb[r] = v[j];
        wave_fence();
#pragma unroll
        for (int c = j + 1; c < SB; ++c) v[c] -= v[j] * colb[c];
        wave_fence();
      }
      if (fail) {
        if (lane == 0) {
          s_fail = 1;
          atomicCAS(info, 0, k + s0 + fail);
        }
      } else if (r < sw) {
#pragma unroll
        for (int c = 0; c < SB; ++c)
          if (c <= r) Ds[(s0 + c) * PLD + s0 + r] = v[c];
        T vr = (T)1;
#pragma unroll
        for (int c = 0; c < SB; ++c) vr = (c == r) ? v[c] : vr;
        rdiag[r] = (T)1 / vr;
      }
    }
    __syncthreads();
    if (s_fail) break;
    // (b) rows below the sub-block: x L11^T = a; the dot products in four independent partial
    // sums, the diagonal applied as a precomputed reciprocal (no division on the chain)
    const int rem = jb - s0 - sw;
    for (int t = tid; t < rem; t += 256) {
      const int i = s0 + sw + t;
      T x[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) x[c] = c < sw ? Ds[(s0 + c) * PLD + i] : (T)0;
#pragma unroll
      for (int c = 0; c < SB; ++c) {
        if (c < sw) {
          T p0 = (T)0, p1 = (T)0, p2 = (T)0, p3 = (T)0;
#pragma unroll
          for (int u = 0; u + 3 < c; u += 4) {
            p0 += x[u] * Ds[(s0 + u) * PLD + s0 + c];
            p1 += x[u + 1] * Ds[(s0 + u + 1) * PLD + s0 + c];
            p2 += x[u + 2] * Ds[(s0 + u + 2) * PLD + s0 + c];
            p3 += x[u + 3] * Ds[(s0 + u + 3) * PLD + s0 + c];
          }
#pragma unroll
          for (int u = c & ~3; u < c; ++u) p0 += x[u] * Ds[(s0 + u) * PLD + s0 + c];
          x[c] = (x[c] - ((p0 + p1) + (p2 + p3))) * rdiag[c];
        }
      }
#pragma unroll
      for (int c = 0; c < SB; ++c)
        if (c < sw) Ds[(s0 + c) * PLD + i] = x[c];
    }
    __syncthreads();
    // (c) trailing part of the block on MFMA: 16 x 16 tiles (ti >= tc) of the lower triangle, one
    // tile per wave at a time, D = P_rows P_cols^T with P = the sub-block's columns below it
    {
      constexpr bool F64 = std::is_same<T, double>::value;
      typedef typename std::conditional<F64, d4, f4>::type acc_t;
      const int b0 = s0 + sw, nt = (rem + 15) / 16, ntiles = nt * (nt + 1) / 2;
      const int li = lane & 15, lg = lane >> 4;
      for (int tile = wave; tile < ntiles; tile += 4) {
        int ti = (int)((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
        while (ti * (ti + 1) / 2 > tile) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        const int tc = tile - ti * (ti + 1) / 2;
        const int i0 = b0 + 16 * ti, c0 = b0 + 16 * tc;
        acc_t acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = (T)0;
#pragma unroll
        for (int k4 = 0; k4 < SB; k4 += 4) {
          const int kk = k4 + lg;
          const T a = (kk < sw && i0 + li < jb) ? Ds[(s0 + kk) * PLD + i0 + li] : (T)0;
          const T b = (kk < sw && c0 + li < jb) ? Ds[(s0 + kk) * PLD + c0 + li] : (T)0;
          if constexpr (F64)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
          else
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + (F64 ? (lg + 4 * v) : (4 * lg + v)), c = c0 + li;
          if (i < jb && c <= i) Ds[c * PLD + i] -= acc[v];
        }
      }
    }
    __syncthreads();
  }
  // the factored (or, after a failed pivot, partially factored) lower triangle back to A
  for (int idx = tid; idx < jb * jb; idx += 256) {
    const int r = idx % jb, c = idx / jb;
    if (r >= c) D[r + (size_t)c * lda] = Ds[c * PLD + r];
  }
  // the inverses of the factor's 16 x 16 diagonal blocks for the TRSM below it, from the block in LDS
  // (after a failed pivot the TRSM does not run and these are never read)
  if (linv != nullptr)
    for (int t = tid; t < ((jb + 15) / 16) * 16; t += 256) diag_inv16_column<T, false>(Ds, PLD, jb, t >> 4, t & 15, linv);
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
      if (jb <= PJB) {
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
      if (jb > PJB && launch_diag_inv16<T>(A + k + (size_t)k * lda, lda, 0, jb, 0, linv, 0, 1, st) != hipSuccess)
        return CDS_HIP_ERROR;
      if (launch_trsm16<T>(A + k + (size_t)k * lda, lda, 0, linv, 0, A + (k + jb) + (size_t)k * lda, lda, 0, jb, rem,
                           1, 1, info, st) != hipSuccess)
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
  // A[r0:r1, c0:c1] -= L21(r0:r1) L21(c0:c1)^T with L21 = A[k+jb:n, k:k+jb]; lower: only the tiles on
  // or below the diagonal (r0 == c0, r1 == c1).  par: the operand-scale region of block column k.
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
      st = syrk(k, jb, kn, kn + jbn, kn, kn + jbn, true, par, s);   // the next diagonal block
      if (st != CDS_SUCCESS) return st;
      st = syrk(k, jb, kn + jbn, n, kn, kn + jbn, false, par, s);  // the rows below it
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
