// Many SPD systems of uneven size in one persistent launch (Cholesky, Sec. 2,
// applied to a batch).  Each workgroup takes systems from a ticket counter
// (largest first when the caller passes that order) and, inside the workgroup:
//   1. factors A with a left-looking blocked Cholesky into an FP32 row-major
//      scratch factor padded with an identity block to a multiple of the block
//      width JW (32 or 64); each FP64 element of A is read and rounded once, when
//      its block column is updated.  Per block column, the
//      rank-j0 delayed update of 64-row chunks runs on MFMA (both operands are
//      rows of the row-major factor, read as float4 straight into registers,
//      several k-slabs in flight), one wave factors the JW x JW diagonal block
//      in registers and forms its inverse, and the rows below are solved by an
//      MFMA product with that inverse;
//   2. solves in FP32 with the stored diagonal-block inverses (the only serial
//      step per block is one dependent load round trip), and
//   3. refines with an FP64 residual in which every thread owns whole rows:
//      the row part of row i reads A(i, 0:i) (coalesced across threads), the
//      column part reads A(i+1:n, i) (one column per lane), so no cross-lane
//      reductions and a fixed summation order (graph replays are bitwise equal).
// No grid-wide synchronisation, no host interaction: the launch can be captured.
// The LDS footprint (about 68 KB) leaves room for two workgroups per CU, so the
// serial diagonal-block and solve phases of one system overlap the MFMA phases
// of another.
#include "common.hpp"
#include "kernels.hpp"
#include "vbatched.hpp"
#include <algorithm>

namespace cds {

namespace {

constexpr int VNT = 256;
constexpr int VNMAX = 1024;
constexpr int VNR = 4;      // right-hand sides per pass
constexpr int CH = 64;      // rows per update chunk
constexpr int WPAD = 32;    // extra floats per scratch row (spreads rows over channels)
constexpr int SP = 68;      // LDS row stride (floats) of the chunk and inverse tiles
constexpr int PD = 3;       // k-slabs (32 wide) in flight in the update
constexpr int WG_PER_CU = 2;

struct VbArgs {
  int batch, nrhs;
  const int32_t* n;
  const double* const* A; const int64_t* lda;
  const double* const* B; const int64_t* ldb;
  double* const* X; const int64_t* ldx;
  const int32_t* order;
  float* ws;
  size_t wg_elems;   // floats of scratch per workgroup
  size_t w_elems;    // floats of the factor region (the inverses follow)
  int* ticket;
  cds_ir_result_t* res;
  uint64_t* t_start; uint64_t* t_end;
  double tol, success_tol;
  int max_iter;
  int jw32_max_n;    // systems with n <= this use 32-wide block columns, larger ones 64
};

struct VbShared {
  double xs[VNMAX][VNR];                 // FP64 solution of the current pass
  union {
    struct { float S[CH][SP]; float Li[64][SP]; float col[64]; } f;      // factorization
    struct { float y[VNMAX][VNR]; float part[4096]; float t[64][VNR]; } s;  // solves / residual out
  } u;
  double red[4][2 * VNR + 1];
  double anorm;
  int info;
  int ticket;
};

__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// One wave: factor the JW x JW diagonal block held in S (lower part) in place,
// L_JJ to S and to Wd (row-major, ld ldw), 1 / L(r, r) to col[], the inverse
// L_JJ^{-1} to Li and to Wi (row-major JW x JW).  Returns 0, or the 1-based
// column of the first non-positive pivot.  Kept out of line: its register
// allocation then does not compete with the update loop around it.
template <int JW>
__device__ __attribute__((noinline)) int vb_diag(float* Wd, int ldw, float* Wi, VbShared& sh) {
  const int lane = threadIdx.x & 63;
  const int r = lane;   // row r of the block in lane r
  float v[JW];
#pragma unroll
  for (int c = 0; c < JW; ++c) v[c] = (r < JW && c <= r) ? sh.u.f.S[r < JW ? r : 0][c] : 0.f;
#pragma unroll
  for (int j = 0; j < JW; ++j) {
    const float d = lane_read(v[j], j);
    if (!(d > 0.f)) return j + 1;
    const float ljj = sqrtf(d), rinv = 1.0f / ljj;
    v[j] = (r == j) ? ljj : (r > j ? v[j] * rinv : 0.f);
    sh.u.f.col[r] = v[j];
    wave_fence();
#pragma unroll
    for (int c = j + 1; c < JW; ++c) v[c] -= v[j] * sh.u.f.col[c];
    wave_fence();
  }
  if (r < JW) {
#pragma unroll
    for (int c = 0; c < JW; ++c) {
      const float x = c <= r ? v[c] : 0.f;
      sh.u.f.S[r][c] = x;
      Wd[(size_t)r * ldw + c] = x;
    }
  }
  float vr = 1.f;
#pragma unroll
  for (int c = 0; c < JW; ++c) vr = (c == r) ? v[c] : vr;
  sh.u.f.col[r] = 1.0f / vr;
  wave_fence();
  // lane c forms column c of L_JJ^{-1} by forward substitution
  const int c = lane;
  float y[JW];
#pragma unroll
  for (int i = 0; i < JW; ++i) {
    float s0 = (i == c) ? 1.f : 0.f, s1 = 0.f;
#pragma unroll
    for (int t = 0; t + 1 < i; t += 2) {
      s0 -= sh.u.f.S[i][t] * y[t];
      s1 -= sh.u.f.S[i][t + 1] * y[t + 1];
    }
    if (i & 1) s0 -= sh.u.f.S[i][i - 1] * y[i - 1];
    y[i] = (s0 + s1) * sh.u.f.col[i];
  }
  if (c < JW) {
#pragma unroll
    for (int i = 0; i < JW; ++i) {
      sh.u.f.Li[i][c] = y[i];
      Wi[i * JW + c] = y[i];
    }
  }
  return 0;
}

// Left-looking blocked Cholesky of A (n x n, FP64, column-major, lower triangle
// read), padded with an identity block to np, into W (np x np, FP32, row-major,
// lower).  Each element of A is read once, when its block column is updated, and
// rounded to FP32 there.  The inverse of every JW x JW diagonal block goes to
// Winv (row-major, JW x JW per block).  sh.info = 0, or the 1-based column of the
// first non-positive pivot.
template <int JW>
__device__ void vb_potrf(const double* A, int64_t lda, int n, float* W, int ldw, float* Winv, int np, VbShared& sh) {
  constexpr int RT = JW == 64 ? 2 : 1;   // 16-row tiles per wave
  constexpr int CT = 2;                  // 16-column tiles per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int rtb = JW == 64 ? 2 * (wave >> 1) : wave;
  const int ctb = JW == 64 ? 2 * (wave & 1) : 0;
  if (tid == 0) sh.info = 0;
  __syncthreads();
  const int nbJ = np / JW;
  for (int J = 0; J < nbJ; ++J) {
    const int j0 = J * JW;
    const int nsl = j0 / 32;
    for (int r0 = j0; r0 < np; r0 += CH) {
      const bool active = r0 + 16 * rtb < np;   // whole row tiles are in or out (np % 32 == 0)
      // ---- S = A(chunk, block column) - L(chunk, 0:j0) L(block, 0:j0)^T; the A loads are issued
      // first and consumed after the MFMA loop
      double ao[RT][CT][4];
      f4 acc[RT][CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          acc[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = r0 + 16 * (rtb + rt) + 4 * lg + v, col = j0 + 16 * (ctb + ct) + li;
            ao[rt][ct][v] = (row < n && col < n) ? (row >= col ? A[row + (size_t)col * lda] : 0.0)
                                                 : (row == col ? 1.0 : 0.0);
          }
        }
      if (active && nsl > 0) {
        const float* Ap[RT];
        const float* Bp[CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) Ap[rt] = W + (size_t)(r0 + 16 * (rtb + rt) + li) * ldw + 4 * lg;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) Bp[ct] = W + (size_t)(j0 + 16 * (ctb + ct) + li) * ldw + 4 * lg;
        f4 a[PD][RT][2], b[PD][CT][2];
        // slab s covers k = 32 s .. 32 s + 31; lane (i, g) holds k = 32 s + 16 h + 4 g + q in a[..][h][q]
        auto load = [&](int p, int s) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[p][rt][h] = *reinterpret_cast<const f4*>(Ap[rt] + 32 * s + 16 * h);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) b[p][ct][h] = *reinterpret_cast<const f4*>(Bp[ct] + 32 * s + 16 * h);
          }
        };
#pragma unroll
        for (int p = 0; p < PD; ++p)
          if (p < nsl) load(p, p);
        for (int s0 = 0; s0 < nsl; s0 += PD) {
#pragma unroll
          for (int p = 0; p < PD; ++p) {
            const int s = s0 + p;
            if (s < nsl) {
#pragma unroll
              for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                      acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p][rt][h][q], b[p][ct][h][q],
                                                                         acc[rt][ct], 0, 0, 0);
              if (s + PD < nsl) load(p, s + PD);
            }
          }
        }
      }
      // (MFMA C layout: row 4 g + v, column i of each 16 x 16 tile)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            sh.u.f.S[16 * (rtb + rt) + 4 * lg + v][16 * (ctb + ct) + li] = (float)ao[rt][ct][v] - acc[rt][ct][v];
      __syncthreads();
      if (r0 == j0) {
        // ---- diagonal block: one wave, row r in lane r, right-looking in registers
        if (wave == 0) {
          const int fail = vb_diag<JW>(W + (size_t)j0 * ldw + j0, ldw, Winv + (size_t)J * JW * JW, sh);
          if (fail && lane == 0) sh.info = j0 + fail;
        }
        __syncthreads();
        if (sh.info != 0) return;
      }
      // ---- rows below the diagonal block: X = S L_JJ^{-T} (MFMA, operands from LDS)
      const int rt_lo = (r0 == j0) ? JW / 16 : 0;
      if (active && rtb >= rt_lo) {
        f4 d[RT][CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) d[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < JW; kk += 16) {
          f4 av[RT], bv[CT];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            av[rt] = *reinterpret_cast<const f4*>(&sh.u.f.S[16 * (rtb + rt) + li][kk + 4 * lg]);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
            bv[ct] = *reinterpret_cast<const f4*>(&sh.u.f.Li[16 * (ctb + ct) + li][kk + 4 * lg]);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
              for (int ct = 0; ct < CT; ++ct)
                d[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt][q], bv[ct][q], d[rt][ct], 0, 0, 0);
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              W[(size_t)(r0 + 16 * (rtb + rt) + 4 * lg + v) * ldw + j0 + 16 * (ctb + ct) + li] = d[rt][ct][v];
      }
      __syncthreads();   // S and the factor stores are complete before the next chunk
    }
  }
}

// y <- L^{-T} L^{-1} y (FP32, VNR right-hand sides, y = sh.u.s.y over np rows).
// L is the row-major factor in W, Winv holds the inverses of its diagonal blocks.
template <int JW>
__device__ void vb_potrs(const float* W, int ldw, const float* Winv, int np, VbShared& sh) {
  const int tid = threadIdx.x;
  float(*y)[VNR] = sh.u.s.y;
  float* part = sh.u.s.part;
  float(*t)[VNR] = sh.u.s.t;
  const int nbJ = np / JW;
  constexpr int KP = VNT / JW;   // k partitions of the forward update (4 or 8)
  constexpr int UN = 4;
  // ---- forward: y_J = Linv_J (y_J - L(J, 0:j0) y(0:j0))
  for (int J = 0; J < nbJ; ++J) {
    const int j0 = J * JW;
    const int i = tid % JW, p = tid / JW;
    // the GEMV thread (i, q = p) prefetches row i of the inverse
    f4 lv[JW / 4];
    if (p < VNR) {
      const float* Li = Winv + (size_t)J * JW * JW + i * JW;
#pragma unroll
      for (int c = 0; c < JW / 4; ++c) lv[c] = *reinterpret_cast<const f4*>(Li + 4 * c);
    }
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* Lr = W + (size_t)(j0 + i) * ldw;
    for (int k0 = 4 * p; k0 < j0; k0 += 4 * KP * UN) {
      f4 lk[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int k = k0 + 4 * KP * u;
        lk[u] = k < j0 ? *reinterpret_cast<const f4*>(Lr + k) : f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int k = min(k0 + 4 * KP * u, np - 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const f4 yk = *reinterpret_cast<const f4*>(y[k + e]);
          acc += lk[u][e] * yk;
        }
      }
    }
    *reinterpret_cast<f4*>(&part[(p * JW + i) * VNR]) = acc;
    __syncthreads();
    if (p < VNR) {
      float s = y[j0 + i][p];
#pragma unroll
      for (int pp = 0; pp < KP; ++pp) s -= part[(pp * JW + i) * VNR + p];
      t[i][p] = s;
    }
    __syncthreads();
    if (p < VNR) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < JW / 4; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) s += lv[c][e] * t[4 * c + e][p];
      y[j0 + i][p] = s;
    }
    __syncthreads();
  }
  // ---- backward: x_J = Linv_J^T (y_J - L(j0+JW:np, J)^T x(j0+JW:np))
  constexpr int CQ = JW / 4;        // column quads
  constexpr int RP = VNT / CQ;      // row partitions (16 or 32)
  constexpr int UB = 8;
  for (int J = nbJ - 1; J >= 0; --J) {
    const int j0 = J * JW;
    const int i = tid % JW, p = tid / JW;
    float lc[JW];
    if (p < VNR) {
      const float* Li = Winv + (size_t)J * JW * JW;
#pragma unroll
      for (int r = 0; r < JW; ++r) lc[r] = Li[r * JW + i];   // column i of the inverse
    }
    const int cq = tid % CQ, rp = tid / CQ;
    f4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int r0 = j0 + JW + rp; r0 < np; r0 += RP * UB) {
      f4 lr[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int r = r0 + RP * u;
        lr[u] = r < np ? *reinterpret_cast<const f4*>(W + (size_t)r * ldw + j0 + 4 * cq) : f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int r = min(r0 + RP * u, np - 1);
        const f4 xr = *reinterpret_cast<const f4*>(y[r]);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += lr[u][c] * xr;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) *reinterpret_cast<f4*>(&part[(rp * JW + 4 * cq + c) * VNR]) = acc[c];
    __syncthreads();
    if (p < VNR) {
      float s = y[j0 + i][p];
      for (int pp = 0; pp < RP; ++pp) s -= part[(pp * JW + i) * VNR + p];
      t[i][p] = s;
    }
    __syncthreads();
    if (p < VNR) {
      float s = 0.f;
#pragma unroll
      for (int r = 0; r < JW; ++r) s += lc[r] * t[r][p];
      y[j0 + i][p] = s;
    }
    __syncthreads();
  }
}

// Residual r = B - A xs in FP64 (A symmetric, lower triangle, column-major); y = fp32(r)
// (zero on the padding rows).  Returns max_c ||r_c||_inf / (||A||_inf ||x_c||_inf); computes
// ||A||_inf into sh.anorm when `norm` is set.
__device__ double vb_residual(const double* A, int64_t lda, const double* B, int64_t ldb, int n, int np, int nr,
                              bool norm, VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int UN = 8;
  double rmax[VNR] = {0.0, 0.0, 0.0, 0.0}, xmax[VNR] = {0.0, 0.0, 0.0, 0.0}, amax = 0.0;
  for (int base = 0; base < np; base += VNT) {
    const int i = base + tid;
    const int wlo = base + 64 * wave;                     // first row of this wave
    const int whi = min(n - 1, wlo + 63);                 // last valid row of this wave
    double s[VNR] = {0.0, 0.0, 0.0, 0.0}, ab = 0.0;
    if (wlo < n) {
      // row part: A(i, 0:i)
      for (int j0 = 0; j0 <= whi; j0 += UN) {
        double a[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int j = j0 + u;
          a[u] = (i < n && j <= i) ? A[i + (size_t)j * lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int j = min(j0 + u, n - 1);
          ab += fabs(a[u]);
#pragma unroll
          for (int q = 0; q < VNR; ++q) s[q] = fma(a[u], sh.xs[j][q], s[q]);
        }
      }
      // column part: A(i+1:n, i), one column per lane
      const double* Ac = A + (size_t)min(i, n - 1) * lda;
      for (int c0 = wlo + 1; c0 < n; c0 += UN) {
        double a[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int c = c0 + u;
          a[u] = (i < n && c > i && c < n) ? Ac[c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int c = min(c0 + u, n - 1);
          ab += fabs(a[u]);
#pragma unroll
          for (int q = 0; q < VNR; ++q) s[q] = fma(a[u], sh.xs[c][q], s[q]);
        }
      }
    }
    if (i < np) {
#pragma unroll
      for (int q = 0; q < VNR; ++q) {
        float rf = 0.f;
        if (i < n && q < nr) {
          const double r = B[i + (size_t)q * ldb] - s[q];
          rf = (float)r;
          rmax[q] = fmax(rmax[q], fabs(r));
          xmax[q] = fmax(xmax[q], fabs(sh.xs[i][q]));
        }
        sh.u.s.y[i][q] = rf;
      }
    }
    amax = fmax(amax, ab);
  }
  // workgroup maxima (exact, order-free)
#pragma unroll
  for (int q = 0; q < VNR; ++q) {
    rmax[q] = wave_max(rmax[q]);
    xmax[q] = wave_max(xmax[q]);
  }
  amax = wave_max(amax);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < VNR; ++q) {
      sh.red[wave][q] = rmax[q];
      sh.red[wave][VNR + q] = xmax[q];
    }
    sh.red[wave][2 * VNR] = amax;
  }
  __syncthreads();
  if (norm) {
    if (tid == 0) sh.anorm = fmax(fmax(sh.red[0][2 * VNR], sh.red[1][2 * VNR]), fmax(sh.red[2][2 * VNR], sh.red[3][2 * VNR]));
    __syncthreads();
  }
  double eta = 0.0;
#pragma unroll
  for (int q = 0; q < VNR; ++q) {
    if (q < nr) {
      const double rr = fmax(fmax(sh.red[0][q], sh.red[1][q]), fmax(sh.red[2][q], sh.red[3][q]));
      const double xx = fmax(fmax(sh.red[0][VNR + q], sh.red[1][VNR + q]), fmax(sh.red[2][VNR + q], sh.red[3][VNR + q]));
      const double e = rr == 0.0 ? 0.0 : (sh.anorm * xx > 0.0 ? rr / (sh.anorm * xx) : INFINITY);
      if (!(e <= eta)) eta = e;
    }
  }
  __syncthreads();   // red[] is reused by the next call
  return eta;
}

template <int JW>
__device__ void vb_system(const VbArgs& a, int sys, float* W, float* Winv, VbShared& sh) {
  const int tid = threadIdx.x;
  const int n = a.n[sys];
  const int np = (n + JW - 1) / JW * JW;
  const int ldw = np + WPAD;
  const double* A = a.A[sys];
  const int64_t lda = a.lda[sys];
  cds_ir_result_t* res = a.res + sys;
  if (tid == 0 && a.t_start) a.t_start[sys] = wall_clock64();
  vb_potrf<JW>(A, lda, n, W, ldw, Winv, np, sh);
  const int info = sh.info;
  if (info != 0) {
    if (tid == 0) {
      res->info = info; res->converged = 0; res->fell_back = 0; res->iters = 0;
      res->eta = INFINITY; res->eta0 = INFINITY; res->stop_reason = 5; res->reserved = 0;
      if (a.t_end) a.t_end[sys] = wall_clock64();
    }
    __syncthreads();
    return;
  }
  int last_reason = 0, last_iters = 0;
  double last_eta = 0.0, first_eta = 0.0;
  for (int c0 = 0; c0 < a.nrhs; c0 += VNR) {
    const int nr = min(VNR, a.nrhs - c0);
    const double* B = a.B[sys] + (size_t)c0 * a.ldb[sys];
    const int64_t ldb = a.ldb[sys];
    double* X = a.X[sys] + (size_t)c0 * a.ldx[sys];
    const int64_t ldx = a.ldx[sys];
    // x0 = solve(b)
    for (int i = tid; i < np; i += VNT)
#pragma unroll
      for (int q = 0; q < VNR; ++q) sh.u.s.y[i][q] = (i < n && q < nr) ? (float)B[i + (size_t)q * ldb] : 0.f;
    __syncthreads();
    vb_potrs<JW>(W, ldw, Winv, np, sh);
    for (int i = tid; i < np; i += VNT)
#pragma unroll
      for (int q = 0; q < VNR; ++q) sh.xs[i][q] = (double)sh.u.s.y[i][q];
    __syncthreads();
    double eta_prev = INFINITY, eta_prev2 = INFINITY;
    int it = 0, reason = 0;
    double eta = 0.0;
    for (it = 0;; ++it) {
      eta = vb_residual(A, lda, B, ldb, n, np, nr, c0 == 0 && it == 0, sh);
      if (it == 0 && c0 == 0) first_eta = eta;
      if (!(eta == eta) || eta == INFINITY) reason = 4;
      else if (eta <= a.tol) reason = 1;
      else if (it >= 2 && eta > 0.5 * eta_prev && eta_prev > 0.5 * eta_prev2) reason = 2;
      else if (it >= a.max_iter) reason = 3;
      if (reason) break;
      eta_prev2 = eta_prev;
      eta_prev = eta;
      vb_potrs<JW>(W, ldw, Winv, np, sh);
      for (int i = tid; i < np; i += VNT)
#pragma unroll
        for (int q = 0; q < VNR; ++q) sh.xs[i][q] += (double)sh.u.s.y[i][q];
      __syncthreads();
    }
    for (int i = tid; i < n; i += VNT)
      for (int q = 0; q < nr; ++q) X[i + (size_t)q * ldx] = sh.xs[i][q];
    if (!(eta <= last_eta)) last_eta = eta;
    if (reason > last_reason) last_reason = reason;
    last_iters = max(last_iters, it);
    __syncthreads();
  }
  if (tid == 0) {
    res->info = 0;
    res->iters = last_iters;
    res->eta = last_eta;
    res->eta0 = first_eta;
    res->stop_reason = last_reason;
    res->converged = last_eta <= a.success_tol ? 1 : 0;
    res->fell_back = 0;
    res->reserved = 0;
    if (a.t_end) a.t_end[sys] = wall_clock64();
  }
  __syncthreads();
}

__global__ void __launch_bounds__(VNT, WG_PER_CU) vbatched_kernel(VbArgs a) {
  __shared__ VbShared sh;
  float* W = a.ws + (size_t)blockIdx.x * a.wg_elems;
  float* Winv = W + a.w_elems;
  while (true) {
    if (threadIdx.x == 0) sh.ticket = atomicAdd(a.ticket, 1);
    __syncthreads();
    const int t = sh.ticket;
    __syncthreads();
    if (t >= a.batch) break;
    const int sys = a.order ? a.order[t] : t;
    if (sys < 0 || sys >= a.batch) continue;
    const int n = a.n[sys];
    if (n < 1 || n > VNMAX || (size_t)((n + 63) / 64 * 64) * ((n + 63) / 64 * 64 + WPAD) > a.w_elems) {
      // invalid size: report and skip (no memory outside the scratch matrix is touched)
      if (threadIdx.x == 0) {
        cds_ir_result_t* r = a.res + sys;
        r->info = -1; r->converged = 0; r->fell_back = 0; r->iters = 0;
        r->eta = INFINITY; r->eta0 = INFINITY; r->stop_reason = 5; r->reserved = 0;
      }
      continue;
    }
    if (n <= a.jw32_max_n) vb_system<32>(a, sys, W, Winv, sh);
    else vb_system<64>(a, sys, W, Winv, sh);
  }
}

__global__ void reset_kernel(int* p) { *p = 0; }

int round64(int n) { return (n + 63) / 64 * 64; }

size_t vb_w_elems(int nmax) { return (size_t)round64(nmax) * (round64(nmax) + WPAD); }
size_t vb_wg_elems(int nmax) { return vb_w_elems(nmax) + (size_t)round64(nmax) * 64; }

}  // namespace

int vbatched_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return WG_PER_CU * cus;
}

size_t vbatched_ws_bytes(int batch, int nmax, int nrhs) {
  (void)nrhs;
  const int grid = std::max(1, std::min(vbatched_grid(), batch));
  return kErrRegion + 256 + (size_t)grid * vb_wg_elems(nmax) * sizeof(float);
}

cds_status_t vbatched_run(Ctx& c, int batch, int nmax, const int32_t* n, const double* const* A, const int64_t* lda,
                          const double* const* B, const int64_t* ldb, double* const* X, const int64_t* ldx, int nrhs,
                          const int32_t* order, const cds_ir_params_t& prm, cds_ir_result_t* res, uint64_t* t_start,
                          uint64_t* t_end, int jw32_max_n) {
  if (batch == 0) return CDS_SUCCESS;
  if (nmax > VNMAX) return CDS_UNSUPPORTED;
  if (c.ws_bytes < vbatched_ws_bytes(batch, nmax, nrhs)) return CDS_WORKSPACE_TOO_SMALL;
  char* base = (char*)c.ws + kErrRegion;
  int* ticket = (int*)base;
  float* ws = (float*)(base + 256);
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, c.s0, ticket);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  VbArgs a;
  a.batch = batch; a.nrhs = nrhs;
  a.n = n; a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.X = X; a.ldx = ldx; a.order = order;
  a.ws = ws; a.wg_elems = vb_wg_elems(nmax); a.w_elems = vb_w_elems(nmax);
  a.ticket = ticket; a.res = res; a.t_start = t_start; a.t_end = t_end;
  a.tol = prm.tol; a.success_tol = prm.success_tol; a.max_iter = prm.max_iter;
  a.jw32_max_n = jw32_max_n;
  const int grid = std::max(1, std::min(vbatched_grid(), batch));
  hipLaunchKernelGGL(vbatched_kernel, dim3(grid), dim3(VNT), 0, c.s0, a);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

}  // namespace cds
