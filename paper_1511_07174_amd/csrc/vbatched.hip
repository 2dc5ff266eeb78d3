// Many SPD systems of uneven size in one persistent launch (Cholesky, Sec. 2,
// applied to a batch).  Each workgroup takes systems from a ticket counter
// (largest first when the caller passes that order) and, inside the workgroup:
//   1. factors A with a left-looking blocked Cholesky into an FP32 row-major
//      scratch factor padded with an identity block to a multiple of the block
//      width JW (32 or 64); each FP64 element of A is read and rounded once, when
//      its block column is updated.  Per block column, the
//      rank-j0 delayed update of 128-row chunks runs on MFMA (both operands are
//      rows of the row-major factor, read as float4 straight into registers,
//      several k-slabs in flight), one wave factors the JW x JW diagonal block
//      in registers and forms its inverse, and the rows below are solved by an
//      MFMA product with that inverse;
//   2. solves in FP32 with the stored diagonal-block inverses (the only serial
//      step per block is one dependent load round trip), and
//   3. refines with an FP64 residual that reads every stored element of A twice,
//      both times coalesced: once along its row (a thread per row), once along
//      its column (16 lanes per column); every sum has a fixed order, so graph
//      replays are bitwise equal.
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
constexpr int WPAD = 32;    // extra floats per scratch row (spreads rows over channels)
constexpr int SP = 68;      // LDS row stride (floats) of the chunk and inverse tiles
constexpr int PD = 3;       // k-slabs (32 wide) in flight in the update
constexpr int WG_PER_CU = 2;

struct VbArgs {
  int batch, nrhs, nmax;
  const int32_t* n;
  const double* const* A; const int64_t* lda;
  const double* const* B; const int64_t* ldb;
  double* const* X; const int64_t* ldx;
  const int32_t* order;
  float* ws;
  size_t wg_elems;   // floats of scratch per workgroup
  size_t w_elems;    // floats of the factor region (the inverses follow)
  size_t inv_elems;  // floats of the inverse region (the column sums of the residual follow)
  int* ticket;
  int* err;          // device error word
  cds_ir_result_t* res;
  uint64_t* t_start; uint64_t* t_end;
  double tol, success_tol;
  int max_iter;
  int jw32_max_n;    // systems with n <= this use 32-wide block columns, larger ones 64
};

struct VbShared {
  double xs[VNMAX][VNR];                 // FP64 solution of the current pass
  union {
    struct { float S[64][SP]; float Li[64][SP]; float col[64]; float tr[4][16][17]; } f;   // factorization
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

// use(buf, b) for the batches b = 0 .. nb-1, the loads of batch b + 1 in flight while batch b is
// consumed (two register buffers, ping-pong).
template <int UN, typename T, typename LoadF, typename UseF>
__device__ __forceinline__ void pipelined(int nb, LoadF&& load, UseF&& use) {
  T b0[UN], b1[UN];
  if (nb > 0) load(b0, 0);
  for (int b = 0; b < nb; b += 2) {
    if (b + 1 < nb) load(b1, b + 1);
    use(b0, b);
    if (b + 1 >= nb) break;
    if (b + 2 < nb) load(b0, b + 2);
    use(b1, b + 1);
  }
}

// A flattened software pipeline over work items: `it` starts at the first item,
// next(it) advances it, valid(it) tells whether it exists; load(buf, it) issues an
// item's loads, use(buf, it) consumes them.  The next item's loads are in flight
// while the current one is consumed, across item boundaries.
template <int UN, typename T, typename Item, typename NextF, typename ValidF, typename LoadF, typename UseF>
__device__ __forceinline__ void pipelined_items(Item it, NextF&& next, ValidF&& valid, LoadF&& load, UseF&& use) {
  T b0[UN], b1[UN];
  if (!valid(it)) return;
  load(b0, it);
  while (true) {
    Item i1 = next(it);
    const bool v1 = valid(i1);
    if (v1) load(b1, i1);
    use(b0, it);
    if (!v1) break;
    Item i2 = next(i1);
    const bool v2 = valid(i2);
    if (v2) load(b0, i2);
    use(b1, i1);
    if (!v2) break;
    it = i2;
  }
}

struct VbItem { int g, b; };

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
    const float ljj = sqrtf(d), rinv = __builtin_amdgcn_rsqf(d);   // hardware 1/sqrt (about 1 ulp): the factor is refined in FP64
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
// rounded to FP32 there.  Per block column the rows are taken in chunks of 128; a
// wave owns 32 consecutive rows of the chunk across the whole block column, so each
// slab of the block's own rows (the second operand) is shared by 128 rows and no
// wave reads another wave's rows.  The inverse of every JW x JW diagonal block goes
// to Winv (row-major, JW x JW per block).  sh.info = 0, or the 1-based column of the
// first non-positive pivot.
template <int JW>
__device__ __attribute__((noinline)) void vb_potrf(const double* A, int64_t lda, int n, float* W, int ldw, float* Winv,
                                                   int np, VbShared& sh) {
  constexpr int RT = 2;          // 16-row tiles per wave (32 rows)
  constexpr int CT = JW / 16;    // 16-column tiles: the whole block column
  constexpr int CHR = 128;       // rows per chunk
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  float(*T16)[17] = sh.u.f.tr[wave];
  if (tid == 0) sh.info = 0;
  __syncthreads();
  const int nbJ = np / JW;
  for (int J = 0; J < nbJ; ++J) {
    const int j0 = J * JW;
    const int nsl = j0 / 32;
    for (int r0 = j0; r0 < np; r0 += CHR) {
      const int wr0 = r0 + 32 * wave;     // this wave's first row
      const bool active = wr0 < np;       // np % 32 == 0: a wave's 32 rows are all in or all out
      // ---- S = A(rows, block column) - L(rows, 0:j0) L(block, 0:j0)^T; the A loads are issued
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
            const int row = wr0 + 16 * rt + 4 * lg + v, col = j0 + 16 * ct + li;
            ao[rt][ct][v] = (row < n && col < n) ? (row >= col ? A[row + (size_t)col * lda] : 0.0)
                                                 : (row == col ? 1.0 : 0.0);
          }
        }
      if (active && nsl > 0) {
        const float* Ap[RT];
        const float* Bp[CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) Ap[rt] = W + (size_t)(wr0 + 16 * rt + li) * ldw + 4 * lg;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) Bp[ct] = W + (size_t)(j0 + 16 * ct + li) * ldw + 4 * lg;
        constexpr int PDL = 2;
        f4 a[PDL][RT][2], b[PDL][CT][2];
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
        for (int p = 0; p < PDL; ++p)
          if (p < nsl) load(p, p);
        for (int s0 = 0; s0 < nsl; s0 += PDL) {
#pragma unroll
          for (int p = 0; p < PDL; ++p) {
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
              if (s + PDL < nsl) load(p, s + PDL);
            }
          }
        }
      }
      // acc <- S (MFMA C layout: row 4 g + v, column i of each 16 x 16 tile)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[rt][ct][v] = (float)ao[rt][ct][v] - acc[rt][ct][v];
      const int nd = (r0 == j0) ? JW / 32 : 0;   // waves holding rows of the diagonal block
      if (r0 == j0) {
        // ---- diagonal block: its rows go to S, one wave factors it and forms the inverse
        if (wave < nd) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
              for (int v = 0; v < 4; ++v) sh.u.f.S[32 * wave + 16 * rt + 4 * lg + v][16 * ct + li] = acc[rt][ct][v];
        }
        __syncthreads();
        if (wave == 0) {
          const int fail = vb_diag<JW>(W + (size_t)j0 * ldw + j0, ldw, Winv + (size_t)J * JW * JW, sh);
          if (fail && lane == 0) sh.info = j0 + fail;
        }
        __syncthreads();
        if (sh.info != 0) return;
      }
      // ---- this wave's rows below the diagonal block: X = S L_JJ^{-T} (MFMA; the S tiles go
      // from the C layout to the operand layout through a per-wave 16 x 16 LDS tile)
      if (active && wave >= nd) {
        f4 d[RT][CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) d[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
          for (int kt = 0; kt < CT; ++kt) {
            wave_fence();   // the previous tile's reads are done
#pragma unroll
            for (int v = 0; v < 4; ++v) T16[4 * lg + v][li] = acc[rt][kt][v];
            wave_fence();
            f4 av;
#pragma unroll
            for (int q = 0; q < 4; ++q) av[q] = T16[li][4 * lg + q];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const f4 bv = *reinterpret_cast<const f4*>(&sh.u.f.Li[16 * ct + li][16 * kt + 4 * lg]);
#pragma unroll
              for (int q = 0; q < 4; ++q)
                d[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], d[rt][ct], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              W[(size_t)(wr0 + 16 * rt + 4 * lg + v) * ldw + j0 + 16 * ct + li] = d[rt][ct][v];
      }
      // the next chunk's S / T16 writes and the factor stores: ordered by the barrier below
      __syncthreads();
    }
  }
}

// y <- L^{-T} L^{-1} y (FP32, VNR right-hand sides, y = sh.u.s.y over np rows).
// L is the row-major factor in W, Winv holds the inverses of its diagonal blocks.
template <int JW>
__device__ __attribute__((noinline)) void vb_potrs(const float* W, int ldw, const float* Winv, int np, VbShared& sh) {
  const int tid = threadIdx.x;
  float(*y)[VNR] = sh.u.s.y;
  float* part = sh.u.s.part;
  float(*t)[VNR] = sh.u.s.t;
  const int nbJ = np / JW;
  constexpr int KP = VNT / JW;   // k partitions of the forward update (4 or 8)
  constexpr int UN = 16;
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
    const float* Lr = W + (size_t)(j0 + i) * ldw + 4 * p;
    const int nbt = (j0 + 4 * KP * UN - 1) / (4 * KP * UN);
    pipelined<UN, f4>(
        nbt,
        [&](f4(&lk)[UN], int bt) {
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int k = 4 * p + 4 * KP * (bt * UN + u);
            lk[u] = k < j0 ? *reinterpret_cast<const f4*>(Lr + 4 * KP * (bt * UN + u)) : f4{0.f, 0.f, 0.f, 0.f};
          }
        },
        [&](f4(&lk)[UN], int bt) {
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int k = min(4 * p + 4 * KP * (bt * UN + u), np - 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const f4 yk = *reinterpret_cast<const f4*>(y[k + e]);
              acc += lk[u][e] * yk;
            }
          }
        });
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
    const int nbt = (np - j0 - JW + RP * UB - 1) / (RP * UB);
    const float* Lc = W + (size_t)(j0 + JW + rp) * ldw + j0 + 4 * cq;
    pipelined<UB, f4>(
        nbt,
        [&](f4(&lr)[UB], int bt) {
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const int r = j0 + JW + rp + RP * (bt * UB + u);
            lr[u] = r < np ? *reinterpret_cast<const f4*>(Lc + (size_t)RP * (bt * UB + u) * ldw) : f4{0.f, 0.f, 0.f, 0.f};
          }
        },
        [&](f4(&lr)[UB], int bt) {
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const int r = min(j0 + JW + rp + RP * (bt * UB + u), np - 1);
            const f4 xr = *reinterpret_cast<const f4*>(y[r]);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += lr[u][c] * xr;
          }
        });
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
// ||A||_inf into sh.anorm when `norm` is set.  (A xs)_i = sum_{j<=i} A(i,j) x_j + sum_{c>i} A(c,i) x_c:
//   column part: a wave takes 4 columns at a time, 16 lanes per column walking its rows
//     (4 x 128 B per load), the 16 partial sums combined inside each 16-lane row; the
//     per-column sums (4 right-hand sides and sum |A(c,i)|) go to cp (global, this
//     workgroup's scratch);
//   row part: thread i walks row i (64 consecutive rows per load) and adds cp[i].
// Both sweeps run as one software pipeline over all their batches, so the loads of the
// next column group or row set are in flight while the current one finishes.  Every sum
// has a fixed order, so the result does not depend on timing.
__device__ __attribute__((noinline)) double vb_residual(const double* A, int64_t lda, const double* B, int64_t ldb,
                                                       int n, int np, int nr, bool norm, double* cp, VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int UN = 16;
  // ---- column part: items (column group g of 4 columns, batch b of 16 UN rows), g = wave, wave + 4, ...
  {
    const int cc = lane >> 4, r = lane & 15;
    const int ng = (n + 3) / 4;
    double s[VNR] = {0.0, 0.0, 0.0, 0.0}, ab = 0.0;
    auto nbat = [&](int g) { return (n - 4 * g - 1 + 16 * UN - 1) / (16 * UN); };
    VbItem first{wave, 0};
    while (first.g < ng && nbat(first.g) == 0) first.g += 4;   // groups without rows below
    pipelined_items<UN, double>(
        first,
        [&](VbItem t) {
          if (t.b + 1 < nbat(t.g)) return VbItem{t.g, t.b + 1};
          int g = t.g + 4;
          while (g < ng && nbat(g) == 0) g += 4;
          return VbItem{g, 0};
        },
        [&](VbItem t) { return t.g < ng; },
        [&](double(&a)[UN], VbItem t) {
          const int i = 4 * t.g + cc;
          const double* Ac = A + (size_t)min(i, n - 1) * lda;
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int c = 4 * t.g + 1 + r + 16 * (t.b * UN + u);
            a[u] = (i < n && c > i && c < n) ? Ac[c] : 0.0;
          }
        },
        [&](double(&a)[UN], VbItem t) {
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int c = min(4 * t.g + 1 + r + 16 * (t.b * UN + u), n - 1);
            ab += fabs(a[u]);
#pragma unroll
            for (int q = 0; q < VNR; ++q) s[q] = fma(a[u], sh.xs[c][q], s[q]);
          }
          if (t.b + 1 == nbat(t.g)) {   // last batch of the group: combine the 16 lanes of each column
#pragma unroll
            for (int q = 0; q < VNR; ++q) s[q] = row16_sum(s[q]);
            ab = row16_sum(ab);
            const int i = 4 * t.g + cc;
            if (r == 0 && i < n) {
              double* o = cp + (size_t)i * 8;
#pragma unroll
              for (int q = 0; q < VNR; ++q) o[q] = s[q];
              o[VNR] = ab;
            }
#pragma unroll
            for (int q = 0; q < VNR; ++q) s[q] = 0.0;
            ab = 0.0;
          }
        });
    // columns of groups with no rows below (the last column at least) have no column part
    for (int i = 4 * wave + cc; i < n; i += 16) {
      if (r == 0 && nbat(i / 4) == 0) {
        double* o = cp + (size_t)i * 8;
#pragma unroll
        for (int q = 0; q <= VNR; ++q) o[q] = 0.0;
      }
    }
  }
  __syncthreads();
  // ---- row part: items (row set m of 256 rows, batch b of UN columns); thread i = 256 m + tid
  double rmax[VNR] = {0.0, 0.0, 0.0, 0.0}, xmax[VNR] = {0.0, 0.0, 0.0, 0.0}, amax = 0.0;
  {
    const int nm = (np + VNT - 1) / VNT;
    double s[VNR] = {0.0, 0.0, 0.0, 0.0}, ab = 0.0;
    // batches of the wave's rows in set m: columns 0 .. min(n - 1, last row of the wave)
    auto nbat = [&](int m) {
      const int wlo = VNT * m + 64 * wave;
      return wlo < n ? (min(n - 1, wlo + 63) + UN) / UN : 0;
    };
    auto finish = [&](int m) {
      const int i = VNT * m + tid;
      const bool rv = i < n;
      if (rv) {
        const double* o = cp + (size_t)i * 8;
#pragma unroll
        for (int q = 0; q < VNR; ++q) s[q] += o[q];
        ab += o[VNR];
      }
      if (i < np) {
#pragma unroll
        for (int q = 0; q < VNR; ++q) {
          float rf = 0.f;
          if (rv && q < nr) {
            const double rr = B[i + (size_t)q * ldb] - s[q];
            rf = (float)rr;
            rmax[q] = fmax(rmax[q], fabs(rr));
            xmax[q] = fmax(xmax[q], fabs(sh.xs[i][q]));
          }
          sh.u.s.y[i][q] = rf;
        }
      }
      amax = fmax(amax, ab);
#pragma unroll
      for (int q = 0; q < VNR; ++q) s[q] = 0.0;
      ab = 0.0;
    };
    // sets with no valid row of this wave form a suffix: the pipeline stops at the first one
    pipelined_items<UN, double>(
        VbItem{0, 0},
        [&](VbItem t) {
          if (t.b + 1 < nbat(t.g)) return VbItem{t.g, t.b + 1};
          return VbItem{t.g + 1, 0};
        },
        [&](VbItem t) { return t.g < nm && nbat(t.g) > 0; },
        [&](double(&a)[UN], VbItem t) {
          const int i = VNT * t.g + tid;
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int j = t.b * UN + u;
            a[u] = (i < n && j <= i) ? A[i + (size_t)j * lda] : 0.0;
          }
        },
        [&](double(&a)[UN], VbItem t) {
#pragma unroll
          for (int u = 0; u < UN; ++u) {
            const int j = min(t.b * UN + u, n - 1);
            ab += fabs(a[u]);
#pragma unroll
            for (int q = 0; q < VNR; ++q) s[q] = fma(a[u], sh.xs[j][q], s[q]);
          }
          if (t.b + 1 == nbat(t.g)) finish(t.g);
        });
    for (int m = 0; m < nm; ++m)
      if (nbat(m) == 0) finish(m);
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
  __syncthreads();   // red[] and cp are reused by the next call
  return eta;
}

template <int JW>
__device__ void vb_system(const VbArgs& a, int sys, float* W, float* Winv, double* cp, VbShared& sh) {
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
      eta = vb_residual(A, lda, B, ldb, n, np, nr, c0 == 0 && it == 0, cp, sh);
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
  double* cp = reinterpret_cast<double*>(Winv + a.inv_elems);
  // A workgroup draws at most batch + 1 tickets (the counter only grows); more draws mean the
  // counter was not reset, and the loop stops with an error instead of running on.
  for (int draws = 0;; ++draws) {
    if (threadIdx.x == 0) sh.ticket = atomicAdd(a.ticket, 1);
    __syncthreads();
    const int t = sh.ticket;
    __syncthreads();
    if (t >= a.batch) break;
    if (t < 0 || draws > a.batch) {
      if (threadIdx.x == 0) atomicExch(a.err, (int)kErrNoProgress);
      break;
    }
    const int sys = a.order ? a.order[t] : t;
    if (sys < 0 || sys >= a.batch) continue;
    const int n = a.n[sys];
    if (n < 1 || n > a.nmax || n > VNMAX) {
      // invalid size: report and skip (no memory outside the scratch matrix is touched)
      if (threadIdx.x == 0) {
        cds_ir_result_t* r = a.res + sys;
        r->info = -1; r->converged = 0; r->fell_back = 0; r->iters = 0;
        r->eta = INFINITY; r->eta0 = INFINITY; r->stop_reason = 5; r->reserved = 0;
      }
      continue;
    }
    if (n <= a.jw32_max_n) vb_system<32>(a, sys, W, Winv, cp, sh);
    else vb_system<64>(a, sys, W, Winv, cp, sh);
  }
}

__global__ void reset_kernel(int* p) { *p = 0; }

int round64(int n) { return (n + 63) / 64 * 64; }

size_t vb_w_elems(int nmax) { return (size_t)round64(nmax) * (round64(nmax) + WPAD); }
size_t vb_inv_elems(int nmax) { return (size_t)round64(nmax) * 64; }
// factor, diagonal-block inverses, residual column sums (8 doubles per row)
size_t vb_wg_elems(int nmax) { return vb_w_elems(nmax) + vb_inv_elems(nmax) + (size_t)round64(nmax) * 16; }

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
  a.batch = batch; a.nrhs = nrhs; a.nmax = nmax;
  a.n = n; a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.X = X; a.ldx = ldx; a.order = order;
  a.ws = ws; a.wg_elems = vb_wg_elems(nmax); a.w_elems = vb_w_elems(nmax); a.inv_elems = vb_inv_elems(nmax);
  a.ticket = ticket; a.err = c.err; a.res = res; a.t_start = t_start; a.t_end = t_end;
  a.tol = prm.tol; a.success_tol = prm.success_tol; a.max_iter = prm.max_iter;
  a.jw32_max_n = jw32_max_n;
  const int grid = std::max(1, std::min(vbatched_grid(), batch));
  hipLaunchKernelGGL(vbatched_kernel, dim3(grid), dim3(VNT), 0, c.s0, a);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

}  // namespace cds
