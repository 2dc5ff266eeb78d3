// Trailing-matrix update  C += alpha * A * op(B)  on MFMA (gfx950).
//
// This is the delayed rank-k update of blocked LU (A22 -= L21 U12) and, in
// lower-tile mode, the symmetric update of blocked Cholesky (A22 -= L21 L21^T):
// Sec. 2 of the paper, where k rank-1 updates are replaced by one rank-k update
// (level-3 BLAS).  It carries ~all of the O(n^3) flops.
//
// Design: 256-thread workgroups (4 waves, 2 x 2), a 128 x 128 C tile per
// workgroup, 64 x 64 per wave = 4 x 4 MFMA 16x16 blocks held in accumulators.
// Launches with fewer than two 128-tiles per compute unit (the look-ahead's
// next-panel columns, the last trailing matrices) take 64 x 64 tiles, so that
// four times as many workgroups share the k-loop.
// A and B tiles are staged through LDS, double-buffered with a register
// prefetch of the next K-slice.  FP64 uses v_mfma_f64_16x16x4, FP32
// v_mfma_f32_16x16x4; the mixed variants read FP32 data, round it to BF16 or
// FP16 while staging into LDS and use v_mfma_f32_16x16x32_{bf16,f16} with
// FP32 accumulation.  Tiles are ordered so that consecutive workgroups on the
// same XCD share the same A row-panel (XCD-aware block remapping).
#include "common.hpp"
#include "kernels.hpp"

#ifndef CDS_GEMM_SCHED
#define CDS_GEMM_SCHED 1
#endif

namespace cds {

namespace {

constexpr int BM = 128, BN = 128, NT = 256;

template <typename T, int MODE> struct GemmCfg;
// MODE 0: native precision MFMA
template <> struct GemmCfg<double, 0> { static constexpr int BK = 16; };
template <> struct GemmCfg<float, 0> { static constexpr int BK = 16; };
// MODE 1: bf16 operands, MODE 2: fp16 operands (T = float storage)
template <> struct GemmCfg<float, 1> { static constexpr int BK = 32; };
template <> struct GemmCfg<float, 2> { static constexpr int BK = 32; };

// Tiles of a launch; lower (m >= n): only tiles with tile_m >= tile_n, the triangle of the top
// tiles_n tile rows and the full tile rows below it.
__host__ __device__ __forceinline__ int tile_count(int tiles_m, int tiles_n, int lower) {
  return lower ? tiles_n * (tiles_n + 1) / 2 + (tiles_m - tiles_n) * tiles_n : tiles_m * tiles_n;
}

// Map a linear workgroup id to a (tile_m, tile_n) pair.
__device__ __forceinline__ void tile_coords(int w, int tiles_m, int tiles_n, int lower, int& tm, int& tn) {
  int total = tile_count(tiles_m, tiles_n, lower);
  // XCD-aware remap: workgroup w runs on XCD (w % 8).  Give each XCD a
  // contiguous range of tile ids so that its L2 sees neighbouring tiles.
  int per = total / 8;
  int t;
  if (per > 0 && w < per * 8) {
    t = (w % 8) * per + (w / 8);
  } else {
    t = w;
  }
  if (!lower) {
    // bands of GM tile rows, each walked column by column: the tiles an XCD runs at once (a few
    // dozen consecutive t) share GM A panels, which stay in its L2 for the whole band, and a
    // handful of B panels (a plain column-major walk would stream every A panel once per column)
    constexpr int GM = 16;
    const int band = t / (GM * tiles_n), r = t - band * GM * tiles_n;
    const int rows = min(GM, tiles_m - band * GM);
    tm = band * GM + r % rows;
    tn = r / rows;
  } else if (t < tiles_n * (tiles_n + 1) / 2) {
    // t -> (tm, tn) with tm >= tn, rows of the lower triangle of tiles
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    tm = r;
    tn = t - r * (r + 1) / 2;
  } else {
    // the full tile rows below the triangle (m > n)
    const int q = t - tiles_n * (tiles_n + 1) / 2;
    tm = tiles_n + q / tiles_n;
    tn = q - (q / tiles_n) * tiles_n;
  }
}

template <typename T>
__device__ __forceinline__ T ldg_or_zero(const T* p, bool ok) { return ok ? *p : (T)0; }

// ------------------------------------------------------------------------------------
// Native-precision kernel (double: f64 MFMA; float: f32 MFMA).
// VEC: 16-byte global loads (host checked the alignment of A, B and the leading
// dimensions); edge vectors fall back to element loads with bounds checks.
// ------------------------------------------------------------------------------------
template <typename T, bool VEC, int TB>
__global__ void __launch_bounds__(NT, (sizeof(T) == 4 && VEC) ? 3 : 2)
gemm_native_kernel(GemmArgs<T> g) {
  if (g.guard && *g.guard != 0) return;
  constexpr int BK = GemmCfg<T, 0>::BK;
  constexpr int BM = TB, BN = TB;   // C tile
  constexpr int MB = TB / 32;       // 16 x 16 blocks per wave and dimension (2 x 2 waves)
  constexpr int PADM = BM + 4;  // row pitch in LDS (elements); PADM * sizeof(T) is a multiple of 16
  constexpr int NV = VEC ? 16 / (int)sizeof(T) : 1;   // elements per global load
  __shared__ __attribute__((aligned(16))) T As[2][BK][PADM];
  __shared__ __attribute__((aligned(16))) T Bs[2][BK][PADM];

  const int b = blockIdx.y;
  const T* __restrict__ A = g.A + (size_t)b * g.strideA;
  const T* __restrict__ B = g.B + (size_t)b * g.strideB;
  T* __restrict__ C = g.C + (size_t)b * g.strideC;

  int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, g.lower, tm, tn);
  const int row0 = tm * BM, col0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave & 1) * (TB / 2), wc = (wave >> 1) * (TB / 2);

  constexpr int A_PER = BM * BK / NT / NV;  // vectors per thread per tile
  constexpr int B_PER = BK * BN / NT / NV;
  T ra[A_PER][NV], rb[B_PER][NV];

  // A tile (BM x BK): vectors run down a column (rows contiguous)
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
      const int e = tid + r * NT;
      const int i = (e % (BM / NV)) * NV, kk = e / (BM / NV);
      const int gi = row0 + i, gk = k0 + kk;
      const T* p = A + gi + (size_t)gk * g.lda;
      if (VEC && gk < g.k && gi + NV <= g.m) {
        if constexpr (VEC) {
          typedef T v_t __attribute__((ext_vector_type(NV)));
          v_t v = *reinterpret_cast<const v_t*>(p);
#pragma unroll
          for (int t = 0; t < NV; ++t) ra[r][t] = v[t];
        }
      } else {
#pragma unroll
        for (int t = 0; t < NV; ++t) ra[r][t] = ldg_or_zero(p + t, gi + t < g.m && gk < g.k);
      }
    }
    if (!g.transB) {
      // B(k, j) = B[k + j ldb]: vectors run along k inside a column
#pragma unroll
      for (int r = 0; r < B_PER; ++r) {
        const int e = tid + r * NT;
        const int kk = (e % (BK / NV)) * NV, j = e / (BK / NV);
        const int gk = k0 + kk, gj = col0 + j;
        const T* p = B + gk + (size_t)gj * g.ldb;
        if (VEC && gj < g.n && gk + NV <= g.k) {
          if constexpr (VEC) {
            typedef T v_t __attribute__((ext_vector_type(NV)));
            v_t v = *reinterpret_cast<const v_t*>(p);
#pragma unroll
            for (int t = 0; t < NV; ++t) rb[r][t] = v[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < NV; ++t) rb[r][t] = ldg_or_zero(p + t, gk + t < g.k && gj < g.n);
        }
      }
    } else {
      // B(k, j) = B[j + k ldb]: vectors run along j
#pragma unroll
      for (int r = 0; r < B_PER; ++r) {
        const int e = tid + r * NT;
        const int j = (e % (BN / NV)) * NV, kk = e / (BN / NV);
        const int gk = k0 + kk, gj = col0 + j;
        const T* p = B + gj + (size_t)gk * g.ldb;
        if (VEC && gk < g.k && gj + NV <= g.n) {
          if constexpr (VEC) {
            typedef T v_t __attribute__((ext_vector_type(NV)));
            v_t v = *reinterpret_cast<const v_t*>(p);
#pragma unroll
            for (int t = 0; t < NV; ++t) rb[r][t] = v[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < NV; ++t) rb[r][t] = ldg_or_zero(p + t, gk < g.k && gj + t < g.n);
        }
      }
    }
  };
  const T alpha = g.alpha;
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
      const int e = tid + r * NT;
      const int i = (e % (BM / NV)) * NV, kk = e / (BM / NV);
#pragma unroll
      for (int t = 0; t < NV; ++t) As[buf][kk][i + t] = alpha * ra[r][t];
    }
    if (!g.transB) {
#pragma unroll
      for (int r = 0; r < B_PER; ++r) {
        const int e = tid + r * NT;
        const int kk = (e % (BK / NV)) * NV, j = e / (BK / NV);
#pragma unroll
        for (int t = 0; t < NV; ++t) Bs[buf][kk + t][j] = rb[r][t];
      }
    } else {
#pragma unroll
      for (int r = 0; r < B_PER; ++r) {
        const int e = tid + r * NT;
        const int j = (e % (BN / NV)) * NV, kk = e / (BN / NV);
#pragma unroll
        for (int t = 0; t < NV; ++t) Bs[buf][kk][j + t] = rb[r][t];
      }
    }
  };

  // The accumulators start from C (loaded together with the first A/B tiles, so
  // the read overlaps the prologue) and alpha is applied to the staged A
  // operand (exact for alpha = -1), which leaves a store-only epilogue.
  typedef typename std::conditional<std::is_same<T, double>::value, d4, f4>::type acc_t;
  // FP32: a lane's four accumulators of a 16 x 16 block are four consecutive rows of one
  // column, so C moves as one 16-byte access per block wherever the group is whole and aligned
  constexpr bool CV4 = std::is_same<T, float>::value;
  const bool c_al = CV4 && ((uintptr_t)C % 16 == 0) && (g.ldc % 4 == 0);
  auto c_group = [&](int mi, int ni, int& gi0, int& gj) {
    gi0 = row0 + wr + mi * 16 + 4 * (lane / 16);
    gj = col0 + wc + ni * 16 + (lane & 15);
    return c_al && gi0 + 3 < g.m && gj < g.n && (!g.lower || gi0 >= gj);
  };
  // element (gi, gj) of C held in accumulator v of block (mi, ni): FP32 keeps the MFMA layout
  // (row 4 (lane / 16) + v, column lane & 15); FP64 computes the transposed block, so its
  // rows are lane & 15 (16 lanes cover 16 consecutive rows) and its columns lane / 16 + 4 v
  auto acc_pos = [&](int mi, int ni, int v, int& gi, int& gj) {
    if constexpr (std::is_same<T, double>::value) {
      gi = row0 + wr + mi * 16 + (lane & 15);
      gj = col0 + wc + ni * 16 + lane / 16 + 4 * v;
    } else {
      gi = row0 + wr + mi * 16 + 4 * (lane / 16) + v;
      gj = col0 + wc + ni * 16 + (lane & 15);
    }
  };
  acc_t acc[MB][MB];
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < MB; ++ni) {
      int gi0, gj0;
      if (c_group(mi, ni, gi0, gj0)) {
        if constexpr (CV4) acc[mi][ni] = *reinterpret_cast<const f4*>(C + gi0 + (size_t)gj0 * g.ldc);
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        acc_pos(mi, ni, v, gi, gj);
        acc[mi][ni][v] = (gi < g.m && gj < g.n && (!g.lower || gi >= gj)) ? C[gi + (size_t)gj * g.ldc] : (T)0;
      }
    }

  const int ktiles = (g.k + BK - 1) / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < ktiles) load_tile((kt + 1) * BK);
    // fragments of k-step s + 1 are read from LDS while the MFMAs of step s run
    T af[2][MB], bf[2][MB];
#pragma unroll
    for (int mi = 0; mi < MB; ++mi) af[0][mi] = As[buf][lane / 16][wr + mi * 16 + (lane & 15)];
#pragma unroll
    for (int ni = 0; ni < MB; ++ni) bf[0][ni] = Bs[buf][lane / 16][wc + ni * 16 + (lane & 15)];
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int cur = s & 1, nxt = cur ^ 1;
      if (s + 1 < BK / 4) {
#pragma unroll
        for (int mi = 0; mi < MB; ++mi) af[nxt][mi] = As[buf][(s + 1) * 4 + lane / 16][wr + mi * 16 + (lane & 15)];
#pragma unroll
        for (int ni = 0; ni < MB; ++ni) bf[nxt][ni] = Bs[buf][(s + 1) * 4 + lane / 16][wc + ni * 16 + (lane & 15)];
      }
#pragma unroll
      for (int mi = 0; mi < MB; ++mi)
#pragma unroll
        for (int ni = 0; ni < MB; ++ni) {
          // FP64 forms the transposed block (operands swapped): lane & 15 then runs down the rows of C
          if constexpr (std::is_same<T, double>::value)
            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[cur][ni], af[cur][mi], acc[mi][ni], 0, 0, 0);
          else
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[cur][mi], bf[cur][ni], acc[mi][ni], 0, 0, 0);
        }
#if CDS_GEMM_SCHED
      // spread the next step's 2 MB fragment reads between this step's MB^2 MFMAs
      if (s + 1 < BK / 4) {
#pragma unroll
        for (int q = 0; q < 2 * MB; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, MB / 2, 0);   // MB / 2 MFMA
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);        // 1 LDS read
        }
      }
#endif
    }
    if (kt + 1 < ktiles) store_tile(buf ^ 1);
    __syncthreads();
  }

  // epilogue: store only
#pragma unroll
  for (int mi = 0; mi < MB; ++mi)
#pragma unroll
    for (int ni = 0; ni < MB; ++ni) {
      int gi0, gj0;
      if (c_group(mi, ni, gi0, gj0)) {
        if constexpr (CV4) *reinterpret_cast<f4*>(C + gi0 + (size_t)gj0 * g.ldc) = acc[mi][ni];
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        acc_pos(mi, ni, v, gi, gj);
        if (gi < g.m && gj < g.n && (!g.lower || gi >= gj)) C[gi + (size_t)gj * g.ldc] = acc[mi][ni][v];
      }
    }
}

// ------------------------------------------------------------------------------------
// Mixed kernel: FP32 data, BF16 (MODE 1) or FP16 (MODE 2) operands, FP32 accumulate.
// For FP16, op(B) is multiplied by 2^e while staging and the product by 2^-e, both
// exact; e comes from the partial maxima of |op(B)| (one wave reduces them).
// ------------------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(NT, 2)
gemm_mixed_kernel(GemmArgs<float> g) {
  if (g.guard && *g.guard != 0) return;
  constexpr int BK = 32;
  constexpr int PITCH = BK + 8;  // halfwords per LDS row (16 B aligned, skewed)
  typedef typename std::conditional<MODE == 1, __bf16, _Float16>::type h_t;
  typedef typename std::conditional<MODE == 1, bf16x8, f16x8>::type h8_t;
  __shared__ __attribute__((aligned(16))) h_t As[2][BM][PITCH];
  __shared__ __attribute__((aligned(16))) h_t Bs[2][BN][PITCH];

  const int b = blockIdx.y;
  const float* __restrict__ A = g.A + (size_t)b * g.strideA;
  const float* __restrict__ B = g.B + (size_t)b * g.strideB;
  float* __restrict__ C = g.C + (size_t)b * g.strideC;
  float bscale = 1.0f, ascale = 1.0f, unscale = 1.0f;
  static_assert(kScaleParts == 64, "one partial maximum per lane");
  if (MODE == 2 && g.scale_part != nullptr) {
    const float t = wave_max(g.scale_part[(size_t)b * kScaleParts + (threadIdx.x & 63)]);
    const int lim = g.scaleA ? 50 : 100;   // 2^-2e stays a normal FP32 number
    int e = 0;
    if (t > 0.f && t == t && t < INFINITY) {
      int ex;
      frexpf(t, &ex);   // t in [2^(ex-1), 2^ex)
      e = max(-lim, min(lim, 14 - ex));
    }
    bscale = ldexpf(1.0f, e);
    if (g.scaleA) ascale = bscale;
    unscale = ldexpf(1.0f, g.scaleA ? -2 * e : -e);
  }

  int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, g.lower, tm, tn);
  const int row0 = tm * BM, col0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;

  // each thread stages 2 units of 8 k-values for A and 2 for B; with B not transposed a unit is 8
  // consecutive elements of a column, read as two 16-byte vectors where aligned and whole
  float ra[2][8], rb[2][8];
  const bool bvec = !g.transB && ((uintptr_t)B % 16 == 0) && (g.ldb % 4 == 0);
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int u = tid + r * NT;
      int i = u % BM, kg = u / BM;
      int gi = row0 + i;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        int gk = k0 + kg * 8 + t;
        ra[r][t] = ldg_or_zero(A + gi + (size_t)gk * g.lda, gi < g.m && gk < g.k);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int u = tid + r * NT;
      int j, kg;
      if (!g.transB) { kg = u % 4; j = u / 4; } else { j = u % BN; kg = u / BN; }
      int gj = col0 + j;
      if (bvec && gj < g.n && k0 + kg * 8 + 8 <= g.k) {
        const f4* p = reinterpret_cast<const f4*>(B + (k0 + kg * 8) + (size_t)gj * g.ldb);
        const f4 v0 = p[0], v1 = p[1];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          rb[r][t] = v0[t];
          rb[r][4 + t] = v1[t];
        }
        continue;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        int gk = k0 + kg * 8 + t;
        const float* p = g.transB ? (B + gj + (size_t)gk * g.ldb) : (B + gk + (size_t)gj * g.ldb);
        rb[r][t] = ldg_or_zero(p, gk < g.k && gj < g.n);
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int u = tid + r * NT;
      int i = u % BM, kg = u / BM;
      h8_t v;
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = (h_t)(ra[r][t] * ascale);
      *reinterpret_cast<h8_t*>(&As[buf][i][kg * 8]) = v;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int u = tid + r * NT;
      int j, kg;
      if (!g.transB) { kg = u % 4; j = u / 4; } else { j = u % BN; kg = u / BN; }
      h8_t v;
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = (h_t)(rb[r][t] * bscale);
      *reinterpret_cast<h8_t*>(&Bs[buf][j][kg * 8]) = v;
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (f4){0, 0, 0, 0};

  const int ktiles = (g.k + BK - 1) / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < ktiles) load_tile((kt + 1) * BK);
    h8_t af[4], bf[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) af[mi] = *reinterpret_cast<const h8_t*>(&As[buf][wr + mi * 16 + (lane & 15)][8 * (lane / 16)]);
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) bf[ni] = *reinterpret_cast<const h8_t*>(&Bs[buf][wc + ni * 16 + (lane & 15)][8 * (lane / 16)]);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) {
        if constexpr (MODE == 1)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        else
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
      }
    if (kt + 1 < ktiles) store_tile(buf ^ 1);
    __syncthreads();
  }
  // epilogue C += alpha (acc 2^-e): a lane's four accumulators of a block are four consecutive rows
  // of one column, so C moves as one 16-byte access where the group is whole and aligned (every
  // read is issued before the first write)
  const bool c_al = ((uintptr_t)C % 16 == 0) && (g.ldc % 4 == 0);
  f4 cv[4][4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int gi0 = row0 + wr + mi * 16 + 4 * (lane / 16), gj = col0 + wc + ni * 16 + (lane & 15);
      if (c_al && gi0 + 3 < g.m && gj < g.n && (!g.lower || gi0 >= gj))
        cv[mi][ni] = *reinterpret_cast<const f4*>(C + gi0 + (size_t)gj * g.ldc);
    }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int gi0 = row0 + wr + mi * 16 + 4 * (lane / 16), gj = col0 + wc + ni * 16 + (lane & 15);
      if (c_al && gi0 + 3 < g.m && gj < g.n && (!g.lower || gi0 >= gj)) {
        f4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = cv[mi][ni][v] + g.alpha * (acc[mi][ni][v] * unscale);
        *reinterpret_cast<f4*>(C + gi0 + (size_t)gj * g.ldc) = o;
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = gi0 + v;
        if (gi < g.m && gj < g.n && (!g.lower || gi >= gj)) {
          float* p = C + gi + (size_t)gj * g.ldc;
          *p = *p + g.alpha * (acc[mi][ni][v] * unscale);
        }
      }
    }
}

}  // namespace

template <typename T>
hipError_t launch_gemm(const GemmArgs<T>& g, int batch, int mode, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.k <= 0 || batch <= 0) return hipSuccess;
  if (g.lower && g.m < g.n) return hipErrorInvalidValue;
  int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  int tiles = tile_count(tiles_m, tiles_n, g.lower);
  dim3 grid(tiles, batch);
  // 16-byte loads need 16-byte aligned bases and leading dimensions that keep every column aligned
  constexpr int nv = 16 / (int)sizeof(T);
  const bool vec = ((uintptr_t)g.A % 16 == 0) && ((uintptr_t)g.B % 16 == 0) && (g.lda % nv == 0) &&
                   (g.ldb % nv == 0) && (g.strideA % nv == 0) && (g.strideB % nv == 0);
  if (mode == 0) {
    if (tiles < 2 * 256) {
      const int tm64 = (g.m + 63) / 64, tn64 = (g.n + 63) / 64;
      const dim3 grid64(tile_count(tm64, tn64, g.lower), batch);
      if (vec)
        hipLaunchKernelGGL((gemm_native_kernel<T, true, 64>), grid64, dim3(NT), 0, s, g);
      else
        hipLaunchKernelGGL((gemm_native_kernel<T, false, 64>), grid64, dim3(NT), 0, s, g);
    } else if (vec) {
      hipLaunchKernelGGL((gemm_native_kernel<T, true, 128>), grid, dim3(NT), 0, s, g);
    } else {
      hipLaunchKernelGGL((gemm_native_kernel<T, false, 128>), grid, dim3(NT), 0, s, g);
    }
  } else {
    if constexpr (std::is_same<T, float>::value) {
      if (mode == 1)
        hipLaunchKernelGGL(gemm_mixed_kernel<1>, grid, dim3(NT), 0, s, g);
      else
        hipLaunchKernelGGL(gemm_mixed_kernel<2>, grid, dim3(NT), 0, s, g);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmArgs<double>&, int, int, hipStream_t);
template hipError_t launch_gemm<float>(const GemmArgs<float>&, int, int, hipStream_t);

}  // namespace cds
