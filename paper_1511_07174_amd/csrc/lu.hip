// Blocked right-looking LU with partial pivoting (Sec. 2 of the paper: A = LU,
// L unit lower, partial pivoting; k rank-1 updates delayed into one rank-k
// update).  Kernels:
//   panel_kernel   factors the m x jb panel A[k:n, k:k+jb] in one persistent
//                  launch of G workgroups (256 rows each).  Each column step is
//                  one all-to-all exchange of (|pivot candidate|, row) through
//                  flag+payload words: every workgroup finds its local arg-max
//                  with wave shuffles, publishes it, reads everybody's, and
//                  agrees on the global pivot (lowest row on ties).  The panel
//                  is processed in leaves of W columns held in registers; after
//                  each leaf the row interchanges, the small triangular solve
//                  and the update of the rest of the panel are done in the same
//                  launch from the published rows.
//   laswp_kernel   applies the panel's interchanges to the other columns as
//                  per-leaf gather/scatter lists (coalesced over the contiguous
//                  top rows, one line per scattered pivot row).
//   trsm_kernel    U12 = L11^{-1} A12 (unit lower), LDS-blocked.
// The trailing update A22 -= L21 U12 is the MFMA GEMM (gemm.hip).
#include "common.hpp"
#include "kernels.hpp"
#include "mixed.hpp"
#include <algorithm>

namespace cds {

namespace {

constexpr int PNT = 256;    // threads (= rows) per panel workgroup
constexpr int PCH = 224;    // column chunk of the in-panel update (the whole right part for nb <= 256)

template <typename T>
struct PanelArgs {
  T* A; int64_t lda; int64_t strideA;
  int n, k, jb;
  int32_t* ipiv; int64_t strideP;
  int32_t* info;
  uint64_t* slots; int64_t slot_stride;   // words per matrix
  int2* pairs; int* pair_cnt; int64_t pairs_stride;  // per matrix: [leaf][3W] pairs, [leaf] counts
  int cnt_stride;                                     // counts per matrix
  int* err;
  int G;
  double* linv; int64_t strideI;   // L11's 16 x 16 diagonal-block inverses (nullptr: not formed here)
};

template <typename T, int W>
struct SlotLayout {
  static constexpr int LLW = LLWords<T>::n;
  int G, jb;
  __host__ __device__ int64_t hdr_words() const { return 4; }
  __host__ __device__ int64_t cs_par() const { return (int64_t)G * 4 + (int64_t)G * W * LLW + W * LLW; }
  __host__ __device__ int64_t sw_par() const { return (int64_t)3 * W * jb * LLW; }
  __host__ __device__ int64_t total() const { return 2 * cs_par() + 2 * sw_par(); }
  __host__ __device__ int64_t hdr(int par, int g) const { return par * cs_par() + (int64_t)g * 4; }
  __host__ __device__ int64_t cand(int par, int g) const { return par * cs_par() + (int64_t)G * 4 + (int64_t)g * W * LLW; }
  __host__ __device__ int64_t rowj(int par) const { return par * cs_par() + (int64_t)G * 4 + (int64_t)G * W * LLW; }
  __host__ __device__ int64_t sw(int par, int e) const { return 2 * cs_par() + par * sw_par() + (int64_t)e * jb * LLW; }
};

// A barrier that orders LDS accesses only: global loads and stores issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Gather half of a column step for up to 64 workgroups.  Lane i polls
// workgroup i's header, and lane l < wl value l of row j.  Each poll round also
// fetches, with one coalesced load per word, the candidate row of the best
// header seen so far.  The loop ends when every header and row j are in and
// the row held is that of the final best.  If the last header to arrive does
// not change the best, the pivot row is then already in registers and costs no
// round trip of its own.  Same outputs as colstep_exchange.
template <typename T, int W>
__device__ __forceinline__ void colstep_gather_fast(const uint64_t* slots, const SlotLayout<T, W>& L, int m, int wl,
                                                    int cc, int j, int par, uint32_t flag, T* prow, T* prm, T* jrow,
                                                    int* s_p, int* err) {
  constexpr int LLW = LLWords<T>::n;
  const int lane = lane_id();
  const bool hv = lane < L.G;
  const uint64_t* hp = slots + L.hdr(par, hv ? lane : 0);
  const uint64_t* jp = slots + L.rowj(par) + (lane < wl ? lane : 0) * LLW;
  bool h_ok = !hv, j_ok = lane >= wl, r_ok = true;
  T hm = (T)-1;
  int hr = 0x7fffffff;
  uint32_t jv[LLW], rv[LLW];
#pragma unroll
  for (int h = 0; h < LLW; ++h) jv[h] = rv[h] = 0u;
  int row_of = -1;   // workgroup whose candidate row rv holds (wave-uniform)
  T bm;
  int br;
  auto value = [](const uint32_t* w) -> T {
    if constexpr (LLW == 2)
      return __longlong_as_double((long long)(((uint64_t)w[1] << 32) | (uint64_t)w[0]));
    else
      return __uint_as_float(w[0]);
  };
  auto fresh = [&](const uint64_t* w, int nw) {
    bool ok = true;
    for (int h = 0; h < nw; ++h) ok = ok && (uint32_t)(w[h] >> 32) == flag;
    return ok;
  };
  long long spins = 0;
  while (true) {
    wave_pivot_search<T>(hm, hr, h_ok, bm, br);
    const int bw = bm >= (T)0 ? br / PNT : -1;
    if (bw != row_of) {
      row_of = bw;
      r_ok = lane >= wl || bw < 0;
    }
    if (__all(h_ok && j_ok && r_ok)) break;
    uint64_t hw[LLW + 1], rw[LLW], jw[LLW];
#pragma unroll
    for (int h = 0; h < LLW + 1; ++h) hw[h] = 0;
#pragma unroll
    for (int h = 0; h < LLW; ++h) rw[h] = jw[h] = 0;
    if (!h_ok) {
#pragma unroll
      for (int h = 0; h < LLW + 1; ++h)
        hw[h] = __hip_atomic_load(const_cast<uint64_t*>(hp + h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!r_ok) {
      const uint64_t* rp = slots + L.cand(par, row_of) + lane * LLW;
#pragma unroll
      for (int h = 0; h < LLW; ++h)
        rw[h] = __hip_atomic_load(const_cast<uint64_t*>(rp + h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!j_ok) {
#pragma unroll
      for (int h = 0; h < LLW; ++h)
        jw[h] = __hip_atomic_load(const_cast<uint64_t*>(jp + h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!h_ok && fresh(hw, LLW + 1)) {
      h_ok = true;
      uint32_t mw[LLW];
#pragma unroll
      for (int h = 0; h < LLW; ++h) mw[h] = (uint32_t)hw[h];
      hm = value(mw);
      hr = (int)(uint32_t)hw[LLW];
    }
    if (!r_ok && fresh(rw, LLW)) {
      r_ok = true;
#pragma unroll
      for (int h = 0; h < LLW; ++h) rv[h] = (uint32_t)rw[h];
    }
    if (!j_ok && fresh(jw, LLW)) {
      j_ok = true;
#pragma unroll
      for (int h = 0; h < LLW; ++h) jv[h] = (uint32_t)jw[h];
    }
    ++spins;
    if ((spins & 1023) == 0) {
      const bool stop =
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spins > (kSpinLimit >> 2);
      if (stop) {
        if (spins > (kSpinLimit >> 2)) atomicExch(err, (int)kErrSpinTimeout);
        break;
      }
    }
  }
  // a column without any comparable candidate (NaN entries) keeps row j, taken from row j's message
  const int p = (br >= j && br < m) ? br : j;
  const bool from_cand = p == br;
  if (lane < W) {
    const T x = lane < wl ? value(from_cand ? rv : jv) : (T)0;
    prow[lane] = x;
    prm[lane] = lane > cc ? x : (T)0;
    if (p != j) jrow[lane] = lane < wl ? value(jv) : (T)0;
  }
  if (lane == 0) *s_p = p;
}

// Column-step exchange, executed by wave 0 of every panel workgroup: this
// workgroup's best candidate (from the per-wave results) is published with its
// row, then every workgroup's header is read and the global pivot agreed on.
// rowbuf[w] holds the leaf row of wave w's best candidate, jbuf row j (staged
// by their owner threads before the barrier that precedes the exchange).
// Outputs: prow = the pivot row (zero beyond wl), prm = prow restricted to the
// columns the elimination updates (cc < c < wl), jrow = row j, *s_p = pivot row.
template <typename T, int W>
__device__ __forceinline__ void colstep_exchange(uint64_t* slots, const SlotLayout<T, W>& L, int g, int m, int wl,
                                                 int cc, int j, int par, uint32_t flag, const T* red_mag,
                                                 const int* red_row, const T (*rowbuf)[W], const T* jbuf, T* prow,
                                                 T* prm, T* jrow, int* s_p, int* err) {
  constexpr int LLW = LLWords<T>::n;
  const int lane = lane_id();
  T mag = red_mag[0];
  int row = red_row[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    const T om = red_mag[w];
    const int orow = red_row[w];
    if (om > mag || (om == mag && orow < row)) {
      mag = om;
      row = orow;
    }
  }
  uint64_t* hdr = slots + L.hdr(par, g);
  if (lane == 0) {
    ll_store_val(hdr, mag, flag);
    ll_store(hdr + LLW, (uint32_t)row, flag);
  }
  // the candidate row goes out even without a candidate (zeros), so a reader may poll it unconditionally
  if (lane < wl)
    ll_store_val(slots + L.cand(par, g) + lane * LLW, mag >= (T)0 ? rowbuf[(row - g * PNT) >> 6][lane] : (T)0,
                 flag);
  if (j / PNT == g && lane < wl) ll_store_val(slots + L.rowj(par) + lane * LLW, jbuf[lane], flag);
  // one-word values only: for FP64 the per-round pivot reduction over two-word magnitudes cost more
  // than the saved round trip (FP64 getrf+getrs at n = 16384: 158.5 ms against 154.6 ms)
  if constexpr (LLW == 1) {
    if (L.G <= kWave) {
      colstep_gather_fast<T, W>(slots, L, m, wl, cc, j, par, flag, prow, prm, jrow, s_p, err);
      return;
    }
  }
  // every workgroup's header (one combined wait per header)
  T bm = (T)-1;
  int br = 0x7fffffff;
  for (int i = lane; i < L.G; i += kWave) {
    uint32_t wv3[LLW + 1];
    ll_wait_words<LLW + 1>(slots + L.hdr(par, i), flag, err, wv3);
    T mi;
    if constexpr (LLW == 2)
      mi = __longlong_as_double((long long)(((uint64_t)wv3[1] << 32) | (uint64_t)wv3[0]));
    else
      mi = __uint_as_float(wv3[0]);
    const int ri = (int)wv3[LLW];
    if (mi > bm || (mi == bm && ri < br)) {
      bm = mi;
      br = ri;
    }
  }
  T gm;
  int gr;
  wave_pivot_search<T>(bm, br, true, gm, gr);
  // a column without any comparable candidate (NaN entries) keeps row j; the row then comes from
  // row j's own message, which its owner always publishes
  const int p = (gr >= j && gr < m) ? gr : j;
  const int gp = p / PNT;
  if (lane < W) {
    T v[2] = {(T)0, (T)0};
    if (lane < wl) {
      const uint64_t* ptr[2] = {slots + (p == j ? L.rowj(par) : L.cand(par, gp)) + lane * LLW,
                                slots + L.rowj(par) + lane * LLW};
      const bool valid[2] = {true, p != j};
      ll_wait_vals<T, 2>(ptr, valid, flag, err, v);
    }
    prow[lane] = v[0];
    prm[lane] = lane > cc ? v[0] : (T)0;
    if (p != j) jrow[lane] = v[1];
  }
  if (lane == 0) *s_p = p;
}

// Compose the leaf's sequential interchanges (c0+cc <-> piv[cc]) into a list of
// (dst, src) moves.  Entries 0..wl-1 are the top positions c0..c0+wl-1 (src may
// equal dst); later entries are the other moved positions (pivot rows below the
// leaf, each once, in the order of first use).  Every lane traces its position
// back through the interchanges in reverse order, so there is no serial table
// update.  Wave 0 only; returns the entry count in every lane.
template <int W, bool FULL>
__device__ __forceinline__ int compose_leaf(const int* s_piv, int c0, int wl_, int* s_dst, int* s_src, int* s_ne) {
  const int wl = FULL ? W : wl_;   // FULL: a whole leaf, so that no column needs a bounds mask
  const int lane = lane_id();
  const int c1 = c0 + wl;
  const int mypiv = lane < wl ? s_piv[lane] : -1;
  // lane cc names the pivot row of column cc when it lies below the leaf and no earlier column chose it.
  // The pivots come from LDS four at a time (every lane reads the same words), entries at or beyond
  // wl (left from an earlier leaf) read as -1, which no valid lane holds.
  const int4* pv4 = reinterpret_cast<const int4*>(s_piv);
  bool other = mypiv >= c1;
#pragma unroll
  for (int q = 0; q < W / 4; ++q) {
    const int4 pv = pv4[q];
    const int pcs[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = 4 * q + u;
      const int pc = cc < wl ? pcs[u] : -1;
      other = other && !(cc < lane && pc == mypiv);
    }
  }
  int src = c0 + lane, osrc = mypiv;
#pragma unroll
  for (int q = W / 4 - 1; q >= 0; --q) {
    const int4 pv = pv4[q];
    const int pcs[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
    for (int u = 3; u >= 0; --u) {
      const int cc = 4 * q + u;
      const int a = c0 + cc, b = pcs[u];
      const bool on = cc < wl;
      src = on ? (src == a ? b : (src == b ? a : src)) : src;
      osrc = on ? (osrc == a ? b : (osrc == b ? a : osrc)) : osrc;
    }
  }
  if (lane < wl) {
    s_dst[lane] = c0 + lane;
    s_src[lane] = src;
  }
  const uint64_t mo = __ballot(other);
  if (other) {
    const int idx = wl + __popcll(mo & ((1ull << lane) - 1ull));
    s_dst[idx] = mypiv;
    s_src[idx] = osrc;
  }
  const int ne = wl + __popcll(mo);
  if (lane == 0) *s_ne = ne;
  return ne;
}

// Compact the entries of a leaf's move list whose source (src_side) or
// destination row lies in this workgroup's rows.  Wave 0 only; ne <= 3W <= 128.
__device__ __forceinline__ void compact_entries(const int* s_dst, const int* s_src, int ne, int g, int* s_own, int* s_nown,
                                int* s_dl, int* s_ndl) {
  const int lane = lane_id();
  int no = 0, nd = 0;
  for (int e0 = 0; e0 < ne; e0 += kWave) {
    const int e = e0 + lane;
    const bool in = e < ne;
    const bool so = in && s_src[e] / PNT == g;
    const bool dO = in && s_dst[e] / PNT == g && s_dst[e] != s_src[e];
    const uint64_t mo = __ballot(so), md = __ballot(dO);
    const uint64_t below = (1ull << lane) - 1ull;
    if (so) s_own[no + __popcll(mo & below)] = e;
    if (dO) s_dl[nd + __popcll(md & below)] = e;
    no += __popcll(mo);
    nd += __popcll(md);
  }
  if (lane == 0) {
    *s_nown = no;
    *s_ndl = nd;
  }
}

// A thread's row of a 32-column leaf, held in registers.  Columns are read and
// written at compile-time indices in unrolled loops, and at the column step's
// wave-uniform index through relative register addressing (a short
// s_set_gpr_idx sequence, not a chain of selects and not scratch memory).
template <typename T> struct LeafRow;
template <> struct LeafRow<float> {
  typedef float vt __attribute__((ext_vector_type(32)));
  vt a;
  __device__ __forceinline__ float get(int c) const { return a[c]; }
  __device__ __forceinline__ void set(int c, float x) { a[c] = x; }
};
template <> struct LeafRow<double> {
  typedef double vt __attribute__((ext_vector_type(16)));
  vt lo, hi;
  __device__ __forceinline__ double get(int c) const { return c < 16 ? lo[c] : hi[c - 16]; }
  __device__ __forceinline__ void set(int c, double x) {
    if (c < 16) lo[c] = x;
    else hi[c - 16] = x;
  }
};

// The panel: G workgroups of PNT rows.  Per leaf of W columns, each thread
// keeps its row of the leaf in registers through the column loop; after the
// leaf, the leaf's interchanges move rows between workgroups in one
// publish/consume round of flag+payload words, every workgroup forms
// U_right = L11^{-1} P_top for the right part of the panel, and updates its own
// rows with an MFMA product.  About 70 KiB of LDS (FP64), so that a panel
// workgroup fits beside a trailing-update workgroup on one compute unit.
template <typename T, int W>
__global__ void __launch_bounds__(PNT, 2) panel_kernel(PanelArgs<T> P) {
  constexpr int LLW = LLWords<T>::n;
  constexpr bool F64 = std::is_same<T, double>::value;
  typedef typename std::conditional<F64, d4, f4>::type acc_t;
  static_assert(W == 32, "the MFMA update assumes 32-column leaves");
  const int g = blockIdx.x, b = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = P.n - P.k, jb = P.jb;
  const int64_t lda = P.lda;
  T* __restrict__ A = P.A + (size_t)b * P.strideA + P.k + (size_t)P.k * lda;
  int32_t* ipiv = P.ipiv + (size_t)b * P.strideP + P.k;
  uint64_t* slots = P.slots + (size_t)b * P.slot_stride;
  int2* pairs = P.pairs + (size_t)b * P.pairs_stride;
  int* pair_cnt = P.pair_cnt + (size_t)b * P.cnt_stride;
  SlotLayout<T, W> L{P.G, jb};
  const int row = g * PNT + tid;
  const bool own = row < m;
  // the panel is the critical path; its waves win issue arbitration over a co-resident trailing update
  __builtin_amdgcn_s_setprio(3);

  __shared__ T rowbuf[4][W];        // per-wave best candidate row
  __shared__ T jbuf[W];             // row j (owner workgroup)
  __shared__ T red_mag[4];
  __shared__ int red_row[4];
  __shared__ T prow[W];
  __shared__ T prm[W];
  __shared__ T jrow[W];
  __shared__ int s_p;
  __shared__ T L11[W][W + 1];
  __shared__ __align__(16) int s_piv[W];
  __shared__ int s_dst[3 * W], s_src[3 * W];
  __shared__ int s_own[3 * W], s_dl[3 * W];
  __shared__ int s_ne, s_nown, s_ndl;
  __shared__ T Ubuf[W][PCH + 8];
  __shared__ double Li2[2][16][17];   // inverses of L11's two unit-lower 16 x 16 diagonal blocks

  int leafc = 0;
  for (int c0 = 0; c0 < jb; c0 += W, ++leafc) {
    const int wl = min(W, jb - c0);
    const int c1 = c0 + wl;
    const bool act = own && row >= c0;
    LeafRow<T> v;
#pragma unroll
    for (int cc = 0; cc < W; ++cc) v.set(cc, (act && cc < wl) ? A[row + (size_t)(c0 + cc) * lda] : (T)0);
    for (int cc = 0; cc < wl; ++cc) {
      const int j = c0 + cc;
      const int par = j & 1;
      const uint32_t flag = (uint32_t)(P.k + j + 1);
      T x = v.get(cc);
      T wbm;
      int wbr;
      wave_pivot_search<T>(fabs(x), row, own && row >= j, wbm, wbr);
      if (row == wbr) {
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) rowbuf[wave][c2] = v.get(c2);
      }
      if (own && row == j) {
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) jbuf[c2] = v.get(c2);
      }
      if (lane == 0) { red_mag[wave] = wbm; red_row[wave] = wbr; }
      __syncthreads();
      if (wave == 0)
        colstep_exchange<T, W>(slots, L, g, m, wl, cc, j, par, flag, red_mag, red_row, rowbuf, jbuf, prow, prm, jrow,
                               &s_p, P.err);
      __syncthreads();
      const int p = s_p;
      const T piv = prow[cc];
      if (own && row == j) {
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) v.set(c2, prow[c2]);
      } else if (own && row == p) {
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) v.set(c2, jrow[c2]);
        x = jrow[cc];
      }
      if (own && row > j && piv != (T)0) {
        // prm is zero outside (cc, wl): one unconditional fused update per column, then the
        // multiplier into column cc
        const T lmul = x / piv;
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) v.set(c2, fma(-lmul, prm[c2], v.get(c2)));
        v.set(cc, lmul);
      }
      if (tid < W) L11[cc][tid] = prow[tid];
      if (tid == 0) {
        s_piv[cc] = p;
        // a zero pivot is recorded at once (rare); ipiv is written once per leaf
        if (g == 0 && piv == (T)0) atomicCAS(P.info + b, 0, P.k + j + 1);
      }
    }
    // the leaf's final values (up to later interchanges) and the MFMA operand copy: a wave-uniform
    // column base and one 32-bit row offset for every column, so that no store waits for the one
    // before it to release an address register
    if (act) {
      const uint32_t urow = (uint32_t)row;
      if (wl == W) {
#pragma unroll
        for (int cc = 0; cc < W; ++cc) (A + (size_t)(c0 + cc) * lda)[urow] = v.get(cc);
      } else {
#pragma unroll
        for (int cc = 0; cc < W; ++cc)
          if (cc < wl) (A + (size_t)(c0 + cc) * lda)[urow] = v.get(cc);
      }
    }
    // these two barriers order LDS only (the pivots, L11 and the move lists); nothing reads the
    // leaf columns just stored before the full barriers further down
    lds_barrier();
    if (wave == 0) {
      const int ne0 = wl == W ? compose_leaf<W, true>(s_piv, c0, wl, s_dst, s_src, &s_ne)
                              : compose_leaf<W, false>(s_piv, c0, wl, s_dst, s_src, &s_ne);
      // the lists written by other lanes of this wave are read below: order the LDS accesses
      wave_fence();
      compact_entries(s_dst, s_src, ne0, g, s_own, &s_nown, s_dl, &s_ndl);
    } else if (F64 && wave == 1 && lane < 32) {
      // meanwhile (FP64 panels): lane c, column c % 16 of the inverse of L11's unit-lower diagonal
      // block c / 16, by forward substitution (the terms q < c multiply y[q] = 0); rows at or beyond
      // wl act as the identity
      const int bb = lane >> 4, c = lane & 15, r0 = 16 * bb;
      double y[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double sacc = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) sacc -= (double)L11[r0 + i][r0 + q] * y[q];
        y[i] = r0 + i >= wl ? ((i == c) ? 1.0 : 0.0) : (i < c ? 0.0 : sacc);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Li2[bb][i][c] = y[i];
    }
    lds_barrier();
    if (g == 0 && tid < wl) ipiv[c0 + tid] = P.k + s_piv[tid] + 1;
    const int ne = s_ne;
    const int spar = leafc & 1;
    const uint32_t sflag = (uint32_t)(P.k + c0 + 1);
    const int nv = jb - wl;   // non-leaf columns of the panel: [0, c0) and [c1, jb)
    if (g == 0) {
      for (int e = tid; e < ne; e += PNT) pairs[leafc * 3 * W + e] = make_int2(s_dst[e] + P.k, s_src[e] + P.k);
      if (tid == 0) pair_cnt[leafc] = ne;
    }
    if (nv == 0) continue;
    constexpr int SB = 8;
    // publish the non-leaf columns of the rows this workgroup is the source of
    {
      const int nown = s_nown;
      const int total = nown * nv;
      for (int base = 0; base < total; base += PNT * SB) {
        T vv[SB];
        int64_t off[SB];
        bool ok[SB];
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          const int it = base + q * PNT + tid;
          ok[q] = it < total;
          off[q] = 0;
          vv[q] = (T)0;
          if (ok[q]) {
            const int ei = it / nv, idx = it - ei * nv;
            const int e = s_own[ei];
            const int col = idx < c0 ? idx : idx + wl;
            off[q] = (int64_t)L.sw(spar, e) + (int64_t)idx * LLW;
            vv[q] = A[s_src[e] + (size_t)col * lda];
          }
        }
#pragma unroll
        for (int q = 0; q < SB; ++q)
          if (ok[q]) ll_store_val(slots + off[q], vv[q], sflag);
      }
    }
    __syncthreads();   // every read of a source row of this workgroup precedes the writes below
    const int ndl = s_ndl;
    // the MFMA B operand, L21 of this wave's rows: lane l takes column 4 kc + l / 16 of the row held
    // by lane 16 rt + l % 16 (four lane shuffles, one per column offset, and a select)
    const int wr = wave * 64;                      // first row of this wave within the workgroup
    T bop[4][W / 4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int kc = 0; kc < W / 4; ++kc) {
        const int src = rt * 16 + (lane & 15);
        T sel = (T)0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T t = __shfl(v.get(4 * kc + q), src, kWave);
          sel = ((lane >> 4) == q) ? t : sel;
        }
        bop[rt][kc] = sel;
      }
    bool first = true;
    // the first pass also takes the rows this workgroup receives, so it runs for the last leaf too
    for (int x0 = c1; x0 < jb || first; x0 += PCH, first = false) {
      const int cw = max(0, min(PCH, jb - x0));
      // one combined wait: P_top's columns [x0, x0 + cw) into Ubuf and (first chunk) the rows this
      // workgroup receives (top destinations take only the left part; U_right overwrites the rest)
      {
        const int nU = wl * cw;
        const int total = nU + (first ? ndl * nv : 0);
        for (int base = 0; base < total; base += PNT * SB) {
          const uint64_t* ptr[SB];
          bool ok[SB];
          int64_t dsto[SB];
          T vv[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const int it = base + q * PNT + tid;
            ok[q] = it < total;
            if (it < nU) {
              const int cc = it / cw, x = it - cc * cw;
              ptr[q] = slots + L.sw(spar, cc) + (int64_t)(x0 + x - wl) * LLW;
              dsto[q] = -1 - (int64_t)(cc * (PCH + 8) + x);
            } else if (ok[q]) {
              const int it2 = it - nU;
              const int ei = it2 / nv, idx = it2 - ei * nv;
              const int e = s_dl[ei];
              const int col = idx < c0 ? idx : idx + wl;
              ok[q] = e >= wl || idx < c0;
              ptr[q] = slots + L.sw(spar, e) + (int64_t)idx * LLW;
              dsto[q] = (int64_t)s_dst[e] + (int64_t)col * lda;
            } else {
              ptr[q] = slots;
              dsto[q] = 0;
            }
          }
          ll_wait_vals<T, SB>(ptr, ok, sflag, P.err, vv);
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            if (!ok[q]) continue;
            if (dsto[q] < 0) (&Ubuf[0][0])[-1 - dsto[q]] = vv[q];
            else A[dsto[q]] = vv[q];
          }
        }
      }
      __syncthreads();
      if (cw == 0) break;
      // U_right = L11^{-1} P_top.  FP64: on MFMA tiles of 16 columns (wave w: tiles w, w + 4, ...), by
      // 16 x 16 blocks: X0 = inv(L00) P0, P1 -= L10 X0, X1 = inv(L11) P1 (products exact on small
      // dyadic data, as in the TRSM).  Accumulator v of a product holds row k64(v) of column l % 16,
      // and every product takes its k index so that the previous product's accumulators are its B
      // operand.  FP32 (where the extra registers slowed the column loop more than this saves): one
      // thread per column, by columns of L11: as soon as u[t] is final it is taken out of every
      // later row, so each u[i] still subtracts L11[i][t] u[t] in the order t = 0, 1, ..., i - 1,
      // while the dependent chain is W steps long instead of W^2 / 2.
      if constexpr (F64) {
        const int li = lane & 15, kl = lane >> 4;
        auto k64 = [&](int v) { return kl + 4 * v; };
        auto kout = [&](int v) { return F64 ? kl + 4 * v : 4 * kl + v; };
        for (int ct = wave; 16 * ct < cw; ct += 4) {
          const int cx = 16 * ct + li;   // column of the chunk
          d4 x0 = {0.0, 0.0, 0.0, 0.0}, x1 = {0.0, 0.0, 0.0, 0.0};
          acc_t p1;
#pragma unroll
          for (int v = 0; v < 4; ++v) p1[v] = 16 + kout(v) < wl ? Ubuf[16 + kout(v)][cx] : (T)0;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = k64(s);
            x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Li2[0][li][k], k < wl ? (double)Ubuf[k][cx] : 0.0, x0, 0, 0, 0);
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const T a = 16 + li < wl ? -L11[16 + li][k64(s)] : (T)0;
            if constexpr (F64)
              p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, x0[s], p1, 0, 0, 0);
            else
              p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, (T)x0[s], p1, 0, 0, 0);
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
            x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Li2[1][li][kout(s)], (double)p1[s], x1, 0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Ubuf[k64(v)][cx] = (T)x0[v];
            Ubuf[16 + k64(v)][cx] = (T)x1[v];
          }
        }
      } else if (tid < cw) {
        T u[W];
#pragma unroll
        for (int i = 0; i < W; ++i) u[i] = (i < wl) ? Ubuf[i][tid] : (T)0;
#pragma unroll
        for (int t = 0; t < W - 1; ++t) {
          const T ut = u[t];
#pragma unroll
          for (int i = t + 1; i < W; ++i) u[i] = (i < wl) ? u[i] - L11[i][t] * ut : (T)0;
        }
#pragma unroll
        for (int i = 0; i < W; ++i) Ubuf[i][tid] = u[i];
      }
      __syncthreads();
      // the top rows take U_right
      for (int idx = tid; idx < wl * cw; idx += PNT) {
        const int cc = idx / cw, x = idx - cc * cw;
        const int r = c0 + cc;
        if (r / PNT == g) A[r + (size_t)(x0 + x) * lda] = Ubuf[cc][x];
      }
      // rows >= c1 of this wave: C[rows, cols] -= L21[rows, :] U_right[:, cols] on 16x16x4 MFMA tiles,
      // computed transposed (D = -U^T L21^T) so that a lane's accumulators run down a column.
      // Tiles of 16 columns.
      {
        const int ntile = 2 * ((cw + 31) / 32);
        const int rr0 = g * PNT + wr + (lane & 15);
        // a tile whose 64 rows all lie in [c1, m) and whose 16 columns all exist takes unmasked loads
        // and stores (wave-uniform test); the others mask element by element
        const bool rows_full = g * PNT + wr >= c1 && g * PNT + wr + 63 < m;
        auto load_c = [&](acc_t (&a)[4], int t) {
          const int xs = x0 + (t >> 1) * 32, cws = min(32, x0 + cw - xs), ct = t & 1;
          if (rows_full && ct * 16 + 16 <= cws) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
              for (int vq = 0; vq < 4; ++vq) {
                const int ci = ct * 16 + (F64 ? ((lane >> 4) + 4 * vq) : (4 * (lane >> 4) + vq));
                a[rt][vq] = A[rr0 + rt * 16 + (size_t)(xs + ci) * lda];
              }
            return;
          }
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int vq = 0; vq < 4; ++vq) {
              const int ci = ct * 16 + (F64 ? ((lane >> 4) + 4 * vq) : (4 * (lane >> 4) + vq));
              const int rr = rr0 + rt * 16;
              const bool ok = rr < m && rr >= c1 && ci < cws;
              a[rt][vq] = ok ? A[rr + (size_t)(xs + ci) * lda] : (T)0;
            }
        };
        auto mfma_store = [&](acc_t (&a)[4], int t) {
          const int xs = x0 + (t >> 1) * 32, cws = min(32, x0 + cw - xs), ct = t & 1;
          T aop[W / 4];
#pragma unroll
          for (int kc = 0; kc < W / 4; ++kc) aop[kc] = -Ubuf[4 * kc + (lane >> 4)][xs - x0 + ct * 16 + (lane & 15)];
#pragma unroll
          for (int kc = 0; kc < W / 4; ++kc) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              if constexpr (F64)
                a[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[kc], bop[rt][kc], a[rt], 0, 0, 0);
              else
                a[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[kc], bop[rt][kc], a[rt], 0, 0, 0);
            }
          }
          if (rows_full && ct * 16 + 16 <= cws) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
              for (int vq = 0; vq < 4; ++vq) {
                const int ci = ct * 16 + (F64 ? ((lane >> 4) + 4 * vq) : (4 * (lane >> 4) + vq));
                A[rr0 + rt * 16 + (size_t)(xs + ci) * lda] = a[rt][vq];
              }
            return;
          }
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int vq = 0; vq < 4; ++vq) {
              const int ci = ct * 16 + (F64 ? ((lane >> 4) + 4 * vq) : (4 * (lane >> 4) + vq));
              const int rr = rr0 + rt * 16;
              if (rr < m && rr >= c1 && ci < cws) A[rr + (size_t)(xs + ci) * lda] = a[rt][vq];
            }
        };
        // three tiles of C in flight: a tile's MFMAs take far less time than its loads
        acc_t b0[4], b1[4], b2[4];
        if (ntile > 0) load_c(b0, 0);
        if (ntile > 1) load_c(b1, 1);
        for (int t = 0; t < ntile; t += 3) {
          if (t + 2 < ntile) load_c(b2, t + 2);
          mfma_store(b0, t);
          if (t + 1 >= ntile) break;
          if (t + 3 < ntile) load_c(b0, t + 3);
          mfma_store(b1, t + 1);
          if (t + 2 >= ntile) break;
          if (t + 4 < ntile) load_c(b1, t + 4);
          mfma_store(b2, t + 2);
        }
      }
      __syncthreads();   // Ubuf is reloaded by the next chunk
    }
  }
  // The panel's top jb <= PNT rows, L11 among them, are rows of workgroup 0 and were written by
  // its own threads: once they are all stored, it forms the inverses of L11's unit 16 x 16
  // diagonal blocks for the TRSMs that follow.
  if (P.linv != nullptr && g == 0) {
    __syncthreads();
    double* Li = P.linv + (size_t)b * P.strideI;
    for (int t = tid; t < ((jb + 15) / 16) * 16; t += PNT) diag_inv16_column<T, true>(A, lda, jb, t >> 4, t & 15, Li);
  }
}

// Apply the panel's interchanges (per-leaf move lists) to column ranges
// [c_lo1, c_hi1) and [c_lo2, c_hi2), and (rowid non-null) to the int32 row-order
// vector rowid, which then follows the rows as one more column.  One wave per
// column at a time.
template <typename T, int W>
__global__ void __launch_bounds__(256) laswp_kernel(T* A0, int64_t lda, int64_t strideA, const int2* pairs0,
                                                    const int* cnt0, int64_t pairs_stride, int cnt_stride,
                                                    int nleaves, int c_lo1, int c_hi1, int c_lo2, int c_hi2,
                                                    int32_t* rowid0, int64_t strideR) {
  const int b = blockIdx.y;
  T* A = A0 + (size_t)b * strideA;
  const int2* pairs = pairs0 + (size_t)b * pairs_stride;
  const int* cnt = cnt0 + (size_t)b * cnt_stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n1 = c_hi1 - c_lo1, n2 = c_hi2 - c_lo2, ncols = n1 + n2 + (rowid0 != nullptr ? 1 : 0);
  constexpr int MAXE = 3 * W;
  constexpr int PER = (MAXE + 63) / 64;
  auto move = [&](auto* colp) {
    typedef typename std::remove_pointer<decltype(colp)>::type E;
    for (int l = 0; l < nleaves; ++l) {
      const int ne = cnt[l];
      const int2* pl = pairs + l * MAXE;
      E v[PER];
      int dst[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = lane + 64 * q;
        dst[q] = -1;
        if (e < ne) {
          int2 pr = pl[e];
          if (pr.x != pr.y) { dst[q] = pr.x; v[q] = colp[pr.y]; }
        }
      }
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (dst[q] >= 0) colp[dst[q]] = v[q];
    }
  };
  for (int cidx = blockIdx.x * 4 + wave; cidx < ncols; cidx += gridDim.x * 4) {
    if (cidx == n1 + n2) {
      move(rowid0 + (size_t)b * strideR);
    } else {
      const int col = cidx < n1 ? c_lo1 + cidx : c_lo2 + (cidx - n1);
      move(A + (size_t)col * lda);
    }
  }
}

__global__ void iota_kernel(int32_t* p0, int64_t stride, int n) {
  int32_t* p = p0 + (size_t)blockIdx.y * stride;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

constexpr int kLeaf = 32;

int default_nb(int n) {
  if (n <= 2048) return 128;
  return 256;
}

}  // namespace

size_t getrf_ws_bytes(int n, int nb, int leaf, int batch, size_t elem) {
  (void)leaf;
  int jb = std::min(nb, std::max(n, 1));
  int G = (std::max(n, 1) + PNT - 1) / PNT;
  int llw = elem == 8 ? 2 : 1;
  int64_t cs = (int64_t)G * 4 + (int64_t)G * kLeaf * llw + kLeaf * llw;
  int64_t sw = (int64_t)3 * kLeaf * jb * llw;
  int64_t slot_words = 2 * cs + 2 * sw;
  int nleaves = (jb + kLeaf - 1) / kLeaf;
  size_t slots = (size_t)slot_words * 8 * batch;
  size_t pairs = (size_t)2 * batch * nleaves * 3 * kLeaf * sizeof(int2);
  size_t cnts = (size_t)2 * batch * nleaves * sizeof(int);
  size_t inv = (size_t)2 * batch * trsm16_inv_elems(jb) * sizeof(double);   // L11 diagonal-block inverses, by parity
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return kErrRegion + al(slots) + al(pairs) + al(cnts) + al(inv);
}

template <typename T>
cds_status_t getrf_run_mode(Ctx& c, int n, T* A, int64_t lda, int64_t strideA, int32_t* ipiv, int64_t strideP,
                            int32_t* info, int batch, int nb, int mode, float* scale_part, int32_t* perm_out) {
  if (batch <= 0) return CDS_SUCCESS;
  if (n == 0) {
    if (launch_fill_i32(info, batch, 0, c.s0) != hipSuccess) return CDS_HIP_ERROR;
    return CDS_SUCCESS;
  }
  if (nb <= 0) nb = default_nb(n);
  nb = std::min(512, std::max(kLeaf, (nb / kLeaf) * kLeaf));
  const int W = kLeaf;
  const int G = (n + PNT - 1) / PNT;
  const int jbmax = std::min(nb, n);
  const int llw = LLWords<T>::n;
  const int64_t cs = (int64_t)G * 4 + (int64_t)G * W * llw + W * llw;
  const int64_t swp = (int64_t)3 * W * jbmax * llw;
  const int64_t slot_words = 2 * cs + 2 * swp;
  const int nleaves = (jbmax + W - 1) / W;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t need = getrf_ws_bytes(n, nb, W, batch, sizeof(T));
  if (c.ws == nullptr || c.ws_bytes < need) return CDS_WORKSPACE_TOO_SMALL;
  char* base = (char*)c.ws + kErrRegion;
  uint64_t* slots = (uint64_t*)base;
  size_t slots_b = al((size_t)slot_words * 8 * batch);
  int2* pairs = (int2*)(base + slots_b);
  size_t pairs_b = al((size_t)2 * batch * nleaves * 3 * W * sizeof(int2));
  int* cnts = (int*)(base + slots_b + pairs_b);
  size_t cnts_b = al((size_t)2 * batch * nleaves * sizeof(int));
  double* linv = (double*)(base + slots_b + pairs_b + cnts_b);
  const int64_t inv_stride = (int64_t)trsm16_inv_elems(jbmax);   // per matrix
  const int64_t pairs_stride = (int64_t)nleaves * 3 * W;   // per matrix per parity

  hipStream_t s0 = c.s0, s1 = c.s1;
  if (launch_fill_i32(info, batch, 0, s0) != hipSuccess) return CDS_HIP_ERROR;
  if (launch_fill_zero(slots, (size_t)slot_words * 8 * batch, s0) != hipSuccess) return CDS_HIP_ERROR;
  if (perm_out != nullptr) {
    // the row order starts as the identity and follows every interchange (n per matrix)
    hipLaunchKernelGGL(iota_kernel, dim3(std::min(1024, (n + 255) / 256), batch), dim3(256), 0, s0, perm_out,
                       (int64_t)n, n);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  }

  const bool la = c.lookahead && n > nb && batch == 1;
  // s1 joins s0's work so far
  if (la) {
    if (hipEventRecord(c.ev[0], s0) != hipSuccess) return CDS_HIP_ERROR;
    if (hipStreamWaitEvent(s1, c.ev[0], 0) != hipSuccess) return CDS_HIP_ERROR;
  }

  auto panel = [&](int k, int jb, int parity, hipStream_t s) -> hipError_t {
    PanelArgs<T> P;
    P.A = A; P.lda = lda; P.strideA = strideA;
    P.n = n; P.k = k; P.jb = jb;
    P.ipiv = ipiv; P.strideP = strideP; P.info = info;
    P.slots = slots; P.slot_stride = slot_words;
    P.pairs = pairs + (size_t)parity * batch * pairs_stride;
    P.pair_cnt = cnts + (size_t)parity * batch * nleaves;
    P.pairs_stride = pairs_stride;
    P.cnt_stride = nleaves;
    P.err = c.err;
    P.G = (n - k + PNT - 1) / PNT;
    double* li = linv + (size_t)parity * batch * inv_stride;
    const bool fused_inv = jb <= PNT;   // then workgroup 0 holds all of L11
    P.linv = fused_inv ? li : nullptr;
    P.strideI = inv_stride;
    const double m = n - k;
    {
      KScope ks(c.timer, CDS_KC_PANEL, s, batch * (m * jb * jb - (double)jb * jb * jb / 3.0),
                batch * 2.0 * m * jb * sizeof(T));
      hipLaunchKernelGGL((panel_kernel<T, kLeaf>), dim3(P.G, batch), dim3(PNT), 0, s, P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || fused_inv) return e;
    // inverses of L11's 16 x 16 diagonal blocks for this panel's TRSMs
    KScope kt(c.timer, CDS_KC_TRSM, s, 0.0, 0.0);
    return launch_diag_inv16<T>(A + k + (size_t)k * lda, lda, strideA, jb, 1, li, inv_stride, batch, s);
  };
  // interchanges + trsm + gemm on columns [cb, ce) for the panel at k (width jb)
  auto update = [&](int k, int jb, int parity, int cb, int ce, bool left, hipStream_t s) -> hipError_t {
    const int nl = (jb + W - 1) / W;
    const int2* pr = pairs + (size_t)parity * batch * pairs_stride;
    const int* pc = cnts + (size_t)parity * batch * nleaves;
    int lo1 = 0, hi1 = left ? k : 0;
    int ncols = (hi1 - lo1) + (ce - cb);
    // the row order follows each panel's interchanges once, with the left columns
    int32_t* rid = left ? perm_out : nullptr;
    if (ncols > 0 || rid != nullptr) {
      int blocks = std::min(4096, (ncols + (rid ? 1 : 0) + 3) / 4);
      KScope ks(c.timer, CDS_KC_LASWP, s, 0.0, batch * 4.0 * sizeof(T) * jb * (double)ncols);
      hipLaunchKernelGGL((laswp_kernel<T, kLeaf>), dim3(blocks, batch), dim3(256), 0, s, A, lda, strideA, pr, pc,
                         pairs_stride, nleaves, nl, lo1, hi1, cb, ce, rid, (int64_t)n);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (ce > cb) {
      const int nc = ce - cb;
      // U12 = L11^{-1} A12 on MFMA tiles, from the panel's diagonal-block inverses
      hipError_t e;
      {
        KScope kt(c.timer, CDS_KC_TRSM, s, batch * (double)jb * jb * nc, 0.0);
        e = launch_trsm16<T>(A + k + (size_t)k * lda, lda, strideA, linv + (size_t)parity * batch * inv_stride,
                             inv_stride, A + k + (size_t)cb * lda, lda, strideA, jb, nc, 0, batch, nullptr, s);
      }
      if (e != hipSuccess) return e;
      const int mrem = n - k - jb;
      const float* sc = nullptr;
      if (mrem > 0 && mode == 2 && scale_part != nullptr) {
        // partial maxima of this launch's U12 block for its power-of-two scale (one region per stream)
        float* slot = scale_part + (s == c.s0 ? 0 : (size_t)batch * kScaleParts);
        if constexpr (std::is_same<T, float>::value) {
          e = launch_maxabs_part(A + k + (size_t)cb * lda, lda, strideA, jb, nc, slot, batch, s);
          if (e != hipSuccess) return e;
        }
        sc = slot;
      }
      if (mrem > 0) {
        GemmArgs<T> ga;
        ga.m = mrem; ga.n = nc; ga.k = jb;
        ga.A = A + (k + jb) + (size_t)k * lda; ga.lda = lda; ga.strideA = strideA;
        ga.B = A + k + (size_t)cb * lda; ga.ldb = lda; ga.strideB = strideA;
        ga.C = A + (k + jb) + (size_t)cb * lda; ga.ldc = lda; ga.strideC = strideA;
        ga.alpha = (T)-1; ga.transB = 0; ga.lower = 0; ga.scale_part = sc; ga.scaleA = 0; ga.guard = nullptr;
        KScope ks(c.timer, CDS_KC_UPDATE, s, batch * 2.0 * mrem * (double)nc * jb,
                  batch * (double)sizeof(T) * (2.0 * mrem * nc + (double)mrem * jb + (double)jb * nc));
        e = launch_gemm<T>(ga, batch, mode, s);
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  };

  int step = 0;
  if (!la) {
    for (int k = 0; k < n; k += nb, ++step) {
      const int jb = std::min(nb, n - k);
      const int par = step & 1;
      if (panel(k, jb, par, s0) != hipSuccess) return CDS_HIP_ERROR;
      if (update(k, jb, par, k + jb, n, true, s0) != hipSuccess) return CDS_HIP_ERROR;
    }
    return CDS_SUCCESS;
  }
  // look-ahead: s0 carries panels and the next panel's columns, s1 the rest.  The rest of step
  // k starts once the next panel's columns are updated: that short chain sits on the critical
  // path and runs faster without the rest's interchanges and TRSM beside it, while the rest
  // still overlaps the whole of the next panel.
  hipEvent_t evL = c.ev[1], evR = c.ev[2];
  if (panel(0, std::min(nb, n), 0, s0) != hipSuccess) return CDS_HIP_ERROR;
  bool have_rest = false;
  for (int k = 0; k < n; k += nb, ++step) {
    const int jb = std::min(nb, n - k);
    const int par = step & 1;
    const int kn = k + jb;                       // next panel start
    const int jbn = std::min(nb, n - kn);        // next panel width (<= 0 if none)
    // s0: next panel's columns (need the previous rest update to have reached them)
    if (jbn > 0) {
      if (have_rest && hipStreamWaitEvent(s0, evR, 0) != hipSuccess) return CDS_HIP_ERROR;
      if (update(k, jb, par, kn, kn + jbn, false, s0) != hipSuccess) return CDS_HIP_ERROR;
    }
    // panel k (and, with a next panel, its columns) done
    if (hipEventRecord(evL, s0) != hipSuccess) return CDS_HIP_ERROR;
    if (jbn > 0 && panel(kn, jbn, par ^ 1, s0) != hipSuccess) return CDS_HIP_ERROR;
    // s1: rest of the trailing matrix and the left interchanges
    if (hipStreamWaitEvent(s1, evL, 0) != hipSuccess) return CDS_HIP_ERROR;
    if (update(k, jb, par, jbn > 0 ? kn + jbn : n, n, true, s1) != hipSuccess) return CDS_HIP_ERROR;
    if (hipEventRecord(evR, s1) != hipSuccess) return CDS_HIP_ERROR;
    have_rest = true;
  }
  // join
  if (hipStreamWaitEvent(s0, evR, 0) != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

template <typename T>
cds_status_t getrf_run(Ctx& c, int n, T* A, int64_t lda, int64_t strideA, int32_t* ipiv, int64_t strideP,
                       int32_t* info, int batch, int nb) {
  return getrf_run_mode<T>(c, n, A, lda, strideA, ipiv, strideP, info, batch, nb, 0, nullptr, nullptr);
}

template cds_status_t getrf_run<double>(Ctx&, int, double*, int64_t, int64_t, int32_t*, int64_t, int32_t*, int, int);
template cds_status_t getrf_run<float>(Ctx&, int, float*, int64_t, int64_t, int32_t*, int64_t, int32_t*, int, int);
template cds_status_t getrf_run_mode<float>(Ctx&, int, float*, int64_t, int64_t, int32_t*, int64_t, int32_t*, int,
                                            int, int, float*, int32_t*);
template cds_status_t getrf_run_mode<double>(Ctx&, int, double*, int64_t, int64_t, int32_t*, int64_t, int32_t*, int,
                                             int, int, float*, int32_t*);

}  // namespace cds
