// Triangular solves of the direct method (Sec. 2, step 2: Ly = b, Ux = y, by
// forward and back substitution), and the row interchanges of P b.
//
//   perm_kernel        ipiv (sequential interchanges) -> row order perm, every
//                      position traced backwards in parallel.
//   gather / scatter   Y = B[perm] (op N) or X[perm] = W (op T), with type
//                      conversion so that the refinement loop can solve in FP32
//                      for an FP64 residual and add the correction in FP64.
//   trsv_kernel        persistent, flag-synchronised blocked substitution.
//                      Workgroups take 64-row blocks in dependency order from a
//                      ticket counter (so a block only waits on blocks whose
//                      workgroups are already running).  A block accumulates
//                      the products with every solved block as soon as that
//                      block's solution appears, solves its 64 x 64 diagonal
//                      block in one wave, and publishes its solution through
//                      flag+payload words.  The factor is read once per RHS
//                      group.
#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"
#include <algorithm>

namespace cds {

namespace {

constexpr int BS = 64;      // rows per block
constexpr int TNT = 256;    // threads per workgroup

// ipiv -> perm: perm[i] = original row found at position i after all the
// interchanges (k <-> ipiv[k] - 1, k = 0, 1, ...).  Each thread traces its
// position backwards through the interchanges: position cur after interchange
// k held, before it, the row at k when cur = ipiv[k] - 1, at ipiv[k] - 1 when
// cur = k, else the row at cur.  Since ipiv[k] - 1 >= k, interchanges above a
// workgroup's last position never touch its rows and are skipped.  ipiv is
// staged in LDS in chunks read by every lane at once (a broadcast).
// Interchange entries out of range are ignored.
constexpr int PERM_CH = 4096;
__global__ void __launch_bounds__(256) perm_kernel(const int32_t* ipiv0, int64_t strideP, int n, int32_t* perm0,
                                                   int64_t strideQ) {
  __shared__ int sp[PERM_CH];
  const int b = blockIdx.y;
  const int32_t* ipiv = ipiv0 + (size_t)b * strideP;
  int32_t* perm = perm0 + (size_t)b * strideQ;
  const int i0 = blockIdx.x * 256;
  int cur = i0 + (int)threadIdx.x;
  const int kmax = min(n, i0 + 256) - 1;
  for (int khi = kmax; khi >= 0; khi -= PERM_CH) {
    const int klo = max(0, khi - PERM_CH + 1);
    __syncthreads();
    for (int k = klo + (int)threadIdx.x; k <= khi; k += 256) {
      const int pv = ipiv[k] - 1;
      sp[k - klo] = (pv > k && pv < n) ? pv : k;   // an invalid entry becomes k <-> k
    }
    __syncthreads();
    int k = khi;
    for (; k - 7 >= klo; k -= 8) {
      int pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = sp[k - u - klo];   // issued together, off the chain
#pragma unroll
      for (int u = 0; u < 8; ++u) cur = (cur == k - u) ? pv[u] : ((cur == pv[u]) ? k - u : cur);
    }
    for (; k >= klo; --k) {
      const int pv = sp[k - klo];
      cur = (cur == k) ? pv : ((cur == pv) ? k : cur);
    }
  }
  if (i0 + (int)threadIdx.x < n) perm[i0 + threadIdx.x] = cur;
}

// The same permutation in two steps, for n up to what one workgroup's LDS holds.
// perm_chunk_kernel: the interchanges in chunks of PCH; for each chunk, the moves it makes:
// position p (the chunk's own positions, and partners past the chunk) receives the row that
// stood at src before the chunk, found by tracing p back through the chunk's interchanges
// (2 PCH move slots per chunk, unused ones p = -1; a position listed twice moves the same row).
// perm_apply_kernel: one workgroup applies the chunks' moves in order to the identity, held in
// LDS: every source of a chunk is read before any of its writes.
constexpr int PCH = 256;
constexpr int kPermLdsMax = 32768;   // positions held in LDS by perm_apply_kernel (128 KB)
__global__ void __launch_bounds__(PCH) perm_chunk_kernel(const int32_t* ipiv0, int64_t strideP, int n, int2* mv0,
                                                         int64_t strideM) {
  __shared__ int sp[PCH];
  const int b = blockIdx.y, c = blockIdx.x, t = threadIdx.x;
  const int32_t* ipiv = ipiv0 + (size_t)b * strideP;
  int2* mv = mv0 + (size_t)b * strideM + (size_t)c * 2 * PCH;
  const int k0 = c * PCH, kc = min(PCH, n - k0);
  {
    const int k = k0 + t;
    const int pv = t < kc ? ipiv[k] - 1 : k;
    sp[t] = (t < kc && pv > k && pv < n) ? pv : k;   // an invalid entry becomes k <-> k
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p = h == 0 ? k0 + t : sp[t];
    const bool cand = t < kc && (h == 0 || p >= k0 + kc);
    int src = p;
    for (int i = kc - 1; i >= 0; --i) {
      const int a = k0 + i, bb = sp[i];
      src = (src == a) ? bb : ((src == bb) ? a : src);
    }
    mv[h * PCH + t] = (cand && src != p) ? make_int2(p, src) : make_int2(-1, -1);
  }
}

__global__ void __launch_bounds__(2 * PCH) perm_apply_kernel(const int2* mv0, int64_t strideM, int n, int nchunk,
                                                             int32_t* perm0, int64_t strideQ) {
  extern __shared__ int content[];
  const int b = blockIdx.y, t = threadIdx.x;
  const int2* mv = mv0 + (size_t)b * strideM;
  int32_t* perm = perm0 + (size_t)b * strideQ;
  for (int i = t; i < n; i += 2 * PCH) content[i] = i;
  int2 nxt = nchunk > 0 ? mv[t] : make_int2(-1, -1);
  for (int c = 0; c < nchunk; ++c) {
    const int2 m = nxt;
    if (c + 1 < nchunk) nxt = mv[(size_t)(c + 1) * 2 * PCH + t];   // one chunk ahead
    __syncthreads();   // the previous chunk's writes (or the identity) are in place
    const int v = m.x >= 0 ? content[m.y] : 0;
    __syncthreads();
    if (m.x >= 0) content[m.x] = v;
  }
  __syncthreads();
  for (int i = t; i < n; i += 2 * PCH) perm[i] = content[i];
}

// Y[i, c] = (T) B[src(i), c] with src = perm[i] (gather = 1) or identity; skipped when active[b] == 0
template <typename S, typename T>
__global__ void gather_kernel(const S* B0, int64_t ldb, int64_t strideB, T* Y0, int64_t ldy, int64_t strideY,
                              const int32_t* perm0, int64_t strideQ, int n, int nrhs, const int* active) {
  const int b = blockIdx.y;
  if (active && active[b] == 0) return;
  const S* B = B0 + (size_t)b * strideB;
  T* Y = Y0 + (size_t)b * strideY;
  const int32_t* perm = perm0 ? perm0 + (size_t)b * strideQ : nullptr;
  const int64_t total = (int64_t)n * nrhs;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % n), c = (int)(idx / n);
    const int src = perm ? perm[i] : i;
    Y[i + (size_t)c * ldy] = (T)B[src + (size_t)c * ldb];
  }
}

// X[dst(i), c] = W[i, c] (or += when accumulate), dst = perm[i] (scatter) or identity
template <typename T, typename S>
__global__ void scatter_kernel(const T* W0, int64_t ldw, int64_t strideW, S* X0, int64_t ldx, int64_t strideX,
                               const int32_t* perm0, int64_t strideQ, int n, int nrhs, int accumulate,
                               const int* active) {
  const int b = blockIdx.y;
  if (active && active[b] == 0) return;
  const T* W = W0 + (size_t)b * strideW;
  S* X = X0 + (size_t)b * strideX;
  const int32_t* perm = perm0 ? perm0 + (size_t)b * strideQ : nullptr;
  const int64_t total = (int64_t)n * nrhs;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % n), c = (int)(idx / n);
    const int dst = perm ? perm[i] : i;
    S* p = X + dst + (size_t)c * ldx;
    const S v = (S)W[i + (size_t)c * ldw];
    *p = accumulate ? (*p + v) : v;
  }
}

template <typename T>
struct TrsvArgs {
  const T* M; int64_t lda; int64_t strideA;
  int n, nrhs, nblk, groups;
  int trans, upper, unit;
  T* Y; int64_t ldy; int64_t strideY;
  uint64_t* slots; int64_t slot_stride;   // words per (batch, group)
  int* tickets;                            // one per (batch, group)
  int* err;
  const int* active;
  uint32_t flag;
};

// M(i, j) of the operator being solved: the stored triangle, or its transpose.
template <typename T>
__device__ __forceinline__ T mel(const TrsvArgs<T>& a, const T* M, int i, int j) {
  return a.trans ? M[j + (size_t)i * a.lda] : M[i + (size_t)j * a.lda];
}

template <typename T, int NR>
__global__ void __launch_bounds__(TNT) trsv_kernel(TrsvArgs<T> a) {
  constexpr int LLW = LLWords<T>::n;
  const int b = blockIdx.z, grp = blockIdx.y;
  if (a.active && a.active[b] == 0) return;
  const T* M = a.M + (size_t)b * a.strideA;
  T* Y = a.Y + (size_t)b * a.strideY;
  uint64_t* slots = a.slots + ((size_t)b * a.groups + grp) * a.slot_stride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c_lo = grp * NR, nr = min(NR, a.nrhs - c_lo);

  __shared__ int s_ticket;
  __shared__ T Ms[BS][BS + 1];
  __shared__ T ys[BS][NR];
  __shared__ T red[4][BS][NR];
  if (tid == 0) s_ticket = atomicAdd(a.tickets + (size_t)b * a.groups + grp, 1);
  __syncthreads();
  const int lb = s_ticket;
  if (lb >= a.nblk) return;
  const int bk = a.upper ? (a.nblk - 1 - lb) : lb;
  const int r0 = bk * BS, rb = min(BS, a.n - r0);

  // thread (i = row in block, q = quarter of the columns of a dependency block)
  const int i = tid & 63, q = tid >> 6;
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = (T)0;

  // cooperative load of the 64 x 64 block of the operator (rows r0.., cols c0..) into registers:
  // element e = tid + 256 * u, (ii, jj) chosen so that global reads are coalesced.
  T mreg[16];
  auto load_block = [&](int cb) {
    const int c0 = cb * BS, cw = min(BS, a.n - c0);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + TNT * u;
      const int fast = e & 63, slow = e >> 6;
      // non-trans: M[r0+fast, c0+slow] contiguous in fast; trans: M^T(r0+slow, c0+fast) = A[c0+fast + (r0+slow)*lda]
      int ii, jj;
      if (!a.trans) { ii = fast; jj = slow; } else { ii = slow; jj = fast; }
      mreg[u] = (ii < rb && jj < cw) ? mel(a, M, r0 + ii, c0 + jj) : (T)0;
    }
  };
  auto store_block = [&]() {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + TNT * u;
      const int fast = e & 63, slow = e >> 6;
      if (!a.trans) Ms[fast][slow] = mreg[u]; else Ms[slow][fast] = mreg[u];
    }
  };

  const int ndep = lb;   // number of dependency blocks
  auto dep_block = [&](int d) { return a.upper ? (a.nblk - 1 - d) : d; };
  if (ndep > 0) load_block(dep_block(0));
  for (int d = 0; d < ndep; ++d) {
    const int cb = dep_block(d);
    store_block();
    if (d + 1 < ndep) load_block(dep_block(d + 1));
    // solution of block cb
    const int c0 = cb * BS, cw = min(BS, a.n - c0);
    for (int idx = tid; idx < BS * NR; idx += TNT) {
      const int cc = idx % BS, r = idx / BS;
      T v = (T)0;
      if (cc < cw && r < nr) v = ll_load_val<T>(slots + ((size_t)cb * BS * NR + (size_t)r * BS + cc) * LLW, a.flag, a.err);
      ys[cc][r] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int cc = q * 16; cc < q * 16 + 16; ++cc) {
      const T mv = Ms[i][cc];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] += mv * ys[cc][r];
    }
    __syncthreads();
  }
  // reduce the four quarters, form the right-hand side
#pragma unroll
  for (int r = 0; r < NR; ++r) red[q][i][r] = acc[r];
  load_block(bk);
  store_block();
  __syncthreads();
  // diagonal block: wave w solves the right-hand sides r = w, w + 4, ...
  {
    const T dii = (lane < rb) ? Ms[lane][lane] : (T)1;
    for (int r = wave; r < nr; r += 4) {
      T rhs = (lane < rb) ? Y[r0 + lane + (size_t)(c_lo + r) * a.ldy] : (T)0;
      T val = rhs - (red[0][lane][r] + red[1][lane][r] + red[2][lane][r] + red[3][lane][r]);
      if (!a.upper) {
        for (int t = 0; t < rb; ++t) {
          T xt = __shfl(val, t);
          if (!a.unit) xt = xt / __shfl(dii, t);
          if (lane == t) val = xt;
          if (lane > t) val -= Ms[lane][t] * xt;
        }
      } else {
        for (int t = rb - 1; t >= 0; --t) {
          T xt = __shfl(val, t);
          if (!a.unit) xt = xt / __shfl(dii, t);
          if (lane == t) val = xt;
          if (lane < t) val -= Ms[lane][t] * xt;
        }
      }
      if (lane < rb) {
        ll_store_val(slots + ((size_t)bk * BS * NR + (size_t)r * BS + lane) * LLW, val, a.flag);
        Y[r0 + lane + (size_t)(c_lo + r) * a.ldy] = val;
      }
    }
  }
}

// Single right-hand side: every wave streams its quarter of each dependency
// block straight from memory (DEPTH blocks of prefetch in registers) and waits
// only for the flag+payload words of the solution values it needs, so the
// dependency loop has no workgroup barrier.
//   op N:  thread (i = lane, q = wave) accumulates M(r0+i, c0+16q..16q+15) . y
//   op T:  thread (j = lane, q = wave) accumulates M(r0+16q+t, c0+j) * y_j for
//          t < 16 and the rows are summed over the wave at the end.
// The most recent dependency is left out of that loop: its block goes to LDS
// and wave 0 alone waits for its solution, forms its product and runs the
// substitution, so no barrier separates the arrival of that solution from the
// substitution.  The diagonal block is staged, scaled and the right-hand side
// read before any waiting.
template <typename T, int DEPTH>
__global__ void __launch_bounds__(TNT) trsv1_kernel(TrsvArgs<T> a) {
  constexpr int LLW = LLWords<T>::n;
  const int b = blockIdx.z;
  if (a.active && a.active[b] == 0) return;
  const T* M = a.M + (size_t)b * a.strideA;
  T* Y = a.Y + (size_t)b * a.strideY;
  uint64_t* slots = a.slots + (size_t)b * a.groups * a.slot_stride;
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;

  __shared__ int s_ticket;
  __shared__ T Ms[BS][BS + 1];     // diagonal block; wave 0 turns its rows into the scaled strict triangle
  __shared__ T Ml[BS][BS + 1];     // block of the most recent dependency
  __shared__ T red[4][BS];
  if (tid == 0) s_ticket = atomicAdd(a.tickets + (size_t)b * a.groups, 1);
  __syncthreads();
  const int lb = s_ticket;
  if (lb >= a.nblk) return;
  const int bk = a.upper ? (a.nblk - 1 - lb) : lb;
  const int r0 = bk * BS, rb = min(BS, a.n - r0);
  const int ndep = lb;
  auto dep_block = [&](int d) { return a.upper ? (a.nblk - 1 - d) : d; };

  // the right-hand side and the diagonal block (independent of every other block)
  const T rhs = (q == 0 && lane < rb) ? Y[r0 + lane] : (T)0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + TNT * u;
    const int fast = e & 63, slow = e >> 6;
    int ii, jj;
    if (!a.trans) { ii = fast; jj = slow; } else { ii = slow; jj = fast; }
    Ms[ii][jj] = (ii < rb && jj < rb) ? mel(a, M, r0 + ii, r0 + jj) : (T)0;
  }

  T mbuf[DEPTH][16];
  auto load = [&](T* dst, int cb) {
    const int c0 = cb * BS;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (!a.trans) {
        const int col = c0 + q * 16 + t;
        dst[t] = (lane < rb && col < a.n) ? M[(r0 + lane) + (size_t)col * a.lda] : (T)0;
      } else {
        const int row = q * 16 + t, col = c0 + lane;
        dst[t] = (row < rb && col < a.n) ? M[col + (size_t)(r0 + row) * a.lda] : (T)0;
      }
    }
  };
  T acc = (T)0;
  T acct[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acct[t] = (T)0;
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
    if (s < ndep) load(mbuf[s], dep_block(s));
  __syncthreads();
  T rdi = (T)1;
  if (q == 0) {
    // Substitution form: every row scaled by the reciprocal of its diagonal entry, w_l = val_l / d_l
    // and m'_lt = m_lt / d_l on the strict triangle, zero elsewhere (and for rows past the end)
    const T dii = (lane < rb) ? Ms[lane][lane] : (T)1;
    rdi = a.unit ? (T)1 : (T)1 / dii;
#pragma unroll
    for (int t = 0; t < BS; ++t) {
      const bool strict = a.upper ? (t > lane) : (t < lane);
      Ms[lane][t] = (strict && lane < rb && t < rb) ? Ms[lane][t] * rdi : (T)0;
    }
  }

  auto wait_ptr = [&](int d, const uint64_t*& ptr, bool& valid) {
    const int cb = d < ndep ? dep_block(d) : 0, c0 = cb * BS;
    const uint64_t* yb = slots + (size_t)cb * BS * LLW;
    if (!a.trans) {
      // lanes 0..15 fetch the wave's 16 solution values; readlane broadcasts them
      ptr = yb + (size_t)(q * 16 + (lane & 15)) * LLW;
      valid = d < ndep && lane < 16 && c0 + q * 16 + lane < a.n;
    } else {
      ptr = yb + (size_t)lane * LLW;
      valid = d < ndep && c0 + lane < a.n;
    }
  };
  for (int d0 = 0; d0 < ndep; d0 += DEPTH) {
    // one combined wait for the group's blocks (the most recent dependency excluded)
    const uint64_t* ptr[DEPTH];
    bool valid[DEPTH];
    T yv[DEPTH];
#pragma unroll
    for (int s = 0; s < DEPTH; ++s) {
      wait_ptr(d0 + s, ptr[s], valid[s]);
      valid[s] = valid[s] && d0 + s < ndep - 1;
    }
    ll_wait_vals<T, DEPTH>(ptr, valid, a.flag, a.err, yv);
#pragma unroll
    for (int s = 0; s < DEPTH; ++s) {
      const int d = d0 + s;
      if (d < ndep - 1) {
        if (!a.trans) {
          T p0 = (T)0, p1 = (T)0;
#pragma unroll
          for (int t = 0; t < 16; t += 2) {
            p0 += mbuf[s][t] * lane_bcast(yv[s], t);
            p1 += mbuf[s][t + 1] * lane_bcast(yv[s], t + 1);
          }
          acc += p0 + p1;
        } else {
#pragma unroll
          for (int t = 0; t < 16; ++t) acct[t] += mbuf[s][t] * yv[s];
        }
        if (d + DEPTH < ndep) load(mbuf[s], dep_block(d + DEPTH));
      } else if (d == ndep - 1) {
        // the most recent dependency's block to LDS, in (row, column) order of the operator
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          if (!a.trans) Ml[lane][q * 16 + t] = mbuf[s][t]; else Ml[q * 16 + t][lane] = mbuf[s][t];
        }
      }
    }
  }
  if (!a.trans) {
    red[q][lane] = acc;
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const T v = wave_sum(acct[t]);
      if (lane == 0) red[0][q * 16 + t] = v;
    }
  }
  __syncthreads();
  if (q == 0) {
    T val = rhs - (a.trans ? red[0][lane] : ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])));
    if (ndep > 0) {
      const int cb = dep_block(ndep - 1), c0 = cb * BS;
      const uint64_t* p1[1] = {slots + ((size_t)cb * BS + lane) * LLW};
      const bool v1[1] = {c0 + lane < a.n};
      T y1[1];
      ll_wait_vals<T, 1>(p1, v1, a.flag, a.err, y1);
      T p[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
      for (int t = 0; t < BS; ++t) p[t & 3] += Ml[lane][t] * lane_bcast(y1[0], t);
      val -= (p[0] + p[1]) + (p[2] + p[3]);
    }
    // substitution: step t broadcasts the finished x_t = w_t, every lane does w_l -= m'_lt x_t
    T mrow[BS];
#pragma unroll
    for (int t = 0; t < BS; ++t) mrow[t] = Ms[lane][t];
    T w = (lane < rb) ? val * rdi : (T)0;
    if (!a.upper) {
#pragma unroll
      for (int t = 0; t < BS; ++t) w = fma(-mrow[t], lane_bcast(w, t), w);
    } else {
#pragma unroll
      for (int t = BS - 1; t >= 0; --t) w = fma(-mrow[t], lane_bcast(w, t), w);
    }
    if (lane < rb) {
      ll_store_val(slots + ((size_t)bk * BS + lane) * LLW, w, a.flag);
      Y[r0 + lane] = w;
    }
  }
}

// ------------------------------------------------------------------------------------
// Block-inverse substitution for one FP32 right-hand side: the refinement's correction
// solves L y = P r, U d = y with the FP32 LU factors (Sec. 2, steps of the iterative
// refinement).  With 128-row diagonal blocks D_b and the block M_{b,p} of the most
// recent dependency p (b - 1 for L, b + 1 for U), block b's part of the solution is
//     x_b = D_b^{-1} (r_b - sum_{c != p} M_{b,c} x_c) - K_b x_p,   K_b = D_b^{-1} M_{b,p}.
// D_b^{-1} and K_b are formed once per factorization (binv_prep_kernel).  Everything
// but the K_b x_p product uses blocks solved at least two steps earlier, so the chain
// from one block to the next is one wait and one 128 x 128 matrix-vector product,
// where substitution needs the product and 64-128 dependent steps.  The block solve
// through D_b^{-1} has forward error of order cond(D_b) u instead of substitution's
// componentwise backward stability; the refinement absorbs that, and getrs / potrs keep
// the substitution kernels.
// ------------------------------------------------------------------------------------
constexpr int BB = 128;

// grid (nblk, 2, batch): block bk of triangle tri (0: L, unit lower; 1: U, upper) of matrix b.
// Output: D^{-1} then K, each 128 x 128 with element (i, t) at t * 128 + i, zero outside the
// block's rows and columns (K: outside the dependency's columns; not written without one).
// D^{-1} by 16 x 16 blocks: the diagonal blocks' inverses by substitution, then block row by
// block row (from the top for L, from the bottom for U) X_IJ = -X_II sum_K D_IK X_KJ.  K = D^{-1} M
// on MFMA (16 x 16 x 4 FP32), each wave a 64 x 64 quarter.
__global__ void __launch_bounds__(256) binv_prep_kernel(const float* M0, int64_t lda, int64_t strideA, int n, int nblk,
                                                        float* out0, int64_t strideO) {
  const int bk = blockIdx.x, tri = blockIdx.y, b = blockIdx.z;
  const float* M = M0 + (size_t)b * strideA;
  float* Dinv = out0 + (size_t)b * strideO + ((size_t)tri * nblk + bk) * 2 * BB * BB;
  float* K = Dinv + BB * BB;
  __shared__ float D[BB][BB + 1];
  __shared__ float X[BB][BB + 1];
  __shared__ float S[7][16][17];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = bk * BB, rb = min(BB, n - r0);
  // the diagonal block; past the matrix's end the identity (so that the padded part inverts to it)
  for (int e = tid; e < BB * BB; e += 256) {
    const int i = e % BB, t = e / BB;
    D[i][t] = (i < rb && t < rb) ? M[(r0 + i) + (size_t)(r0 + t) * lda] : (i == t ? 1.f : 0.f);
    X[i][t] = 0.f;
  }
  __syncthreads();
  // diagonal 16 x 16 blocks: thread (I, c) solves column c of block I by substitution
  if (tid < BB) {
    const int I = tid >> 4, c = tid & 15, o = 16 * I;
    if (tri == 0) {
      for (int i = 0; i < 16; ++i) {
        float s = (i == c) ? 1.f : 0.f;
        for (int m = 0; m < i; ++m) s = fmaf(-D[o + i][o + m], X[o + m][o + c], s);
        X[o + i][o + c] = (i >= c) ? s : 0.f;
      }
    } else {
      for (int i = 15; i >= 0; --i) {
        float s = (i == c) ? 1.f : 0.f;
        for (int m = i + 1; m < 16; ++m) s = fmaf(-D[o + i][o + m], X[o + m][o + c], s);
        X[o + i][o + c] = (i <= c) ? s / D[o + i][o + i] : 0.f;
      }
    }
  }
  __syncthreads();
  // off-diagonal blocks, one block row per step
  for (int st = 1; st < 8; ++st) {
    const int I = tri == 0 ? st : 7 - st;
    // S_J = sum over K between J and I (exclusive of I) of D_IK X_KJ, for the st blocks J on I's far side
    for (int e = tid; e < st * 256; e += 256) {
      const int jj = e >> 8, r = (e >> 4) & 15, c = e & 15;
      const int J = tri == 0 ? jj : I + 1 + jj;
      const int k0 = tri == 0 ? J : I + 1, k1 = tri == 0 ? I : J + 1;   // K in [k0, k1)
      float acc = 0.f;
      for (int Kb = k0; Kb < k1; ++Kb)
#pragma unroll
        for (int m = 0; m < 16; ++m) acc = fmaf(D[16 * I + r][16 * Kb + m], X[16 * Kb + m][16 * J + c], acc);
      S[jj][r][c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < st * 256; e += 256) {
      const int jj = e >> 8, r = (e >> 4) & 15, c = e & 15;
      const int J = tri == 0 ? jj : I + 1 + jj;
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < 16; ++m) acc = fmaf(X[16 * I + r][16 * I + m], S[jj][m][c], acc);
      X[16 * I + r][16 * J + c] = -acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < BB * BB; e += 256) {
    const int i = e % BB, t = e / BB;
    Dinv[e] = (i < rb && t < rb) ? X[i][t] : 0.f;
  }
  const int dep = tri == 0 ? bk - 1 : bk + 1;
  if (dep < 0 || dep >= nblk) return;   // uniform over the workgroup
  const int c0 = dep * BB, cw = min(BB, n - c0);
  __syncthreads();   // D is free (the inverse is complete)
  for (int e = tid; e < BB * BB; e += 256) {
    const int u = e % BB, t = e / BB;
    D[u][t] = (u < rb && t < cw) ? M[(r0 + u) + (size_t)(c0 + t) * lda] : 0.f;
  }
  for (int e = tid; e < BB * BB; e += 256) {   // rows and columns of X past the block's end count as zero
    const int i = e % BB, t = e / BB;
    if (i >= rb || t >= rb) X[i][t] = 0.f;
  }
  __syncthreads();
  // K = X D on MFMA: wave w takes rows 64 (w & 1) .., columns 64 (w >> 1) .., as 4 x 4 blocks of 16 x 16
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;
  f4 acc[4][4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = (f4){0.f, 0.f, 0.f, 0.f};
  for (int u0 = 0; u0 < BB; u0 += 4) {
    float af[4], bf[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) af[mi] = X[wr + mi * 16 + (lane & 15)][u0 + (lane >> 4)];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) bf[ni] = D[u0 + (lane >> 4)][wc + ni * 16 + (lane & 15)];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
  }
  // accumulator v of block (mi, ni): row wr + 16 mi + 4 (lane / 16) + v, column wc + 16 ni + (lane & 15)
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wr + mi * 16 + 4 * (lane >> 4) + v, t = wc + ni * 16 + (lane & 15);
        K[(size_t)t * BB + i] = acc[mi][ni][v];
      }
}

struct BinvArgs {
  const float* M; int64_t lda; int64_t strideA;
  const float* P; int64_t strideP;          // binv_prep_kernel's output per matrix
  float* Y; int64_t strideY;                // right-hand side in, solution out (n per matrix)
  uint64_t* slots; int64_t slot_stride;     // flag+payload word per row
  int* tickets;                             // one per matrix
  int* err;
  const int* active;
  int n, nblk, upper;
  uint32_t flag;
};

// Persistent, ticket-ordered like trsv1_kernel.  Wave q covers rows 64 (q & 1) + lane of the
// block and columns 64 (q >> 1) .. + 63 of every 128 x 128 block it multiplies; the two column
// halves meet in LDS.  D_b^{-1} and K_b are staged in LDS before any waiting.
template <int DEPTH>
__global__ void __launch_bounds__(TNT, 1) trsv1_binv_kernel(BinvArgs a) {
  const int b = blockIdx.z;
  if (a.active && a.active[b] == 0) return;
  const float* M = a.M + (size_t)b * a.strideA;
  float* Y = a.Y + (size_t)b * a.strideY;
  uint64_t* slots = a.slots + (size_t)b * a.slot_stride;
  const int tid = threadIdx.x, lane = tid & 63;
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, kept in a scalar register
  const int ch = q >> 1;                  // column half
  const int row = (q & 1) * 64 + lane;    // row of the block
  __shared__ int s_ticket;
  __shared__ float sD[BB][BB];            // D^{-1}: element (i, t) at [t][i]
  __shared__ float sv[BB];
  __shared__ float red[2][BB];
  __shared__ float red2[2][BB];
  __shared__ __attribute__((aligned(16))) float sy[4][64];
  if (tid == 0) s_ticket = atomicAdd(a.tickets + b, 1);
  __syncthreads();
  const int lb = s_ticket;
  if (lb >= a.nblk) return;
  const int bk = a.upper ? (a.nblk - 1 - lb) : lb;
  const int r0 = bk * BB, rb = min(BB, a.n - r0);
  const bool rok = row < rb;
  const int ndep = lb;
  auto dep_block = [&](int d) { return a.upper ? (a.nblk - 1 - d) : d; };
  const float* Pb = a.P + (size_t)b * a.strideP + ((size_t)a.upper * a.nblk + bk) * 2 * BB * BB;

  // independent of every other block: D^{-1} and K to LDS, the right-hand side
  for (int e = tid; e < BB * BB; e += TNT) (&sD[0][0])[e] = Pb[e];
  const float rhs = (ch == 0 && rok) ? Y[r0 + row] : 0.f;

  float mbuf[DEPTH][64];
  // A wave-uniform base per block of columns and a 32-bit element offset per lane, advanced by
  // lda per column (64 lda + 128 stays far below 2^32).  The offset is made opaque after every
  // step so that the 64 offsets are formed one at a time instead of being kept live across the
  // loop.  Rows past the end read the block's last row (their results are discarded); columns
  // past the end are read only in the last, partial block of columns, under a mask.
  const unsigned ldu = (unsigned)a.lda;
  const unsigned rowc = (unsigned)(rok ? row : rb - 1);
  auto load = [&](float* dst, int cb) {
    const int c0 = cb * BB + ch * 64;
    const float* base = M + r0 + (size_t)c0 * a.lda;
    unsigned off = rowc;
    if (c0 + 64 <= a.n) {
#pragma unroll
      for (int t = 0; t < 64; ++t) {
        dst[t] = base[off];
        off += ldu;
        asm volatile("" : "+v"(off));
      }
    } else {
#pragma unroll
      for (int t = 0; t < 64; ++t) {
        dst[t] = c0 + t < a.n ? base[off] : 0.f;
        off += ldu;
        asm volatile("" : "+v"(off));
      }
    }
  };
  const int nstream = ndep > 0 ? ndep - 1 : 0;   // dependencies before the most recent one
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
    if (s < nstream) load(mbuf[s], dep_block(s));
  float acc0 = 0.f, acc1 = 0.f;
  for (int d0 = 0; d0 < nstream; d0 += DEPTH) {
#pragma unroll
    for (int s = 0; s < DEPTH; ++s) {
      const int d = d0 + s;
      if (d < nstream) {
        const int idx = dep_block(d) * BB + ch * 64 + lane;
        const uint64_t* p[1] = {slots + idx};
        const bool v[1] = {idx < a.n};
        float y[1];
        ll_wait_vals<float, 1>(p, v, a.flag, a.err, y);
#pragma unroll
        for (int t = 0; t < 64; t += 2) {
          acc0 = fmaf(mbuf[s][t], lane_bcast(y[0], t), acc0);
          acc1 = fmaf(mbuf[s][t + 1], lane_bcast(y[0], t + 1), acc1);
        }
        if (d + DEPTH < nstream) load(mbuf[s], dep_block(d + DEPTH));
      }
    }
  }
  // this thread's 64 entries of K (row `row`, the wave's half of the columns; element (i, t) at
  // t BB + i), held in registers for the chain step, loaded while D^{-1} v is formed
  float kreg[64];
  if (ndep > 0) {
    const float* Kp = Pb + BB * BB + (size_t)(ch * 64) * BB + row;
#pragma unroll
    for (int t = 0; t < 64; ++t) kreg[t] = Kp[(size_t)t * BB];
  }
  // v = r - (products so far), then c = D^{-1} v
  red[ch][row] = acc0 + acc1;
  __syncthreads();
  if (ch == 0) sv[row] = rok ? rhs - (red[0][row] + red[1][row]) : 0.f;
  __syncthreads();
  float c0p = 0.f, c1p = 0.f;
#pragma unroll 8
  for (int t = 0; t < 64; t += 2) {
    c0p = fmaf(sD[ch * 64 + t][row], sv[ch * 64 + t], c0p);
    c1p = fmaf(sD[ch * 64 + t + 1][row], sv[ch * 64 + t + 1], c1p);
  }
  red[ch][row] = c0p + c1p;   // the reads of red above finished before the last barrier
  __syncthreads();
  float x = red[0][row] + red[1][row];
  if (ndep > 0) {
    // the chain step: x -= K x_p as soon as x_p is published
    const int idx = dep_block(ndep - 1) * BB + ch * 64 + lane;
    const uint64_t* p[1] = {slots + idx};
    const bool v[1] = {idx < a.n};
    float y[1];
    ll_wait_vals<float, 1>(p, v, a.flag, a.err, y);
    // x_p's 64 values of this wave go through LDS and come back as 16-byte broadcast reads (every
    // lane reads the same address), in place of 64 cross-lane reads
    sy[q][lane] = y[0];
    wave_fence();
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
    for (int t = 0; t < 64; t += 4) {
      const f4 yv = *reinterpret_cast<const f4*>(&sy[q][t]);
      p0 = fmaf(kreg[t], yv[0], p0);
      p1 = fmaf(kreg[t + 1], yv[1], p1);
      p2 = fmaf(kreg[t + 2], yv[2], p2);
      p3 = fmaf(kreg[t + 3], yv[3], p3);
    }
    red2[ch][row] = (p0 + p1) + (p2 + p3);
    __syncthreads();
    x -= red2[0][row] + red2[1][row];
  }
  if (ch == 0 && rok) {
    ll_store_val(slots + (r0 + row), x, a.flag);
    Y[r0 + row] = x;
  }
}

template <typename T, int NR>
hipError_t launch_trsv_nr(const TrsvArgs<T>& a, int batch, hipStream_t s) {
  dim3 grid(a.nblk, a.groups, batch);
  hipLaunchKernelGGL((trsv_kernel<T, NR>), grid, dim3(TNT), 0, s, a);
  return hipGetLastError();
}

int pick_nr(int nrhs) { return nrhs <= 1 ? 1 : (nrhs <= 8 ? 8 : 32); }

}  // namespace

size_t trsv_slot_bytes(int n, int nrhs, int batch, size_t elem) {
  const int nr = pick_nr(nrhs);
  const int groups = (nrhs + nr - 1) / nr;
  const int nblk = (n + BS - 1) / BS;
  const int llw = elem == 8 ? 2 : 1;
  // one right-hand side may also take the block-inverse kernel (128-row blocks)
  const size_t rows = nr == 1 ? std::max<size_t>((size_t)nblk * BS, (size_t)((n + BB - 1) / BB) * BB)
                              : (size_t)nblk * BS;
  return (size_t)batch * groups * rows * nr * llw * 8;
}

size_t binv_elems(int n) { return (size_t)2 * ((n + BB - 1) / BB) * 2 * BB * BB; }

hipError_t launch_binv_prep(const float* LU, int64_t lda, int64_t strideA, int n, float* out, int64_t strideO,
                            int batch, hipStream_t s) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  const int nblk = (n + BB - 1) / BB;
  hipLaunchKernelGGL(binv_prep_kernel, dim3(nblk, 2, batch), dim3(256), 0, s, LU, lda, strideA, n, nblk, out, strideO);
  return hipGetLastError();
}

size_t getrs_ws_bytes(int n, int nrhs, int batch, size_t elem) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t perm = al((size_t)batch * n * 4);
  size_t gmap = al((size_t)batch * perm_moves_ints(n) * 4);
  size_t temp = al((size_t)batch * n * std::max(nrhs, 1) * elem);
  size_t slots = al(trsv_slot_bytes(n, nrhs, batch, elem));
  size_t tick = al((size_t)batch * 64 * 4);
  return kErrRegion + perm + gmap + temp + slots + tick;
}

size_t perm_moves_ints(int n) { return (size_t)((std::max(n, 1) + PCH - 1) / PCH) * 2 * PCH * 2; }

hipError_t launch_perm(const int32_t* ipiv, int64_t strideP, int n, int32_t* perm, int64_t strideQ, int32_t* gmap,
                       int batch, hipStream_t s) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (gmap != nullptr && n <= kPermLdsMax) {
    // chunked: gmap holds perm_moves_ints(n) ints per matrix
    const int nchunk = (n + PCH - 1) / PCH;
    const int64_t strideM = (int64_t)perm_moves_ints(n) / 2;
    int2* mv = reinterpret_cast<int2*>(gmap);
    hipLaunchKernelGGL(perm_chunk_kernel, dim3(nchunk, batch), dim3(PCH), 0, s, ipiv, strideP, n, mv, strideM);
    hipLaunchKernelGGL(perm_apply_kernel, dim3(1, batch), dim3(2 * PCH), (size_t)n * 4, s, (const int2*)mv, strideM,
                       n, nchunk, perm, strideQ);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(perm_kernel, dim3((n + 255) / 256, batch), dim3(256), 0, s, ipiv, strideP, n, perm, strideQ);
  return hipGetLastError();
}

template <typename T, typename S>
cds_status_t getrs_core(Ctx& c, const GetrsCore<T, S>& g) {
  const int n = g.n, nrhs = g.nrhs, batch = g.batch;
  if (n == 0 || nrhs == 0 || batch == 0) return CDS_SUCCESS;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* base = (char*)g.ws + kErrRegion;
  int32_t* perm = (int32_t*)base;
  base += al((size_t)batch * n * 4);
  int32_t* gmap = (int32_t*)base;
  base += al((size_t)batch * perm_moves_ints(n) * 4);
  T* temp = (T*)base;
  base += al((size_t)batch * n * nrhs * sizeof(T));
  uint64_t* slots = (uint64_t*)base;
  const size_t slot_b = trsv_slot_bytes(n, nrhs, batch, sizeof(T));
  base += al(slot_b);
  int* tickets = (int*)base;
  base += al((size_t)batch * 64 * 4);
  if ((size_t)(base - (char*)g.ws) > g.ws_bytes) return CDS_WORKSPACE_TOO_SMALL;
  hipStream_t s = c.s0;

  const int32_t* P = g.perm;
  int64_t strideQ = g.strideQ;
  if (g.ipiv && !P) {
    if (launch_perm(g.ipiv, g.strideP, n, perm, n, gmap, batch, s) != hipSuccess) return CDS_HIP_ERROR;
    P = perm;
    strideQ = n;
  }
  const int64_t strideT = (int64_t)n * nrhs;
  const int gblocks = (int)std::min<int64_t>(2048, ((int64_t)n * nrhs + 255) / 256);
  // right-hand side into the working buffer (permuted for op N)
  hipLaunchKernelGGL((gather_kernel<S, T>), dim3(gblocks, batch), dim3(256), 0, s, g.B, g.ldb, g.strideB, temp,
                     (int64_t)n, strideT, g.trans ? (const int32_t*)nullptr : P, strideQ, n, nrhs, g.active);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;

  const int nr = pick_nr(nrhs);
  const int groups = (nrhs + nr - 1) / nr;
  const int nblk = (n + BS - 1) / BS;
  const int64_t slot_stride = (int64_t)nblk * BS * nr * LLWords<T>::n;
  for (int pass = 0; pass < 2; ++pass) {
    TrsvArgs<T> a;
    a.M = g.M; a.lda = g.lda; a.strideA = g.strideA;
    a.n = n; a.nrhs = nrhs; a.nblk = nblk; a.groups = groups;
    a.Y = temp; a.ldy = n; a.strideY = strideT;
    a.slots = slots; a.slot_stride = slot_stride;
    a.tickets = tickets;
    a.err = c.err;
    a.active = g.active;
    a.flag = (uint32_t)(pass + 1);
    if (!g.chol) {
      if (!g.trans) {           // L y = Pb (unit), U x = y
        a.trans = 0; a.upper = pass; a.unit = pass == 0;
      } else {                  // U^T z = b, L^T w = z (unit)
        a.trans = 1; a.upper = pass; a.unit = pass == 1;
      }
    } else {                    // L y = b, L^T x = y
      a.trans = pass; a.upper = pass; a.unit = 0;
    }
    // clear flags and tickets (fill kernels, no memset nodes)
    if (launch_fill_zero(slots, slot_b, s) != hipSuccess) return CDS_HIP_ERROR;
    if (launch_fill_i32(tickets, (int64_t)batch * groups, 0, s) != hipSuccess) return CDS_HIP_ERROR;
    hipError_t e;
    KScope ks(c.timer, CDS_KC_TRSV, s, (double)batch * n * (double)n * nrhs,
              (double)batch * sizeof(T) * ((double)n * n / 2.0 * groups + 2.0 * n * nrhs));
    bool done = false;
    if constexpr (std::is_same<T, float>::value) {
      if (g.binv != nullptr && !g.trans && !g.chol && nrhs == 1) {
        BinvArgs bv;
        bv.M = g.M; bv.lda = g.lda; bv.strideA = g.strideA;
        bv.P = g.binv; bv.strideP = (int64_t)binv_elems(n);
        bv.Y = temp; bv.strideY = strideT;
        bv.n = n; bv.nblk = (n + BB - 1) / BB; bv.upper = pass;
        bv.slots = slots; bv.slot_stride = (int64_t)bv.nblk * BB;
        bv.tickets = tickets; bv.err = c.err; bv.active = g.active; bv.flag = a.flag;
        hipLaunchKernelGGL(trsv1_binv_kernel<2>, dim3(bv.nblk, 1, batch), dim3(TNT), 0, s, bv);
        e = hipGetLastError();
        done = true;
      }
    }
    if (done) {
    } else if (nr == 1) {
      hipLaunchKernelGGL((trsv1_kernel<T, 4>), dim3(a.nblk, 1, batch), dim3(TNT), 0, s, a);
      e = hipGetLastError();
    }
    else if (nr == 8) e = launch_trsv_nr<T, 8>(a, batch, s);
    else e = launch_trsv_nr<T, 32>(a, batch, s);
    if (e != hipSuccess) return CDS_HIP_ERROR;
  }
  hipLaunchKernelGGL((scatter_kernel<T, S>), dim3(gblocks, batch), dim3(256), 0, s, temp, (int64_t)n, strideT, g.X,
                     g.ldx, g.strideX, g.trans ? P : (const int32_t*)nullptr, strideQ, n, nrhs, g.accumulate,
                     g.active);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

template cds_status_t getrs_core<double, double>(Ctx&, const GetrsCore<double, double>&);
template cds_status_t getrs_core<float, float>(Ctx&, const GetrsCore<float, float>&);
template cds_status_t getrs_core<float, double>(Ctx&, const GetrsCore<float, double>&);

template <typename T>
cds_status_t getrs_run(Ctx& c, int trans, int n, int nrhs, const T* LU, int64_t lda, int64_t strideA,
                       const int32_t* ipiv, int64_t strideP, T* B, int64_t ldb, int64_t strideB, int batch,
                       void* ws, size_t ws_bytes) {
  GetrsCore<T, T> g{};
  g.trans = trans; g.chol = 0; g.n = n; g.nrhs = nrhs; g.batch = batch;
  g.M = LU; g.lda = lda; g.strideA = strideA;
  g.ipiv = ipiv; g.strideP = strideP; g.perm = nullptr; g.strideQ = 0;
  g.B = B; g.ldb = ldb; g.strideB = strideB;
  g.X = B; g.ldx = ldb; g.strideX = strideB; g.accumulate = 0;
  g.active = nullptr; g.ws = ws; g.ws_bytes = ws_bytes;
  return getrs_core<T, T>(c, g);
}
template cds_status_t getrs_run<double>(Ctx&, int, int, int, const double*, int64_t, int64_t, const int32_t*,
                                        int64_t, double*, int64_t, int64_t, int, void*, size_t);
template cds_status_t getrs_run<float>(Ctx&, int, int, int, const float*, int64_t, int64_t, const int32_t*,
                                       int64_t, float*, int64_t, int64_t, int, void*, size_t);

template <typename T>
cds_status_t potrs_run(Ctx& c, int n, int nrhs, const T* L, int64_t lda, T* B, int64_t ldb, void* ws,
                       size_t ws_bytes) {
  GetrsCore<T, T> g{};
  g.trans = 0; g.chol = 1; g.n = n; g.nrhs = nrhs; g.batch = 1;
  g.M = L; g.lda = lda; g.strideA = 0;
  g.ipiv = nullptr; g.perm = nullptr;
  g.B = B; g.ldb = ldb; g.strideB = 0;
  g.X = B; g.ldx = ldb; g.strideX = 0; g.accumulate = 0;
  g.active = nullptr; g.ws = ws; g.ws_bytes = ws_bytes;
  return getrs_core<T, T>(c, g);
}
template cds_status_t potrs_run<double>(Ctx&, int, int, const double*, int64_t, double*, int64_t, void*, size_t);
template cds_status_t potrs_run<float>(Ctx&, int, int, const float*, int64_t, float*, int64_t, void*, size_t);

}  // namespace cds
