// Krylov solvers of the paper's iterative family (Sec. 2): conjugate gradient
// for SPD A, BiCG (residuals with A, shadow residuals with A^T), BiCGSTAB, and
// GMRES restarted after a fixed number of Arnoldi steps; and GMRES-based
// refinement (FP64 GMRES on the correction equation, left-preconditioned by
// low-precision LU factors).  All arithmetic in FP64 on the device.
//
// The time goes into the products with the dense n x n matrix, which read A
// once each (8 n^2 bytes): they are HBM-bound, so they are written for
// coalescing, not for MFMA.  A product is split over column chunks into
// partial sums (one coalesced column sweep per thread pair of rows), then the
// chunks are added in a fixed order; every dot product is a two-level sum in
// a fixed order (block partials, then every consumer adds the partials the
// same way), so a solve is bitwise reproducible.  Scalars (alpha, beta, ...)
// live in device memory and are formed by the kernels that use them; the host
// only enqueues and, every check_every iterations, reads one state word.
#include "common.hpp"
#include "kernels.hpp"
#include "krylov.hpp"
#include "solve.hpp"
#include <algorithm>
#include <cmath>
#include <vector>

namespace cds {

namespace {

constexpr int KNT = 256;          // threads per block
constexpr int KRB = 512;          // rows per product block (two per thread)
constexpr int KCW = 256;          // columns per product chunk
constexpr int KMAXP = 256;        // at most this many block partials per dot product

struct KState {
  int done;          // 1 converged, 2 iteration budget spent, 3 breakdown
  int iters;
  int cycle_k;       // GMRES: Arnoldi steps taken in the current cycle
  int pad;
  double bnorm;      // ||b||_2 (of the preconditioned right-hand side for GMRES)
  double relres;
  double rho[2];     // CG: r.r; BiCG / BiCGSTAB: rho, double-buffered by iteration parity
  double alpha, omega;
  double hn_inv;     // GMRES: 1 / ||w|| of the newest Arnoldi vector
  double beta0;      // GMRES: ||r|| at the cycle start
};

// blocks of the vector kernels (and so the count of each dot product's partials): one row per thread
int nparts(int n) { return std::max(1, std::min(KMAXP, (n + KNT - 1) / KNT)); }
int nchunks(int n) { return std::max(1, (n + KCW - 1) / KCW); }

// sum of `np` partials in a fixed order, the same in every block (wave 0 only)
__device__ __forceinline__ double sum_parts(const double* part, int np) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < np; i += 64) s += part[i];
  return wave_sum(s);
}

// block sum of v (fixed order), valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < KNT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------ products with A
// part[c * n + i] = sum over column chunk c of A(i, j) x(j) (scale * x if xs is given)
__global__ void __launch_bounds__(KNT) gemv_n_part(const double* __restrict__ A, int64_t lda, int n,
                                                   const double* __restrict__ x, const double* xs_inv,
                                                   double* __restrict__ part, const KState* st) {
  if (st && st->done) return;
  const int r0 = blockIdx.x * KRB + threadIdx.x;
  const int r1 = r0 + KNT;
  const int c = blockIdx.y;
  const int j0 = c * KCW, j1 = min(n, j0 + KCW);
  const double sc = xs_inv ? *xs_inv : 1.0;
  const bool ok0 = r0 < n, ok1 = r1 < n;
  const double* a0 = A + (size_t)min(r0, n - 1);
  const double* a1 = A + (size_t)min(r1, n - 1);
  double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    double u0[8], u1[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      u0[q] = a0[(size_t)(j + q) * lda];
      u1[q] = a1[(size_t)(j + q) * lda];
      xv[q] = x[j + q];
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      s0 = fma(u0[q], xv[q], s0);
      t0 = fma(u0[q + 1], xv[q + 1], t0);
      s1 = fma(u1[q], xv[q], s1);
      t1 = fma(u1[q + 1], xv[q + 1], t1);
    }
  }
  for (; j < j1; ++j) {
    s0 = fma(a0[(size_t)j * lda], x[j], s0);
    s1 = fma(a1[(size_t)j * lda], x[j], s1);
  }
  if (ok0) part[(size_t)c * n + r0] = (s0 + t0) * sc;
  if (ok1) part[(size_t)c * n + r1] = (s1 + t1) * sc;
}

// part[j * ... ]: y(j) = sum_i A(i, j) x(i), one wave per column, lanes down the rows
__global__ void __launch_bounds__(KNT) gemv_t_kernel(const double* __restrict__ A, int64_t lda, int n,
                                                     const double* __restrict__ x, double* __restrict__ y,
                                                     const KState* st) {
  if (st && st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * (KNT / 64) + wave;
  if (col >= n) return;
  const double* a = A + (size_t)col * lda;
  double s0 = 0.0, s1 = 0.0;
  int i = lane;
  for (; i + 7 * 64 < n; i += 8 * 64) {
    double u[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      u[q] = a[i + q * 64];
      xv[q] = x[i + q * 64];
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      s0 = fma(u[q], xv[q], s0);
      s1 = fma(u[q + 1], xv[q + 1], s1);
    }
  }
  for (; i < n; i += 64) s0 = fma(a[i], x[i], s0);
  const double s = wave_sum(s0 + s1);
  if (lane == 0) y[col] = s;
}

// y = s_sum * sum_c part[c] + s_z * z; optional dot partials dp[blk] = sum y_i w_i
__global__ void __launch_bounds__(KNT) reduce_rows(const double* __restrict__ part, int nc, int n, double s_sum,
                                                   const double* z, double s_z, double* __restrict__ y,
                                                   const double* w, double* dp, const KState* st) {
  __shared__ double red[KNT / 64];
  if (st && st->done) return;
  double d = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += part[(size_t)c * n + i];
    double v = s_sum * s;
    if (z) v = fma(s_z, z[i], v);
    y[i] = v;
    if (w) d = fma(v, w[i], d);
  }
  if (dp) {
    const double b = block_sum(d, red);
    if (threadIdx.x == 0) dp[blockIdx.x] = b;
  }
}

// dp[blk] = sum x_i y_i over the block's grid-stride rows
__global__ void __launch_bounds__(KNT) dot_part(int n, const double* x, const double* y, double* dp,
                                                const KState* st) {
  __shared__ double red[KNT / 64];
  if (st && st->done) return;
  double d = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) d = fma(x[i], y[i], d);
  const double b = block_sum(d, red);
  if (threadIdx.x == 0) dp[blockIdx.x] = b;
}

// ------------------------------------------------------------------ CG
// alpha = rho / (p.q); x += alpha p; r -= alpha q; dp = partials of r.r
__global__ void __launch_bounds__(KNT) cg_step(int n, const double* pq, int np, KState* st, double* x, double* r,
                                               const double* p, const double* q, double* dp, int par) {
  __shared__ double red[KNT / 64];
  __shared__ double s_alpha;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double den = sum_parts(pq, np);
    if (threadIdx.x == 0) s_alpha = st->rho[par] / den;
  }
  __syncthreads();
  const double alpha = s_alpha;
  double d = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    d = fma(ri, ri, d);
  }
  const double b = block_sum(d, red);
  if (threadIdx.x == 0) dp[blockIdx.x] = b;
}

// rho' = r.r; test; beta = rho' / rho; p = r + beta p
__global__ void __launch_bounds__(KNT) cg_dir(int n, const double* rr, int np, KState* st, const double* r, double* p,
                                              int par, double tol, int max_iter) {
  __shared__ double s_rho;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(rr, np);
    if (threadIdx.x == 0) s_rho = v;
  }
  __syncthreads();
  const double rho1 = s_rho;
  const double rho0 = st->rho[par];
  const double beta = rho1 / rho0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) p[i] = fma(beta, p[i], r[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rho[par ^ 1] = rho1;
    st->iters += 1;
    st->relres = sqrt(rho1) / st->bnorm;
  }
}

// after the last block of cg_dir: the stopping test (a separate launch so that every block of cg_dir
// read the state before it changes)
__global__ void krylov_test(KState* st, double tol, int max_iter) {
  if (st->done) return;
  if (!(st->relres > tol)) st->done = 1;   // also stops on NaN
  else if (st->iters >= max_iter) st->done = 2;
}

__global__ void krylov_init(KState* st, const double* bb, int np, const double* rr, int np2) {
  // bb: partials of b.b; rr: partials of r0.r0
  if (threadIdx.x < 64) {
    const double b2 = sum_parts(bb, np);
    const double r2 = sum_parts(rr, np2);
    if (threadIdx.x == 0) {
      st->done = 0;
      st->iters = 0;
      st->cycle_k = 0;
      st->bnorm = b2 > 0.0 ? sqrt(b2) : 1.0;
      st->relres = sqrt(r2) / st->bnorm;
      st->rho[0] = r2;
      st->rho[1] = 0.0;
      st->alpha = st->omega = 0.0;
      st->hn_inv = 0.0;
      st->beta0 = sqrt(r2);
    }
  }
}

// ------------------------------------------------------------------ BiCG
// alpha = rho / (pt.q); x += alpha p; r -= alpha q; rt -= alpha qt; partials of rt.r and r.r
__global__ void __launch_bounds__(KNT) bicg_step(int n, const double* ptq, int np, KState* st, double* x, double* r,
                                                 double* rt, const double* p, const double* q, const double* qt,
                                                 double* dp_rho, double* dp_rr, int par) {
  __shared__ double red[KNT / 64];
  __shared__ double s_alpha;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double den = sum_parts(ptq, np);
    if (threadIdx.x == 0) s_alpha = st->rho[par] / den;
  }
  __syncthreads();
  const double alpha = s_alpha;
  double d1 = 0.0, d2 = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    const double rti = fma(-alpha, qt[i], rt[i]);
    r[i] = ri;
    rt[i] = rti;
    d1 = fma(rti, ri, d1);
    d2 = fma(ri, ri, d2);
  }
  const double b1 = block_sum(d1, red);
  const double b2 = block_sum(d2, red);
  if (threadIdx.x == 0) {
    dp_rho[blockIdx.x] = b1;
    dp_rr[blockIdx.x] = b2;
  }
}

__global__ void __launch_bounds__(KNT) bicg_dir(int n, const double* rho_p, const double* rr_p, int np, KState* st,
                                                const double* r, const double* rt, double* p, double* pt, int par) {
  __shared__ double s_rho, s_rr;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(rho_p, np);
    const double w = sum_parts(rr_p, np);
    if (threadIdx.x == 0) { s_rho = v; s_rr = w; }
  }
  __syncthreads();
  const double beta = s_rho / st->rho[par];
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    p[i] = fma(beta, p[i], r[i]);
    pt[i] = fma(beta, pt[i], rt[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rho[par ^ 1] = s_rho;
    st->iters += 1;
    st->relres = sqrt(s_rr) / st->bnorm;
    if (s_rho == 0.0 && s_rr != 0.0) st->done = 3;
  }
}

// ------------------------------------------------------------------ BiCGSTAB
// first half: rho' = rh.r (partials given); p = r (first iteration) or r + beta (p - omega v)
__global__ void __launch_bounds__(KNT) bcs_dir(int n, const double* rho_p, int np, KState* st, const double* r,
                                               double* p, const double* v, int par, int first) {
  __shared__ double s_rho;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double x = sum_parts(rho_p, np);
    if (threadIdx.x == 0) s_rho = x;
  }
  __syncthreads();
  const double rho1 = s_rho;
  if (first) {
    for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) p[i] = r[i];
  } else {
    const double beta = (rho1 / st->rho[par]) * (st->alpha / st->omega);
    const double om = st->omega;
    for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT)
      p[i] = fma(beta, fma(-om, v[i], p[i]), r[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->rho[par ^ 1] = rho1;
}

// alpha = rho' / (rh.v); s = r - alpha v; partials of s.s
__global__ void __launch_bounds__(KNT) bcs_half(int n, const double* rhv, int np, KState* st, const double* r,
                                                const double* v, double* s, double* dp_ss, int par) {
  __shared__ double red[KNT / 64];
  __shared__ double s_alpha;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double den = sum_parts(rhv, np);
    if (threadIdx.x == 0) s_alpha = st->rho[par ^ 1] / den;
  }
  __syncthreads();
  const double alpha = s_alpha;
  double d = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    const double si = fma(-alpha, v[i], r[i]);
    s[i] = si;
    d = fma(si, si, d);
  }
  const double b = block_sum(d, red);
  if (threadIdx.x == 0) dp_ss[blockIdx.x] = b;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->alpha = alpha;
}

// early exit on ||s||: x += alpha p, r = s, done (a separate launch reads the finished partials)
__global__ void __launch_bounds__(KNT) bcs_half_test(int n, const double* ss, int np, KState* st, double* x,
                                                     const double* p, double* r, const double* s, double tol,
                                                     double* flag) {
  __shared__ double s_rel;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(ss, np);
    if (threadIdx.x == 0) s_rel = sqrt(v) / st->bnorm;
  }
  __syncthreads();
  const bool stop = !(s_rel > tol);
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = stop ? 1.0 : 0.0;
  if (!stop) return;
  const double alpha = st->alpha;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = s[i];
  }
}

// the state after an early exit (a separate launch so that every block of bcs_half_test saw done == 0)
__global__ void bcs_half_done(KState* st, const double* flag, const double* ss, int np) {
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(ss, np);
    if (threadIdx.x == 0 && *flag != 0.0) {
      st->iters += 1;
      st->relres = sqrt(v) / st->bnorm;
      st->done = 1;
    }
  }
}

// omega = (t.s) / (t.t); x += alpha p + omega s; r = s - omega t; partials of r.r and rh.r
__global__ void __launch_bounds__(KNT) bcs_full(int n, const double* ts, const double* tt, int np, KState* st,
                                                double* x, double* r, const double* p, const double* s,
                                                const double* t, const double* rh, double* dp_rr, double* dp_rho) {
  __shared__ double red[KNT / 64];
  __shared__ double s_om;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double a = sum_parts(ts, np);
    const double b = sum_parts(tt, np);
    if (threadIdx.x == 0) s_om = a / b;
  }
  __syncthreads();
  const double om = s_om, alpha = st->alpha;
  double d1 = 0.0, d2 = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    x[i] = fma(om, s[i], fma(alpha, p[i], x[i]));
    const double ri = fma(-om, t[i], s[i]);
    r[i] = ri;
    d1 = fma(ri, ri, d1);
    d2 = fma(rh[i], ri, d2);
  }
  const double b1 = block_sum(d1, red);
  const double b2 = block_sum(d2, red);
  if (threadIdx.x == 0) {
    dp_rr[blockIdx.x] = b1;
    dp_rho[blockIdx.x] = b2;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->omega = om;
}

__global__ void bcs_account(KState* st, const double* rr, int np) {
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(rr, np);
    if (threadIdx.x == 0) {
      st->iters += 1;
      st->relres = sqrt(v) / st->bnorm;
      if (st->omega == 0.0 && v != 0.0) st->done = 3;
    }
  }
}

// partials of t.s and t.t in one pass
__global__ void __launch_bounds__(KNT) dot2_part(int n, const double* t, const double* s, double* dp_ts,
                                                 double* dp_tt, const KState* st) {
  __shared__ double red[KNT / 64];
  if (st && st->done) return;
  double a = 0.0, b = 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    a = fma(t[i], s[i], a);
    b = fma(t[i], t[i], b);
  }
  const double ba = block_sum(a, red);
  const double bb = block_sum(b, red);
  if (threadIdx.x == 0) {
    dp_ts[blockIdx.x] = ba;
    dp_tt[blockIdx.x] = bb;
  }
}

// ------------------------------------------------------------------ GMRES
// hp[blk * (k1) + c] = sum over the block's rows of V(i, c) w(i), c < k1 (V n x k1, ld ldv)
__global__ void __launch_bounds__(KNT) gs_dots(int n, const double* V, int64_t ldv, int k1, const double* w,
                                               double* hp, const KState* st) {
  __shared__ double red[KNT / 64];
  if (st && st->done) return;
  const int r0 = blockIdx.x * KRB + threadIdx.x, r1 = r0 + KNT;
  const double w0 = r0 < n ? w[r0] : 0.0, w1 = r1 < n ? w[r1] : 0.0;
  for (int c = 0; c < k1; ++c) {
    const double* v = V + (size_t)c * ldv;
    double d = 0.0;
    if (r0 < n) d = fma(v[r0], w0, d);
    if (r1 < n) d = fma(v[r1], w1, d);
    const double b = block_sum(d, red);
    if (threadIdx.x == 0) hp[(size_t)blockIdx.x * k1 + c] = b;
  }
}

// h = sum of the partials (fixed order); w -= V h; h accumulated into H(:, k) (hacc: add, else set);
// then (second pass) the partials of V^T w (pass2 = 1) or of w.w (pass2 = 0)
__global__ void __launch_bounds__(KNT) gs_sub(int n, double* V, int64_t ldv, int k1, double* w, const double* hp,
                                              int nblk, double* Hk, int hacc, double* hp2, double* wwp, int pass2,
                                              const KState* st) {
  __shared__ double red[KNT / 64];
  __shared__ double h[129];
  if (st && st->done) return;
  // every block forms the same h from the partials
  for (int c = threadIdx.x >> 6; c < k1; c += KNT / 64) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += hp[(size_t)b * k1 + c];
    s = wave_sum(s);
    if (lane == 0) h[c] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < k1) Hk[threadIdx.x] = hacc ? Hk[threadIdx.x] + h[threadIdx.x] : h[threadIdx.x];
  const int r0 = blockIdx.x * KRB + threadIdx.x, r1 = r0 + KNT;
  double w0 = r0 < n ? w[r0] : 0.0, w1 = r1 < n ? w[r1] : 0.0;
  for (int c = 0; c < k1; ++c) {
    const double* v = V + (size_t)c * ldv;
    if (r0 < n) w0 = fma(-h[c], v[r0], w0);
    if (r1 < n) w1 = fma(-h[c], v[r1], w1);
  }
  if (r0 < n) w[r0] = w0;
  if (r1 < n) w[r1] = w1;
  if (pass2) {
    for (int c = 0; c < k1; ++c) {
      const double* v = V + (size_t)c * ldv;
      double d = 0.0;
      if (r0 < n) d = fma(v[r0], w0, d);
      if (r1 < n) d = fma(v[r1], w1, d);
      const double b = block_sum(d, red);
      if (threadIdx.x == 0) hp2[(size_t)blockIdx.x * k1 + c] = b;
    }
  } else {
    const double b = block_sum(w0 * w0 + w1 * w1, red);
    if (threadIdx.x == 0) wwp[blockIdx.x] = b;
  }
}

struct GmCycle {
  double* H;    // (m + 1) x m, column-major, ld m + 1
  double* cs;   // m
  double* sn;   // m
  double* g;    // m + 1
  double* y;    // m
  int m;
};

// Column k of H is in place (h = V^T w accumulated over both passes); its norm partials are in wwp.
// Apply the earlier rotations, form the new one, update g and the residual estimate, decide.
__global__ void gm_givens(GmCycle c, int k, const double* wwp, int nblk, KState* st, double tol, int max_iter) {
  if (st->done) return;
  if (threadIdx.x >= 64) return;
  const double ww = sum_parts(wwp, nblk);
  if (threadIdx.x != 0) return;
  const int ldh = c.m + 1;
  double* Hk = c.H + (size_t)k * ldh;
  const double hn = sqrt(ww);
  Hk[k + 1] = hn;
  for (int i = 0; i < k; ++i) {
    const double a = Hk[i], b = Hk[i + 1];
    Hk[i] = c.cs[i] * a + c.sn[i] * b;
    Hk[i + 1] = -c.sn[i] * a + c.cs[i] * b;
  }
  double cs = 1.0, sn = 0.0;
  if (Hk[k + 1] != 0.0) {
    const double h = hypot(Hk[k], Hk[k + 1]);
    cs = Hk[k] / h;
    sn = Hk[k + 1] / h;
  }
  c.cs[k] = cs;
  c.sn[k] = sn;
  Hk[k] = cs * Hk[k] + sn * Hk[k + 1];
  Hk[k + 1] = 0.0;
  c.g[k + 1] = -sn * c.g[k];
  c.g[k] = cs * c.g[k];
  st->iters += 1;
  st->cycle_k = k + 1;
  st->relres = fabs(c.g[k + 1]) / st->bnorm;
  st->hn_inv = hn != 0.0 ? 1.0 / hn : 0.0;
  if (!(st->relres > tol)) st->done = 1;
  else if (st->iters >= max_iter) st->done = 2;
  else if (hn == 0.0) st->done = 1;
}

// v_{k+1} = w / ||w||
__global__ void __launch_bounds__(KNT) gm_scale(int n, const double* w, double* v, const KState* st) {
  if (st->done) return;
  const double s = st->hn_inv;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) v[i] = w[i] * s;
}

// end of a cycle: y = H^{-1} g over the steps taken (back substitution), in one wave
__global__ void gm_solve_y(GmCycle c, const KState* st) {
  if (threadIdx.x != 0) return;
  const int kk = st->cycle_k;
  const int ldh = c.m + 1;
  for (int i = kk - 1; i >= 0; --i) {
    double s = c.g[i];
    for (int j = i + 1; j < kk; ++j) s -= c.H[i + (size_t)j * ldh] * c.y[j];
    c.y[i] = s / c.H[i + (size_t)i * ldh];
  }
  for (int i = kk; i < c.m; ++i) c.y[i] = 0.0;
}

// x += V y over the cycle's steps (y zero beyond them)
__global__ void __launch_bounds__(KNT) gm_update_x(int n, const double* V, int64_t ldv, int m, const double* y,
                                                   double* x) {
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s = fma(V[(size_t)c * ldv + i], y[c], s);
    x[i] += s;
  }
}

// cycle start: beta = ||r|| (partials), v0 = r / beta, g = (beta, 0, ...), H = 0; a fresh cycle
// replaces the residual estimate with the true (preconditioned) residual
__global__ void __launch_bounds__(KNT) gm_start(int n, const double* r, const double* rr, int np, double* v0,
                                                GmCycle c, KState* st, double tol) {
  __shared__ double s_b;
  if (st->done) return;
  if (threadIdx.x < 64) {
    const double v = sum_parts(rr, np);
    if (threadIdx.x == 0) s_b = sqrt(v);
  }
  __syncthreads();
  const double beta = s_b;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) v0[i] = r[i] * inv;
  if (blockIdx.x == 0) {
    const int ldh = c.m + 1;
    for (int i = threadIdx.x; i < ldh * c.m; i += KNT) c.H[i] = 0.0;
    for (int i = threadIdx.x; i <= c.m; i += KNT) c.g[i] = i == 0 ? beta : 0.0;
  }
}

__global__ void gm_start_state(KState* st, const double* rr, int np, double tol, int first) {
  if (st->done) return;
  if (threadIdx.x >= 64) return;
  const double v = sum_parts(rr, np);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(v);
  st->beta0 = beta;
  st->cycle_k = 0;
  if (first) st->bnorm = st->bnorm > 0.0 ? st->bnorm : 1.0;
  st->relres = beta / st->bnorm;
  if (!(st->relres > tol) || beta == 0.0) st->done = 1;
}

__global__ void bnorm_kernel(KState* st, const double* bb, int np) {
  if (threadIdx.x >= 64) return;
  const double v = sum_parts(bb, np);
  if (threadIdx.x == 0) {
    st->done = 0;
    st->iters = 0;
    st->cycle_k = 0;
    st->bnorm = v > 0.0 ? sqrt(v) : 1.0;
  }
}

__global__ void write_result(const KState* st, cds_krylov_result_t* res) {
  res->iters = st->iters;
  res->converged = st->done == 1 ? 1 : 0;
  res->breakdown = st->done == 3 ? 1 : 0;
  res->reserved = 0;
  res->relres = st->relres;
}

__global__ void copy_kernel(int n, const double* a, double* b) {
  for (int i = blockIdx.x * KNT + threadIdx.x; i < n; i += gridDim.x * KNT) b[i] = a[i];
}

// ------------------------------------------------------------------ host side
struct KWs {
  KState* st;
  double* part;            // product partials: nchunks x n
  double* dp[6];           // dot partials (KMAXP each)
  double* vec[8];          // n-vectors
  double* V;               // GMRES basis n x (m + 1)
  GmCycle cyc;
  double* hp;              // Gram-Schmidt partials: nblk x (m + 1), twice
  double* hp2;
  double* flag;
  void* inner; size_t inner_bytes;   // preconditioner (triangular solves) region
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t krylov_bytes(int n, int m, size_t inner, KWs* w, void* base) {
  const size_t nn = (size_t)std::max(n, 1);
  const int nblk = (n + KRB - 1) / KRB;
  char* p = (char*)base;
  size_t off = kErrRegion;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? (void*)(p + off) : nullptr;
    off += al256(bytes);
    return r;
  };
  KWs t{};
  t.st = (KState*)take(sizeof(KState));
  t.part = (double*)take((size_t)nchunks(n) * nn * 8);
  // dot partials: KMAXP for the vector kernels, one per product block for the Gram-Schmidt norms
  for (int i = 0; i < 6; ++i) t.dp[i] = (double*)take((size_t)std::max(KMAXP, nblk) * 8);
  for (int i = 0; i < 8; ++i) t.vec[i] = (double*)take(nn * 8);
  if (m > 0) {
    t.V = (double*)take(nn * (m + 1) * 8);
    t.cyc.m = m;
    t.cyc.H = (double*)take((size_t)(m + 1) * m * 8);
    t.cyc.cs = (double*)take((size_t)m * 8);
    t.cyc.sn = (double*)take((size_t)m * 8);
    t.cyc.g = (double*)take((size_t)(m + 1) * 8);
    t.cyc.y = (double*)take((size_t)m * 8);
    t.hp = (double*)take((size_t)nblk * (m + 1) * 8);
    t.hp2 = (double*)take((size_t)nblk * (m + 1) * 8);
  }
  t.flag = (double*)take(8);
  t.inner = p ? (void*)(p + off - kErrRegion) : nullptr;   // inner drivers see their own error-region view
  t.inner_bytes = inner;
  off += inner;
  if (w) *w = t;
  return off;
}

struct KCtx {
  Ctx* c;
  int n;
  const double* A; int64_t lda;
  int nc, np, nvec_blocks, nblk;
  hipStream_t s;
  KWs w;
};

hipError_t prod_n(KCtx& k, const double* x, const double* xs_inv, double s_sum, const double* z, double s_z,
                  double* y, const double* dotw, double* dp, const KState* st) {
  {
    KScope ks(k.c->timer, CDS_KC_KRYLOV_GEMV, k.s, 2.0 * k.n * (double)k.n, 8.0 * k.n * (double)k.n);
    hipLaunchKernelGGL(gemv_n_part, dim3((k.n + KRB - 1) / KRB, k.nc), dim3(KNT), 0, k.s, k.A, k.lda, k.n, x, xs_inv,
                       k.w.part, st);
  }
  hipLaunchKernelGGL(reduce_rows, dim3(k.np), dim3(KNT), 0, k.s, (const double*)k.w.part, k.nc, k.n, s_sum, z, s_z, y,
                     dotw, dp, st);
  return hipGetLastError();
}

hipError_t prod_t(KCtx& k, const double* x, double* y, const KState* st) {
  KScope ks(k.c->timer, CDS_KC_KRYLOV_GEMV, k.s, 2.0 * k.n * (double)k.n, 8.0 * k.n * (double)k.n);
  hipLaunchKernelGGL(gemv_t_kernel, dim3((k.n + KNT / 64 - 1) / (KNT / 64)), dim3(KNT), 0, k.s, k.A, k.lda, k.n, x, y,
                     st);
  return hipGetLastError();
}

// The host loop: enqueue `step` check_every times between state reads (check_every = 0: the whole
// budget is enqueued; iterations after the stop exit at once).
template <typename StepF>
cds_status_t drive(KCtx& k, const cds_krylov_params_t& p, int max_steps, StepF&& step) {
  const int every = p.check_every > 0 ? p.check_every : max_steps;
  for (int it = 0; it < max_steps;) {
    const int todo = std::min(every, max_steps - it);
    for (int q = 0; q < todo; ++q)
      if (step() != hipSuccess) return CDS_HIP_ERROR;
    it += todo;
    if (it < max_steps) {
      int done = 0;
      if (hipMemcpyAsync(&done, &k.w.st->done, sizeof(int), hipMemcpyDeviceToHost, k.s) != hipSuccess)
        return CDS_HIP_ERROR;
      if (hipStreamSynchronize(k.s) != hipSuccess) return CDS_HIP_ERROR;
      if (done) break;
    }
  }
  return CDS_SUCCESS;
}

}  // namespace

size_t krylov_ws_bytes(int method, int n, int restart, int precond_nb) {
  const int m = method == CDS_KRYLOV_GMRES ? restart : 0;
  size_t inner = precond_nb > 0 ? getrs_ws_bytes(n, 1, 1, 4) : 0;
  return krylov_bytes(n, m, inner, nullptr, nullptr);
}

// x: initial guess in, solution out.  prec (GMRES only): left preconditioner M^{-1} from FP32 LU
// factors (perm = row order of their pivots), or null.
cds_status_t krylov_run(Ctx& c, int method, int n, const double* A, int64_t lda, const double* b, double* x,
                        const cds_krylov_params_t& p, cds_krylov_result_t* res, const float* LUlo,
                        const int32_t* perm) {
  const int m = method == CDS_KRYLOV_GMRES ? p.restart : 0;
  KCtx k;
  k.c = &c;
  k.n = n; k.A = A; k.lda = lda;
  k.nc = nchunks(n);
  k.np = nparts(n);
  k.nblk = (n + KRB - 1) / KRB;
  k.s = c.s0;
  const size_t inner = LUlo ? getrs_ws_bytes(n, 1, 1, 4) : 0;
  if (krylov_bytes(n, m, inner, nullptr, nullptr) > c.ws_bytes) return CDS_WORKSPACE_TOO_SMALL;
  krylov_bytes(n, m, inner, &k.w, c.ws);
  KWs& w = k.w;
  KState* st = w.st;
  hipStream_t s = k.s;
  const int np = k.np;
  const dim3 vg(np), vb(KNT);
  const double tol = p.tol;
  const int maxit = p.max_iter;
  auto apply_prec = [&](double* in, double* out) -> cds_status_t {
    GetrsCore<float, double> g{};
    g.trans = 0; g.chol = 0; g.n = n; g.nrhs = 1; g.batch = 1;
    g.M = LUlo; g.lda = n; g.strideA = 0;
    g.ipiv = nullptr; g.strideP = 0; g.perm = perm; g.strideQ = n;
    g.B = in; g.ldb = n; g.strideB = 0;
    g.X = out; g.ldx = n; g.strideX = 0; g.accumulate = 0;
    g.active = nullptr; g.ws = w.inner; g.ws_bytes = w.inner_bytes;
    Ctx ci = c;
    ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
    return getrs_core<float, double>(ci, g);
  };

  if (method == CDS_KRYLOV_CG) {
    double *r = w.vec[0], *pv = w.vec[1], *q = w.vec[2];
    // r = b - A x, p = r; partials of b.b and r.r
    hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, b, b, w.dp[0], nullptr);
    if (prod_n(k, x, nullptr, -1.0, b, 1.0, r, r, w.dp[1], nullptr) != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, (const double*)r, pv);
    hipLaunchKernelGGL(krylov_init, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[0], np, (const double*)w.dp[1],
                       np);
    hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
    int it = 0;
    cds_status_t e = drive(k, p, maxit, [&]() -> hipError_t {
      const int par = it & 1;
      ++it;
      hipError_t he = prod_n(k, pv, nullptr, 1.0, nullptr, 0.0, q, pv, w.dp[2], st);
      if (he != hipSuccess) return he;
      hipLaunchKernelGGL(cg_step, vg, vb, 0, s, n, (const double*)w.dp[2], np, st, x, r, (const double*)pv,
                         (const double*)q, w.dp[3], par);
      hipLaunchKernelGGL(cg_dir, vg, vb, 0, s, n, (const double*)w.dp[3], np, st, (const double*)r, pv, par, tol,
                         maxit);
      hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
      return hipGetLastError();
    });
    if (e != CDS_SUCCESS) return e;
  } else if (method == CDS_KRYLOV_BICG) {
    double *r = w.vec[0], *rt = w.vec[1], *pv = w.vec[2], *pt = w.vec[3], *q = w.vec[4], *qt = w.vec[5];
    hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, b, b, w.dp[0], nullptr);
    if (prod_n(k, x, nullptr, -1.0, b, 1.0, r, r, w.dp[1], nullptr) != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, (const double*)r, rt);
    hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, (const double*)r, pv);
    hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, (const double*)r, pt);
    hipLaunchKernelGGL(krylov_init, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[0], np, (const double*)w.dp[1],
                       np);
    hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
    int it = 0;
    cds_status_t e = drive(k, p, maxit, [&]() -> hipError_t {
      const int par = it & 1;
      ++it;
      hipError_t he = prod_n(k, pv, nullptr, 1.0, nullptr, 0.0, q, pt, w.dp[2], st);
      if (he != hipSuccess) return he;
      he = prod_t(k, pt, qt, st);
      if (he != hipSuccess) return he;
      hipLaunchKernelGGL(bicg_step, vg, vb, 0, s, n, (const double*)w.dp[2], np, st, x, r, rt, (const double*)pv,
                         (const double*)q, (const double*)qt, w.dp[3], w.dp[4], par);
      hipLaunchKernelGGL(bicg_dir, vg, vb, 0, s, n, (const double*)w.dp[3], (const double*)w.dp[4], np, st,
                         (const double*)r, (const double*)rt, pv, pt, par);
      hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
      return hipGetLastError();
    });
    if (e != CDS_SUCCESS) return e;
  } else if (method == CDS_KRYLOV_BICGSTAB) {
    double *r = w.vec[0], *rh = w.vec[1], *pv = w.vec[2], *v = w.vec[3], *sv = w.vec[4], *t = w.vec[5];
    hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, b, b, w.dp[0], nullptr);
    if (prod_n(k, x, nullptr, -1.0, b, 1.0, r, r, w.dp[1], nullptr) != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, (const double*)r, rh);
    hipLaunchKernelGGL(krylov_init, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[0], np, (const double*)w.dp[1],
                       np);
    hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
    // rho partials for the first iteration: rh.r = r.r
    hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, (const double*)rh, (const double*)r, w.dp[2], nullptr);
    int it = 0;
    cds_status_t e = drive(k, p, maxit, [&]() -> hipError_t {
      const int par = it & 1;
      const int first = it == 0;
      ++it;
      hipLaunchKernelGGL(bcs_dir, vg, vb, 0, s, n, (const double*)w.dp[2], np, st, (const double*)r, pv,
                         (const double*)v, par, first);
      hipError_t he = prod_n(k, pv, nullptr, 1.0, nullptr, 0.0, v, rh, w.dp[3], st);
      if (he != hipSuccess) return he;
      hipLaunchKernelGGL(bcs_half, vg, vb, 0, s, n, (const double*)w.dp[3], np, st, (const double*)r,
                         (const double*)v, sv, w.dp[4], par);
      hipLaunchKernelGGL(bcs_half_test, vg, vb, 0, s, n, (const double*)w.dp[4], np, st, x, (const double*)pv, r,
                         (const double*)sv, tol, w.flag);
      hipLaunchKernelGGL(bcs_half_done, dim3(1), dim3(64), 0, s, st, (const double*)w.flag, (const double*)w.dp[4],
                         np);
      he = prod_n(k, sv, nullptr, 1.0, nullptr, 0.0, t, nullptr, nullptr, st);
      if (he != hipSuccess) return he;
      hipLaunchKernelGGL(dot2_part, vg, vb, 0, s, n, (const double*)t, (const double*)sv, w.dp[5], w.dp[0],
                         (const KState*)st);
      hipLaunchKernelGGL(bcs_full, vg, vb, 0, s, n, (const double*)w.dp[5], (const double*)w.dp[0], np, st, x, r,
                         (const double*)pv, (const double*)sv, (const double*)t, (const double*)rh, w.dp[1], w.dp[2]);
      hipLaunchKernelGGL(bcs_account, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[1], np);
      hipLaunchKernelGGL(krylov_test, dim3(1), dim3(1), 0, s, st, tol, maxit);
      return hipGetLastError();
    });
    if (e != CDS_SUCCESS) return e;
  } else {
    // GMRES(m), classical Gram-Schmidt twice, Givens rotations, optional left preconditioner
    double *r = w.vec[0], *wv = w.vec[1], *t1 = w.vec[2], *pb = w.vec[3];
    const int64_t ldv = n;
    const dim3 pg(k.nblk);
    // ||M^{-1} b||
    if (LUlo) {
      hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, b, t1);
      cds_status_t e = apply_prec(t1, pb);
      if (e != CDS_SUCCESS) return e;
    } else {
      hipLaunchKernelGGL(copy_kernel, vg, vb, 0, s, n, b, pb);
    }
    hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, (const double*)pb, (const double*)pb, w.dp[0], nullptr);
    hipLaunchKernelGGL(bnorm_kernel, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[0], np);
    bool first = true;
    // one cycle: r = M^{-1}(b - A x); Arnoldi steps; x += V y.  The budget check happens per cycle.
    for (int cyc = 0;; ++cyc) {
      if (LUlo) {
        if (prod_n(k, x, nullptr, -1.0, b, 1.0, t1, nullptr, nullptr, st) != hipSuccess) return CDS_HIP_ERROR;
        cds_status_t e = apply_prec(t1, r);
        if (e != CDS_SUCCESS) return e;
        hipLaunchKernelGGL(dot_part, vg, vb, 0, s, n, (const double*)r, (const double*)r, w.dp[1], (const KState*)st);
      } else {
        if (prod_n(k, x, nullptr, -1.0, b, 1.0, r, r, w.dp[1], st) != hipSuccess) return CDS_HIP_ERROR;
      }
      hipLaunchKernelGGL(gm_start_state, dim3(1), dim3(64), 0, s, st, (const double*)w.dp[1], np, tol, first ? 1 : 0);
      hipLaunchKernelGGL(gm_start, vg, vb, 0, s, n, (const double*)r, (const double*)w.dp[1], np, w.V, w.cyc, st, tol);
      first = false;
      int kk = 0;
      cds_status_t e = drive(k, p, m, [&]() -> hipError_t {
        const int kstep = kk++;
        double* vk = w.V + (size_t)kstep * ldv;
        double* Hk = w.cyc.H + (size_t)kstep * (m + 1);
        hipError_t he;
        if (LUlo) {
          he = prod_n(k, vk, nullptr, 1.0, nullptr, 0.0, t1, nullptr, nullptr, st);
          if (he != hipSuccess) return he;
          if (apply_prec(t1, wv) != CDS_SUCCESS) return hipErrorUnknown;
        } else {
          he = prod_n(k, vk, nullptr, 1.0, nullptr, 0.0, wv, nullptr, nullptr, st);
          if (he != hipSuccess) return he;
        }
        const int k1 = kstep + 1;
        hipLaunchKernelGGL(gs_dots, pg, vb, 0, s, n, (const double*)w.V, ldv, k1, (const double*)wv, w.hp,
                           (const KState*)st);
        hipLaunchKernelGGL(gs_sub, pg, vb, 0, s, n, w.V, ldv, k1, wv, (const double*)w.hp, k.nblk, Hk, 0, w.hp2,
                           nullptr, 1, (const KState*)st);
        hipLaunchKernelGGL(gs_sub, pg, vb, 0, s, n, w.V, ldv, k1, wv, (const double*)w.hp2, k.nblk, Hk, 1, nullptr,
                           w.dp[4], 0, (const KState*)st);
        hipLaunchKernelGGL(gm_givens, dim3(1), dim3(64), 0, s, w.cyc, kstep, (const double*)w.dp[4], k.nblk, st, tol,
                           maxit);
        if (kstep + 1 < m)
          hipLaunchKernelGGL(gm_scale, vg, vb, 0, s, n, (const double*)wv, w.V + (size_t)(kstep + 1) * ldv,
                             (const KState*)st);
        return hipGetLastError();
      });
      if (e != CDS_SUCCESS) return e;
      hipLaunchKernelGGL(gm_solve_y, dim3(1), dim3(64), 0, s, w.cyc, (const KState*)st);
      hipLaunchKernelGGL(gm_update_x, vg, vb, 0, s, n, (const double*)w.V, ldv, m, (const double*)w.cyc.y, x);
      if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
      // decide on the host whether another cycle is needed (one read per cycle)
      KState hs;
      if (hipMemcpyAsync(&hs, st, sizeof(KState), hipMemcpyDeviceToHost, s) != hipSuccess) return CDS_HIP_ERROR;
      if (hipStreamSynchronize(s) != hipSuccess) return CDS_HIP_ERROR;
      if (hs.done == 1 || hs.done == 3) break;
      if (hs.done == 2 || hs.iters >= maxit) break;
      // the cycle ended by its length: continue (gm_start_state recomputes the true residual)
    }
  }
  hipLaunchKernelGGL(write_result, dim3(1), dim3(1), 0, s, (const KState*)st, res);
  return hipGetLastError() == hipSuccess ? CDS_SUCCESS : CDS_HIP_ERROR;
}

}  // namespace cds
