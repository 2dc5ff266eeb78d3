// Mixed-precision solve with FP64 iterative refinement (an extension of the
// paper's direct method, Sec. 2: factor once, then triangular solves; here the
// factorization runs in FP32 or with BF16/FP16 update operands and the FP64
// accuracy is recovered by refinement with an FP64 residual).
//
//   convert_kernel   A64 -> A32 (RNE) and the row sums of |A| (for ||A||_inf).
//   residual_kernel  R = B - A X in FP64, with ||R(:,c)||_inf and ||X(:,c)||_inf.
//   control_kernel   backward error eta, stopping rule, per-matrix active flag
//                    that turns every later kernel of the loop into a no-op.
//   outer_kernel     C = alpha X Y^T (the adjoint's Abar = -bbar x^T).
#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"
#include "mixed.hpp"
#include "krylov.hpp"
#include <algorithm>
#include <vector>

namespace cds {

namespace {

// order-preserving atomic max for non-negative doubles (NaN sorts above +inf)
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  atomicMax(reinterpret_cast<unsigned long long*>(p), bits);
}

// One workgroup per 64 rows; wave w streams the columns j = w, w+4, ...  Columns [jlo, jhi) are
// converted; with anorm the row sums run over every column (in the same order whatever jlo and
// jhi), otherwise only [jlo, jhi) is read.
__global__ void __launch_bounds__(256) convert_kernel(const double* A0, int64_t lda, int64_t strideA, float* B0,
                                                      int64_t ldb, int64_t strideB, int n, double* anorm, int jlo,
                                                      int jhi) {
  const int b = blockIdx.y;
  const double* A = A0 + (size_t)b * strideA;
  float* Bf = B0 + (size_t)b * strideB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  __shared__ double part[4][64];
  double s = 0.0;
  const int j0s = anorm ? 0 : jlo, j1s = anorm ? n : jhi;
  if (r < n) {
    // 8 columns per step and wave (32 per workgroup step): 8 loads in flight per lane
    for (int j0 = j0s + wave; j0 < j1s; j0 += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = j0 + 4 * u < j1s ? A[r + (size_t)(j0 + 4 * u) * lda] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + 4 * u < j1s) {
          const int j = j0 + 4 * u;
          if (j >= jlo && j < jhi) Bf[r + (size_t)j * ldb] = (float)v[u];
          s += fabs(v[u]);
        }
    }
  }
  if (anorm == nullptr) return;   // uniform over the workgroup
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0) {
    double t = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    t = wave_max(t);
    if (lane == 0) atomic_max_nonneg(anorm + b, t);
  }
}

// ||A||_inf only (when no conversion is needed)
__global__ void __launch_bounds__(256) rownorm_kernel(const double* A0, int64_t lda, int64_t strideA, int n,
                                                      double* anorm) {
  const int b = blockIdx.y;
  const double* A = A0 + (size_t)b * strideA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  __shared__ double part[4][64];
  double s = 0.0;
  if (r < n)
    for (int j = wave; j < n; j += 4) s += fabs(A[r + (size_t)j * lda]);
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0) {
    double t = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    t = wave_max(t);
    if (lane == 0) atomic_max_nonneg(anorm + b, t);
  }
}

// R = B - op(A) X (FP64).  op N: 64 rows per workgroup, waves split the columns.
// op T: row i of A^T is column i of A: 16 lanes per output, four outputs per wave.
__global__ void __launch_bounds__(256) residual_kernel(const double* A0, int64_t lda, int64_t strideA,
                                                       const double* X0, int64_t ldx, int64_t strideX,
                                                       const double* B0, int64_t ldb, int64_t strideB, double* R0,
                                                       int64_t ldr, int64_t strideR, int n, int nrhs, int trans,
                                                       double* rnorm, double* xnorm, const int* active) {
  const int b = blockIdx.y;
  if (active && active[b] == 0) return;
  const double* A = A0 + (size_t)b * strideA;
  const double* X = X0 + (size_t)b * strideX;
  const double* B = B0 + (size_t)b * strideB;
  double* R = R0 + (size_t)b * strideR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double part[4][64];
  for (int c = 0; c < nrhs; ++c) {
    const double* x = X + (size_t)c * ldx;
    if (!trans) {
      const int r = blockIdx.x * 64 + lane;
      double s = 0.0;
      if (r < n)
        for (int j = wave; j < n; j += 4) s = fma(A[r + (size_t)j * lda], x[j], s);
      part[wave][lane] = s;
      __syncthreads();
      if (wave == 0) {
        double rv = 0.0;
        if (r < n) {
          rv = B[r + (size_t)c * ldb] - ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
          R[r + (size_t)c * ldr] = rv;
        }
        double m = wave_max(fabs(rv));
        double xm = wave_max(r < n ? fabs(x[r]) : 0.0);
        if (lane == 0) {
          atomic_max_nonneg(rnorm + (size_t)b * nrhs + c, m);
          atomic_max_nonneg(xnorm + (size_t)b * nrhs + c, xm);
        }
      }
      __syncthreads();
    } else {
      // op T: 16 outputs (columns of A) per workgroup, 4 per wave, 16 lanes per column walking its
      // rows (4 x 128 B per load, 8 loads in flight per lane), combined inside each 16-lane row
      const int cc = lane >> 4, rl = lane & 15;
      const int i = blockIdx.x * 16 + wave * 4 + cc;
      const double* col = A + (size_t)min(i, n - 1) * lda;
      double s0 = 0.0, s1 = 0.0;
      for (int j0 = rl; j0 < n; j0 += 16 * 8) {
        double a[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = j0 + 16 * u;
          const bool ok = i < n && j < n;
          a[u] = ok ? col[j] : 0.0;
          xv[u] = ok ? x[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0 = fma(a[u], xv[u], s0);
          s1 = fma(a[u + 1], xv[u + 1], s1);
        }
      }
      const double sum = row16_sum(s0 + s1);
      double rv = 0.0, xi = 0.0;
      if (rl == 0 && i < n) {
        rv = B[i + (size_t)c * ldb] - sum;
        R[i + (size_t)c * ldr] = rv;
        xi = x[i];
      }
      const double m = wave_max(fabs(rv)), xm = wave_max(fabs(xi));
      if (lane == 0) {
        atomic_max_nonneg(rnorm + (size_t)b * nrhs + c, m);
        atomic_max_nonneg(xnorm + (size_t)b * nrhs + c, xm);
      }
    }
  }
}

// Residual, op N, split over column chunks: part[chunk][row] = sum over the chunk of A(row, j) x_j.
// 256 rows per workgroup (one per thread, 2 KB contiguous per column), 8 columns per step.
__global__ void __launch_bounds__(256) residual_part_kernel(const double* A0, int64_t lda, int64_t strideA,
                                                            const double* X0, int64_t ldx, int64_t strideX, int n,
                                                            int c, int chunk, double* part, const int* active) {
  const int b = blockIdx.z;
  if (active && active[b] == 0) return;
  const double* A = A0 + (size_t)b * strideA;
  const double* x = X0 + (size_t)b * strideX + (size_t)c * ldx;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * chunk, j1 = min(n, j0 + chunk);
  double s0 = 0.0, s1 = 0.0;
  if (r < n) {
    int j = j0;
    for (; j + 8 <= j1; j += 8) {
      double a[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) a[t] = A[r + (size_t)(j + t) * lda];
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        s0 = fma(a[t], x[j + t], s0);
        s1 = fma(a[t + 1], x[j + t + 1], s1);
      }
    }
    for (; j < j1; ++j) s0 = fma(A[r + (size_t)j * lda], x[j], s0);
    part[((size_t)b * gridDim.y + blockIdx.y) * n + r] = s0 + s1;
  }
}

// R(:, c) = B(:, c) - sum_chunk part[chunk] (fixed order) and the inf-norms of R(:, c), X(:, c).
__global__ void __launch_bounds__(256) residual_finish_kernel(const double* X0, int64_t ldx, int64_t strideX,
                                                              const double* B0, int64_t ldb, int64_t strideB,
                                                              double* R0, int64_t ldr, int64_t strideR, int n, int c,
                                                              int nrhs, int nchunk, const double* part,
                                                              double* rnorm, double* xnorm, const int* active) {
  const int b = blockIdx.y;
  if (active && active[b] == 0) return;
  const int r = blockIdx.x * 256 + threadIdx.x;
  double rv = 0.0, xv = 0.0;
  if (r < n) {
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += part[((size_t)b * nchunk + k) * n + r];
    rv = B0[(size_t)b * strideB + (size_t)c * ldb + r] - s;
    R0[(size_t)b * strideR + (size_t)c * ldr + r] = rv;
    xv = X0[(size_t)b * strideX + (size_t)c * ldx + r];
  }
  double m = wave_max(fabs(rv)), xm = wave_max(fabs(xv));
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(rnorm + (size_t)b * nrhs + c, m);
    atomic_max_nonneg(xnorm + (size_t)b * nrhs + c, xm);
  }
}

// Refinement state per matrix: eta history and the active flag.
struct IrState {
  double eta_prev, eta_prev2;
  int active;
  int done;
};

// One thread per matrix.  it = number of corrections applied so far.
__global__ void control_kernel(int batch, int nrhs, int it, int max_iter, double tol, double success_tol,
                               const double* anorm, double* rnorm, double* xnorm, IrState* st,
                               cds_ir_result_t* res, int* active, const int32_t* info) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  IrState& s = st[b];
  if (it == 0) {
    s.eta_prev = s.eta_prev2 = INFINITY;
    s.done = 0;
    res[b].info = info ? info[b] : 0;
    res[b].fell_back = 0;
    res[b].iters = 0;
  }
  if (s.done) { active[b] = 0; return; }
  double eta = 0.0;
  const double na = anorm[b];
  for (int c = 0; c < nrhs; ++c) {
    const double rn = rnorm[(size_t)b * nrhs + c], xn = xnorm[(size_t)b * nrhs + c];
    double e;
    if (rn == 0.0) e = 0.0;
    else if (na * xn > 0.0) e = rn / (na * xn);
    else e = INFINITY;
    if (!(e <= eta)) eta = e;   // NaN propagates
    rnorm[(size_t)b * nrhs + c] = 0.0;
    xnorm[(size_t)b * nrhs + c] = 0.0;
  }
  if (it == 0) res[b].eta0 = eta;
  res[b].eta = eta;
  res[b].iters = it;
  int reason = 0;
  if (info && info[b] != 0) reason = 5;
  else if (!(eta == eta) || eta == INFINITY) reason = 4;
  else if (eta <= tol) reason = 1;
  else if (it >= 2 && eta > 0.5 * s.eta_prev && s.eta_prev > 0.5 * s.eta_prev2) reason = 2;
  else if (it >= max_iter) reason = 3;
  s.eta_prev2 = s.eta_prev;
  s.eta_prev = eta;
  if (reason) {
    s.done = 1;
    active[b] = 0;
    res[b].stop_reason = reason;
    res[b].converged = (eta <= success_tol) ? 1 : 0;
  } else {
    active[b] = 1;
    res[b].stop_reason = 0;
    res[b].converged = 0;
  }
}

__global__ void outer_kernel(int m, int n, int k, double alpha, const double* X0, int64_t ldx, int64_t strideX,
                             const double* Y0, int64_t ldy, int64_t strideY, double* C0, int64_t ldc,
                             int64_t strideC) {
  const int b = blockIdx.z;
  const double* X = X0 + (size_t)b * strideX;
  const double* Y = Y0 + (size_t)b * strideY;
  double* C = C0 + (size_t)b * strideC;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j0 = blockIdx.y * 64;
  if (i >= m) return;
  for (int jj = threadIdx.x >> 6; jj < 64; jj += 4) {
    const int j = j0 + jj;
    if (j >= n) break;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s = fma(X[i + (size_t)t * ldx], Y[j + (size_t)t * ldy], s);
    C[i + (size_t)j * ldc] = alpha * s;
  }
}

__global__ void set_active_kernel(int* active, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) active[b] = 1;
}

__global__ void copy_d_kernel(const double* A0, int64_t lda, int64_t strideA, double* B0, int64_t ldb,
                              int64_t strideB, int rows, int cols) {
  const int b = blockIdx.y;
  const double* A = A0 + (size_t)b * strideA;
  double* Bd = B0 + (size_t)b * strideB;
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    Bd[i + (size_t)j * ldb] = A[i + (size_t)j * lda];
  }
}

// Partial maxima of |B| for the FP16 operand scale (the update kernel reduces the kScaleParts
// values and derives the power of two).  Block p takes columns 4p + wave, 4p + wave + 4P, ...
// (one wave per column, lanes down the rows).  NaN entries are ignored, as fmaxf does.
__global__ void __launch_bounds__(256) maxabs_part_kernel(const float* B0, int64_t ldb, int64_t strideB, int rows,
                                                          int cols, float* part) {
  const int b = blockIdx.y;
  const float* B = B0 + (size_t)b * strideB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ float red[4];
  float m = 0.f;
  for (int j = blockIdx.x * 4 + wave; j < cols; j += kScaleParts * 4) {
    const float* col = B + (size_t)j * ldb;
    for (int i = lane; i < rows; i += 64) m = fmaxf(m, fabsf(col[i]));
  }
  m = wave_max(m);
  if (lane == 0) red[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)b * kScaleParts + blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// max_j sum_i |A(i, j)| = ||A^T||_inf; one wave per column
__global__ void __launch_bounds__(256) colnorm_kernel(const double* A0, int64_t lda, int64_t strideA, int n,
                                                      double* anorm) {
  const int b = blockIdx.y;
  const double* A = A0 + (size_t)b * strideA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + wave;
  double s = 0.0;
  if (j < n)
    for (int i = lane; i < n; i += 64) s += fabs(A[i + (size_t)j * lda]);
  s = wave_sum(s);
  if (lane == 0 && j < n) atomic_max_nonneg(anorm + b, s);
}

// Symmetric matrix held in its lower triangle: row r of A is A(r, 0..r) followed by
// A(r+1.., r) (column r below the diagonal).  Converts the lower triangle to FP32
// (the strict upper triangle of the copy is not written) and computes ||A||_inf.
// Column part of the symmetric row sums: colabs[i] = sum_{c>i} |A(c,i)| (16 lanes per column, 4 columns
// per wave, 8 loads in flight per lane, combined inside each 16-lane row).
__global__ void __launch_bounds__(256) sym_colabs_kernel(const double* A, int64_t lda, int n, double* colabs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cc = lane >> 4, rl = lane & 15;
  const int g0 = blockIdx.x * 16 + wave * 4;
  const int col = g0 + cc;
  const double* Ac = A + (size_t)min(col, n - 1) * lda;
  double s0 = 0.0, s1 = 0.0;
  for (int i0 = g0 + 1 + rl; i0 < n; i0 += 16 * 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 16 * u;
      a[u] = (col < n && i > col && i < n) ? Ac[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      s0 += fabs(a[u]);
      s1 += fabs(a[u + 1]);
    }
  }
  const double t = row16_sum(s0 + s1);
  if (rl == 0 && col < n) colabs[col] = t;
}

// Lower triangle of A to FP32 (row part of the symmetric row sums on the way) and ||A||_inf with the
// column parts from sym_colabs_kernel.
__global__ void __launch_bounds__(256) convert_sym_kernel(const double* A, int64_t lda, float* Bf, int64_t ldb, int n,
                                                          const double* colabs, double* anorm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  __shared__ double part[4][64];
  double s = 0.0;
  if (r < n) {
    const int jmax = min(n - 1, (int)blockIdx.x * 64 + 63);   // the block's last row
    for (int j0 = wave; j0 <= jmax; j0 += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = j0 + 4 * u <= r ? A[r + (size_t)(j0 + 4 * u) * lda] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + 4 * u <= r) {
          Bf[r + (size_t)(j0 + 4 * u) * ldb] = (float)v[u];
          s += fabs(v[u]);
        }
    }
  }
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0) {
    double t = ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) + (r < n ? colabs[r] : 0.0);
    t = wave_max(t);
    if (lane == 0) atomic_max_nonneg(anorm, t);
  }
}

// Symmetric A held in its lower triangle: (A x)_r = sum_{j<=r} A(r,j) x_j + sum_{i>r} A(i,r) x_i.
// Row part over one column chunk (thread per row, 64 consecutive rows per load): part[chunk][r].
__global__ void __launch_bounds__(256) residual_sym_row_kernel(const double* A, int64_t lda, const double* X,
                                                               int64_t ldx, int n, int c, int chunk, double* part,
                                                               const int* active) {
  if (active && active[0] == 0) return;
  const double* x = X + (size_t)c * ldx;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * chunk;
  const int rmax = min(n - 1, (int)blockIdx.x * 256 + 255);
  const int j1 = min(min(n, j0 + chunk), rmax + 1);   // nothing of the chunk above the block's last row
  double s0 = 0.0, s1 = 0.0;
  if (r < n) {
    int j = j0;
    for (; j + 8 <= j1; j += 8) {
      double a[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) a[t] = (j + t <= r) ? A[r + (size_t)(j + t) * lda] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; t += 2) {
        s0 = fma(a[t], x[j + t], s0);
        s1 = fma(a[t + 1], x[j + t + 1], s1);
      }
    }
    for (; j < j1; ++j)
      if (j <= r) s0 = fma(A[r + (size_t)j * lda], x[j], s0);
    part[(size_t)blockIdx.y * n + r] = s0 + s1;
  }
}

// Column part: sum_{i>r} A(i,r) x_i for 16 columns per workgroup, 4 per wave, 16 lanes per column
// (each load reads 4 x 128 B), combined inside each 16-lane row: out[r].
__global__ void __launch_bounds__(256) residual_sym_col_kernel(const double* A, int64_t lda, const double* X,
                                                               int64_t ldx, int n, int c, double* out,
                                                               const int* active) {
  if (active && active[0] == 0) return;
  const double* x = X + (size_t)c * ldx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cc = lane >> 4, rl = lane & 15;
  const int g0 = blockIdx.x * 16 + wave * 4;      // this wave's first column
  const int col = g0 + cc;
  const double* Ac = A + (size_t)min(col, n - 1) * lda;
  constexpr int UN = 8;
  double s0 = 0.0, s1 = 0.0;
  for (int i0 = g0 + 1 + rl; i0 < n; i0 += 16 * UN) {
    double a[UN], xv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int i = i0 + 16 * u;
      const bool ok = col < n && i > col && i < n;
      a[u] = ok ? Ac[i] : 0.0;
      xv[u] = ok ? x[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; u += 2) {
      s0 = fma(a[u], xv[u], s0);
      s1 = fma(a[u + 1], xv[u + 1], s1);
    }
  }
  const double s = row16_sum(s0 + s1);
  if (rl == 0 && col < n) out[col] = s;
}

// R = B - A X for symmetric A held in its lower triangle (same split as above).
__global__ void __launch_bounds__(256) residual_sym_kernel(const double* A, int64_t lda, const double* X, int64_t ldx,
                                                           const double* B, int64_t ldb, double* R, int64_t ldr,
                                                           int n, int nrhs, double* rnorm, double* xnorm,
                                                           const int* active) {
  if (active && active[0] == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  __shared__ double part[4][64];
  __shared__ double colp[64];
  for (int c = 0; c < nrhs; ++c) {
    const double* x = X + (size_t)c * ldx;
    double s = 0.0;
    if (r < n)
      for (int j = wave; j <= r; j += 4) s = fma(A[r + (size_t)j * lda], x[j], s);
    part[wave][lane] = s;
    for (int o = 0; o < 16; ++o) {
      const int loc = wave * 16 + o;
      const int rr = blockIdx.x * 64 + loc;
      double t = 0.0;
      if (rr < n)
        for (int i = rr + 1 + lane; i < n; i += 64) t = fma(A[i + (size_t)rr * lda], x[i], t);
      t = wave_sum(t);
      if (lane == 0) colp[loc] = t;
    }
    __syncthreads();
    if (wave == 0) {
      double rv = 0.0;
      if (r < n) {
        rv = B[r + (size_t)c * ldb] -
             (((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) + colp[lane]);
        R[r + (size_t)c * ldr] = rv;
      }
      double m = wave_max(fabs(rv));
      double xm = wave_max(r < n ? fabs(x[r]) : 0.0);
      if (lane == 0) {
        atomic_max_nonneg(rnorm + c, m);
        atomic_max_nonneg(xnorm + c, xm);
      }
    }
    __syncthreads();
  }
}

__global__ void fallback_result_kernel(int nrhs, const double* anorm, double* rnorm, double* xnorm,
                                       cds_ir_result_t* res, const int32_t* info, double success_tol) {
  double eta = 0.0;
  for (int c = 0; c < nrhs; ++c) {
    const double rn = rnorm[c], xn = xnorm[c];
    double e = rn == 0.0 ? 0.0 : ((*anorm) * xn > 0.0 ? rn / ((*anorm) * xn) : INFINITY);
    if (!(e <= eta)) eta = e;
    rnorm[c] = 0.0;
    xnorm[c] = 0.0;
  }
  res->eta = eta;
  res->fell_back = 1;
  res->info = *info;
  res->converged = (*info == 0 && eta <= success_tol) ? 1 : 0;
}

}  // namespace

hipError_t launch_maxabs_part(const float* B, int64_t ldb, int64_t strideB, int rows, int cols, float* part, int batch,
                              hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  // an empty block still writes its kScaleParts zeros (no scaling)
  hipLaunchKernelGGL(maxabs_part_kernel, dim3(kScaleParts, batch), dim3(256), 0, s, B, ldb, strideB, std::max(rows, 0),
                     std::max(cols, 0), part);
  return hipGetLastError();
}

hipError_t launch_outer(int m, int n, int k, double alpha, const double* X, int64_t ldx, int64_t strideX,
                        const double* Y, int64_t ldy, int64_t strideY, double* C, int64_t ldc, int64_t strideC,
                        int batch, hipStream_t s) {
  if (m <= 0 || n <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((m + 63) / 64, (n + 63) / 64, batch);
  hipLaunchKernelGGL(outer_kernel, grid, dim3(256), 0, s, m, n, k, alpha, X, ldx, strideX, Y, ldy, strideY, C, ldc,
                     strideC);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// workspace of the refinement loop (after the error region):
//   anorm, rnorm, xnorm, state, active, scale partials (2 x kScaleParts per matrix), info, perm, gmap, R,
//   [FP64 fallback copy and pivots], then the inner region for the factorization /
//   solves (which keeps its own error region view at the same error word).
// ---------------------------------------------------------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr int kResChunks = 16;   // column chunks of the split residual

// the block-inverse data of the FP32 factors (one right-hand side, LU only)
static size_t binv_region(int n, int nrhs, int batch, int chol) {
  return (!chol && nrhs == 1) ? al256((size_t)batch * binv_elems(n) * 4) : 0;
}

static size_t ir_small_bytes(int n, int nrhs, int batch) {
  return al256(batch * 8) + 2 * al256((size_t)batch * nrhs * 8) + al256(batch * sizeof(IrState)) +
         al256(batch * 4) + al256((size_t)batch * 4 * 2 * kScaleParts) + al256(batch * 4) + al256((size_t)batch * n * 4) +
         al256((size_t)batch * perm_moves_ints(n) * 4) +
         al256((size_t)batch * n * nrhs * 8) + al256((size_t)batch * kResChunks * n * 8);
}

size_t ir_ws_bytes(int n, int nrhs, int batch, int nb, int chol, int fallback) {
  size_t inner = chol ? std::max(potrf_ws_bytes(n, nb, 4), getrs_ws_bytes(n, nrhs, batch, 4))
                      : std::max(getrf_ws_bytes(n, nb, 32, batch, 4), getrs_ws_bytes(n, nrhs, batch, 4));
  size_t fb = 0;
  if (fallback) {
    inner = std::max(inner, chol ? potrf_ws_bytes(n, nb, 8) : getrf_ws_bytes(n, nb, 32, batch, 8));
    inner = std::max(inner, getrs_ws_bytes(n, nrhs, batch, 8));
    fb = al256((size_t)batch * n * n * 8) + al256((size_t)batch * n * 4) + al256(batch * 4);
  }
  return kErrRegion + ir_small_bytes(n, nrhs, batch) + binv_region(n, nrhs, batch, chol) + fb + inner;
}

struct IrWs {
  double* anorm; double* rnorm; double* xnorm; IrState* st; int* active; float* scale; int32_t* info;
  int32_t* perm; int32_t* gmap; double* R; double* part;
  float* binv;   // block-inverse data of the factors, or null
  double* fbA; int32_t* fbpiv; int32_t* fbinfo;
  void* inner; size_t inner_bytes;
};

static bool carve(void* ws, size_t ws_bytes, int n, int nrhs, int batch, int fallback, IrWs& w, int binv = 0) {
  w = IrWs{};
  char* p = (char*)ws + kErrRegion;
  w.anorm = (double*)p; p += al256(batch * 8);
  w.rnorm = (double*)p; p += al256((size_t)batch * nrhs * 8);
  w.xnorm = (double*)p; p += al256((size_t)batch * nrhs * 8);
  w.st = (IrState*)p; p += al256(batch * sizeof(IrState));
  w.active = (int*)p; p += al256(batch * 4);
  w.scale = (float*)p; p += al256((size_t)batch * 4 * 2 * kScaleParts);
  w.info = (int32_t*)p; p += al256(batch * 4);
  w.perm = (int32_t*)p; p += al256((size_t)batch * n * 4);
  w.gmap = (int32_t*)p; p += al256((size_t)batch * perm_moves_ints(n) * 4);
  w.R = (double*)p; p += al256((size_t)batch * n * nrhs * 8);
  w.part = (double*)p; p += al256((size_t)batch * kResChunks * n * 8);
  if (binv) {
    w.binv = (float*)p;
    p += binv_region(n, nrhs, batch, 0);
  }
  if (fallback) {
    w.fbA = (double*)p; p += al256((size_t)batch * n * n * 8);
    w.fbpiv = (int32_t*)p; p += al256((size_t)batch * n * 4);
    w.fbinfo = (int32_t*)p; p += al256(batch * 4);
  }
  // inner drivers address their regions from (base + kErrRegion); give them a base
  // whose "error region" overlaps the end of ours, and point their error word at ours.
  w.inner = (void*)(p - kErrRegion);
  size_t used = (size_t)(p - (char*)ws);
  if (ws_bytes < used) return false;
  w.inner_bytes = ws_bytes - used + kErrRegion;
  return true;
}

// GMRES as the correction solver of the refinement (one system, one right-hand side).
struct GmresCorr {
  const cds_krylov_params_t* p;
  void* kws; size_t kbytes;    // the Krylov solver's workspace
  double* d;                   // the correction
  cds_krylov_result_t* kres;   // the last inner solve's result (device)
};

__global__ void add_vec_kernel(int n, const double* d, double* x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] += d[i];
}
__global__ void add_inner_iters_kernel(cds_ir_result_t* res, const cds_krylov_result_t* kres, int reset) {
  res->reserved = (reset ? 0 : res->reserved) + (kres ? kres->iters : 0);
}

// The refinement loop on existing low-precision factors: x0 = solve_lo(b), then
// r = b - op(A) x (FP64), eta, stop test, d = solve_lo(r), x += d (FP64).  With gm,
// d solves A d = r by GMRES left-preconditioned with the low-precision factors.
static cds_status_t refine(Ctx& c, const IrWs& w, int trans, int chol, int n, int nrhs, const double* A, int64_t lda,
                           int64_t strideA, const float* LU, int64_t ldlu, int64_t strideLU, const int32_t* perm,
                           int64_t strideQ, const double* B, int64_t ldb, int64_t strideB, double* X, int64_t ldx,
                           int64_t strideX, const cds_ir_params_t& prm, cds_ir_result_t* res, const int32_t* info,
                           int batch, const GmresCorr* gm = nullptr) {
  hipStream_t s = c.s0;
  const int rblocks = (n + 63) / 64;
  GetrsCore<float, double> g{};
  g.trans = trans; g.chol = chol; g.n = n; g.nrhs = nrhs; g.batch = batch;
  g.M = LU; g.lda = ldlu; g.strideA = strideLU;
  g.ipiv = nullptr; g.strideP = 0; g.perm = perm; g.strideQ = strideQ;
  g.B = B; g.ldb = ldb; g.strideB = strideB;
  g.X = X; g.ldx = ldx; g.strideX = strideX; g.accumulate = 0;
  g.active = nullptr; g.ws = w.inner; g.ws_bytes = w.inner_bytes;
  g.binv = (!trans && !chol && nrhs == 1) ? w.binv : nullptr;
  cds_status_t st = getrs_core<float, double>(c, g);
  if (st != CDS_SUCCESS) return st;
  if (launch_fill_zero(w.rnorm, (size_t)batch * nrhs * 8, s) != hipSuccess) return CDS_HIP_ERROR;
  if (launch_fill_zero(w.xnorm, (size_t)batch * nrhs * 8, s) != hipSuccess) return CDS_HIP_ERROR;
  hipLaunchKernelGGL(set_active_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, w.active, batch);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  const int max_iter = prm.max_iter;
  std::vector<int> h_active;
  for (int it = 0; it <= max_iter; ++it) {
    KScope* ks = new KScope(c.timer, CDS_KC_RESIDUAL, s, 2.0 * batch * n * (double)n * nrhs,
                            8.0 * batch * ((chol ? 0.5 : 1.0) * n * (double)n * nrhs + 3.0 * n * nrhs));
    if (!chol && !trans) {
      const int rb256 = (n + 255) / 256;
      const int nchunk = std::max(1, std::min(kResChunks, 1024 / std::max(1, rb256 * batch)));
      const int chunk = (n + nchunk - 1) / nchunk;
      for (int cc = 0; cc < nrhs; ++cc) {
        hipLaunchKernelGGL(residual_part_kernel, dim3(rb256, nchunk, batch), dim3(256), 0, s, A, lda, strideA,
                           (const double*)X, ldx, strideX, n, cc, chunk, w.part, (const int*)w.active);
        hipLaunchKernelGGL(residual_finish_kernel, dim3(rb256, batch), dim3(256), 0, s, (const double*)X, ldx,
                           strideX, B, ldb, strideB, w.R, (int64_t)n, (int64_t)n * nrhs, n, cc, nrhs, nchunk,
                           (const double*)w.part, w.rnorm, w.xnorm, (const int*)w.active);
      }
    } else if (!chol) {
      hipLaunchKernelGGL(residual_kernel, dim3(trans ? (n + 15) / 16 : rblocks, batch), dim3(256), 0, s, A, lda, strideA, (const double*)X,
                         ldx, strideX, B, ldb, strideB, w.R, (int64_t)n, (int64_t)n * nrhs, n, nrhs, trans, w.rnorm,
                         w.xnorm, (const int*)w.active);
    } else if (batch == 1) {
      // symmetric: row parts over column chunks, the column part in the last slot, then the fixed-order sum
      const int rb256 = (n + 255) / 256;
      const int nchunk = std::max(1, std::min(kResChunks - 1, 1024 / std::max(1, rb256)));
      const int chunk = (n + nchunk - 1) / nchunk;
      for (int cc = 0; cc < nrhs; ++cc) {
        hipLaunchKernelGGL(residual_sym_row_kernel, dim3(rb256, nchunk), dim3(256), 0, s, A, lda, (const double*)X, ldx,
                           n, cc, chunk, w.part, (const int*)w.active);
        hipLaunchKernelGGL(residual_sym_col_kernel, dim3((n + 15) / 16), dim3(256), 0, s, A, lda, (const double*)X, ldx,
                           n, cc, w.part + (size_t)nchunk * n, (const int*)w.active);
        hipLaunchKernelGGL(residual_finish_kernel, dim3(rb256, 1), dim3(256), 0, s, (const double*)X, ldx, (int64_t)0,
                           B, ldb, (int64_t)0, w.R, (int64_t)n, (int64_t)n * nrhs, n, cc, nrhs, nchunk + 1,
                           (const double*)w.part, w.rnorm, w.xnorm, (const int*)w.active);
      }
    } else {
      hipLaunchKernelGGL(residual_sym_kernel, dim3(rblocks), dim3(256), 0, s, A, lda, (const double*)X, ldx, B, ldb,
                         w.R, (int64_t)n, n, nrhs, w.rnorm, w.xnorm, (const int*)w.active);
    }
    delete ks;
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(control_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, batch, nrhs, it, max_iter, prm.tol,
                       prm.success_tol, (const double*)w.anorm, w.rnorm, w.xnorm, w.st, res, w.active, info);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    if (it == max_iter) break;
    if (gm) {
      // the host decides whether another correction is needed (the GMRES solve is host-driven)
      int act = 0;
      if (hipMemcpyAsync(&act, w.active, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return CDS_HIP_ERROR;
      if (hipStreamSynchronize(s) != hipSuccess) return CDS_HIP_ERROR;
      if (!act) break;
      if (launch_fill_zero(gm->d, (size_t)n * 8, s) != hipSuccess) return CDS_HIP_ERROR;
      Ctx ck = c;
      ck.ws = gm->kws;
      ck.ws_bytes = gm->kbytes;
      st = krylov_run(ck, CDS_KRYLOV_GMRES, n, A, lda, w.R, gm->d, *gm->p, gm->kres, LU, perm);
      if (st != CDS_SUCCESS) return st;
      hipLaunchKernelGGL(add_inner_iters_kernel, dim3(1), dim3(1), 0, s, res, (const cds_krylov_result_t*)gm->kres, 0);
      hipLaunchKernelGGL(add_vec_kernel, dim3(std::min(1024, (n + 255) / 256)), dim3(256), 0, s, n,
                         (const double*)gm->d, X);
      if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
      continue;
    }
    // With host_check the host reads the stop flags of this step and leaves early.  The flags are
    // copied on the second stream after this step's control kernel, while the correction solve is
    // already queued on the first: the device runs the solve while the host waits, and a solve
    // queued after the last step finds no active system and returns at once.
    if (prm.host_check && hipEventRecord(c.ev[3], s) != hipSuccess) return CDS_HIP_ERROR;
    GetrsCore<float, double> d = g;
    d.B = w.R; d.ldb = n; d.strideB = (int64_t)n * nrhs;
    d.accumulate = 1;
    d.active = w.active;
    st = getrs_core<float, double>(c, d);
    if (st != CDS_SUCCESS) return st;
    if (prm.host_check) {
      h_active.resize(batch);
      if (hipStreamWaitEvent(c.s1, c.ev[3], 0) != hipSuccess) return CDS_HIP_ERROR;
      if (hipMemcpyAsync(h_active.data(), w.active, sizeof(int) * batch, hipMemcpyDeviceToHost, c.s1) != hipSuccess)
        return CDS_HIP_ERROR;
      if (hipStreamSynchronize(c.s1) != hipSuccess) return CDS_HIP_ERROR;
      bool any = false;
      for (int v : h_active) any = any || v;
      if (!any) break;
    }
  }
  return CDS_SUCCESS;
}

size_t gmres_ir_ws_bytes(int n, int nb, int restart) {
  const size_t kr = krylov_ws_bytes(CDS_KRYLOV_GMRES, n, restart, 1);
  const size_t corr = al256(kr) + al256((size_t)n * 8) + al256(sizeof(cds_krylov_result_t));
  return ir_ws_bytes(n, 1, 1, nb, 0, 0) + corr;
}

// GMRES-based refinement: the factorization of gesv_mixed_run, then corrections from GMRES
// left-preconditioned with the low-precision factors.
cds_status_t gesv_gmres_ir_run(Ctx& c, int prec, int n, const double* A, int64_t lda, const double* b, double* x,
                               float* LU, int32_t* ipiv, const cds_ir_params_t& prm, const cds_krylov_params_t& kp,
                               cds_ir_result_t* res, int nb) {
  if (n == 0) return CDS_SUCCESS;
  hipStream_t s = c.s0;
  const size_t kr = krylov_ws_bytes(CDS_KRYLOV_GMRES, n, kp.restart, 1);
  const size_t corr = al256(kr) + al256((size_t)n * 8) + al256(sizeof(cds_krylov_result_t));
  if (c.ws_bytes < corr + kErrRegion) return CDS_WORKSPACE_TOO_SMALL;
  // the correction solver's regions at the end of the workspace, the refinement's before them
  char* top = (char*)c.ws + c.ws_bytes - corr;
  top = (char*)((uintptr_t)top & ~(uintptr_t)255);
  GmresCorr gm;
  gm.p = &kp;
  gm.kws = top;
  gm.kbytes = kr;
  gm.d = (double*)(top + al256(kr));
  gm.kres = (cds_krylov_result_t*)(top + al256(kr) + al256((size_t)n * 8));
  const size_t lower = (size_t)(top - (char*)c.ws);
  IrWs w;
  if (!carve(c.ws, lower, n, 1, 1, 0, w)) return CDS_WORKSPACE_TOO_SMALL;
  if (launch_fill_zero(w.anorm, 8, s) != hipSuccess) return CDS_HIP_ERROR;
  hipLaunchKernelGGL(convert_kernel, dim3((n + 63) / 64, 1), dim3(256), 0, s, A, lda, (int64_t)0, LU, (int64_t)n,
                     (int64_t)0, n, w.anorm, 0, n);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  Ctx ci = c;
  ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
  cds_status_t st = getrf_run_mode<float>(ci, n, LU, n, 0, ipiv, 0, w.info, 1, nb, prec, w.scale, w.perm);
  if (st != CDS_SUCCESS) return st;
  hipLaunchKernelGGL(add_inner_iters_kernel, dim3(1), dim3(1), 0, s, res, (const cds_krylov_result_t*)nullptr, 1);
  return refine(ci, w, 0, 0, n, 1, A, lda, 0, LU, n, 0, w.perm, n, b, n, 0, x, n, 0, prm, res, w.info, 1, &gm);
}

// FP64 redo of the systems whose refinement did not converge (host decides).
static cds_status_t fallback_fp64(Ctx& c, const IrWs& w, int chol, int trans, int n, int nrhs, const double* A,
                                  int64_t lda, int64_t strideA, const double* B, int64_t ldb, int64_t strideB,
                                  double* X, int64_t ldx, int64_t strideX, cds_ir_result_t* res, int batch, int nb,
                                  double success_tol) {
  hipStream_t s = c.s0;
  std::vector<cds_ir_result_t> h(batch);
  if (hipMemcpyAsync(h.data(), res, sizeof(cds_ir_result_t) * batch, hipMemcpyDeviceToHost, s) != hipSuccess)
    return CDS_HIP_ERROR;
  if (hipStreamSynchronize(s) != hipSuccess) return CDS_HIP_ERROR;
  Ctx ci = c;
  ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
  for (int b = 0; b < batch; ++b) {
    if (h[b].converged) continue;
    double* Ab = w.fbA + (size_t)b * n * n;
    hipLaunchKernelGGL(copy_d_kernel, dim3(std::min(4096, (n * n + 255) / 256), 1), dim3(256), 0, s,
                       A + (size_t)b * strideA, lda, (int64_t)0, Ab, (int64_t)n, (int64_t)0, n, n);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(copy_d_kernel, dim3(std::min(4096, (n * nrhs + 255) / 256), 1), dim3(256), 0, s,
                       B + (size_t)b * strideB, ldb, (int64_t)0, X + (size_t)b * strideX, ldx, (int64_t)0, n, nrhs);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    cds_status_t st;
    if (!chol) {
      st = getrf_run<double>(ci, n, Ab, n, 0, w.fbpiv, 0, w.fbinfo, 1, nb);
      if (st != CDS_SUCCESS) return st;
      st = getrs_run<double>(ci, trans, n, nrhs, Ab, n, 0, w.fbpiv, 0, X + (size_t)b * strideX, ldx, 0, 1, ci.ws,
                             ci.ws_bytes);
    } else {
      st = potrf_run<double>(ci, n, Ab, n, w.fbinfo, nb);
      if (st != CDS_SUCCESS) return st;
      st = potrs_run<double>(ci, n, nrhs, Ab, n, X + (size_t)b * strideX, ldx, ci.ws, ci.ws_bytes);
    }
    if (st != CDS_SUCCESS) return st;
    // residual of the FP64 solution into the result struct
    if (launch_fill_zero(w.rnorm, (size_t)nrhs * 8, s) != hipSuccess) return CDS_HIP_ERROR;
    if (launch_fill_zero(w.xnorm, (size_t)nrhs * 8, s) != hipSuccess) return CDS_HIP_ERROR;
    if (!chol) {
      hipLaunchKernelGGL(residual_kernel, dim3(trans ? (n + 15) / 16 : (n + 63) / 64, 1), dim3(256), 0, s, A + (size_t)b * strideA, lda,
                         (int64_t)0, (const double*)(X + (size_t)b * strideX), ldx, (int64_t)0,
                         B + (size_t)b * strideB, ldb, (int64_t)0, w.R, (int64_t)n, (int64_t)0, n, nrhs, trans,
                         w.rnorm, w.xnorm, (const int*)nullptr);
    } else {
      hipLaunchKernelGGL(residual_sym_kernel, dim3((n + 63) / 64), dim3(256), 0, s, A, lda, (const double*)X, ldx, B,
                         ldb, w.R, (int64_t)n, n, nrhs, w.rnorm, w.xnorm, (const int*)nullptr);
    }
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(fallback_result_kernel, dim3(1), dim3(1), 0, s, nrhs, w.anorm + b, w.rnorm, w.xnorm, res + b,
                       (const int32_t*)w.fbinfo, success_tol);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  }
  return CDS_SUCCESS;
}

cds_status_t gesv_mixed_run(Ctx& c, int prec, int n, int nrhs, const double* A, int64_t lda, int64_t strideA,
                            const double* B, int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                            float* LU, int64_t strideLU, int32_t* ipiv, int64_t strideP, const cds_ir_params_t& prm,
                            cds_ir_result_t* res, int batch, int nb) {
  if (batch == 0 || n == 0 || nrhs == 0) return CDS_SUCCESS;
  hipStream_t s = c.s0;
  IrWs w;
  if (!carve(c.ws, c.ws_bytes, n, nrhs, batch, prm.fallback, w, nrhs == 1)) return CDS_WORKSPACE_TOO_SMALL;
  if (launch_fill_zero(w.anorm, batch * 8, s) != hipSuccess) return CDS_HIP_ERROR;
  // With the look-ahead, the first 1024 columns (at least the first two panels', a panel being at
  // most 512 wide) are converted first and the rest (with ||A||_inf) on the second stream, beside
  // the first panel: the factorization's later work on the first stream follows the second
  // stream's, and the second stream's own work follows it in order.  n > 1024 implies the
  // factorization takes the look-ahead schedule.
  const int c1 = std::min(n, 1024);
  const bool split = c.lookahead && batch == 1 && n > c1;
  if (split) {
    hipLaunchKernelGGL(convert_kernel, dim3((n + 63) / 64, 1), dim3(256), 0, s, A, lda, strideA, LU, (int64_t)n,
                       strideLU, n, (double*)nullptr, 0, c1);
    if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
    if (hipEventRecord(c.ev[3], s) != hipSuccess) return CDS_HIP_ERROR;
    if (hipStreamWaitEvent(c.s1, c.ev[3], 0) != hipSuccess) return CDS_HIP_ERROR;
    hipLaunchKernelGGL(convert_kernel, dim3((n + 63) / 64, 1), dim3(256), 0, c.s1, A, lda, strideA, LU, (int64_t)n,
                       strideLU, n, w.anorm, c1, n);
  } else {
    hipLaunchKernelGGL(convert_kernel, dim3((n + 63) / 64, batch), dim3(256), 0, s, A, lda, strideA, LU, (int64_t)n,
                       strideLU, n, w.anorm, 0, n);
  }
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  Ctx ci = c;
  ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
  cds_status_t st = getrf_run_mode<float>(ci, n, LU, n, strideLU, ipiv, strideP, w.info, batch, nb, prec, w.scale,
                                          w.perm);
  if (st != CDS_SUCCESS) return st;
  if (w.binv) {
    KScope kb(c.timer, CDS_KC_TRSV, s, 0.0, 0.0);
    if (launch_binv_prep(LU, n, strideLU, n, w.binv, (int64_t)binv_elems(n), batch, s) != hipSuccess)
      return CDS_HIP_ERROR;
  }
  st = refine(ci, w, 0, 0, n, nrhs, A, lda, strideA, LU, n, strideLU, w.perm, n, B, ldb, strideB, X, ldx, strideX,
              prm, res, w.info, batch);
  if (st != CDS_SUCCESS) return st;
  if (prm.fallback) return fallback_fp64(c, w, 0, 0, n, nrhs, A, lda, strideA, B, ldb, strideB, X, ldx, strideX, res,
                                         batch, nb, prm.success_tol);
  return CDS_SUCCESS;
}

cds_status_t getrs_mixed_run(Ctx& c, int trans, int n, int nrhs, const double* A, int64_t lda, int64_t strideA,
                             const float* LU, int64_t strideLU, const int32_t* ipiv, int64_t strideP, const double* B,
                             int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                             const cds_ir_params_t& prm, cds_ir_result_t* res, int batch) {
  if (batch == 0 || n == 0 || nrhs == 0) return CDS_SUCCESS;
  hipStream_t s = c.s0;
  IrWs w;
  if (!carve(c.ws, c.ws_bytes, n, nrhs, batch, 0, w)) return CDS_WORKSPACE_TOO_SMALL;
  if (launch_fill_zero(w.anorm, batch * 8, s) != hipSuccess) return CDS_HIP_ERROR;
  // ||op(A)||_inf: for A^T that is the largest column sum of |A|
  if (!trans) {
    hipLaunchKernelGGL(rownorm_kernel, dim3((n + 63) / 64, batch), dim3(256), 0, s, A, lda, strideA, n, w.anorm);
  } else {
    hipLaunchKernelGGL(colnorm_kernel, dim3((n + 3) / 4, batch), dim3(256), 0, s, A, lda, strideA, n, w.anorm);
  }
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  if (launch_fill_i32(w.info, batch, 0, s) != hipSuccess) return CDS_HIP_ERROR;
  if (launch_perm(ipiv, strideP, n, w.perm, n, w.gmap, batch, s) != hipSuccess) return CDS_HIP_ERROR;
  Ctx ci = c;
  ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
  return refine(ci, w, trans, 0, n, nrhs, A, lda, strideA, LU, n, strideLU, w.perm, n, B, ldb, strideB, X, ldx,
                strideX, prm, res, w.info, batch);
}

cds_status_t posv_mixed_run(Ctx& c, int prec, int n, int nrhs, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* X, int64_t ldx, float* L, const cds_ir_params_t& prm,
                            cds_ir_result_t* res, int nb) {
  if (n == 0 || nrhs == 0) return CDS_SUCCESS;
  hipStream_t s = c.s0;
  IrWs w;
  if (!carve(c.ws, c.ws_bytes, n, nrhs, 1, prm.fallback, w)) return CDS_WORKSPACE_TOO_SMALL;
  if (launch_fill_zero(w.anorm, 8, s) != hipSuccess) return CDS_HIP_ERROR;
  // lower triangle to FP32 and the norm of the symmetric matrix
  hipLaunchKernelGGL(sym_colabs_kernel, dim3((n + 15) / 16), dim3(256), 0, s, A, lda, n, w.part);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  hipLaunchKernelGGL(convert_sym_kernel, dim3((n + 63) / 64, 1), dim3(256), 0, s, A, lda, L, (int64_t)n, n,
                     (const double*)w.part, w.anorm);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  Ctx ci = c;
  ci.ws = w.inner; ci.ws_bytes = w.inner_bytes;
  cds_status_t st = potrf_run_mode<float>(ci, n, L, n, w.info, nb, prec, w.scale);
  if (st != CDS_SUCCESS) return st;
  st = refine(ci, w, 0, 1, n, nrhs, A, lda, 0, L, n, 0, nullptr, 0, B, ldb, 0, X, ldx, 0, prm, res, w.info, 1);
  if (st != CDS_SUCCESS) return st;
  if (prm.fallback) return fallback_fp64(c, w, 1, 0, n, nrhs, A, lda, 0, B, ldb, 0, X, ldx, 0, res, 1, nb, prm.success_tol);
  return CDS_SUCCESS;
}

}  // namespace cds
