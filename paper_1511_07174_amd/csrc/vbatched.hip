// Many SPD systems of uneven size in one persistent launch (Cholesky, Sec. 2,
// applied to a batch): each workgroup takes systems from a ticket counter
// (largest first when the caller passes that order), converts the lower
// triangle of A to FP32 in its own scratch matrix, factors it with a blocked
// left-looking Cholesky (only the current block column is written, the left
// part is read once per block column), solves in FP32 and refines the solution
// with an FP64 residual, all inside the workgroup.  No grid-wide
// synchronisation, no host interaction: the launch can be captured in a graph.
#include "common.hpp"
#include "kernels.hpp"
#include "vbatched.hpp"
#include <algorithm>

namespace cds {

namespace {

constexpr int VNT = 256;
constexpr int VNMAX = 1024;
constexpr int VNR = 4;      // right-hand sides handled per pass

struct VbArgs {
  int batch, nmax, nrhs;
  const int32_t* n;
  const double* const* A; const int64_t* lda;
  const double* const* B; const int64_t* ldb;
  double* const* X; const int64_t* ldx;
  const int32_t* order;
  float* ws;
  int* ticket;
  cds_ir_result_t* res;
  uint64_t* t_start; uint64_t* t_end;
  double tol, success_tol;
  int max_iter;
  int jw16_max_n;   // systems with n <= this use 16-wide block columns, larger ones 32
};

struct VbShared {
  float ys[VNMAX][VNR];
  double xs[VNMAX][VNR];
  double rs[VNMAX][VNR];
  float Ld[32][33];
  float Lrow[64][33];   // [k][column of the block]
  double red[4][VNR];
  double anorm;
  int info;
  int ticket;
};

// ||A||_inf of the symmetric matrix held in the lower triangle, and W = fp32(lower(A)).
__device__ void vb_convert(const double* A, int64_t lda, float* W, int n, VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // lower parts: thread per row; column parts below the diagonal: wave per column
  for (int i = tid; i < n; i += VNT) {
    double s = 0.0;
    for (int j = 0; j <= i; ++j) {
      const double v = A[i + (size_t)j * lda];
      W[i + (size_t)j * n] = (float)v;
      s += fabs(v);
    }
    sh.rs[i][0] = s;
  }
  __syncthreads();
  for (int j = wave; j < n; j += 4) {
    double s = 0.0;
    for (int i = j + 1 + lane; i < n; i += 64) s += fabs(A[i + (size_t)j * lda]);
    s = wave_sum(s);
    if (lane == 0) sh.rs[j][0] += s;
  }
  __syncthreads();
  double m = 0.0;
  for (int i = tid; i < n; i += VNT) m = fmax(m, sh.rs[i][0]);
  m = wave_max(m);
  if (lane == 0) sh.red[wave][0] = m;
  __syncthreads();
  if (tid == 0) sh.anorm = fmax(fmax(sh.red[0][0], sh.red[1][0]), fmax(sh.red[2][0], sh.red[3][0]));
  __syncthreads();
}

// Left-looking blocked Cholesky of W (n x n, ld n, lower).  Returns info via sh.info.
template <int JW>
__device__ void vb_potrf(float* W, int n, VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) sh.info = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += JW) {
    const int jw = min(JW, n - j0);
    // rows of this block column, one row per thread, in chunks of VNT rows
    for (int r0 = j0; r0 < n; r0 += VNT) {
      const int r = r0 + tid;
      float acc[JW];
#pragma unroll
      for (int c = 0; c < JW; ++c) acc[c] = (r < n && c < jw && r >= j0 + c) ? W[r + (size_t)(j0 + c) * n] : 0.f;
      // acc -= L[r, 0:j0] * L[j0:j0+jw, 0:j0]^T, k in slabs of 64 staged in LDS
      for (int k0 = 0; k0 < j0; k0 += 64) {
        const int kw = min(64, j0 - k0);
        __syncthreads();
        for (int idx = tid; idx < jw * kw; idx += VNT) {
          const int c = idx % jw, kk = idx / jw;
          sh.Lrow[kk][c] = W[(j0 + c) + (size_t)(k0 + kk) * n];
        }
        __syncthreads();
        if (r < n) {
          for (int kk = 0; kk < kw; ++kk) {
            const float a = W[r + (size_t)(k0 + kk) * n];
#pragma unroll
            for (int c = 0; c < JW; ++c) acc[c] -= a * sh.Lrow[kk][c];
          }
        }
      }
      if (r0 == j0) {
        // factor the diagonal block in LDS (rows j0..j0+jw belong to this first chunk)
        if (tid < jw) {
#pragma unroll
          for (int c = 0; c < JW; ++c)
            if (c < jw) sh.Ld[tid][c] = acc[c];
        }
        __syncthreads();
        if (wave == 0) {
          int fail = 0;
          for (int j = 0; j < jw; ++j) {
            const float d = sh.Ld[j][j];
            if (!(d > 0.f)) { fail = j + 1; break; }
            const float ljj = sqrtf(d);
            wave_fence();
            if (lane == j) sh.Ld[j][j] = ljj;
            if (lane > j && lane < jw) sh.Ld[lane][j] = sh.Ld[lane][j] / ljj;
            wave_fence();
            if (lane > j && lane < jw) {
              const float lrj = sh.Ld[lane][j];
              for (int c = j + 1; c <= lane; ++c) sh.Ld[lane][c] -= lrj * sh.Ld[c][j];
            }
            wave_fence();
          }
          if (lane == 0 && fail) sh.info = j0 + fail;
        }
        __syncthreads();
        if (sh.info != 0) return;
        if (tid < jw) {
#pragma unroll
          for (int c = 0; c < JW; ++c)
            if (c <= tid && c < jw) W[(j0 + tid) + (size_t)(j0 + c) * n] = sh.Ld[tid][c];
        }
      }
      // rows below the diagonal block: x L_dd^T = acc
      if (r < n && r >= j0 + jw) {
#pragma unroll
        for (int c = 0; c < JW; ++c) {
          if (c < jw) {
            float v = acc[c];
#pragma unroll
            for (int t = 0; t < c; ++t) v -= acc[t] * sh.Ld[c][t];
            acc[c] = v / sh.Ld[c][c];
          }
        }
#pragma unroll
        for (int c = 0; c < JW; ++c)
          if (c < jw) W[r + (size_t)(j0 + c) * n] = acc[c];
      }
    }
    __syncthreads();
  }
}

// ys <- L^{-T} L^{-1} ys (FP32, nr right-hand sides), L = lower(W).
template <int JB>
__device__ void vb_potrs(const float* W, int n, int nr, VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // forward: L y = b
  for (int j0 = 0; j0 < n; j0 += JB) {
    const int jw = min(JB, n - j0);
    for (int idx = tid; idx < jw * jw; idx += VNT) {
      const int i = idx % jw, c = idx / jw;
      if (i >= c) sh.Ld[i][c] = W[(j0 + i) + (size_t)(j0 + c) * n];
    }
    __syncthreads();
    if (wave == 0) {
      for (int r = 0; r < nr; ++r) {
        float v = lane < jw ? sh.ys[j0 + lane][r] : 0.f;
        for (int t = 0; t < jw; ++t) {
          float xt = __shfl(v, t) / sh.Ld[t][t];
          if (lane == t) v = xt;
          if (lane > t && lane < jw) v -= sh.Ld[lane][t] * xt;
        }
        if (lane < jw) sh.ys[j0 + lane][r] = v;
      }
    }
    __syncthreads();
    for (int i = j0 + jw + tid; i < n; i += VNT) {
      float v[VNR];
#pragma unroll
      for (int r = 0; r < VNR; ++r) v[r] = sh.ys[i][r];
      for (int t = 0; t < jw; ++t) {
        const float l = W[i + (size_t)(j0 + t) * n];
#pragma unroll
        for (int r = 0; r < VNR; ++r) v[r] -= l * sh.ys[j0 + t][r];
      }
#pragma unroll
      for (int r = 0; r < VNR; ++r) sh.ys[i][r] = v[r];
    }
    __syncthreads();
  }
  // backward: L^T x = y
  const int nblk = (n + JB - 1) / JB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int j0 = bk * JB, jw = min(JB, n - j0);
    // s_r = sum_{c >= j0+jw} L[c, r] x_c for r in the block: wave per row
    for (int rr = wave; rr < jw; rr += 4) {
      const int r = j0 + rr;
      float s[VNR] = {0.f, 0.f, 0.f, 0.f};
      for (int c = j0 + jw + lane; c < n; c += 64) {
        const float l = W[c + (size_t)r * n];
#pragma unroll
        for (int q = 0; q < VNR; ++q) s[q] += l * sh.ys[c][q];
      }
#pragma unroll
      for (int q = 0; q < VNR; ++q) s[q] = wave_sum(s[q]);
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < VNR; ++q) sh.rs[r][q] = (double)s[q];
    }
    for (int idx = tid; idx < jw * jw; idx += VNT) {
      const int i = idx % jw, c = idx / jw;
      if (i >= c) sh.Ld[i][c] = W[(j0 + i) + (size_t)(j0 + c) * n];
    }
    __syncthreads();
    if (wave == 0) {
      for (int r = 0; r < nr; ++r) {
        float v = lane < jw ? sh.ys[j0 + lane][r] - (float)sh.rs[j0 + lane][r] : 0.f;
        for (int t = jw - 1; t >= 0; --t) {
          float xt = __shfl(v, t) / sh.Ld[t][t];
          if (lane == t) v = xt;
          if (lane < t) v -= sh.Ld[t][lane] * xt;
        }
        if (lane < jw) sh.ys[j0 + lane][r] = v;
      }
    }
    __syncthreads();
  }
}

// rs = B - A xs (FP64, A symmetric in its lower triangle); returns max_c ||r_c|| / (||A|| ||x_c||) in sh.red
__device__ double vb_residual(const double* A, int64_t lda, const double* B, int64_t ldb, int n, int nr,
                              VbShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // column parts first (wave per row): sum_{c > i} A[c, i] x_c
  for (int i = wave; i < n; i += 4) {
    double s[VNR] = {0.0, 0.0, 0.0, 0.0};
    for (int c = i + 1 + lane; c < n; c += 64) {
      const double a = A[c + (size_t)i * lda];
#pragma unroll
      for (int q = 0; q < VNR; ++q) s[q] = fma(a, sh.xs[c][q], s[q]);
    }
#pragma unroll
    for (int q = 0; q < VNR; ++q) s[q] = wave_sum(s[q]);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < VNR; ++q) sh.rs[i][q] = s[q];
  }
  __syncthreads();
  double rmax[VNR] = {0.0, 0.0, 0.0, 0.0}, xmax[VNR] = {0.0, 0.0, 0.0, 0.0};
  for (int i = tid; i < n; i += VNT) {
    double s[VNR];
#pragma unroll
    for (int q = 0; q < VNR; ++q) s[q] = sh.rs[i][q];
    for (int j = 0; j <= i; ++j) {
      const double a = A[i + (size_t)j * lda];
#pragma unroll
      for (int q = 0; q < VNR; ++q) s[q] = fma(a, sh.xs[j][q], s[q]);
    }
#pragma unroll
    for (int q = 0; q < VNR; ++q) {
      if (q < nr) {
        const double r = B[i + (size_t)q * ldb] - s[q];
        sh.rs[i][q] = r;
        rmax[q] = fmax(rmax[q], fabs(r));
        xmax[q] = fmax(xmax[q], fabs(sh.xs[i][q]));
      }
    }
  }
  __syncthreads();
  double eta = 0.0;
#pragma unroll
  for (int q = 0; q < VNR; ++q) {
    double rm = wave_max(rmax[q]), xm = wave_max(xmax[q]);
    if (lane == 0) { sh.red[wave][q] = rm; }
    __syncthreads();
    if (tid == 0) {
      double a = fmax(fmax(sh.red[0][q], sh.red[1][q]), fmax(sh.red[2][q], sh.red[3][q]));
      sh.red[0][q] = a;
    }
    __syncthreads();
    const double rr = sh.red[0][q];
    __syncthreads();
    if (lane == 0) sh.red[wave][q] = xm;
    __syncthreads();
    const double xx = fmax(fmax(sh.red[0][q], sh.red[1][q]), fmax(sh.red[2][q], sh.red[3][q]));
    __syncthreads();
    if (q < nr) {
      double e = rr == 0.0 ? 0.0 : (sh.anorm * xx > 0.0 ? rr / (sh.anorm * xx) : INFINITY);
      if (!(e <= eta)) eta = e;
    }
  }
  return eta;
}

template <int JW>
__device__ void vb_system(const VbArgs& a, int sys, float* W, VbShared& sh) {
  const int tid = threadIdx.x;
  const int n = a.n[sys];
  const double* A = a.A[sys];
  const int64_t lda = a.lda[sys];
  cds_ir_result_t* res = a.res + sys;
  if (tid == 0 && a.t_start) a.t_start[sys] = wall_clock64();
  vb_convert(A, lda, W, n, sh);
  vb_potrf<JW>(W, n, sh);
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
    for (int i = tid; i < n; i += VNT)
#pragma unroll
      for (int q = 0; q < VNR; ++q) sh.ys[i][q] = q < nr ? (float)B[i + (size_t)q * ldb] : 0.f;
    __syncthreads();
    vb_potrs<32>(W, n, nr, sh);
    for (int i = tid; i < n; i += VNT)
#pragma unroll
      for (int q = 0; q < VNR; ++q) sh.xs[i][q] = (double)sh.ys[i][q];
    __syncthreads();
    double eta_prev = INFINITY, eta_prev2 = INFINITY;
    int it = 0, reason = 0;
    double eta = 0.0;
    for (it = 0;; ++it) {
      eta = vb_residual(A, lda, B, ldb, n, nr, sh);
      if (it == 0 && c0 == 0) first_eta = eta;
      if (!(eta == eta) || eta == INFINITY) reason = 4;
      else if (eta <= a.tol) reason = 1;
      else if (it >= 2 && eta > 0.5 * eta_prev && eta_prev > 0.5 * eta_prev2) reason = 2;
      else if (it >= a.max_iter) reason = 3;
      if (reason) break;
      eta_prev2 = eta_prev;
      eta_prev = eta;
      for (int i = tid; i < n; i += VNT)
#pragma unroll
        for (int q = 0; q < VNR; ++q) sh.ys[i][q] = (float)sh.rs[i][q];
      __syncthreads();
      vb_potrs<32>(W, n, nr, sh);
      for (int i = tid; i < n; i += VNT)
#pragma unroll
        for (int q = 0; q < VNR; ++q) sh.xs[i][q] += (double)sh.ys[i][q];
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

__global__ void __launch_bounds__(VNT) vbatched_kernel(VbArgs a) {
  __shared__ VbShared sh;
  float* W = a.ws + (size_t)blockIdx.x * a.nmax * a.nmax;
  while (true) {
    if (threadIdx.x == 0) sh.ticket = atomicAdd(a.ticket, 1);
    __syncthreads();
    const int t = sh.ticket;
    __syncthreads();
    if (t >= a.batch) break;
    const int sys = a.order ? a.order[t] : t;
    if (sys < 0 || sys >= a.batch) continue;
    const int n = a.n[sys];
    if (n < 1 || n > a.nmax) {
      // invalid size: report and skip (no memory outside the scratch matrix is touched)
      if (threadIdx.x == 0) {
        cds_ir_result_t* r = a.res + sys;
        r->info = -1; r->converged = 0; r->fell_back = 0; r->iters = 0;
        r->eta = INFINITY; r->eta0 = INFINITY; r->stop_reason = 5; r->reserved = 0;
      }
      continue;
    }
    if (n <= a.jw16_max_n) vb_system<16>(a, sys, W, sh);
    else vb_system<32>(a, sys, W, sh);
  }
}

__global__ void reset_kernel(int* p) { *p = 0; }

}  // namespace

int vbatched_grid() { return 256; }

size_t vbatched_ws_bytes(int batch, int nmax, int nrhs) {
  (void)batch; (void)nrhs;
  return kErrRegion + 256 + (size_t)vbatched_grid() * nmax * nmax * sizeof(float);
}

cds_status_t vbatched_run(Ctx& c, int batch, int nmax, const int32_t* n, const double* const* A, const int64_t* lda,
                          const double* const* B, const int64_t* ldb, double* const* X, const int64_t* ldx, int nrhs,
                          const int32_t* order, const cds_ir_params_t& prm, cds_ir_result_t* res, uint64_t* t_start,
                          uint64_t* t_end, int jw16_max_n) {
  if (batch == 0) return CDS_SUCCESS;
  if (nmax > VNMAX) return CDS_UNSUPPORTED;
  if (c.ws_bytes < vbatched_ws_bytes(batch, nmax, nrhs)) return CDS_WORKSPACE_TOO_SMALL;
  char* base = (char*)c.ws + kErrRegion;
  int* ticket = (int*)base;
  float* ws = (float*)(base + 256);
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(1), 0, c.s0, ticket);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  VbArgs a;
  a.batch = batch; a.nmax = nmax; a.nrhs = nrhs;
  a.n = n; a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.X = X; a.ldx = ldx; a.order = order;
  a.ws = ws; a.ticket = ticket; a.res = res; a.t_start = t_start; a.t_end = t_end;
  a.tol = prm.tol; a.success_tol = prm.success_tol; a.max_iter = prm.max_iter;
  a.jw16_max_n = jw16_max_n;
  hipLaunchKernelGGL(vbatched_kernel, dim3(std::min(vbatched_grid(), batch)), dim3(VNT), 0, c.s0, a);
  if (hipGetLastError() != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

}  // namespace cds
