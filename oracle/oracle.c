/*
 * Plain CPU FP64 oracle for the direct solvers of Oancea & Andrei,
 * "Developing a High Performance Software Library with MPI and CUDA for
 * Matrix Computations" (arXiv 1511.07174).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Sec. 2 of the paper, on the serial iterative and direct
 * methods): the direct method for Ax = b in two steps, (1) factor A = LU with
 * L unit lower triangular and partial pivoting (the textbook algorithm the
 * paper cites from Golub & Van Loan), or A = L L^T for SPD A, then (2) the two
 * triangular solves Ly = b and Ux = y.  Blocked right-looking LU (delayed
 * updating, Sec. 2 last paragraph) is a reordering of exactly these
 * operations, so the oracle is the unblocked definition, one column at a time.
 *
 * Conventions (readings where the paper is silent): column-major storage with
 * a leading dimension; pivots 1-based with sequential-interchange semantics;
 * ties in the pivot search go to the lowest row index; a zero pivot records
 * info = k+1 (1-based) and elimination continues without dividing; Cholesky
 * uses and writes only the lower triangle and stops at the first non-positive
 * (or NaN) pivot.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction,
 * so every product and sum is rounded exactly as written; the only explicit
 * fma() calls are the error-free transformations of the double-double
 * residual).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(M, ld, i, j) (M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)]

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Gaussian elimination with partial pivoting, outer-product (kji) form
 * (Sec. 2: the first step of the direct method, A = LU with unit-diagonal L).
 * For k = 0..n-1:
 *   mu = argmax_{i >= k} |a_ik|   (lowest i on ties);  ipiv[k] = mu + 1;
 *   swap whole rows k and mu (all n columns);
 *   if a_kk != 0: a_ik /= a_kk (i > k), then a_ij -= a_ik * a_kj (i, j > k);
 *   else: info = k + 1 if still 0, and go on.
 * On return A holds L (strictly below the diagonal) and U (on and above).
 * Returns info.
 */
int64_t oracle_dgetrf(int64_t n, double* A, int64_t lda, int32_t* ipiv) {
  int64_t info = 0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t mu = k;
    double best = fabs(AT(A, lda, k, k));
    for (int64_t i = k + 1; i < n; ++i) {
      double v = fabs(AT(A, lda, i, k));
      if (v > best) { best = v; mu = i; }   /* strict '>' keeps the lowest index on ties */
    }
    ipiv[k] = (int32_t)(mu + 1);
    if (mu != k) {
      for (int64_t j = 0; j < n; ++j) {
        double t = AT(A, lda, k, j);
        AT(A, lda, k, j) = AT(A, lda, mu, j);
        AT(A, lda, mu, j) = t;
      }
    }
    double piv = AT(A, lda, k, k);
    if (piv != 0.0) {
      for (int64_t i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / piv;
      /* rank-1 update of the trailing matrix; columns are independent */
#pragma omp parallel for schedule(static) if (n - k > 256)
      for (int64_t j = k + 1; j < n; ++j) {
        double ukj = AT(A, lda, k, j);
        if (ukj != 0.0) {
          for (int64_t i = k + 1; i < n; ++i) {
            double prod = AT(A, lda, i, k) * ukj;
            AT(A, lda, i, j) = AT(A, lda, i, j) - prod;
          }
        }
      }
    } else if (info == 0) {
      info = k + 1;
    }
  }
  return info;
}

/*
 * The same elimination carried out in single precision (the paper runs its
 * solvers in single as well as double precision, Sec. 4).  Every stored value,
 * product and difference is a float, so the pivot decisions are taken in FP32,
 * the precision of the FP32 factorization it is compared with.  Same steps and
 * conventions as oracle_dgetrf.  Returns info.
 */
int64_t oracle_sgetrf(int64_t n, float* A, int64_t lda, int32_t* ipiv) {
  int64_t info = 0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t mu = k;
    float best = fabsf(AT(A, lda, k, k));
    for (int64_t i = k + 1; i < n; ++i) {
      float v = fabsf(AT(A, lda, i, k));
      if (v > best) { best = v; mu = i; }
    }
    ipiv[k] = (int32_t)(mu + 1);
    if (mu != k) {
      for (int64_t j = 0; j < n; ++j) {
        float t = AT(A, lda, k, j);
        AT(A, lda, k, j) = AT(A, lda, mu, j);
        AT(A, lda, mu, j) = t;
      }
    }
    float piv = AT(A, lda, k, k);
    if (piv != 0.0f) {
      for (int64_t i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / piv;
#pragma omp parallel for schedule(static) if (n - k > 256)
      for (int64_t j = k + 1; j < n; ++j) {
        float ukj = AT(A, lda, k, j);
        if (ukj != 0.0f) {
          for (int64_t i = k + 1; i < n; ++i) {
            float prod = AT(A, lda, i, k) * ukj;
            AT(A, lda, i, j) = AT(A, lda, i, j) - prod;
          }
        }
      }
    } else if (info == 0) {
      info = k + 1;
    }
  }
  return info;
}

/*
 * Second step of the direct method (Sec. 2): with P A = L U,
 *   trans = 0: solve A X = B:   apply the interchanges to B in order k = 0..n-1,
 *              forward substitution L Y = P B (unit diagonal), back substitution U X = Y.
 *   trans = 1: solve A^T X = B: U^T Z = B (forward), L^T W = Z (backward, unit),
 *              then undo the interchanges in reverse order k = n-1..0.
 * B (n x nrhs, leading dimension ldb) is overwritten with X.
 */
void oracle_dgetrs(int trans, int64_t n, int64_t nrhs, const double* LU, int64_t lda,
                   const int32_t* ipiv, double* B, int64_t ldb) {
  /* right-hand sides are independent: one thread per column, each solved in the order below */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nrhs; ++c) {
    double* b = B + (size_t)c * (size_t)ldb;
    if (!trans) {
      for (int64_t k = 0; k < n; ++k) {
        int64_t p = ipiv[k] - 1;
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
      }
      for (int64_t i = 0; i < n; ++i) {        /* L y = Pb, unit diagonal */
        double s = b[i];
        for (int64_t j = 0; j < i; ++j) s = s - AT(LU, lda, i, j) * b[j];
        b[i] = s;
      }
      for (int64_t i = n - 1; i >= 0; --i) {   /* U x = y */
        double s = b[i];
        for (int64_t j = i + 1; j < n; ++j) s = s - AT(LU, lda, i, j) * b[j];
        b[i] = s / AT(LU, lda, i, i);
      }
    } else {
      for (int64_t i = 0; i < n; ++i) {        /* U^T z = b */
        double s = b[i];
        for (int64_t j = 0; j < i; ++j) s = s - AT(LU, lda, j, i) * b[j];
        b[i] = s / AT(LU, lda, i, i);
      }
      for (int64_t i = n - 1; i >= 0; --i) {   /* L^T w = z, unit diagonal */
        double s = b[i];
        for (int64_t j = i + 1; j < n; ++j) s = s - AT(LU, lda, j, i) * b[j];
        b[i] = s;
      }
      for (int64_t k = n - 1; k >= 0; --k) {   /* x = P^T w */
        int64_t p = ipiv[k] - 1;
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
      }
    }
  }
}

/*
 * Cholesky A = L L^T of an SPD matrix (Sec. 2: the symmetric positive
 * definite case of the direct method), lower triangle, column (gaxpy / jki)
 * form:
 *   s = a_jj - sum_{k<j} l_jk^2;  if !(s > 0): info = j + 1, stop;
 *   l_jj = sqrt(s);  l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj  (i > j).
 * Every sum runs over k = 0, 1, ..., j-1 in that order.  The rows i > j are
 * taken in chunks, and inside a chunk the loop over k is the outer one, so the
 * columns of L are read contiguously; each row still subtracts its terms in
 * the order k = 0..j-1, so the rounding is that of the formula as written.
 * Reads and writes the lower triangle only.  Returns info.
 */
int64_t oracle_dpotrf(int64_t n, double* A, int64_t lda) {
  enum { CH = 256 };
  for (int64_t j = 0; j < n; ++j) {
    double s = AT(A, lda, j, j);
    for (int64_t k = 0; k < j; ++k) s = s - AT(A, lda, j, k) * AT(A, lda, j, k);
    if (!(s > 0.0)) return j + 1;
    double ljj = sqrt(s);
    AT(A, lda, j, j) = ljj;
    const int64_t nch = (n - j - 1 + CH - 1) / CH;
#pragma omp parallel for schedule(static) if (n - j > 512)
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t i0 = j + 1 + c * CH;
      const int64_t i1 = i0 + CH < n ? i0 + CH : n;
      double t[CH];
      for (int64_t i = i0; i < i1; ++i) t[i - i0] = AT(A, lda, i, j);
      for (int64_t k = 0; k < j; ++k) {
        const double ljk = AT(A, lda, j, k);
        const double* col = &AT(A, lda, 0, k);
        for (int64_t i = i0; i < i1; ++i) t[i - i0] = t[i - i0] - col[i] * ljk;
      }
      for (int64_t i = i0; i < i1; ++i) AT(A, lda, i, j) = t[i - i0] / ljj;
    }
  }
  return 0;
}

/* Solve A X = B with A = L L^T: L Y = B (forward), L^T X = Y (backward). */
void oracle_dpotrs(int64_t n, int64_t nrhs, const double* L, int64_t lda, double* B, int64_t ldb) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nrhs; ++c) {
    double* b = B + (size_t)c * (size_t)ldb;
    for (int64_t i = 0; i < n; ++i) {
      double s = b[i];
      for (int64_t j = 0; j < i; ++j) s = s - AT(L, lda, i, j) * b[j];
      b[i] = s / AT(L, lda, i, i);
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = b[i];
      for (int64_t j = i + 1; j < n; ++j) s = s - AT(L, lda, j, i) * b[j];
      b[i] = s / AT(L, lda, i, i);
    }
  }
}

/* Error-free transformations (Knuth TwoSum; TwoProduct through one fma). */
static inline void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double bb = x - a;
  *e = (a - (x - bb)) + (b - bb);
  *s = x;
}
static inline void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}
/* (hi, lo) += v, double-double accumulation */
static inline void dd_add(double* hi, double* lo, double v) {
  double s, e;
  two_sum(*hi, v, &s, &e);
  e = e + *lo;
  double h2, l2;
  two_sum(s, e, &h2, &l2);
  *hi = h2;
  *lo = l2;
}

/*
 * Residual R = B - op(A) X accumulated in double-double and rounded once, so
 * that the reported backward error is that of X itself, not of the residual
 * computation.  trans = 0 uses A, trans = 1 uses A^T.
 */
void oracle_residual_dd(int trans, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                        const double* X, int64_t ldx, const double* B, int64_t ldb,
                        double* R, int64_t ldr) {
  for (int64_t c = 0; c < nrhs; ++c) {
    const double* x = X + (size_t)c * (size_t)ldx;
    const double* b = B + (size_t)c * (size_t)ldb;
    double* r = R + (size_t)c * (size_t)ldr;
#pragma omp parallel for schedule(static) if (n > 256)
    for (int64_t i = 0; i < n; ++i) {
      double hi = b[i], lo = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        double a = trans ? AT(A, lda, j, i) : AT(A, lda, i, j);
        double p, e;
        two_prod(a, x[j], &p, &e);
        dd_add(&hi, &lo, -p);
        dd_add(&hi, &lo, -e);
      }
      r[i] = hi + lo;
    }
  }
}

/* ||A||_inf = max_i sum_j |a_ij| (rows of an n x m column-major matrix). */
double oracle_norm_inf(int64_t n, int64_t m, const double* A, int64_t lda) {
  double best = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) s = s + fabs(AT(A, lda, i, j));
    if (s > best || s != s) best = s;
  }
  return best;
}
