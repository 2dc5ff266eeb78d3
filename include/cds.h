/*
 * cds.h — C-ABI of the dense direct solvers for one AMD MI355X (gfx950).
 *
 * The operations follow the direct method of Oancea & Andrei, "Developing a
 * High Performance Software Library with MPI and CUDA for Matrix
 * Computations" (arXiv 1511.07174), Sec. 2: solve Ax = b by (1) factoring
 * A = LU, L unit lower triangular, with partial pivoting (A = L L^T for SPD A),
 * computed blockwise by delayed (rank-k) updates, then (2) the triangular
 * solves Ly = b and Ux = y.  The library keeps the paper's goal of a simple
 * interface behind an opaque object (Sec. 3) and LAPACK's naming and argument
 * order (the paper names LAPACK the de-facto standard, Sec. 3).
 *
 * Conventions for every call below:
 *  - Matrices are column-major with a leading dimension (ld >= max(1, rows)).
 *  - Every matrix and vector pointer is a DEVICE pointer unless its name
 *    starts with h_ or it is a parameter struct.  The caller allocates and
 *    frees all of them; the library never allocates device memory.
 *  - Calls only enqueue work on the handle's stream (asynchronous; no host
 *    synchronisation, no host<->device copies) unless documented otherwise.
 *    Numerical outcomes (info, IR results) are written to device memory.
 *  - Argument errors return CDS_INVALID_VALUE before anything is enqueued.
 *  - Pivots are 1-based int32 with LAPACK sequential-interchange meaning: for
 *    k = 0..n-1, row k was interchanged with row ipiv[k]-1.  Ties in the pivot
 *    search go to the lowest row index.
 *  - The workspace (cds_set_workspace) must be at least the size the matching
 *    *_bufferSize call reports; it is scratch between calls.  Calls that share
 *    one handle must not run concurrently.
 *  - Sizes are int64_t; n = 0 (or batch = 0) is a valid no-op.
 */
#ifndef CDS_H
#define CDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cds_handle_s* cds_handle_t;

typedef enum {
  CDS_SUCCESS = 0,
  CDS_INVALID_VALUE = 1,      /* bad argument; nothing was enqueued */
  CDS_NOT_INITIALIZED = 2,    /* null handle */
  CDS_HIP_ERROR = 3,          /* a HIP runtime call or kernel launch failed */
  CDS_ARCH_MISMATCH = 4,      /* the current device is not gfx950 */
  CDS_WORKSPACE_TOO_SMALL = 5,
  CDS_UNSUPPORTED = 6,
  CDS_DEVICE_FAULT = 7        /* a kernel's bounded wait timed out (see cds_device_error) */
} cds_status_t;

typedef enum { CDS_OP_N = 0, CDS_OP_T = 1 } cds_op_t;
typedef enum { CDS_LOWER = 0 } cds_fill_t;
typedef enum { CDS_R_64F = 0, CDS_R_32F = 1 } cds_dtype_t;

/* Precision of the factorization inside the mixed-precision solvers.
 * FP32: panel, trailing matrix and update all FP32.
 * BF16 / FP16: factors stored in FP32 and the panel in FP32; only the operands
 * of the trailing-matrix update are rounded (to nearest even) to BF16 / FP16,
 * with FP32 accumulation.  FP16 operands get a per-step power-of-two scale. */
typedef enum { CDS_PREC_FP32 = 0, CDS_PREC_BF16 = 1, CDS_PREC_FP16 = 2 } cds_prec_t;

typedef enum {
  CDS_OPT_NB = 0,           /* block size override for getrf/potrf (0 = tuning table / default) */
  CDS_OPT_LOOKAHEAD = 1,    /* 1 (default): overlap the next panel with the trailing update */
  CDS_OPT_LEAF = 2,         /* panel leaf width: 0 (default) or 32, the one width the panel is built for */
  CDS_OPT_PANEL_WGS = 3,    /* reserved: 0 only (the panel runs one workgroup per 256 of its rows) */
  CDS_OPT_KERNEL_TIMING = 4 /* 1: record a pair of events around every launch of the kernel classes
                               below, on the stream the kernel runs on (see cds_kernel_timing) */
} cds_option_t;

/* Kernel classes for cds_kernel_timing. */
typedef enum {
  CDS_KC_UPDATE = 0,     /* trailing-matrix update (MFMA GEMM / SYRK) */
  CDS_KC_PANEL = 1,      /* panel factorization (LU) or diagonal block (Cholesky) */
  CDS_KC_LASWP = 2,      /* row interchanges outside the panel */
  CDS_KC_TRSM = 3,       /* U12 / L21 triangular solves of the factorization */
  CDS_KC_TRSV = 4,       /* triangular solves of getrs / potrs */
  CDS_KC_RESIDUAL = 5,   /* FP64 residual of the refinement */
  CDS_KC_KRYLOV_GEMV = 6,/* products with A (or A^T) inside the Krylov solvers */
  CDS_KC_COUNT = 7
} cds_kernel_class_t;

/* Keys of the tuning table (cds_tune_set). */
typedef enum {
  CDS_TUNE_GETRF_NB = 0,    /* value: block size nb */
  CDS_TUNE_POTRF_NB = 1,    /* value: block size nb */
  CDS_TUNE_VBATCH_TILE = 2  /* value: block-column width (32 or 64) of the batched Cholesky for systems of size <= n_max */
} cds_tune_key_t;

/* Handle: holds the stream, the workspace pointer, options and the tuning
 * table (host state only).  cds_create checks that device 0.. current device
 * is gfx950 (else CDS_ARCH_MISMATCH) and creates one internal stream at the
 * default priority plus events, used to overlap the panel factorization with
 * the trailing update.  Not thread-safe: use one handle per host thread. */
cds_status_t cds_create(cds_handle_t* handle);
cds_status_t cds_destroy(cds_handle_t handle);
/* stream: a hipStream_t (0 = the null stream). */
cds_status_t cds_set_stream(cds_handle_t handle, void* stream);
cds_status_t cds_get_stream(cds_handle_t handle, void** stream);
cds_status_t cds_set_workspace(cds_handle_t handle, void* d_workspace, size_t bytes);
cds_status_t cds_set_option(cds_handle_t handle, cds_option_t option, int64_t value);
/* Tuning table: for problems of size n, the entry with the smallest n_max >= n
 * of (key, dtype) is used.  value <= 0 is rejected. */
cds_status_t cds_tune_set(cds_handle_t handle, cds_tune_key_t key, cds_dtype_t dtype, int64_t n_max, int64_t value);
cds_status_t cds_tune_clear(cds_handle_t handle);
/* Install the autotuner's table from a JSON file (host work only: the file is
 * read and parsed on the host, nothing is enqueued).  The file is an object
 * with an "entries" array of {"key": "getrf_nb" | "potrf_nb" | "vbatch_tile",
 * "dtype": "f64" | "f32", "n_max": int, "value": int} records (the form the
 * autotuner writes); other members are ignored.  Every entry must pass the
 * checks of cds_tune_set, else CDS_INVALID_VALUE; a table whose "arch" member
 * names another device than gfx950 gives CDS_ARCH_MISMATCH.  On any error the
 * handle's table is left unchanged; on success it is replaced by the file's.
 * The tuned quantities are the block size of the blocked factorizations (the
 * rank of the delayed update, Sec. 2) and the batched kernel's tile width. */
cds_status_t cds_tune(cds_handle_t handle, const char* table_path);
/* Validate a table file as cds_tune would, without a handle (no GPU needed):
 * *h_entries receives the number of entries on success. */
cds_status_t cds_tune_check(const char* table_path, int64_t* h_entries);
/* Synchronises the handle's stream, then reads and clears the device error
 * word of the workspace: *h_err = 0 when every bounded wait completed. */
cds_status_t cds_device_error(cds_handle_t handle, int32_t* h_err);
const char* cds_status_string(cds_status_t status);
/* Timing of the launches recorded since the last reset (CDS_OPT_KERNEL_TIMING = 1):
 * synchronises, then returns the number of launches of class kc, their summed
 * duration in ms (from the events around each launch) and their summed
 * algorithmic flops and bytes (the operation's own count: 2mnk for an update,
 * bytes read and written once for the bandwidth-bound kernels).  Host outputs. */
cds_status_t cds_kernel_timing(cds_handle_t handle, int32_t kc, int64_t* h_launches, double* h_ms, double* h_flops,
                               double* h_bytes);
cds_status_t cds_kernel_timing_reset(cds_handle_t handle);

typedef struct cds_ir_params_s cds_ir_params_t;

/* ---------------------------------------------------------------------------
 * Workspace sizes (bytes) for each operation, for the handle's current options.
 * ------------------------------------------------------------------------- */
cds_status_t cds_getrf_bufferSize(cds_handle_t handle, cds_dtype_t dtype, int64_t n, int64_t batch, size_t* h_bytes);
cds_status_t cds_getrs_bufferSize(cds_handle_t handle, cds_dtype_t dtype, int64_t n, int64_t nrhs, int64_t batch, size_t* h_bytes);
cds_status_t cds_potrf_bufferSize(cds_handle_t handle, cds_dtype_t dtype, int64_t n, size_t* h_bytes);
cds_status_t cds_potrs_bufferSize(cds_handle_t handle, cds_dtype_t dtype, int64_t n, int64_t nrhs, size_t* h_bytes);
/* The mixed-precision sizes depend on params->fallback (NULL = defaults). */
cds_status_t cds_gesv_mixed_bufferSize(cds_handle_t handle, cds_prec_t prec, int64_t n, int64_t nrhs, int64_t batch,
                                       const cds_ir_params_t* params, size_t* h_bytes);
cds_status_t cds_posv_mixed_bufferSize(cds_handle_t handle, cds_prec_t prec, int64_t n, int64_t nrhs,
                                       const cds_ir_params_t* params, size_t* h_bytes);
cds_status_t cds_posv_mixed_vbatched_bufferSize(cds_handle_t handle, int64_t batch, int64_t nmax, int64_t nrhs, size_t* h_bytes);

/* ---------------------------------------------------------------------------
 * LU with partial pivoting (Sec. 2, step 1): P A = L U, blocked right-looking
 * with rank-nb delayed updates.
 *   A (n x n, lda)  in: the matrix; out: L strictly below the diagonal (unit
 *                   diagonal implied) and U on and above it.
 *   ipiv (n)        out: 1-based pivots.
 *   info (1)        out: 0, or k > 0 if U(k,k) (1-based) is exactly zero; the
 *                   factorization still completes, no division by zero is done.
 * The strided-batched form factors `batch` independent matrices A + b*strideA
 * with pivots ipiv + b*strideP and info[b].
 * ------------------------------------------------------------------------- */
cds_status_t cds_dgetrf(cds_handle_t handle, int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t* info);
cds_status_t cds_sgetrf(cds_handle_t handle, int64_t n, float* A, int64_t lda, int32_t* ipiv, int32_t* info);
cds_status_t cds_dgetrf_strided_batched(cds_handle_t handle, int64_t n, double* A, int64_t lda, int64_t strideA,
                                        int32_t* ipiv, int64_t strideP, int32_t* info, int64_t batch);
cds_status_t cds_sgetrf_strided_batched(cds_handle_t handle, int64_t n, float* A, int64_t lda, int64_t strideA,
                                        int32_t* ipiv, int64_t strideP, int32_t* info, int64_t batch);

/* ---------------------------------------------------------------------------
 * Solve with LU factors (Sec. 2, step 2): op = N: A X = B via P B, L Y = P B,
 * U X = Y.  op = T: A^T X = B via U^T Z = B, L^T W = Z, X = P^T W.
 *   LU, ipiv: output of getrf.  B (n x nrhs, ldb): in right-hand sides, out X.
 * Singularity is not checked (as in LAPACK).
 * ------------------------------------------------------------------------- */
cds_status_t cds_dgetrs(cds_handle_t handle, cds_op_t op, int64_t n, int64_t nrhs, const double* LU, int64_t lda,
                        const int32_t* ipiv, double* B, int64_t ldb);
cds_status_t cds_sgetrs(cds_handle_t handle, cds_op_t op, int64_t n, int64_t nrhs, const float* LU, int64_t lda,
                        const int32_t* ipiv, float* B, int64_t ldb);
cds_status_t cds_dgetrs_strided_batched(cds_handle_t handle, cds_op_t op, int64_t n, int64_t nrhs, const double* LU,
                                        int64_t lda, int64_t strideA, const int32_t* ipiv, int64_t strideP,
                                        double* B, int64_t ldb, int64_t strideB, int64_t batch);

/* ---------------------------------------------------------------------------
 * Cholesky A = L L^T of an SPD matrix (Sec. 2), lower.
 *   A (n x n, lda): in the SPD matrix (lower triangle read); out L in the lower
 *   triangle.  The strict upper triangle is never read or written.
 *   info: 0, or k > 0 if the leading minor of order k is not positive
 *   definite (or NaN); the factorization stops there.
 * potrs: L Y = B, L^T X = Y; B overwritten with X.
 * ------------------------------------------------------------------------- */
cds_status_t cds_dpotrf(cds_handle_t handle, cds_fill_t fill, int64_t n, double* A, int64_t lda, int32_t* info);
cds_status_t cds_spotrf(cds_handle_t handle, cds_fill_t fill, int64_t n, float* A, int64_t lda, int32_t* info);
cds_status_t cds_dpotrs(cds_handle_t handle, cds_fill_t fill, int64_t n, int64_t nrhs, const double* L, int64_t lda,
                        double* B, int64_t ldb);
cds_status_t cds_spotrs(cds_handle_t handle, cds_fill_t fill, int64_t n, int64_t nrhs, const float* L, int64_t lda,
                        float* B, int64_t ldb);

/* ---------------------------------------------------------------------------
 * Mixed precision with FP64 iterative refinement.  The factorization runs in
 * `prec` (see cds_prec_t); then x0 = solve_lo(b) and, per iteration,
 * r = b - A x (FP64), eta = ||r||_inf / (||A||_inf ||x||_inf), d = solve_lo(r),
 * x += d (FP64), all on the device.  Stop when eta <= tol, when eta has not
 * halved over two iterations (stagnation), or after max_iter updates.
 * converged = (final eta <= success_tol).  With fallback = 1 a non-converged
 * solve is redone in FP64 (getrf + getrs + refinement); that decision reads
 * the device result, so fallback = 1 synchronises the stream.  fallback = 0
 * keeps the call free of host synchronisation (graph-capture safe).
 * ------------------------------------------------------------------------- */
struct cds_ir_params_s {
  double tol;          /* default 1e-15 */
  double success_tol;  /* default 1e-14 */
  int32_t max_iter;    /* default 30 */
  int32_t fallback;    /* default 0 */
  int32_t host_check;  /* default 0; 1: read the convergence flags on the host after every
                          iteration and stop enqueueing once all systems are done
                          (synchronises the stream; saves the no-op launches of the
                          remaining iterations) */
  int32_t reserved;
};

/* Written to device memory, one per system. stop_reason: 1 eta <= tol,
 * 2 stagnation, 3 max_iter, 4 non-finite, 5 factorization failed (info != 0). */
typedef struct {
  int32_t iters;       /* refinement updates applied */
  int32_t info;        /* factorization info */
  int32_t converged;
  int32_t fell_back;
  double eta;          /* final backward error */
  double eta0;         /* backward error of the unrefined low-precision solve */
  int32_t stop_reason;
  int32_t reserved;
} cds_ir_result_t;

/* A (n x n, lda) and B (n x nrhs, ldb) are read only.  X (n x nrhs, ldx) out.
 * LUlo (n x n, leading dimension n, FP32): out, the low-precision factors;
 * ipiv (n): out.  result (1): out, device. params: host pointer or NULL. */
cds_status_t cds_dgesv_mixed(cds_handle_t handle, cds_prec_t prec, int64_t n, int64_t nrhs, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* X, int64_t ldx, float* LUlo,
                             int32_t* ipiv, const cds_ir_params_t* params, cds_ir_result_t* result);
cds_status_t cds_dgesv_mixed_strided_batched(cds_handle_t handle, cds_prec_t prec, int64_t n, int64_t nrhs,
                                             const double* A, int64_t lda, int64_t strideA, const double* B,
                                             int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                                             float* LUlo, int64_t strideLU, int32_t* ipiv, int64_t strideP,
                                             const cds_ir_params_t* params, cds_ir_result_t* results, int64_t batch);
/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): cds_dgesv_mixed with
 * the same arguments and results, but its scratch is a fixed 72 MiB device
 * array inside the library (one per GPU, held until the process ends) instead
 * of the handle's workspace; no workspace need be set.  The call allocates
 * nothing.  Limits: the scratch must hold what cds_gesv_mixed_bufferSize
 * reports for (prec, n, nrhs, batch 1) with params->fallback = 0, which covers
 * n <= 32768 with nrhs <= 32; larger sizes return CDS_WORKSPACE_TOO_SMALL and
 * fallback = 1 returns CDS_UNSUPPORTED, both before anything is enqueued.
 * Every call on one GPU shares that GPU's scratch: calls that overlap in time
 * on one GPU (other streams, other handles, other threads) race and must be
 * ordered by the caller.  A timed-out bounded wait is reported by
 * cds_device_error on the calling handle. */
cds_status_t cds_dgesv_mixed_noalloc(cds_handle_t handle, cds_prec_t prec, int64_t n, int64_t nrhs, const double* A,
                                     int64_t lda, const double* B, int64_t ldb, double* X, int64_t ldx, float* LUlo,
                                     int32_t* ipiv, const cds_ir_params_t* params, cds_ir_result_t* result);
/* Refinement only, from existing low-precision LU factors (e.g. for the
 * transposed solve of a gradient): op(A) X = B, op = N or T.  Workspace: the
 * size cds_gesv_mixed_bufferSize reports for CDS_PREC_FP32, the same n, nrhs
 * and batch; params->fallback is ignored (no FP64 fallback without A's
 * factorization). */
cds_status_t cds_dgetrs_mixed_strided_batched(cds_handle_t handle, cds_op_t op, int64_t n, int64_t nrhs,
                                              const double* A, int64_t lda, int64_t strideA, const float* LUlo,
                                              int64_t strideLU, const int32_t* ipiv, int64_t strideP,
                                              const double* B, int64_t ldb, int64_t strideB, double* X,
                                              int64_t ldx, int64_t strideX, const cds_ir_params_t* params,
                                              cds_ir_result_t* results, int64_t batch);
/* SPD version: Cholesky in `prec`, FP64 refinement.  Llo (n x n, ld n, FP32) out. */
cds_status_t cds_dposv_mixed(cds_handle_t handle, cds_prec_t prec, cds_fill_t fill, int64_t n, int64_t nrhs,
                             const double* A, int64_t lda, const double* B, int64_t ldb, double* X, int64_t ldx,
                             float* Llo, const cds_ir_params_t* params, cds_ir_result_t* result);

/* ---------------------------------------------------------------------------
 * Many SPD systems of uneven size in one persistent launch: FP32 Cholesky and
 * FP32 triangular solves inside one workgroup per system, FP64 refinement.
 * Systems are taken largest-first from a device ticket counter.  All arrays
 * are device arrays of length batch.  n[i] in [1, nmax] (a system outside it is
 * skipped with results[i].info = -1, nothing of it read); A[i] (n x n, lda[i]);
 * B[i], X[i] (n x nrhs, ldb[i] / ldx[i]).  results[i] as above.  t_start[i] /
 * t_end[i] (may be NULL): device wall-clock ticks (100 MHz) when the system's
 * work started / ended.  order (may be NULL): processing order (a permutation
 * of 0..batch-1, e.g. sorted by decreasing n); NULL = index order.
 * No host synchronisation and no allocation: capture-safe.  prec must be FP32.
 * ------------------------------------------------------------------------- */
cds_status_t cds_dposv_mixed_vbatched(cds_handle_t handle, cds_prec_t prec, int64_t batch, int64_t nmax,
                                      const int32_t* n, const double* const* A, const int64_t* lda,
                                      const double* const* B, const int64_t* ldb, double* const* X,
                                      const int64_t* ldx, int64_t nrhs, const int32_t* order,
                                      const cds_ir_params_t* params, cds_ir_result_t* results,
                                      uint64_t* t_start, uint64_t* t_end);

/* ---------------------------------------------------------------------------
 * Krylov solvers (Sec. 2, the iterative family): conjugate gradient for SPD A,
 * BiCG (residuals with A, shadow residuals with A^T, shadow start r0), its
 * stabilised form BiCGSTAB, and GMRES restarted after `restart` Arnoldi steps
 * (Gram-Schmidt applied twice per step, Givens rotations for the small
 * least-squares problem).  FP64 throughout; A is dense n x n column-major
 * (lda), read only; b (n) read only; x (n) holds the initial guess on entry and
 * the solution on exit.  The solve stops when the relative residual of the
 * method's recurrence, ||r||_2 / ||b||_2, is <= params->tol, or after
 * params->max_iter iterations: one iteration is one product with A (CG,
 * GMRES), one with A and one with A^T (BiCG), or two with A (BiCGSTAB).  For
 * GMRES a cycle's end and every restart recompute the true residual.
 * result (device, 1): iters, converged, breakdown (a zero inner product ended
 * the recurrence), relres.  Enqueue-only except that the host reads one state
 * word every params->check_every iterations (and once per GMRES cycle) to stop
 * enqueueing after convergence; check_every = 0 enqueues the whole budget
 * (iterations after the stop exit at once).  Workspace: cds_krylov_bufferSize.
 * ------------------------------------------------------------------------- */
typedef enum { CDS_KRYLOV_CG = 0, CDS_KRYLOV_BICG = 1, CDS_KRYLOV_BICGSTAB = 2, CDS_KRYLOV_GMRES = 3 } cds_krylov_t;
typedef struct {
  double tol;           /* default 1e-10 */
  int32_t max_iter;     /* default 1000 */
  int32_t restart;      /* GMRES steps per cycle, 1..128; default 30 */
  int32_t check_every;  /* default 10 */
  int32_t reserved;
} cds_krylov_params_t;
typedef struct {
  int32_t iters;
  int32_t converged;
  int32_t breakdown;
  int32_t reserved;
  double relres;
} cds_krylov_result_t;
cds_status_t cds_krylov_bufferSize(cds_handle_t handle, cds_krylov_t method, int64_t n, int32_t restart,
                                   size_t* bytes);
cds_status_t cds_dkrylov(cds_handle_t handle, cds_krylov_t method, int64_t n, const double* A, int64_t lda,
                         const double* b, double* x, const cds_krylov_params_t* params, cds_krylov_result_t* result);

/* GMRES-based iterative refinement for one right-hand side: the factorization
 * of cds_dgesv_mixed in `prec` (LUlo, ipiv out), x0 from the low-precision
 * factors, then repeatedly r = b - A x (FP64), A d = r solved by GMRES in FP64
 * left-preconditioned with the low-precision factors (inner params: tol is the
 * preconditioned relative residual, default 1e-4; restart; max_iter per
 * correction), x += d, until eta = ||r||_inf / (||A||_inf ||x||_inf) <=
 * ir->tol or ir->max_iter corrections.  result (device): iters = corrections,
 * eta, eta0, converged (eta <= ir->success_tol), stop_reason as for the mixed
 * solvers, reserved = the total number of GMRES iterations.  The FP64 fallback
 * is not offered (ir->fallback must be 0).  Workspace:
 * cds_gesv_gmres_ir_bufferSize. */
cds_status_t cds_gesv_gmres_ir_bufferSize(cds_handle_t handle, cds_prec_t prec, int64_t n, int32_t restart,
                                          size_t* bytes);
cds_status_t cds_dgesv_gmres_ir(cds_handle_t handle, cds_prec_t prec, int64_t n, const double* A, int64_t lda,
                                const double* b, double* x, float* LUlo, int32_t* ipiv, const cds_ir_params_t* ir,
                                const cds_krylov_params_t* inner, cds_ir_result_t* result);

/* ---------------------------------------------------------------------------
 * Outer-product update used by the adjoint of the solve (Abar = -bbar x^T):
 * C = alpha * X * Y^T, with X (m x k, ldx), Y (n x k, ldy), C (m x n, ldc)
 * overwritten; strided over `batch`.
 * ------------------------------------------------------------------------- */
cds_status_t cds_douter_strided_batched(cds_handle_t handle, int64_t m, int64_t n, int64_t k, double alpha,
                                        const double* X, int64_t ldx, int64_t strideX, const double* Y,
                                        int64_t ldy, int64_t strideY, double* C, int64_t ldc, int64_t strideC,
                                        int64_t batch);

#ifdef __cplusplus
}
#endif
#endif /* CDS_H */
