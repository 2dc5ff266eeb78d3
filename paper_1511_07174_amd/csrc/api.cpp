// C-ABI of the dense direct solvers: handle, argument validation, workspace
// queries and dispatch to the drivers.  Every check that can fail happens
// before any work is enqueued.
#include <hip/hip_runtime.h>
#include <string.h>
#include <algorithm>
#include <mutex>
#include <vector>
#include "kernels.hpp"
#include "krylov.hpp"
#include "mixed.hpp"
#include "solve.hpp"
#include "tune_table.hpp"
#include "vbatched.hpp"

namespace {

struct TuneEntry {
  int key, dtype;
  int64_t n_max, value;
};

}  // namespace

struct cds_handle_s {
  hipStream_t stream = nullptr;
  hipStream_t s1 = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int nb_override = 0, lookahead = 1, leaf = 0, timing = 0;
  std::vector<TuneEntry> tune;
  cds::KTimer timer;
  void* noalloc_err = nullptr;   // error word of the fixed scratch, once a no-allocation call has used it
};

namespace {

using cds::Ctx;

int64_t tune_lookup(const cds_handle_s* h, int key, int dtype, int64_t n) {
  int64_t best_nmax = -1, val = 0;
  for (const auto& e : h->tune) {
    if (e.key != key || e.dtype != dtype || e.n_max < n) continue;
    if (best_nmax < 0 || e.n_max < best_nmax) { best_nmax = e.n_max; val = e.value; }
  }
  return val;
}

int getrf_nb(const cds_handle_s* h, int dtype, int64_t n) {
  if (h->nb_override > 0) return h->nb_override;
  return (int)tune_lookup(h, CDS_TUNE_GETRF_NB, dtype, n);
}
int potrf_nb(const cds_handle_s* h, int dtype, int64_t n) {
  if (h->nb_override > 0) return h->nb_override;
  return (int)tune_lookup(h, CDS_TUNE_POTRF_NB, dtype, n);
}
// getrf needs the resolved nb for its workspace size
int resolved_nb(int nb, int64_t n) {
  if (nb <= 0) nb = n <= 2048 ? 128 : 256;
  return std::min(512, std::max(32, (nb / 32) * 32));
}

Ctx make_ctx(cds_handle_s* h) {
  Ctx c{};
  c.s0 = h->stream;
  c.s1 = h->s1;
  for (int i = 0; i < 4; ++i) c.ev[i] = h->ev[i];
  c.ws = h->ws;
  c.ws_bytes = h->ws_bytes;
  c.err = (int*)h->ws;
  c.nb_override = h->nb_override;
  c.lookahead = h->lookahead;
  c.leaf = h->leaf;
  c.timer = h->timing ? &h->timer : nullptr;
  return c;
}

bool bad_dim(int64_t n) { return n < 0 || n > (int64_t)1 << 30; }
bool bad_ld(int64_t ld, int64_t rows) { return ld < std::max<int64_t>(1, rows); }
bool misaligned(const void* p, size_t a) { return ((uintptr_t)p % a) != 0; }

cds_ir_params_t default_params() {
  cds_ir_params_t p;
  p.tol = 1e-15;
  p.success_tol = 1e-14;
  p.max_iter = 30;
  p.fallback = 0;
  p.host_check = 0;
  p.reserved = 0;
  return p;
}
bool bad_params(const cds_ir_params_t& p) {
  return !(p.tol >= 0.0) || !(p.success_tol >= 0.0) || p.max_iter < 0 || p.max_iter > 1000 ||
         (p.fallback != 0 && p.fallback != 1) || (p.host_check != 0 && p.host_check != 1);
}

// The library needs a workspace whenever it enqueues work (the error word lives there).
cds_status_t need_ws(const cds_handle_s* h, size_t bytes) {
  if (h->ws == nullptr || h->ws_bytes < bytes) return CDS_WORKSPACE_TOO_SMALL;
  return CDS_SUCCESS;
}

// Fixed device scratch for the no-allocation entry point.  Every GPU that loads
// the library holds its own copy until the process ends.  Host code never uses
// the array's name as an address: the device address is resolved once per
// device with hipGetSymbolAddress (that device current) and kept in
// g_scratch_addr.
constexpr size_t kNoallocScratchBytes = (size_t)72 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // indexed by device ordinal; nullptr = not resolved yet

// Device address of `scratch` on device `dev`, which must be the current device.
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)dev + 1, nullptr);
  if (g_scratch_addr[dev] == nullptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

template <typename T>
cds_status_t getrf_generic(cds_handle_t h, int64_t n, T* A, int64_t lda, int64_t strideA, int32_t* ipiv,
                           int64_t strideP, int32_t* info, int64_t batch) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (bad_dim(n) || batch < 0 || bad_ld(lda, n)) return CDS_INVALID_VALUE;
  if (batch == 0) return CDS_SUCCESS;
  if (!info) return CDS_INVALID_VALUE;
  if (n > 0 && (!A || !ipiv)) return CDS_INVALID_VALUE;
  if (batch > 1 && n > 0 && (strideA < lda * n || strideP < n)) return CDS_INVALID_VALUE;
  if (misaligned(A, sizeof(T)) || misaligned(ipiv, 4) || misaligned(info, 4)) return CDS_INVALID_VALUE;
  const int dt = sizeof(T) == 8 ? CDS_R_64F : CDS_R_32F;
  const int nb = resolved_nb(getrf_nb(h, dt, n), n);
  cds_status_t st = need_ws(h, cds::getrf_ws_bytes((int)n, nb, 32, (int)batch, sizeof(T)));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::getrf_run<T>(c, (int)n, A, lda, strideA, ipiv, strideP, info, (int)batch, nb);
}

template <typename T>
cds_status_t getrs_generic(cds_handle_t h, cds_op_t op, int64_t n, int64_t nrhs, const T* LU, int64_t lda,
                           int64_t strideA, const int32_t* ipiv, int64_t strideP, T* B, int64_t ldb, int64_t strideB,
                           int64_t batch) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (op != CDS_OP_N && op != CDS_OP_T) return CDS_INVALID_VALUE;
  if (bad_dim(n) || nrhs < 0 || nrhs > 2048 || batch < 0 || bad_ld(lda, n) || bad_ld(ldb, n)) return CDS_INVALID_VALUE;
  if (batch == 0 || n == 0 || nrhs == 0) return CDS_SUCCESS;
  if (!LU || !ipiv || !B) return CDS_INVALID_VALUE;
  if (batch > 1 && (strideA < lda * n || strideP < n || strideB < ldb * nrhs)) return CDS_INVALID_VALUE;
  if (misaligned(LU, sizeof(T)) || misaligned(B, sizeof(T)) || misaligned(ipiv, 4)) return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::getrs_ws_bytes((int)n, (int)nrhs, (int)batch, sizeof(T)));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::getrs_run<T>(c, op == CDS_OP_T, (int)n, (int)nrhs, LU, lda, strideA, ipiv, strideP, B, ldb, strideB,
                           (int)batch, h->ws, h->ws_bytes);
}

template <typename T>
cds_status_t potrf_generic(cds_handle_t h, cds_fill_t fill, int64_t n, T* A, int64_t lda, int32_t* info) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (fill != CDS_LOWER || bad_dim(n) || bad_ld(lda, n)) return CDS_INVALID_VALUE;
  if (!info || (n > 0 && !A)) return CDS_INVALID_VALUE;
  if (misaligned(A, sizeof(T)) || misaligned(info, 4)) return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::potrf_ws_bytes((int)n, 0, sizeof(T)));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  const int dt = sizeof(T) == 8 ? CDS_R_64F : CDS_R_32F;
  return cds::potrf_run<T>(c, (int)n, A, lda, info, potrf_nb(h, dt, n));
}

template <typename T>
cds_status_t potrs_generic(cds_handle_t h, cds_fill_t fill, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B,
                           int64_t ldb) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (fill != CDS_LOWER || bad_dim(n) || nrhs < 0 || nrhs > 2048 || bad_ld(lda, n) || bad_ld(ldb, n))
    return CDS_INVALID_VALUE;
  if (n == 0 || nrhs == 0) return CDS_SUCCESS;
  if (!L || !B) return CDS_INVALID_VALUE;
  if (misaligned(L, sizeof(T)) || misaligned(B, sizeof(T))) return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::getrs_ws_bytes((int)n, (int)nrhs, 1, sizeof(T)));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::potrs_run<T>(c, (int)n, (int)nrhs, L, lda, B, ldb, h->ws, h->ws_bytes);
}

bool bad_tune_entry(int key, int dtype, int64_t n_max, int64_t value);
bool bad_prec(cds_prec_t p) { return p != CDS_PREC_FP32 && p != CDS_PREC_BF16 && p != CDS_PREC_FP16; }

// Argument checks of the mixed LU solvers; *nothing = true for a valid call with no work.
cds_status_t gesv_mixed_args(cds_prec_t prec, int64_t n, int64_t nrhs, const double* A, int64_t lda, int64_t strideA,
                             const double* B, int64_t ldb, int64_t strideB, const double* X, int64_t ldx,
                             int64_t strideX, const float* LUlo, int64_t strideLU, const int32_t* ipiv,
                             int64_t strideP, const cds_ir_params_t& p, const cds_ir_result_t* results,
                             int64_t batch, bool* nothing) {
  *nothing = false;
  if (bad_prec(prec) || bad_dim(n) || nrhs < 0 || nrhs > 2048 || batch < 0) return CDS_INVALID_VALUE;
  if (bad_ld(lda, n) || bad_ld(ldb, n) || bad_ld(ldx, n)) return CDS_INVALID_VALUE;
  if (bad_params(p)) return CDS_INVALID_VALUE;
  if (batch == 0 || n == 0 || nrhs == 0) {
    *nothing = true;
    return CDS_SUCCESS;
  }
  if (!A || !B || !X || !LUlo || !ipiv || !results) return CDS_INVALID_VALUE;
  if (batch > 1 && (strideA < lda * n || strideB < ldb * nrhs || strideX < ldx * nrhs || strideLU < n * n ||
                    strideP < n))
    return CDS_INVALID_VALUE;
  if (misaligned(A, 8) || misaligned(B, 8) || misaligned(X, 8) || misaligned(LUlo, 4) || misaligned(ipiv, 4) ||
      misaligned(results, 8))
    return CDS_INVALID_VALUE;
  return CDS_SUCCESS;
}


}  // namespace

// Krylov solver parameters
namespace {
cds_krylov_params_t krylov_defaults() {
  cds_krylov_params_t p;
  p.tol = 1e-10;
  p.max_iter = 1000;
  p.restart = 30;
  p.check_every = 10;
  p.reserved = 0;
  return p;
}
bool bad_krylov(const cds_krylov_params_t& p) {
  return !(p.tol >= 0.0) || p.max_iter < 0 || p.max_iter > (1 << 24) || p.restart < 1 || p.restart > 128 ||
         p.check_every < 0;
}
bool bad_method(int m) { return m < CDS_KRYLOV_CG || m > CDS_KRYLOV_GMRES; }
}  // namespace

extern "C" {

const char* cds_status_string(cds_status_t s) {
  switch (s) {
    case CDS_SUCCESS: return "CDS_SUCCESS";
    case CDS_INVALID_VALUE: return "CDS_INVALID_VALUE";
    case CDS_NOT_INITIALIZED: return "CDS_NOT_INITIALIZED";
    case CDS_HIP_ERROR: return "CDS_HIP_ERROR";
    case CDS_ARCH_MISMATCH: return "CDS_ARCH_MISMATCH";
    case CDS_WORKSPACE_TOO_SMALL: return "CDS_WORKSPACE_TOO_SMALL";
    case CDS_UNSUPPORTED: return "CDS_UNSUPPORTED";
    case CDS_DEVICE_FAULT: return "CDS_DEVICE_FAULT";
  }
  return "CDS_UNKNOWN_STATUS";
}

cds_status_t cds_create(cds_handle_t* out) {
  if (!out) return CDS_INVALID_VALUE;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CDS_HIP_ERROR;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CDS_HIP_ERROR;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CDS_ARCH_MISMATCH;
  // set-up of the no-allocation entry point's scratch on this device (a failure here is
  // reported by that entry point, which resolves the address again on its first call)
  {
    void* sp = nullptr;
    (void)scratch_address(dev, &sp);
  }
  cds_handle_s* h = new cds_handle_s();
  if (hipStreamCreateWithFlags(&h->s1, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return CDS_HIP_ERROR;
  }
  for (int i = 0; i < 4; ++i) {
    if (hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(h->ev[j]);
      (void)hipStreamDestroy(h->s1);
      delete h;
      return CDS_HIP_ERROR;
    }
  }
  *out = h;
  return CDS_SUCCESS;
}

cds_status_t cds_destroy(cds_handle_t h) {
  if (!h) return CDS_NOT_INITIALIZED;
  (void)hipStreamSynchronize(h->s1);
  for (int i = 0; i < 4; ++i) (void)hipEventDestroy(h->ev[i]);
  (void)hipStreamDestroy(h->s1);
  delete h;
  return CDS_SUCCESS;
}

cds_status_t cds_set_stream(cds_handle_t h, void* stream) {
  if (!h) return CDS_NOT_INITIALIZED;
  h->stream = (hipStream_t)stream;
  return CDS_SUCCESS;
}

cds_status_t cds_get_stream(cds_handle_t h, void** stream) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!stream) return CDS_INVALID_VALUE;
  *stream = (void*)h->stream;
  return CDS_SUCCESS;
}

cds_status_t cds_set_workspace(cds_handle_t h, void* ws, size_t bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if ((ws == nullptr) != (bytes == 0)) return CDS_INVALID_VALUE;
  if (ws && (misaligned(ws, 256) || bytes < cds::kErrRegion)) return CDS_INVALID_VALUE;
  h->ws = ws;
  h->ws_bytes = bytes;
  if (ws && cds::launch_fill_zero(ws, cds::kErrRegion, h->stream) != hipSuccess) return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

cds_status_t cds_set_option(cds_handle_t h, cds_option_t opt, int64_t v) {
  if (!h) return CDS_NOT_INITIALIZED;
  switch (opt) {
    case CDS_OPT_NB:
      if (v < 0 || v > 512) return CDS_INVALID_VALUE;
      h->nb_override = (int)v;
      return CDS_SUCCESS;
    case CDS_OPT_LOOKAHEAD:
      if (v != 0 && v != 1) return CDS_INVALID_VALUE;
      h->lookahead = (int)v;
      return CDS_SUCCESS;
    case CDS_OPT_LEAF:
      if (v != 0 && v != 32) return CDS_INVALID_VALUE;
      h->leaf = (int)v;
      return CDS_SUCCESS;
    case CDS_OPT_PANEL_WGS:
      return v == 0 ? CDS_SUCCESS : CDS_INVALID_VALUE;
    case CDS_OPT_KERNEL_TIMING:
      if (v != 0 && v != 1) return CDS_INVALID_VALUE;
      h->timing = (int)v;
      return CDS_SUCCESS;
  }
  return CDS_INVALID_VALUE;
}

cds_status_t cds_tune_set(cds_handle_t h, cds_tune_key_t key, cds_dtype_t dtype, int64_t n_max, int64_t value) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (bad_tune_entry(key, dtype, n_max, value)) return CDS_INVALID_VALUE;
  for (auto& e : h->tune)
    if (e.key == key && e.dtype == dtype && e.n_max == n_max) { e.value = value; return CDS_SUCCESS; }
  h->tune.push_back(TuneEntry{key, dtype, n_max, value});
  return CDS_SUCCESS;
}

namespace {
// The checks cds_tune_set applies to one entry.
bool bad_tune_entry(int key, int dtype, int64_t n_max, int64_t value) {
  if (key < CDS_TUNE_GETRF_NB || key > CDS_TUNE_VBATCH_TILE) return true;
  if (dtype != CDS_R_64F && dtype != CDS_R_32F) return true;
  if (n_max < 0 || value <= 0 || value > 512) return true;
  if (key == CDS_TUNE_VBATCH_TILE && value != 32 && value != 64) return true;
  return false;
}
// Reads and validates a table file; arch must name gfx950 when the table names one.
cds_status_t load_tune_file(const char* path, std::vector<cds::TuneRecord>& recs) {
  if (!path) return CDS_INVALID_VALUE;
  std::string arch, err;
  if (cds::read_tune_table(path, recs, arch, err) != 0) return CDS_INVALID_VALUE;
  if (!arch.empty() && arch.compare(0, 6, "gfx950") != 0) return CDS_ARCH_MISMATCH;
  for (const auto& r : recs)
    if (bad_tune_entry(r.key, r.dtype, r.n_max, r.value)) return CDS_INVALID_VALUE;
  return CDS_SUCCESS;
}
}  // namespace

cds_status_t cds_tune(cds_handle_t h, const char* table_path) {
  if (!h) return CDS_NOT_INITIALIZED;
  std::vector<cds::TuneRecord> recs;
  cds_status_t st = load_tune_file(table_path, recs);
  if (st != CDS_SUCCESS) return st;   // the handle's table is left as it was
  h->tune.clear();
  for (const auto& r : recs) {
    bool found = false;
    for (auto& e : h->tune)
      if (e.key == r.key && e.dtype == r.dtype && e.n_max == r.n_max) { e.value = r.value; found = true; }
    if (!found) h->tune.push_back(TuneEntry{r.key, r.dtype, r.n_max, r.value});
  }
  return CDS_SUCCESS;
}

cds_status_t cds_tune_check(const char* table_path, int64_t* h_entries) {
  if (!h_entries) return CDS_INVALID_VALUE;
  *h_entries = 0;
  std::vector<cds::TuneRecord> recs;
  cds_status_t st = load_tune_file(table_path, recs);
  if (st == CDS_SUCCESS) *h_entries = (int64_t)recs.size();
  return st;
}

cds_status_t cds_tune_clear(cds_handle_t h) {
  if (!h) return CDS_NOT_INITIALIZED;
  h->tune.clear();
  return CDS_SUCCESS;
}

cds_status_t cds_device_error(cds_handle_t h, int32_t* h_err) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!h_err) return CDS_INVALID_VALUE;
  *h_err = 0;
  void* words[2] = {h->ws, h->noalloc_err};
  if (!words[0] && !words[1]) return CDS_SUCCESS;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return CDS_HIP_ERROR;
  for (void* w : words) {
    if (!w) continue;
    int32_t v = 0;
    if (hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return CDS_HIP_ERROR;
    if (v != 0) {
      if (*h_err == 0) *h_err = v;
      if (cds::launch_fill_zero(w, cds::kErrRegion, h->stream) != hipSuccess) return CDS_HIP_ERROR;
      if (hipStreamSynchronize(h->stream) != hipSuccess) return CDS_HIP_ERROR;
    }
  }
  return CDS_SUCCESS;
}

cds_status_t cds_kernel_timing(cds_handle_t h, int32_t kc, int64_t* launches, double* ms, double* flops,
                               double* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (kc < 0 || kc >= CDS_KC_COUNT || !launches || !ms || !flops || !bytes) return CDS_INVALID_VALUE;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return CDS_HIP_ERROR;
  if (hipStreamSynchronize(h->s1) != hipSuccess) return CDS_HIP_ERROR;
  int64_t cnt = 0;
  double t = 0.0, f = 0.0, b = 0.0;
  for (const auto& r : h->timer.recs) {
    if (r.kc != kc) continue;
    float e = 0.f;
    if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return CDS_HIP_ERROR;
    ++cnt;
    t += e;
    f += r.flops;
    b += r.bytes;
  }
  *launches = cnt;
  *ms = t;
  *flops = f;
  *bytes = b;
  return CDS_SUCCESS;
}

cds_status_t cds_kernel_timing_reset(cds_handle_t h) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return CDS_HIP_ERROR;
  if (hipStreamSynchronize(h->s1) != hipSuccess) return CDS_HIP_ERROR;
  h->timer.reset();
  return CDS_SUCCESS;
}

// ------------------------------------------------------------------------------- sizes
cds_status_t cds_getrf_bufferSize(cds_handle_t h, cds_dtype_t dt, int64_t n, int64_t batch, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_dim(n) || batch < 0 || (dt != CDS_R_64F && dt != CDS_R_32F)) return CDS_INVALID_VALUE;
  const int nb = resolved_nb(getrf_nb(h, dt, n), n);
  *bytes = cds::getrf_ws_bytes((int)n, nb, 32, (int)std::max<int64_t>(batch, 1), dt == CDS_R_64F ? 8 : 4);
  return CDS_SUCCESS;
}
cds_status_t cds_getrs_bufferSize(cds_handle_t h, cds_dtype_t dt, int64_t n, int64_t nrhs, int64_t batch,
                                  size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_dim(n) || nrhs < 0 || nrhs > 2048 || batch < 0 || (dt != CDS_R_64F && dt != CDS_R_32F))
    return CDS_INVALID_VALUE;
  *bytes = cds::getrs_ws_bytes((int)n, (int)std::max<int64_t>(nrhs, 1), (int)std::max<int64_t>(batch, 1),
                               dt == CDS_R_64F ? 8 : 4);
  return CDS_SUCCESS;
}
cds_status_t cds_potrf_bufferSize(cds_handle_t h, cds_dtype_t dt, int64_t n, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_dim(n) || (dt != CDS_R_64F && dt != CDS_R_32F)) return CDS_INVALID_VALUE;
  *bytes = cds::potrf_ws_bytes((int)n, 0, dt == CDS_R_64F ? 8 : 4);
  return CDS_SUCCESS;
}
cds_status_t cds_potrs_bufferSize(cds_handle_t h, cds_dtype_t dt, int64_t n, int64_t nrhs, size_t* bytes) {
  return cds_getrs_bufferSize(h, dt, n, nrhs, 1, bytes);
}
cds_status_t cds_gesv_mixed_bufferSize(cds_handle_t h, cds_prec_t prec, int64_t n, int64_t nrhs, int64_t batch,
                                       const cds_ir_params_t* params, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_prec(prec) || bad_dim(n) || nrhs < 0 || nrhs > 2048 || batch < 0) return CDS_INVALID_VALUE;
  const cds_ir_params_t p = params ? *params : default_params();
  const int nb = resolved_nb(getrf_nb(h, CDS_R_32F, n), n);
  *bytes = cds::ir_ws_bytes((int)n, (int)std::max<int64_t>(nrhs, 1), (int)std::max<int64_t>(batch, 1), nb, 0,
                            p.fallback);
  return CDS_SUCCESS;
}
cds_status_t cds_posv_mixed_bufferSize(cds_handle_t h, cds_prec_t prec, int64_t n, int64_t nrhs,
                                       const cds_ir_params_t* params, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_prec(prec) || bad_dim(n) || nrhs < 0 || nrhs > 2048) return CDS_INVALID_VALUE;
  const cds_ir_params_t p = params ? *params : default_params();
  *bytes = cds::ir_ws_bytes((int)n, (int)std::max<int64_t>(nrhs, 1), 1, 256, 1, p.fallback);
  return CDS_SUCCESS;
}
cds_status_t cds_posv_mixed_vbatched_bufferSize(cds_handle_t h, int64_t batch, int64_t nmax, int64_t nrhs,
                                                size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || batch < 0 || nmax < 0 || nmax > 1024 || nrhs < 0) return CDS_INVALID_VALUE;
  *bytes = cds::vbatched_ws_bytes((int)batch, (int)nmax, (int)nrhs);
  return CDS_SUCCESS;
}

// ------------------------------------------------------------------------------- LU
cds_status_t cds_dgetrf(cds_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, int32_t* info) {
  return getrf_generic<double>(h, n, A, lda, 0, ipiv, 0, info, 1);
}
cds_status_t cds_sgetrf(cds_handle_t h, int64_t n, float* A, int64_t lda, int32_t* ipiv, int32_t* info) {
  return getrf_generic<float>(h, n, A, lda, 0, ipiv, 0, info, 1);
}
cds_status_t cds_dgetrf_strided_batched(cds_handle_t h, int64_t n, double* A, int64_t lda, int64_t strideA,
                                        int32_t* ipiv, int64_t strideP, int32_t* info, int64_t batch) {
  return getrf_generic<double>(h, n, A, lda, strideA, ipiv, strideP, info, batch);
}
cds_status_t cds_sgetrf_strided_batched(cds_handle_t h, int64_t n, float* A, int64_t lda, int64_t strideA,
                                        int32_t* ipiv, int64_t strideP, int32_t* info, int64_t batch) {
  return getrf_generic<float>(h, n, A, lda, strideA, ipiv, strideP, info, batch);
}
cds_status_t cds_dgetrs(cds_handle_t h, cds_op_t op, int64_t n, int64_t nrhs, const double* LU, int64_t lda,
                        const int32_t* ipiv, double* B, int64_t ldb) {
  return getrs_generic<double>(h, op, n, nrhs, LU, lda, 0, ipiv, 0, B, ldb, 0, 1);
}
cds_status_t cds_sgetrs(cds_handle_t h, cds_op_t op, int64_t n, int64_t nrhs, const float* LU, int64_t lda,
                        const int32_t* ipiv, float* B, int64_t ldb) {
  return getrs_generic<float>(h, op, n, nrhs, LU, lda, 0, ipiv, 0, B, ldb, 0, 1);
}
cds_status_t cds_dgetrs_strided_batched(cds_handle_t h, cds_op_t op, int64_t n, int64_t nrhs, const double* LU,
                                        int64_t lda, int64_t strideA, const int32_t* ipiv, int64_t strideP,
                                        double* B, int64_t ldb, int64_t strideB, int64_t batch) {
  return getrs_generic<double>(h, op, n, nrhs, LU, lda, strideA, ipiv, strideP, B, ldb, strideB, batch);
}

// ------------------------------------------------------------------------------- Cholesky
cds_status_t cds_dpotrf(cds_handle_t h, cds_fill_t fill, int64_t n, double* A, int64_t lda, int32_t* info) {
  return potrf_generic<double>(h, fill, n, A, lda, info);
}
cds_status_t cds_spotrf(cds_handle_t h, cds_fill_t fill, int64_t n, float* A, int64_t lda, int32_t* info) {
  return potrf_generic<float>(h, fill, n, A, lda, info);
}
cds_status_t cds_dpotrs(cds_handle_t h, cds_fill_t fill, int64_t n, int64_t nrhs, const double* L, int64_t lda,
                        double* B, int64_t ldb) {
  return potrs_generic<double>(h, fill, n, nrhs, L, lda, B, ldb);
}
cds_status_t cds_spotrs(cds_handle_t h, cds_fill_t fill, int64_t n, int64_t nrhs, const float* L, int64_t lda,
                        float* B, int64_t ldb) {
  return potrs_generic<float>(h, fill, n, nrhs, L, lda, B, ldb);
}

// ------------------------------------------------------------------------------- mixed precision
cds_status_t cds_dgesv_mixed_strided_batched(cds_handle_t h, cds_prec_t prec, int64_t n, int64_t nrhs,
                                             const double* A, int64_t lda, int64_t strideA, const double* B,
                                             int64_t ldb, int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                                             float* LUlo, int64_t strideLU, int32_t* ipiv, int64_t strideP,
                                             const cds_ir_params_t* params, cds_ir_result_t* results,
                                             int64_t batch) {
  if (!h) return CDS_NOT_INITIALIZED;
  const cds_ir_params_t p = params ? *params : default_params();
  bool nothing = false;
  cds_status_t vst = gesv_mixed_args(prec, n, nrhs, A, lda, strideA, B, ldb, strideB, X, ldx, strideX, LUlo,
                                     strideLU, ipiv, strideP, p, results, batch, &nothing);
  if (vst != CDS_SUCCESS || nothing) return vst;
  const int nb = resolved_nb(getrf_nb(h, CDS_R_32F, n), n);
  cds_status_t st = need_ws(h, cds::ir_ws_bytes((int)n, (int)nrhs, (int)batch, nb, 0, p.fallback));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::gesv_mixed_run(c, (int)prec, (int)n, (int)nrhs, A, lda, strideA, B, ldb, strideB, X, ldx, strideX, LUlo,
                             batch > 1 ? strideLU : n * n, ipiv, strideP, p, results, (int)batch, nb);
}

cds_status_t cds_dgesv_mixed(cds_handle_t h, cds_prec_t prec, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double* X, int64_t ldx, float* LUlo, int32_t* ipiv,
                             const cds_ir_params_t* params, cds_ir_result_t* result) {
  return cds_dgesv_mixed_strided_batched(h, prec, n, nrhs, A, lda, 0, B, ldb, 0, X, ldx, 0, LUlo, 0, ipiv, 0, params,
                                         result, 1);
}

cds_status_t cds_dgesv_mixed_noalloc(cds_handle_t h, cds_prec_t prec, int64_t n, int64_t nrhs, const double* A,
                                     int64_t lda, const double* B, int64_t ldb, double* X, int64_t ldx, float* LUlo,
                                     int32_t* ipiv, const cds_ir_params_t* params, cds_ir_result_t* result) {
  if (!h) return CDS_NOT_INITIALIZED;
  const cds_ir_params_t p = params ? *params : default_params();
  bool nothing = false;
  cds_status_t vst = gesv_mixed_args(prec, n, nrhs, A, lda, 0, B, ldb, 0, X, ldx, 0, LUlo, 0, ipiv, 0, p, result, 1,
                                     &nothing);
  if (vst != CDS_SUCCESS || nothing) return vst;
  if (p.fallback) return CDS_UNSUPPORTED;   // the FP64 fallback needs an n x n copy of A
  const int nb = resolved_nb(getrf_nb(h, CDS_R_32F, n), n);
  if (cds::ir_ws_bytes((int)n, (int)nrhs, 1, nb, 0, 0) > kNoallocScratchBytes) return CDS_WORKSPACE_TOO_SMALL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CDS_HIP_ERROR;
  void* sp = nullptr;
  if (scratch_address(dev, &sp) != hipSuccess) return CDS_HIP_ERROR;
  Ctx c = make_ctx(h);
  c.ws = sp;
  c.ws_bytes = kNoallocScratchBytes;
  c.err = (int*)sp;
  // the error word starts at zero on every call; the rest of the scratch is cleared by the drivers
  if (cds::launch_fill_zero(sp, cds::kErrRegion, h->stream) != hipSuccess) return CDS_HIP_ERROR;
  h->noalloc_err = sp;
  return cds::gesv_mixed_run(c, (int)prec, (int)n, (int)nrhs, A, lda, 0, B, ldb, 0, X, ldx, 0, LUlo, n * n, ipiv, 0, p,
                             result, 1, nb);
}

cds_status_t cds_dgetrs_mixed_strided_batched(cds_handle_t h, cds_op_t op, int64_t n, int64_t nrhs, const double* A,
                                              int64_t lda, int64_t strideA, const float* LUlo, int64_t strideLU,
                                              const int32_t* ipiv, int64_t strideP, const double* B, int64_t ldb,
                                              int64_t strideB, double* X, int64_t ldx, int64_t strideX,
                                              const cds_ir_params_t* params, cds_ir_result_t* results,
                                              int64_t batch) {
  if (!h) return CDS_NOT_INITIALIZED;
  if ((op != CDS_OP_N && op != CDS_OP_T) || bad_dim(n) || nrhs < 0 || nrhs > 2048 || batch < 0)
    return CDS_INVALID_VALUE;
  if (bad_ld(lda, n) || bad_ld(ldb, n) || bad_ld(ldx, n)) return CDS_INVALID_VALUE;
  cds_ir_params_t p = params ? *params : default_params();
  if (bad_params(p)) return CDS_INVALID_VALUE;
  p.fallback = 0;
  if (batch == 0 || n == 0 || nrhs == 0) return CDS_SUCCESS;
  if (!A || !B || !X || !LUlo || !ipiv || !results) return CDS_INVALID_VALUE;
  if (batch > 1 && (strideA < lda * n || strideB < ldb * nrhs || strideX < ldx * nrhs || strideLU < n * n ||
                    strideP < n))
    return CDS_INVALID_VALUE;
  if (misaligned(A, 8) || misaligned(B, 8) || misaligned(X, 8) || misaligned(LUlo, 4) || misaligned(ipiv, 4) ||
      misaligned(results, 8))
    return CDS_INVALID_VALUE;
  // the same requirement as cds_gesv_mixed_bufferSize reports for these sizes
  const int nbq = resolved_nb(getrf_nb(h, CDS_R_32F, n), n);
  cds_status_t st = need_ws(h, cds::ir_ws_bytes((int)n, (int)nrhs, (int)batch, nbq, 0, 0));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::getrs_mixed_run(c, op == CDS_OP_T, (int)n, (int)nrhs, A, lda, strideA, LUlo,
                              batch > 1 ? strideLU : n * n, ipiv, strideP, B, ldb, strideB, X, ldx, strideX, p,
                              results, (int)batch);
}

cds_status_t cds_dposv_mixed(cds_handle_t h, cds_prec_t prec, cds_fill_t fill, int64_t n, int64_t nrhs,
                             const double* A, int64_t lda, const double* B, int64_t ldb, double* X, int64_t ldx,
                             float* Llo, const cds_ir_params_t* params, cds_ir_result_t* result) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (bad_prec(prec) || fill != CDS_LOWER || bad_dim(n) || nrhs < 0 || nrhs > 2048) return CDS_INVALID_VALUE;
  if (bad_ld(lda, n) || bad_ld(ldb, n) || bad_ld(ldx, n)) return CDS_INVALID_VALUE;
  const cds_ir_params_t p = params ? *params : default_params();
  if (bad_params(p)) return CDS_INVALID_VALUE;
  if (n == 0 || nrhs == 0) return CDS_SUCCESS;
  if (!A || !B || !X || !Llo || !result) return CDS_INVALID_VALUE;
  if (misaligned(A, 8) || misaligned(B, 8) || misaligned(X, 8) || misaligned(Llo, 4) || misaligned(result, 8))
    return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::ir_ws_bytes((int)n, (int)nrhs, 1, 256, 1, p.fallback));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::posv_mixed_run(c, (int)prec, (int)n, (int)nrhs, A, lda, B, ldb, X, ldx, Llo, p, result,
                             potrf_nb(h, CDS_R_32F, n));
}

cds_status_t cds_dposv_mixed_vbatched(cds_handle_t h, cds_prec_t prec, int64_t batch, int64_t nmax, const int32_t* n,
                                      const double* const* A, const int64_t* lda, const double* const* B,
                                      const int64_t* ldb, double* const* X, const int64_t* ldx, int64_t nrhs,
                                      const int32_t* order, const cds_ir_params_t* params, cds_ir_result_t* results,
                                      uint64_t* t_start, uint64_t* t_end) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (prec != CDS_PREC_FP32) return CDS_UNSUPPORTED;
  if (batch < 0 || nmax < 1 || nmax > 1024 || nrhs < 0 || batch > (1 << 30)) return CDS_INVALID_VALUE;
  const cds_ir_params_t p = params ? *params : default_params();
  if (bad_params(p) || p.fallback) return CDS_INVALID_VALUE;
  if (batch == 0 || nrhs == 0) return CDS_SUCCESS;
  if (!n || !A || !lda || !B || !ldb || !X || !ldx || !results) return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::vbatched_ws_bytes((int)batch, (int)nmax, (int)nrhs));
  if (st != CDS_SUCCESS) return st;
  // block width per size: systems up to the largest bucket tuned to 32 use 32-wide block columns
  int jw32 = 256;
  {
    int64_t best = -1;
    bool any = false;
    for (const auto& e : h->tune) {
      if (e.key != CDS_TUNE_VBATCH_TILE) continue;
      any = true;
      if (e.value == 32 && e.n_max > best) best = e.n_max;
    }
    if (any) jw32 = (int)std::min<int64_t>(std::max<int64_t>(best, 0), 1 << 30);
  }
  Ctx c = make_ctx(h);
  return cds::vbatched_run(c, (int)batch, (int)nmax, n, A, lda, B, ldb, X, ldx, (int)nrhs, order, p, results, t_start,
                           t_end, jw32);
}

// ------------------------------------------------------------------------- Krylov solvers

cds_status_t cds_krylov_bufferSize(cds_handle_t h, cds_krylov_t method, int64_t n, int32_t restart, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_method(method) || bad_dim(n) || restart < 1 || restart > 128) return CDS_INVALID_VALUE;
  *bytes = cds::krylov_ws_bytes((int)method, (int)n, restart, 0);
  return CDS_SUCCESS;
}

cds_status_t cds_dkrylov(cds_handle_t h, cds_krylov_t method, int64_t n, const double* A, int64_t lda,
                         const double* b, double* x, const cds_krylov_params_t* params, cds_krylov_result_t* result) {
  if (!h) return CDS_NOT_INITIALIZED;
  const cds_krylov_params_t p = params ? *params : krylov_defaults();
  if (bad_method(method) || bad_dim(n) || bad_ld(lda, n) || bad_krylov(p)) return CDS_INVALID_VALUE;
  if (n == 0) return CDS_SUCCESS;
  if (!A || !b || !x || !result) return CDS_INVALID_VALUE;
  if (misaligned(A, 8) || misaligned(b, 8) || misaligned(x, 8) || misaligned(result, 8)) return CDS_INVALID_VALUE;
  cds_status_t st = need_ws(h, cds::krylov_ws_bytes((int)method, (int)n, p.restart, 0));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::krylov_run(c, (int)method, (int)n, A, lda, b, x, p, result, nullptr, nullptr);
}

cds_status_t cds_gesv_gmres_ir_bufferSize(cds_handle_t h, cds_prec_t prec, int64_t n, int32_t restart, size_t* bytes) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (!bytes || bad_prec(prec) || bad_dim(n) || restart < 1 || restart > 128) return CDS_INVALID_VALUE;
  *bytes = cds::gmres_ir_ws_bytes((int)n, resolved_nb(getrf_nb(h, CDS_R_32F, n), n), restart);
  return CDS_SUCCESS;
}

cds_status_t cds_dgesv_gmres_ir(cds_handle_t h, cds_prec_t prec, int64_t n, const double* A, int64_t lda,
                                const double* b, double* x, float* LUlo, int32_t* ipiv, const cds_ir_params_t* ir,
                                const cds_krylov_params_t* inner, cds_ir_result_t* result) {
  if (!h) return CDS_NOT_INITIALIZED;
  const cds_ir_params_t p = ir ? *ir : default_params();
  cds_krylov_params_t kp = krylov_defaults();
  kp.tol = 1e-4;
  kp.max_iter = 60;
  if (inner) kp = *inner;
  if (bad_prec(prec) || bad_dim(n) || bad_ld(lda, n) || bad_params(p) || p.fallback || bad_krylov(kp))
    return CDS_INVALID_VALUE;
  if (n == 0) return CDS_SUCCESS;
  if (!A || !b || !x || !LUlo || !ipiv || !result) return CDS_INVALID_VALUE;
  if (misaligned(A, 8) || misaligned(b, 8) || misaligned(x, 8) || misaligned(LUlo, 4) || misaligned(ipiv, 4) ||
      misaligned(result, 8))
    return CDS_INVALID_VALUE;
  const int nb = resolved_nb(getrf_nb(h, CDS_R_32F, n), n);
  cds_status_t st = need_ws(h, cds::gmres_ir_ws_bytes((int)n, nb, kp.restart));
  if (st != CDS_SUCCESS) return st;
  Ctx c = make_ctx(h);
  return cds::gesv_gmres_ir_run(c, (int)prec, (int)n, A, lda, b, x, LUlo, ipiv, p, kp, result, nb);
}

cds_status_t cds_douter_strided_batched(cds_handle_t h, int64_t m, int64_t n, int64_t k, double alpha,
                                        const double* X, int64_t ldx, int64_t strideX, const double* Y, int64_t ldy,
                                        int64_t strideY, double* C, int64_t ldc, int64_t strideC, int64_t batch) {
  if (!h) return CDS_NOT_INITIALIZED;
  if (bad_dim(m) || bad_dim(n) || k < 0 || batch < 0 || bad_ld(ldc, m)) return CDS_INVALID_VALUE;
  if (k > 0 && (bad_ld(ldx, m) || bad_ld(ldy, n))) return CDS_INVALID_VALUE;
  if (batch == 0 || m == 0 || n == 0) return CDS_SUCCESS;
  if (!C || (k > 0 && (!X || !Y))) return CDS_INVALID_VALUE;
  if (misaligned(C, 8) || misaligned(X, 8) || misaligned(Y, 8)) return CDS_INVALID_VALUE;
  if (cds::launch_outer((int)m, (int)n, (int)k, alpha, X, ldx, strideX, Y, ldy, strideY, C, ldc, strideC, (int)batch,
                        h->stream) != hipSuccess)
    return CDS_HIP_ERROR;
  return CDS_SUCCESS;
}

}  // extern "C"
