// Shared device helpers for the gfx950 kernels of the dense direct solvers.
// Wave64 reductions, MFMA fragment types, the flag+payload ("low-latency")
// message words used for cross-workgroup exchange, and launch checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace cds {

constexpr int kWave = 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Device error word (bounded spins that time out record here; never hang).
// ---------------------------------------------------------------------------
enum DevErr : int { kErrNone = 0, kErrSpinTimeout = 1, kErrNoProgress = 2 };

// ~ several seconds of polling; a correct run never comes close.
constexpr long long kSpinLimit = 1ll << 23;

// ---------------------------------------------------------------------------
// Flag+payload words: a 64-bit word holds 32 bits of payload in the low half
// and a 32-bit flag in the high half.  Written and read with agent-scope
// relaxed atomics, which keep them coherent across the XCDs' separate L2
// caches without a full cache write-back.  A reader spins until the flag it
// expects appears, so each word validates itself and no fence is needed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ll_store(uint64_t* p, uint32_t payload, uint32_t flag) {
  uint64_t w = ((uint64_t)flag << 32) | (uint64_t)payload;
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin until the word's flag equals `flag`; returns the payload.  On time-out
// records kErrSpinTimeout in *err and returns 0 (results are then invalid but
// the kernel still terminates).
__device__ __forceinline__ uint32_t ll_load(const uint64_t* p, uint32_t flag, int* err) {
  long long spins = 0;
  while (true) {
    uint64_t w = __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(w >> 32) == flag) return (uint32_t)w;
    ++spins;
    if ((spins & 4095) == 0) {
      // give up at once if another wait has already timed out
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0u;
      if (spins > kSpinLimit) {
        atomicExch(err, (int)kErrSpinTimeout);
        return 0u;
      }
    }
  }
}

// A double travels as two words (low and high halves).
__device__ __forceinline__ void ll_store_f64(uint64_t* p, double v, uint32_t flag) {
  uint64_t bits = __double_as_longlong(v);
  ll_store(p, (uint32_t)bits, flag);
  ll_store(p + 1, (uint32_t)(bits >> 32), flag);
}
// Both words are requested together (one round trip when the message is there).
__device__ __forceinline__ double ll_load_f64(const uint64_t* p, uint32_t flag, int* err) {
  long long spins = 0;
  while (true) {
    uint64_t w0 = __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t w1 = __hip_atomic_load(const_cast<uint64_t*>(p + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(w0 >> 32) == flag && (uint32_t)(w1 >> 32) == flag)
      return __longlong_as_double((long long)(((w1 & 0xffffffffull) << 32) | (w0 & 0xffffffffull)));
    ++spins;
    if ((spins & 4095) == 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0.0;
      if (spins > kSpinLimit) {
        atomicExch(err, (int)kErrSpinTimeout);
        return 0.0;
      }
    }
  }
}
__device__ __forceinline__ void ll_store_val(uint64_t* p, double v, uint32_t flag) { ll_store_f64(p, v, flag); }
__device__ __forceinline__ void ll_store_val(uint64_t* p, float v, uint32_t flag) {
  ll_store(p, __float_as_uint(v), flag);
}
template <typename T> __device__ __forceinline__ T ll_load_val(const uint64_t* p, uint32_t flag, int* err);
template <> __device__ __forceinline__ double ll_load_val<double>(const uint64_t* p, uint32_t flag, int* err) {
  return ll_load_f64(p, flag, err);
}
template <> __device__ __forceinline__ float ll_load_val<float>(const uint64_t* p, uint32_t flag, int* err) {
  return __uint_as_float(ll_load(p, flag, err));
}

// K values (value k at p + k * stride words) loaded with one combined wait:
// every word is requested before any flag is checked, so a ready message costs
// one round trip instead of K.  valid[k] = false skips value k.
template <typename T, int K>
__device__ __forceinline__ void ll_load_many(const uint64_t* p, int64_t stride, const bool* valid, uint32_t flag,
                                             int* err, T* out) {
  constexpr int LW = sizeof(T) == 8 ? 2 : 1;
  long long spins = 0;
  while (true) {
    uint64_t w[K][LW];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int h = 0; h < LW; ++h)
        w[k][h] = valid[k] ? __hip_atomic_load(const_cast<uint64_t*>(p + k * stride + h), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : ((uint64_t)flag << 32);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int h = 0; h < LW; ++h) ok = ok && ((uint32_t)(w[k][h] >> 32) == flag);
    if (ok) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if constexpr (LW == 2)
          out[k] = __longlong_as_double((long long)(((w[k][1] & 0xffffffffull) << 32) | (w[k][0] & 0xffffffffull)));
        else
          out[k] = __uint_as_float((uint32_t)w[k][0]);
      }
      return;
    }
    ++spins;
    if ((spins & 1023) == 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (T)0;
        return;
      }
      if (spins > (kSpinLimit >> 2)) {
        atomicExch(err, (int)kErrSpinTimeout);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (T)0;
        return;
      }
    }
  }
}

// K values at arbitrary addresses, one combined wait (see ll_load_many).
template <typename T, int K>
__device__ __forceinline__ void ll_wait_vals(const uint64_t* const* ptr, const bool* valid, uint32_t flag, int* err,
                                             T* out) {
  constexpr int LW = sizeof(T) == 8 ? 2 : 1;
  long long spins = 0;
  while (true) {
    uint64_t w[K][LW];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int h = 0; h < LW; ++h)
        w[k][h] = valid[k] ? __hip_atomic_load(const_cast<uint64_t*>(ptr[k] + h), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : ((uint64_t)flag << 32);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int h = 0; h < LW; ++h) ok = ok && ((uint32_t)(w[k][h] >> 32) == flag);
    if (ok) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if constexpr (LW == 2)
          out[k] = __longlong_as_double((long long)(((w[k][1] & 0xffffffffull) << 32) | (w[k][0] & 0xffffffffull)));
        else
          out[k] = __uint_as_float((uint32_t)w[k][0]);
      }
      return;
    }
    ++spins;
    if ((spins & 1023) == 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spins > (kSpinLimit >> 2)) {
        if (spins > (kSpinLimit >> 2)) atomicExch(err, (int)kErrSpinTimeout);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = (T)0;
        return;
      }
    }
  }
}

// N raw 32-bit payloads at p[0..N) with one combined wait.
template <int N>
__device__ __forceinline__ void ll_wait_words(const uint64_t* p, uint32_t flag, int* err, uint32_t* out) {
  long long spins = 0;
  while (true) {
    uint64_t w[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
      w[k] = __hip_atomic_load(const_cast<uint64_t*>(p + k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < N; ++k) ok = ok && ((uint32_t)(w[k] >> 32) == flag);
    if (ok) {
#pragma unroll
      for (int k = 0; k < N; ++k) out[k] = (uint32_t)w[k];
      return;
    }
    ++spins;
    if ((spins & 1023) == 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spins > (kSpinLimit >> 2)) {
        if (spins > (kSpinLimit >> 2)) atomicExch(err, (int)kErrSpinTimeout);
#pragma unroll
        for (int k = 0; k < N; ++k) out[k] = 0u;
        return;
      }
    }
  }
}

// words per value in a message
template <typename T> struct LLWords { static constexpr int n = 2; };
template <> struct LLWords<float> { static constexpr int n = 1; };

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, kWave); }

// (|v|, row) arg-max over the wave: larger magnitude wins, ties go to the lower
// row index.  Invalid entries carry mag = -1.
template <typename T>
__device__ __forceinline__ void wave_argmax(T& mag, int& row) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    T om = shfl_xor(mag, m);
    int orow = shfl_xor(row, m);
    bool take = (om > mag) || (om == mag && orow < row);
    mag = take ? om : mag;
    row = take ? orow : row;
  }
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, shfl_xor(v, m));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
  return v;
}

// Wave-uniform max / min of a 32-bit value: DPP exchanges inside each 16-lane
// row (quad permutes, half-row and row mirrors), then the four row results
// through readlane.  Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  const uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return min(min(a, b), min(c, d));
}

// Pivot search over the wave: the largest magnitude wins, ties go to the lowest
// row.  Lanes with valid = false, a NaN or a negative magnitude take no part.
// Magnitudes are compared through their bit patterns (monotone for values
// >= 0): the high word first, then the low word among the leaders.  The result
// is uniform; with no valid lane best_mag = -1 and best_row = INT_MAX.
template <typename T>
__device__ __forceinline__ void wave_pivot_search(T mag, int row, bool valid, T& best_mag, int& best_row) {
  valid = valid && (mag >= (T)0);   // false for NaN
  bool lead;
  if constexpr (sizeof(T) == 8) {
    const uint64_t bits = (uint64_t)__double_as_longlong(mag);
    const uint32_t hi = valid ? (uint32_t)(bits >> 32) + 1u : 0u;
    const uint32_t mh = wave_max_u32(hi);
    const uint32_t lo = (valid && hi == mh) ? (uint32_t)bits : 0u;
    const uint32_t ml = wave_max_u32(lo);
    lead = valid && hi == mh && (uint32_t)bits == ml;
    best_mag = mh == 0u ? (T)-1 : __longlong_as_double((long long)(((uint64_t)(mh - 1u) << 32) | ml));
  } else {
    const uint32_t k = valid ? __float_as_uint(mag) + 1u : 0u;
    const uint32_t mk = wave_max_u32(k);
    lead = valid && k == mk;
    best_mag = mk == 0u ? (T)-1 : __uint_as_float(mk - 1u);
  }
  best_row = (int)wave_min_u32(lead ? (uint32_t)row : 0x7fffffffu);
}

// Value of lane t (wave-uniform t) in every lane, through readlane (no LDS).
template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int t) {
  if constexpr (sizeof(T) == 8) {
    const long long bits = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), t);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
  }
}

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Orders LDS accesses between the lanes of one wave (lanes run in lockstep and
// the LDS serves one wave's requests in order; this keeps the compiler from
// moving accesses across the point).
// Sum over each 16-lane row of the wave (quad permutes, half-row and row mirrors);
// every lane of the row gets the row's sum, added in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm 1,0,3,2
  v += dpp_move<0x4E>(v);    // quad_perm 2,3,0,1
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return v;
}

// Column c of the inverse of the 16 x 16 diagonal block blk of the lower
// triangle L (unit diagonal when UNIT), by forward substitution in FP64, into
// Linv[blk * 256 + i * 16 + c]; rows of the block at or beyond jb act as the
// identity.
template <typename T, bool UNIT>
__device__ __forceinline__ void diag_inv16_column(const T* L, int64_t lda, int jb, int blk, int c, double* Linv) {
  const int r0 = blk * 16, rb = min(16, jb - r0);
  double y[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i >= rb) {
      y[i] = (i == c) ? 1.0 : 0.0;
      continue;
    }
    double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < i; ++q)
      if (q >= c) s -= (double)L[(r0 + i) + (size_t)(r0 + q) * lda] * y[q];
    y[i] = (i < c) ? 0.0 : (UNIT ? s : s / (double)L[(r0 + i) + (size_t)(r0 + i) * lda]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) Linv[(size_t)blk * 256 + i * 16 + c] = y[i];
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace cds

#define CDS_HIP_CHECK(expr)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return CDS_HIP_ERROR;      \
  } while (0)
