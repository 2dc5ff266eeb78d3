// Small utility kernels: clearing scratch memory with a fill kernel (kept free
// of memset nodes so that the enqueued work can be captured into a graph).
#include "common.hpp"
#include "kernels.hpp"

namespace cds {

namespace {
__global__ void fill_zero_kernel(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  // p is 16-byte aligned for every caller (workspace regions are 256-byte aligned)
  size_t n16 = bytes / 16, ntail = bytes % 16;
  int blocks = (int)std::min<size_t>(4096, (n16 + 255) / 256 + 1);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

hipEvent_t KTimer::next() {
  if (used == pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[used++];
}
void KTimer::reset() {
  recs.clear();
  used = 0;
}
KTimer::~KTimer() {
  for (auto e : pool) (void)hipEventDestroy(e);
}
KScope::KScope(KTimer* timer, int kc, hipStream_t stream, double flops, double bytes) : t(timer), s(stream), idx(0) {
  if (!t) return;
  hipEvent_t a = t->next(), b = t->next();
  if (!a || !b) { t = nullptr; return; }
  (void)hipEventRecord(a, s);
  t->recs.push_back(KTimer::Rec{kc, a, b, flops, bytes});
  idx = t->recs.size() - 1;
}
KScope::~KScope() {
  if (t) (void)hipEventRecord(t->recs[idx].b, s);
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>(1024, (count + 255) / 256);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace cds
