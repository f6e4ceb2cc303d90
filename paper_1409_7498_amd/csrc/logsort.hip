// logsort.hip -- canonical order of a resident system's bond log, on the device.
//
// The log holds rows (step, id_A, id_T) of int32.  The closing kernels append
// the rows of one step together and the steps in order, but within a step in
// the order the workgroups reserved their ranges.  The canonical order of the
// emitted bonds (Table I, step 9: each step's bonds by id_A) is restored here
// by one radix sort of the 64-bit keys (step << 32 | id_A) with id_T as the
// value, written back in place, so that the log in HBM is ordered for any
// consumer and the host copy needs no sorting.  Keys are unique: a particle
// takes at most one bond per step.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <stdint.h>

namespace pr {

namespace {

__global__ void k_log_keys(const int32_t* __restrict__ log, int64_t n,
                           unsigned long long* __restrict__ key, int32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = ((unsigned long long)(uint32_t)log[3 * i] << 32) | (uint32_t)log[3 * i + 1];
  val[i] = log[3 * i + 2];
}

__global__ void k_log_rows(int32_t* __restrict__ log, int64_t n,
                           const unsigned long long* __restrict__ key,
                           const int32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  log[3 * i] = (int32_t)(uint32_t)(key[i] >> 32);
  log[3 * i + 1] = (int32_t)(uint32_t)key[i];
  log[3 * i + 2] = val[i];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Orders rows [0, n) of `log` (device memory, 3 int32 per row) by (step, id_A)
// in place, in stream order on `s`.  Temporary device memory (about 24 bytes
// per row plus the sort's own) is taken from and returned to the stream's
// memory pool.  Returns hipSuccess or the first HIP error.
hipError_t log_order(int32_t* log, int64_t n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  const size_t nn = (size_t)n;
  size_t tmp_bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, (unsigned long long*)nullptr,
                                           (unsigned long long*)nullptr, (int32_t*)nullptr,
                                           (int32_t*)nullptr, nn, 0, 64, s);
  if (e != hipSuccess) return e;
  const size_t kb = align256(nn * sizeof(unsigned long long)), vb = align256(nn * sizeof(int32_t));
  char* buf = nullptr;
  if ((e = hipMallocAsync((void**)&buf, 2 * kb + 2 * vb + align256(tmp_bytes), s)) != hipSuccess)
    return e;
  auto* k0 = (unsigned long long*)buf;
  auto* k1 = (unsigned long long*)(buf + kb);
  auto* v0 = (int32_t*)(buf + 2 * kb);
  auto* v1 = (int32_t*)(buf + 2 * kb + vb);
  void* tmp = buf + 2 * kb + 2 * vb;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  k_log_keys<<<blocks, 256, 0, s>>>(log, n, k0, v0);
  e = hipGetLastError();
  if (e == hipSuccess) e = rocprim::radix_sort_pairs(tmp, tmp_bytes, k0, k1, v0, v1, nn, 0, 64, s);
  if (e == hipSuccess) {
    k_log_rows<<<blocks, 256, 0, s>>>(log, n, k1, v1);
    e = hipGetLastError();
  }
  const hipError_t f = hipFreeAsync(buf, s);
  return e != hipSuccess ? e : f;
}

}  // namespace pr
