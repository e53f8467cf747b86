// A plain streaming copy (16-byte non-temporal loads and stores, a
// persistent grid): the achievable-bandwidth reference the measurements of
// the Kronecker kernels are compared with.  It is not part of the action.
// Its shape is the fastest of a sweep on MI355X (1 GiB, 2 GiB moved): 2 KiB
// per wavefront step and two workgroups per CU, 5.95 TB/s; 4 KiB per step
// gave 5.70-5.76 at one to eight workgroups per CU, 8 KiB per step 3.7-5.5,
// plain (temporal) accesses 1-5 % less, and one contiguous range per
// wavefront 4.3-5.0.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kron.h"
#include "kron_launch.hpp"

namespace kron {
namespace {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void kron_copy_kernel(const u32x4_t* __restrict__ src, u32x4_t* __restrict__ dst,
                                                          int64_t nvec) {
  constexpr int kU = 2;  // vectors per lane in flight: 2 KiB per wavefront step
  const int l = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t base = wave * 64 * kU; base < nvec; base += nwaves * 64 * kU) {
    u32x4_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * 64 + l;
      if (i < nvec) v[u] = __builtin_nontemporal_load(in_global(src) + i);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + u * 64 + l;
      if (i < nvec) __builtin_nontemporal_store(v[u], in_global(dst) + i);
    }
  }
}

}  // namespace
}  // namespace kron

extern "C" int kron_copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  if (!src || (reinterpret_cast<uintptr_t>(src) & 15)) return -1;
  if (!dst || (reinterpret_cast<uintptr_t>(dst) & 15) || dst == src) return -2;
  if (bytes % 16) return -3;
  if (bytes == 0) return 0;
  const int64_t nvec = (int64_t)(bytes / 16);
  auto k = kron::kron_copy_kernel;
  const int64_t waves = (nvec + 127) / 128;
  hipLaunchKernelGGL(k, dim3(kron::grid_blocks(waves, kron::occupancy_blocks(k), 2)), dim3(kron::kBlock), 0, stream,
                     static_cast<const kron::u32x4_t*>(src), static_cast<kron::u32x4_t*>(dst), nvec);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}
