// Plain device-to-device copy: the reference kernel for achievable HBM
// bandwidth on this GPU (a measurement aid, not part of the method).  Every
// figure of the extraction kernels is reported both against the HBM peak
// and against the rate this kernel sustains on the same device.
#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Grid-stride loop over 16-byte chunks; each thread keeps kCopyUnroll loads
// in flight before its stores, consecutive lanes touch consecutive chunks;
// loads and stores carry the non-temporal hint (the data is touched once).
// Measured on one MI355X (1 GiB each way): 4.27 TB/s without the hint at 8
// workgroups per CU, 5.09 TB/s with it at 32 per CU.
__global__ void __launch_bounds__(kCopyThreads)
stream_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
  int64_t i = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    u32x4 r[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) r[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(r[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return hipSuccess;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // 32 workgroups per CU (the fastest of 4, 8, 16, 32 measured); a
  // grid-stride loop covers any size
  const int64_t want = (n + kCopyThreads - 1) / kCopyThreads;
  const int grid = (int)(want < (int64_t)cus * 32 ? want : (int64_t)cus * 32);
  hipLaunchKernelGGL(stream_copy16, dim3(grid), dim3(kCopyThreads), 0, s,
                     static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
  return hipGetLastError();
}

}  // namespace sem
