// Plain device-to-device copy: the reference kernel for achievable HBM
// bandwidth on this GPU (a measurement aid, not part of the method).  Every
// figure of the extraction kernels is reported both against the HBM peak
// and against the rate this kernel sustains on the same device.
#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;

// Grid-stride loop over 16-byte chunks; each thread keeps kCopyUnroll loads
// in flight before its stores, consecutive lanes touch consecutive chunks.
__global__ void __launch_bounds__(kCopyThreads)
stream_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
  int64_t i = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    uint4 r[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) r[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) dst[i + u * stride] = r[u];
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
  // eight workgroups per CU keep every CU busy; a grid-stride loop covers
  // any size
  const int64_t want = (n + kCopyThreads - 1) / kCopyThreads;
  const int grid = (int)(want < (int64_t)cus * 8 ? want : (int64_t)cus * 8);
  hipLaunchKernelGGL(stream_copy16, dim3(grid), dim3(kCopyThreads), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  return hipGetLastError();
}

}  // namespace sem
