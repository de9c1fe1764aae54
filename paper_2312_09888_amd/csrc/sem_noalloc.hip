// Fixed device scratch for sem_extract_noalloc: the per-(isovalue, element)
// triangle counts, their exclusive prefix and the scan's block partials live
// in one statically sized array per GPU instead of a caller workspace.
#include "sem_internal.h"

namespace sem {

// Largest n_iso * n_elem the scratch holds (SEM_NOALLOC_MAX_COUNTS): int32
// counts, int64 offsets (one more than the counts) and int64 scan partials,
// each 256-byte aligned, as iso_workspace_layout places them.
constexpr int64_t kNoallocCounts = SEM_NOALLOC_MAX_COUNTS;
constexpr size_t align_up(size_t b) { return (b + 255) & ~size_t(255); }
// every count up to kNoallocCounts takes the 1,024-count tiles, so the
// largest count has the most tile sums
static_assert(kNoallocCounts <= kScanSmall, "one tile size for every count the scratch takes");
constexpr size_t kNoallocBytes =
    align_up(sizeof(int32_t) * kNoallocCounts) + align_up(sizeof(int64_t) * (kNoallocCounts + 1)) +
    align_up(sizeof(int64_t) * (scan_partials_capacity(kNoallocCounts) + 1));

}  // namespace sem

// One copy per GPU, resident until the process ends.  Host code never
// passes this name to a kernel: it is a host-side stand-in for the device
// symbol, whose device address noalloc_scratch() looks up per device.
static __device__ __align__(256) unsigned char scratch[sem::kNoallocBytes];

namespace sem {

hipError_t noalloc_scratch(void** ptr) {
  *ptr = nullptr;
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

size_t noalloc_scratch_bytes() { return kNoallocBytes; }

}  // namespace sem
