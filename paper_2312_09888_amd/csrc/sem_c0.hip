// C0 averaging over shared GLL nodes, global edge keys and welded output.
//
// Elements store their own copy of every node; a global id per stored node
// says which copies coincide.  The direct-stiffness average (the
// gather-scatter sum of spectral-element codes, Deville, Fischer & Mund
// 2002, ch. 4, divided by the multiplicity) replaces each copy by the mean
// over all copies of its node, which makes per-element derived fields
// continuous and their isosurfaces closed across element faces.
//
// sem_gs_setup turns the ids into a compressed row structure (copies of a
// global node listed in increasing storage order), so every average is
// summed in one fixed order and the result does not depend on scheduling.
// Welding numbers the distinct global edge keys of a triangle soup in order
// of first occurrence: a hash table records each key's first corner, a flag
// marks those corners, and their exclusive prefix gives the vertex index.
#include <hip/hip_runtime.h>

#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kEmpty = ~0ull;

inline unsigned blocks_for(int64_t n) {
  return (unsigned)((n + kThreads - 1) / kThreads > 0 ? (n + kThreads - 1) / kThreads : 1);
}

__global__ void fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// copies per global node
__global__ void gs_count(int64_t n_nodes, const int64_t* __restrict__ gid, int64_t n_global,
                         int32_t* __restrict__ cnt, int32_t* __restrict__ status) {
  const int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (n >= n_nodes) return;
  const int64_t g = gid[n];
  if (g < 0 || g >= n_global) {
    if (status) atomicOr(status, SEM_FLAG_BAD_ID);
    return;
  }
  atomicAdd(&cnt[g], 1);
}

// place every copy in its node's row (arbitrary order within the row)
__global__ void gs_fill(int64_t n_nodes, const int64_t* __restrict__ gid, int64_t n_global,
                        const int64_t* __restrict__ rowptr, int32_t* __restrict__ cursor,
                        int64_t* __restrict__ col) {
  const int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (n >= n_nodes) return;
  const int64_t g = gid[n];
  if (g < 0 || g >= n_global) return;
  col[rowptr[g] + atomicAdd(&cursor[g], 1)] = n;
}

// order each row by storage index (rows are short: the copies of one node)
__global__ void gs_sort(int64_t n_global, const int64_t* __restrict__ rowptr,
                        int64_t* __restrict__ col) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n_global) return;
  const int64_t a = rowptr[g], b = rowptr[g + 1];
  for (int64_t i = a + 1; i < b; ++i) {
    const int64_t v = col[i];
    int64_t j = i - 1;
    while (j >= a && col[j] > v) {
      col[j + 1] = col[j];
      --j;
    }
    col[j + 1] = v;
  }
}

// mean over the copies of each global node, summed in storage order, then
// written back to every copy (in may equal out)
template <typename T>
__global__ void dsavg_k(int64_t n_global, const int64_t* __restrict__ rowptr,
                        const int64_t* __restrict__ col, const T* in, T* out) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (g >= n_global) return;
  const int64_t a = rowptr[g], b = rowptr[g + 1];
  if (a == b) return;
  T s = T(0);
  for (int64_t i = a; i < b; ++i) s += in[col[i]];
  const T avg = s / (T)(b - a);
  for (int64_t i = a; i < b; ++i) out[col[i]] = avg;
}

// element-local key (e P^3 + n_lo) * 3 + axis  ->  (min gid << 32) | max gid
__global__ void global_keys_k(int64_t n_ref, int p, int64_t n_elem,
                              const uint64_t* __restrict__ local,
                              const int64_t* __restrict__ gid, uint64_t* __restrict__ global,
                              int32_t* __restrict__ status) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_ref) return;
  const uint64_t k = local[r];
  const int axis = (int)(k % 3u);
  const uint64_t flat = k / 3u;
  const uint64_t p3 = (uint64_t)p * p * p;
  const uint64_t e = flat / p3, lo = flat % p3;
  const uint64_t step = axis == 0 ? 1u : (axis == 1 ? (uint64_t)p : (uint64_t)p * p);
  const uint64_t hi = lo + step;
  if (e >= (uint64_t)n_elem || hi >= p3) {
    if (status) atomicOr(status, SEM_FLAG_BAD_ID);
    global[r] = kEmpty;
    return;
  }
  const int64_t a = gid[e * p3 + lo], b = gid[e * p3 + hi];
  if (a < 0 || b < 0 || a >= (int64_t)0xffffffffll || b >= (int64_t)0xffffffffll) {
    if (status) atomicOr(status, SEM_FLAG_BAD_ID);
    global[r] = kEmpty;
    return;
  }
  const uint64_t mn = (uint64_t)(a < b ? a : b), mx = (uint64_t)(a < b ? b : a);
  global[r] = (mn << 32) | mx;
}

// 64-bit finaliser of SplitMix64 (Steele, Lea & Flood 2014) as the hash
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// table slot of every corner's key (linear probing; the table is at least
// twice the number of corners, so a free slot is always reached), and the
// smallest corner index per key
__global__ void weld_insert(int64_t n_ref, const uint64_t* __restrict__ keys,
                            uint64_t* __restrict__ tkey, uint64_t* __restrict__ tpos,
                            int32_t* __restrict__ slot, int64_t cap,
                            int32_t* __restrict__ status) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_ref) return;
  const uint64_t k = keys[r];
  if (k == kEmpty) {
    if (status) atomicOr(status, SEM_FLAG_BAD_ID);
    slot[r] = -1;
    return;
  }
  const uint64_t mask = (uint64_t)cap - 1;
  uint64_t h = mix64(k) & mask;
  for (int64_t probe = 0; probe < cap; ++probe) {
    const uint64_t prev = atomicCAS((unsigned long long*)&tkey[h], (unsigned long long)kEmpty,
                                    (unsigned long long)k);
    if (prev == kEmpty || prev == k) {
      atomicMin((unsigned long long*)&tpos[h], (unsigned long long)r);
      slot[r] = (int32_t)h;
      return;
    }
    h = (h + 1) & mask;
  }
  slot[r] = -1;   // unreachable with a half-empty table
  if (status) atomicOr(status, SEM_FLAG_BAD_ID);
}

__global__ void weld_flag(int64_t n_ref, const int32_t* __restrict__ slot,
                          const uint64_t* __restrict__ tpos, int32_t* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_ref) return;
  const int32_t h = slot[r];
  flag[r] = (h >= 0 && tpos[h] == (uint64_t)r) ? 1 : 0;
}

template <typename T>
__global__ void weld_emit(int64_t n_ref, const int32_t* __restrict__ slot,
                          const uint64_t* __restrict__ tpos, const int64_t* __restrict__ offs,
                          const T* __restrict__ tri_xyz, int64_t* __restrict__ tri_index,
                          T* __restrict__ vert_xyz, int64_t vert_cap) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_ref) return;
  const int32_t h = slot[r];
  if (h < 0) {
    tri_index[r] = -1;
    return;
  }
  const int64_t first = (int64_t)tpos[h];
  const int64_t v = offs[first];
  tri_index[r] = v;
  if (first == r && v < vert_cap) {
    vert_xyz[3 * v] = tri_xyz[3 * r];
    vert_xyz[3 * v + 1] = tri_xyz[3 * r + 1];
    vert_xyz[3 * v + 2] = tri_xyz[3 * r + 2];
  }
}

__global__ void weld_total(const int64_t* __restrict__ offs, int64_t n_ref,
                           int64_t* __restrict__ n_vert, int64_t vert_cap,
                           int32_t* __restrict__ status) {
  const int64_t total = offs[n_ref];
  *n_vert = total;
  if (status && total > vert_cap) atomicOr(status, SEM_FLAG_VERT_OVERFLOW);
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

GsLayout gs_layout(void* base, int64_t n_nodes, int64_t n_global) {
  GsLayout l;
  const size_t b_cnt = al256((size_t)n_global * sizeof(int32_t));
  const size_t b_row = al256((size_t)(n_global + 1) * sizeof(int64_t));
  const size_t b_par = al256((size_t)(scan_partials_capacity(n_global) + 1) * sizeof(int64_t));
  const size_t b_col = al256((size_t)n_nodes * sizeof(int64_t));
  char* p = static_cast<char*>(base);
  l.cnt = reinterpret_cast<int32_t*>(p);
  l.rowptr = reinterpret_cast<int64_t*>(p ? p + b_cnt : nullptr);
  l.partial = reinterpret_cast<int64_t*>(p ? p + b_cnt + b_row : nullptr);
  l.col = reinterpret_cast<int64_t*>(p ? p + b_cnt + b_row + b_par : nullptr);
  l.bytes = b_cnt + b_row + b_par + b_col;
  return l;
}

hipError_t launch_gs_setup(int64_t n_nodes, const int64_t* gid, int64_t n_global,
                           const GsLayout& gs, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32, dim3(blocks_for(n_global)), dim3(kThreads), 0, s, gs.cnt,
                     n_global, 0);
  hipLaunchKernelGGL(gs_count, dim3(blocks_for(n_nodes)), dim3(kThreads), 0, s, n_nodes, gid,
                     n_global, gs.cnt, status);
  hipError_t e = launch_exclusive_scan(gs.cnt, n_global, gs.partial, gs.rowptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_i32, dim3(blocks_for(n_global)), dim3(kThreads), 0, s, gs.cnt,
                     n_global, 0);
  hipLaunchKernelGGL(gs_fill, dim3(blocks_for(n_nodes)), dim3(kThreads), 0, s, n_nodes, gid,
                     n_global, gs.rowptr, gs.cnt, gs.col);
  hipLaunchKernelGGL(gs_sort, dim3(blocks_for(n_global)), dim3(kThreads), 0, s, n_global,
                     gs.rowptr, gs.col);
  return hipGetLastError();
}

hipError_t launch_dsavg(sem_dtype dt, int64_t n_global, const GsLayout& gs, const void* in,
                        void* out, hipStream_t s) {
  if (dt == SEM_F64)
    hipLaunchKernelGGL(dsavg_k<double>, dim3(blocks_for(n_global)), dim3(kThreads), 0, s,
                       n_global, (const int64_t*)gs.rowptr, (const int64_t*)gs.col,
                       (const double*)in, (double*)out);
  else
    hipLaunchKernelGGL(dsavg_k<float>, dim3(blocks_for(n_global)), dim3(kThreads), 0, s,
                       n_global, (const int64_t*)gs.rowptr, (const int64_t*)gs.col,
                       (const float*)in, (float*)out);
  return hipGetLastError();
}

hipError_t launch_global_keys(int64_t n_ref, int order, int64_t n_elem, const uint64_t* local,
                              const int64_t* gid, uint64_t* global, int32_t* status,
                              hipStream_t s) {
  hipLaunchKernelGGL(global_keys_k, dim3(blocks_for(n_ref)), dim3(kThreads), 0, s, n_ref,
                     order + 1, n_elem, local, gid, global, status);
  return hipGetLastError();
}

WeldLayout weld_layout(void* base, int64_t n_ref) {
  WeldLayout w;
  int64_t cap = 64;
  while (cap < 2 * n_ref) cap <<= 1;
  w.cap = cap;
  const size_t b_key = al256((size_t)cap * sizeof(uint64_t));
  const size_t b_slot = al256((size_t)n_ref * sizeof(int32_t));
  const size_t b_offs = al256((size_t)(n_ref + 1) * sizeof(int64_t));
  const size_t b_par = al256((size_t)(scan_partials_capacity(n_ref) + 1) * sizeof(int64_t));
  char* p = static_cast<char*>(base);
  size_t o = 0;
  w.key = reinterpret_cast<uint64_t*>(p ? p + o : nullptr);
  o += b_key;
  w.pos = reinterpret_cast<uint64_t*>(p ? p + o : nullptr);
  o += b_key;
  w.slot = reinterpret_cast<int32_t*>(p ? p + o : nullptr);
  o += b_slot;
  w.flag = reinterpret_cast<int32_t*>(p ? p + o : nullptr);
  o += b_slot;
  w.offs = reinterpret_cast<int64_t*>(p ? p + o : nullptr);
  o += b_offs;
  w.partial = reinterpret_cast<int64_t*>(p ? p + o : nullptr);
  o += b_par;
  w.bytes = o;
  return w;
}

hipError_t launch_weld(int64_t n_ref, sem_dtype dt, const void* tri_xyz, const uint64_t* keys,
                       int64_t* tri_index, void* vert_xyz, int64_t vert_cap, int64_t* n_vert,
                       const WeldLayout& w, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64, dim3(blocks_for(w.cap)), dim3(kThreads), 0, s, w.key, w.cap,
                     kEmpty);
  hipLaunchKernelGGL(fill_u64, dim3(blocks_for(w.cap)), dim3(kThreads), 0, s, w.pos, w.cap,
                     kEmpty);
  if (n_ref > 0) {
    hipLaunchKernelGGL(weld_insert, dim3(blocks_for(n_ref)), dim3(kThreads), 0, s, n_ref, keys,
                       w.key, w.pos, w.slot, w.cap, status);
    hipLaunchKernelGGL(weld_flag, dim3(blocks_for(n_ref)), dim3(kThreads), 0, s, n_ref,
                       (const int32_t*)w.slot, (const uint64_t*)w.pos, w.flag);
  }
  hipError_t e = launch_exclusive_scan(w.flag, n_ref, w.partial, w.offs, s);
  if (e != hipSuccess) return e;
  if (n_ref > 0) {
    if (dt == SEM_F64)
      hipLaunchKernelGGL(weld_emit<double>, dim3(blocks_for(n_ref)), dim3(kThreads), 0, s,
                         n_ref, (const int32_t*)w.slot, (const uint64_t*)w.pos,
                         (const int64_t*)w.offs, (const double*)tri_xyz, tri_index,
                         (double*)vert_xyz, vert_cap);
    else
      hipLaunchKernelGGL(weld_emit<float>, dim3(blocks_for(n_ref)), dim3(kThreads), 0, s,
                         n_ref, (const int32_t*)w.slot, (const uint64_t*)w.pos,
                         (const int64_t*)w.offs, (const float*)tri_xyz, tri_index,
                         (float*)vert_xyz, vert_cap);
  }
  hipLaunchKernelGGL(weld_total, dim3(1), dim3(1), 0, s, (const int64_t*)w.offs, n_ref, n_vert,
                     vert_cap, status);
  return hipGetLastError();
}

}  // namespace sem
