// Internal declarations shared by the host files and the kernel file.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "../../include/sem.h"

namespace sem {

constexpr int kMaxBasisOrder = 15;          // host basis queries
constexpr int kMaxOrder = SEM_MAX_ORDER;    // kernels
constexpr int kMcMaxTri = SEM_MC_MAX_TRI;

// FP32 fields: line sums of orders up to kF32SumOrder run in FP32 with the
// FP32-rounded D and even-odd halves; higher orders sum in FP64 with the
// FP64 tables.
constexpr int kF32SumOrder = 8;
constexpr bool f32_line_sums(int order) { return order <= kF32SumOrder; }

// sem_basis.cpp
bool gll_basis(int n, double* nodes, double* weights, double* dmat);
// sem_mctable.cpp
void build_mc_table(uint8_t* ntri, int8_t* tri);

// Device-resident constant tables of one GPU.
struct DeviceTables {
  // D of each order, row-major (N+1)^2, followed by its even-odd halves
  // A[NE][NE], B[NE][NE] (NE = ceil((N+1)/2)): FP64, and the same values
  // rounded to FP32
  const double* d64[kMaxOrder + 1];
  const float* d32[kMaxOrder + 1];
  const uint8_t* ntri;                // [256]
  const int8_t* tri;                  // [256][kMcMaxTri][3]
  const double* eo7;                  // N = 7 even-odd form of D: A[4][4], B[4][4]
  int cu_count;                       // compute units (persistent grids)
  void* scratch;                      // device address of this GPU's copy of the
                                      // fixed scratch array (sem_noalloc.hip)
  int tuned_variant[2][kMaxOrder + 1];  // batch variant + 1 per (dtype, order); 0 = not tuned
};

template <typename T>
struct IsoList {
  T v[SEM_MAX_ISO];
};

// Triangle destinations: one contiguous buffer for all isovalues
// (per_iso == 0: ptr[0], cap[0], global offsets) or one buffer per isovalue
// (per_iso == 1: ptr[s], cap[s], offsets within isovalue s).
template <typename T>
struct IsoOut {
  T* ptr[SEM_MAX_ISO];
  int64_t cap[SEM_MAX_ISO];
  int per_iso;
};

// Isosurface workspace layout (offsets in bytes from the workspace start).
struct IsoWorkspace {
  int32_t* cnt;       // [n_iso * n_elem] triangles per (isovalue, element)
  int64_t* offs;      // [n_iso * n_elem + 1] exclusive prefix of cnt
  int64_t* partial;   // [scan blocks + 1]
  size_t bytes;
};
IsoWorkspace iso_workspace_layout(void* base, int64_t n_elem, int n_iso);

// Exclusive-scan tiling, shared by the kernels and every workspace that
// holds the tile sums: tiles of 1,024 counts up to kScanSmall counts (more
// workgroups, a shorter chain per tile), of 4,096 above.
constexpr int64_t kScanSmall = int64_t(1) << 20;
constexpr int64_t scan_tile(int64_t count) { return count <= kScanSmall ? 1024 : 4096; }
constexpr int64_t scan_tiles(int64_t count) {
  return count <= 0 ? 1 : (count + scan_tile(count) - 1) / scan_tile(count);
}
// Tile sums a scan of `count` values writes (scan_tiles(count)).
int64_t scan_blocks(int64_t count);
// Tile sums to reserve for a scan of `count` values: at least
// scan_tiles(count), and never fewer for a larger count (the tile count
// itself drops where the tile grows), so that workspace sizes grow with
// the problem.
constexpr int64_t scan_partials_capacity(int64_t count) {
  return count <= kScanSmall ? scan_tiles(count)
                             : (scan_tiles(count) > kScanSmall / 1024 ? scan_tiles(count)
                                                                      : kScanSmall / 1024);
}

// Exclusive prefix of count int32 values into offs[0..count] (offs[count] =
// total); partial holds scan_blocks(count) + 1 int64.
hipError_t launch_exclusive_scan(const int32_t* cnt, int64_t count, int64_t* partial,
                                 int64_t* offs, hipStream_t s);

// Batched snapshots: a plan (device) holds a header and one descriptor per
// snapshot; one persistent kernel walks the work items (chunks of `chunk`
// elements of one snapshot) of all snapshots.
struct BatchHeader {
  int32_t n_snap;
  int32_t dt;
  int32_t snap_begin[kMaxOrder + 2];   // descriptors sorted by order: [begin(N), begin(N+1))
  int64_t items[kMaxOrder + 1];        // work items of each order
};
struct BatchSnap {
  int64_t n_elem;
  int64_t item_begin;   // first work item of this snapshot among those of its order
  int32_t order;
  int32_t chunk;        // elements per work item
  int32_t form;         // BatchForm of this order's work items
  int32_t pad;
  const void* f[6];     // x, y, z, u, v, w
  void* q;
  void* om;
  void* qmm;
  const void* dmat;     // D and its halves in the line sums' type (d64 or d32)
  const void* eo;       // even-odd halves of D (order 7)
};
constexpr int kBatchMaxSnap = 4096;
size_t batch_plan_bytes(int n_snap);
// Batch variants: 0, 1, 2 = LDS-tile form with 1, 2, 4 elements per work
// item (256 threads); 3 = register-pencil form (N <= 7); 4 = direct-to-LDS
// form (N = 7, FP64); 5 = one thread per node.  Variants 3-5 take one
// element per work item and are the per-element kernels of sem_qcrit.
constexpr int kBatchVariants = 6;
enum BatchForm { kBatchChunk = 0, kBatchPencil = 1, kBatchDma7 = 2, kBatchNodeTile = 3 };
bool batch_variant_ok(int order, sem_dtype dt, int variant);
int batch_variant_chunk(int order, sem_dtype dt, int variant);   // elements per work item
int batch_variant_form(int variant);
int batch_default_variant(int order, sem_dtype dt);
// Launch code of a plan: 3 bits per order at bit 3N, 0 = no snapshot of
// that order, else 1 + the form its work items use.
inline int launch_code_form(unsigned code, int n) { return (int)((code >> (3 * n)) & 7u) - 1; }
hipError_t launch_qcrit_batch(sem_dtype dt, const void* plan, unsigned launch_code, int grid,
                              int32_t* status, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Batched isosurfaces: a plan (device) holds a header and one descriptor
// per job (one field of one snapshot at up to four isovalues), grouped by
// order; persistent count and emission kernels walk each order's work
// items (one element each).
struct IsoBatchHeader {
  int32_t n_job;
  int32_t dt;
  int32_t job_begin[kMaxOrder + 2];   // descriptors sorted by order: [begin(N), begin(N+1))
  int64_t items[kMaxOrder + 1];       // work items of each order
  int64_t n_slots;                    // count slots of every job
};
struct IsoBatchJob {
  int64_t n_elem;
  int64_t item_begin;   // first work item of this job among those of its order
  int64_t slot_begin;   // count of (isovalue s, element e) at slot_begin + s * n_elem + e
  int32_t order;
  int32_t n_iso;        // 1..4
  int32_t job;          // index in the caller's job array
  int32_t pad;
  const void* x;
  const void* y;
  const void* z;
  const void* field;
  const void* mm;       // element ranges of the field, or NULL
  double isod[4];       // isovalues in the plan's precision
  float isof[4];
};
static_assert(sizeof(IsoBatchHeader) <= 256, "header fits the plan's first 256 bytes");
constexpr int kIsoBatchMaxJob = 16384;
size_t iso_batch_plan_bytes(int n_job);
// Launch code of an isosurface plan: bit N set when some job has order N.
hipError_t launch_iso_batch(sem_dtype dt, const DeviceTables& tab, const void* plan,
                            unsigned launch_code, int n_job, int64_t n_slots, void* tri,
                            int64_t cap, int64_t* tri_offset, int64_t* tri_count,
                            int64_t* active, const IsoWorkspace& ws, int32_t* status,
                            hipStream_t s);

// synthetic well-shaped elements for timing (x, y, z, u, v, w)
hipError_t launch_tune_fill(sem_dtype dt, int order, int64_t n_elem, void* const* f,
                            hipStream_t s);

// sem_c0.hip: gather-scatter structure built by sem_gs_setup in the
// caller's buffer, C0 averaging, global edge keys, welding.
struct GsLayout {
  int32_t* cnt;       // [n_global] copies per global node (then a fill cursor)
  int64_t* rowptr;    // [n_global + 1] first copy of each global node
  int64_t* partial;   // scan partials
  int64_t* col;       // [n_nodes] storage index of each copy, by node, ascending
  size_t bytes;
};
GsLayout gs_layout(void* base, int64_t n_nodes, int64_t n_global);
hipError_t launch_gs_setup(int64_t n_nodes, const int64_t* gid, int64_t n_global,
                           const GsLayout& gs, int32_t* status, hipStream_t s);
hipError_t launch_dsavg(sem_dtype dt, int64_t n_global, const GsLayout& gs, const void* in,
                        void* out, hipStream_t s);
hipError_t launch_global_keys(int64_t n_ref, int order, int64_t n_elem, const uint64_t* local,
                              const int64_t* gid, uint64_t* global, int32_t* status,
                              hipStream_t s);
struct WeldLayout {
  uint64_t* key;      // [cap] hash table keys (all ones = empty)
  uint64_t* pos;      // [cap] first corner holding the key
  int32_t* slot;      // [n_ref] table slot of each corner
  int32_t* flag;      // [n_ref] 1 at a key's first corner
  int64_t* offs;      // [n_ref + 1] exclusive prefix of flag
  int64_t* partial;
  int64_t cap;
  size_t bytes;
};
WeldLayout weld_layout(void* base, int64_t n_ref);
hipError_t launch_weld(int64_t n_ref, sem_dtype dt, const void* tri_xyz, const uint64_t* keys,
                       int64_t* tri_index, void* vert_xyz, int64_t vert_cap, int64_t* n_vert,
                       const WeldLayout& w, int32_t* status, hipStream_t s);

// Kernel-phase timing (sem_api.cpp).  phase_timer() hands out two events
// when timing is on for the current device (else two nulls): the phase's
// first kernel is launched with `start`, its last with `stop`, through
// hipExtLaunchKernelGGL, which stamps them from the kernels' own dispatch
// timestamps (no extra packets on the stream); phase_done() then records
// the span.
struct PhaseTimer {
  hipEvent_t start = nullptr, stop = nullptr;
  int phase = -1, i0 = -1, i1 = -1;
};
PhaseTimer phase_timer(int phase);
void phase_done(const PhaseTimer& t);

// sem_noalloc.hip: device address of the fixed scratch array on the current
// device (looked up once per device by sem_init) and its size in bytes.
hipError_t noalloc_scratch(void** ptr);
size_t noalloc_scratch_bytes();

// sem_bw.hip: plain 16-byte-vector copy (bandwidth reference)
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// sem_kernels.hip -- launchers return hipSuccess or the launch error.
hipError_t launch_derivs(int order, sem_dtype dt, const DeviceTables& tab,
                         int64_t n_elem, const void* x, const void* y,
                         const void* z, const void* f, void* gx, void* gy,
                         void* gz, int32_t* status, hipStream_t s);

hipError_t launch_qcrit(int order, sem_dtype dt, const DeviceTables& tab,
                        int64_t n_elem, const void* x, const void* y,
                        const void* z, const void* u, const void* v,
                        const void* w, void* q, void* om, void* qmm,
                        int32_t* status, hipStream_t s);

hipError_t launch_extract(int order, sem_dtype dt, const DeviceTables& tab, int64_t n_elem,
                          const void* x, const void* y, const void* z, const void* u,
                          const void* v, const void* w, void* q, void* om, void* qmm,
                          int n_iso, const double* iso_host, void* const* tri_xyz,
                          const int64_t* tri_capacity, int64_t* tri_count,
                          int64_t* active_cells, const IsoWorkspace& ws, int32_t* status,
                          hipStream_t s);

hipError_t launch_isosurface(int order, sem_dtype dt, const DeviceTables& tab,
                             int64_t n_elem, const void* x, const void* y,
                             const void* z, const void* field,
                             const void* field_minmax, int n_iso,
                             const double* iso_host, void* tri_xyz,
                             int64_t tri_capacity, uint64_t* tri_edge_key,
                             int64_t* tri_count, int64_t* active_cells,
                             uint8_t* case_idx, const IsoWorkspace& ws,
                             int32_t* status, hipStream_t s);

// Learned compression (sem_ae.hip)
int64_t ae_param_count();
size_t ae_workspace_bytes(int64_t n);
size_t eig_workspace_bytes(int n);
size_t pca_workspace_bytes(int64_t n_pool);
size_t compress_workspace_bytes(int64_t n_elem);
hipError_t launch_ae_scales(int64_t n_elem, const float* const* f, float* scale,
                            uint32_t* gmax_bits, hipStream_t s);
hipError_t launch_ae_pack(int64_t e_begin, int64_t n, const float* const* f, const float* scale,
                          float* x, hipStream_t s);
hipError_t launch_ae_forward(int64_t n, const float* blocks, const float* params, int tanh_mask,
                             float* recon, uint16_t* latent, void* ws, hipStream_t s);
hipError_t launch_ae_grad(int64_t n, const float* pool, int64_t n_pool, const int64_t* idx,
                          const float* params, int tanh_mask, int loss_kind, float* grad,
                          float* loss, void* ws, int32_t* status, hipStream_t s);
hipError_t launch_ae_adam(int64_t n, float* p, const float* g, float* m, float* v, int step,
                          float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_sym_eig(int n, const double* a_in, int r, double* lam, float* w, void* ws,
                          int* sweeps, hipStream_t s);
hipError_t launch_ae_pca_init(int64_t n_pool, const float* pool, float* params, double* lams,
                              void* ws, hipStream_t s);
hipError_t launch_ae_compress(int64_t n_elem, const float* const* f, const float* params,
                              int tanh_mask, uint16_t* latent, float* scale, uint8_t* flags,
                              float* raw, int64_t raw_cap, int64_t* n_raw, void* ws,
                              int32_t* status, hipStream_t s);
hipError_t launch_ae_decompress(int64_t n_elem, const uint16_t* latent, const float* scale,
                                const uint8_t* flags, const float* raw, int64_t raw_count,
                                const float* params, int tanh_mask, float* const* f, void* ws,
                                int32_t* status, hipStream_t s);
hipError_t launch_modal(int64_t n_elem, const float* const* f, const double* xi,
                        const double* wq, float* scale, uint16_t* coef, uint8_t* flags,
                        float* const* recon, void* ws, hipStream_t s);

}  // namespace sem
