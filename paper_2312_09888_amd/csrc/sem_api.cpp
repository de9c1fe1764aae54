// C ABI of libsem: argument validation, per-device constant tables, launches.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kMaxDevices = 64;

struct DeviceState {
  bool ready = false;
  void* buf = nullptr;
  DeviceTables tab{};
};

std::mutex g_mutex;
DeviceState g_dev[kMaxDevices];

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Tables of the current device, or nullptr when sem_init was not called.
const DeviceTables* current_tables() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  return g_dev[dev].ready ? &g_dev[dev].tab : nullptr;
}

// Kernel-phase timing of one device: a pool of events handed out in order,
// and the (phase, start event, end event) of every timed phase execution.
struct Span {
  int phase, ev0, ev1;
};
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  std::vector<Span> spans;
  int64_t dropped = 0;
};
std::mutex g_tmutex;
Timing g_timing[kMaxDevices];

bool mixed_dtype(sem_dtype dt) { return dt >= SEM_MIXED_BF16 && dt <= SEM_MIXED_FP16X3; }

// `derivatives`: the call differentiates (mixed modes then need N = 7).
int check_common(int64_t n_elem, int order, sem_dtype dt, bool derivatives = true) {
  if (dt < SEM_F64 || dt > SEM_MIXED_FP16X3) return SEM_ERR_DTYPE;
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (derivatives && mixed_dtype(dt) && order != 7) return SEM_ERR_ORDER;
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  return SEM_OK;
}

}  // namespace

PhaseTimer phase_timer(int phase) {
  PhaseTimer pt;
  int dev = -1;
  if (phase < 0 || phase >= SEM_NUM_PHASES) return pt;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return pt;
  std::lock_guard<std::mutex> lock(g_tmutex);
  Timing& t = g_timing[dev];
  if (!t.on) return pt;
  if (t.used + 2 > t.ev.size()) {
    ++t.dropped;
    return pt;
  }
  pt.phase = phase;
  pt.i0 = (int)t.used++;
  pt.i1 = (int)t.used++;
  pt.start = t.ev[pt.i0];
  pt.stop = t.ev[pt.i1];
  return pt;
}

void phase_done(const PhaseTimer& pt) {
  int dev = -1;
  if (pt.phase < 0) return;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_tmutex);
  Timing& t = g_timing[dev];
  if (t.on) t.spans.push_back(Span{pt.phase, pt.i0, pt.i1});
}

IsoWorkspace iso_workspace_layout(void* base, int64_t n_elem, int n_iso) {
  const int64_t count = (int64_t)n_iso * n_elem;
  const size_t b_cnt = align256((size_t)count * sizeof(int32_t));
  const size_t b_offs = align256((size_t)(count + 1) * sizeof(int64_t));
  const size_t b_part = align256((size_t)(scan_partials_capacity(count) + 1) * sizeof(int64_t));
  IsoWorkspace ws;
  char* p = static_cast<char*>(base);
  ws.cnt = reinterpret_cast<int32_t*>(p);
  ws.offs = reinterpret_cast<int64_t*>(p ? p + b_cnt : nullptr);
  ws.partial = reinterpret_cast<int64_t*>(p ? p + b_cnt + b_offs : nullptr);
  ws.bytes = b_cnt + b_offs + b_part;
  return ws;
}

namespace {

// sem_extract counts triangles per element, scans the counts and emits
// from the stored Q; Q and its element ranges need storage, taken from the
// workspace when the caller does not want them.
struct ExtractLayout {
  size_t iso_bytes, q_off, mm_off, bytes;
};

ExtractLayout extract_layout(int64_t n_elem, int order, int n_iso, sem_dtype dt) {
  const size_t esz = dt == SEM_F64 ? sizeof(double) : sizeof(float);
  const size_t p3 = (size_t)(order + 1) * (order + 1) * (order + 1);
  ExtractLayout f;
  f.iso_bytes = iso_workspace_layout(nullptr, n_elem, n_iso).bytes;
  f.q_off = f.iso_bytes;
  f.mm_off = f.q_off + align256((size_t)n_elem * p3 * esz);
  f.bytes = f.mm_off + align256((size_t)n_elem * 2 * esz);
  return f;
}

}  // namespace

}  // namespace sem

using namespace sem;

extern "C" {

const char* sem_build_info(void) {
  // both strings are compiler definitions from the build script
  return "sources_sha256=" SEM_SOURCES_SHA256 ";arch=gfx950;hip=" SEM_HIP_VERSION;
}

const char* sem_status_str(int status) {
  switch (status) {
    case SEM_OK: return "ok";
    case SEM_ERR_ARG: return "invalid argument (NULL pointer, negative size or bad count)";
    case SEM_ERR_ORDER: return "polynomial order outside the supported range";
    case SEM_ERR_NOT_INIT: return "sem_init was not called for the current device";
    case SEM_ERR_HIP: return "HIP runtime call or kernel launch failed";
    case SEM_ERR_WORKSPACE: return "isosurface workspace missing or too small";
    case SEM_ERR_DTYPE: return "dtype is not a sem_dtype value";
    default: return "unknown status";
  }
}

int sem_gll(int order, double* nodes, double* weights, double* dmat) {
  if (order < 1 || order > kMaxBasisOrder) return SEM_ERR_ORDER;
  return gll_basis(order, nodes, weights, dmat) ? SEM_OK : SEM_ERR_ORDER;
}

int sem_mc_table(uint8_t* ntri, int8_t* tri) {
  build_mc_table(ntri, tri);
  return SEM_OK;
}

int sem_init(int device) {
  if (device < 0 || device >= kMaxDevices) return SEM_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_mutex);
  DeviceState& st = g_dev[device];
  if (st.ready) return SEM_OK;
  // host tables: D of every order in FP64 and FP32, then the case table
  size_t off64[kMaxOrder + 1], off32[kMaxOrder + 1];
  size_t bytes = 0;
  // FP64 D of order n is followed by its even-odd halves (below)
  for (int n = 1; n <= kMaxOrder; ++n) {
    const int ne = (n + 2) / 2;
    off64[n] = bytes;
    bytes += align256(sizeof(double) * ((n + 1) * (n + 1) + 2 * ne * ne));
  }
  for (int n = 1; n <= kMaxOrder; ++n) {
    const int ne = (n + 2) / 2;
    off32[n] = bytes;
    bytes += align256(sizeof(float) * ((n + 1) * (n + 1) + 2 * ne * ne));
  }
  // the case table directly follows the 256 triangle counts: kernels copy
  // both as one 4 KiB block
  const size_t off_ntri = bytes;
  bytes += align256(256);
  const size_t off_tri = bytes;
  bytes += align256(256 * kMcMaxTri * 3);
  const size_t off_eo7 = bytes;
  bytes += align256(sizeof(double) * 32);
  std::vector<unsigned char> host(bytes, 0);
  for (int n = 1; n <= kMaxOrder; ++n) {
    double* d = reinterpret_cast<double*>(host.data() + off64[n]);
    gll_basis(n, nullptr, nullptr, d);
    // even-odd halves of D (D[P-1-i][P-1-m] = -D[i][m] on the symmetric GLL
    // nodes), P = n + 1, H = P / 2 node pairs, NE = ceil(P / 2) rows:
    // A[i][m] = (D[i][m] + D[i][P-1-m]) / 2 for m < H and A[i][H] = D[i][H]
    // when P is odd (the middle node); B[i][m] = (D[i][m] - D[i][P-1-m]) / 2.
    // With e_m = g_m + g_{P-1-m} (e_H = g_H), o_m = g_m - g_{P-1-m}:
    // (Dg)_i = A_i.e + B_i.o and (Dg)_{P-1-i} = B_i.o - A_i.e.
    const int p = n + 1, hp = p / 2, ne = (p + 1) / 2;
    double* a = d + p * p;
    double* b = a + ne * ne;
    for (int i = 0; i < ne; ++i) {
      for (int m = 0; m < hp; ++m) {
        a[ne * i + m] = 0.5 * (d[p * i + m] + d[p * i + p - 1 - m]);
        b[hp * i + m] = 0.5 * (d[p * i + m] - d[p * i + p - 1 - m]);
      }
      if (p % 2) a[ne * i + hp] = d[p * i + hp];
    }
    // FP32 copy of D and of its halves (each rounded from its FP64 value)
    float* f = reinterpret_cast<float*>(host.data() + off32[n]);
    for (int q = 0; q < p * p + 2 * ne * ne; ++q) f[q] = (float)d[q];
  }
  build_mc_table(host.data() + off_ntri, reinterpret_cast<int8_t*>(host.data() + off_tri));
  {
    // even-odd coefficients of D for N = 7: A = (D[i][m] + D[i][7-m]) / 2,
    // B = (D[i][m] - D[i][7-m]) / 2 for i, m < 4
    const double* d = reinterpret_cast<const double*>(host.data() + off64[7]);
    double* eo = reinterpret_cast<double*>(host.data() + off_eo7);
    for (int i = 0; i < 4; ++i)
      for (int m = 0; m < 4; ++m) {
        eo[4 * i + m] = 0.5 * (d[8 * i + m] + d[8 * i + 7 - m]);
        eo[16 + 4 * i + m] = 0.5 * (d[8 * i + m] - d[8 * i + 7 - m]);
      }
  }

  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return SEM_ERR_HIP;
  if (hipSetDevice(device) != hipSuccess) return SEM_ERR_HIP;
  void* buf = nullptr;
  void* scratch = nullptr;
  int rc = SEM_OK;
  // this device's copy of the fixed scratch array (sem_extract_noalloc)
  if (noalloc_scratch(&scratch) != hipSuccess || !scratch) {
    rc = SEM_ERR_HIP;
  } else if (hipMalloc(&buf, bytes) != hipSuccess ||
             hipMemcpy(buf, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    if (buf) (void)hipFree(buf);
    rc = SEM_ERR_HIP;
  } else {
    st.tab.scratch = scratch;
    st.buf = buf;
    char* b = static_cast<char*>(buf);
    for (int n = 0; n <= kMaxOrder; ++n) {
      st.tab.d64[n] = n ? reinterpret_cast<const double*>(b + off64[n]) : nullptr;
      st.tab.d32[n] = n ? reinterpret_cast<const float*>(b + off32[n]) : nullptr;
    }
    st.tab.ntri = reinterpret_cast<const uint8_t*>(b + off_ntri);
    st.tab.tri = reinterpret_cast<const int8_t*>(b + off_tri);
    st.tab.eo7 = reinterpret_cast<const double*>(b + off_eo7);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess || cus <= 0)
      cus = 256;
    st.tab.cu_count = cus;
    st.ready = true;
  }
  (void)hipSetDevice(prev);
  return rc;
}

void sem_finalize(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  for (int d = 0; d < kMaxDevices; ++d) {
    if (!g_dev[d].ready) continue;
    if (hipSetDevice(d) == hipSuccess) (void)hipFree(g_dev[d].buf);
    g_dev[d] = DeviceState{};
  }
  if (prev >= 0) (void)hipSetDevice(prev);
}

int sem_derivs(int64_t n_elem, int order, sem_dtype dt, const void* x, const void* y,
               const void* z, const void* f, void* dfdx, void* dfdy, void* dfdz,
               int32_t* status_word, void* stream) {
  int rc = check_common(n_elem, order, dt);
  if (rc) return rc;
  if (n_elem == 0) return SEM_OK;
  if (!x || !y || !z || !f || !dfdx || !dfdy || !dfdz) return SEM_ERR_ARG;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  hipError_t e = launch_derivs(order, dt, *tab, n_elem, x, y, z, f, dfdx, dfdy, dfdz,
                               status_word, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_qcrit(int64_t n_elem, int order, sem_dtype dt, const void* x, const void* y,
              const void* z, const void* u, const void* v, const void* w, void* q,
              void* omega_mag, void* q_minmax, int32_t* status_word, void* stream) {
  int rc = check_common(n_elem, order, dt);
  if (rc) return rc;
  if (n_elem == 0) return SEM_OK;
  if (!x || !y || !z || !u || !v || !w) return SEM_ERR_ARG;
  if (!q && !omega_mag && !q_minmax) return SEM_ERR_ARG;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  hipError_t e = launch_qcrit(order, dt, *tab, n_elem, x, y, z, u, v, w, q, omega_mag, q_minmax,
                              status_word, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

size_t sem_extract_workspace_bytes(int64_t n_elem, int order, int n_iso, sem_dtype dt) {
  if (check_common(n_elem, order, dt) != SEM_OK || n_iso < 1 || n_iso > SEM_MAX_ISO) return 0;
  return extract_layout(n_elem, order, n_iso, dt).bytes;
}

int sem_extract(int64_t n_elem, int order, sem_dtype dt, const void* x, const void* y,
                const void* z, const void* u, const void* v, const void* w, void* q,
                void* omega_mag, void* q_minmax, int n_iso, const double* iso_host,
                void* const* tri_xyz, const int64_t* tri_capacity, int64_t* tri_count,
                int64_t* active_cells, void* workspace, size_t workspace_bytes,
                int32_t* status_word, void* stream) {
  int rc = check_common(n_elem, order, dt);
  if (rc) return rc;
  if (n_iso < 1 || n_iso > SEM_MAX_ISO || !iso_host || !tri_count) return SEM_ERR_ARG;
  if (!tri_xyz || !tri_capacity) return SEM_ERR_ARG;
  for (int k = 0; k < n_iso; ++k)
    if (tri_capacity[k] < 0 || (tri_capacity[k] > 0 && !tri_xyz[k])) return SEM_ERR_ARG;
  if ((int64_t)n_iso * n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  if (n_elem > 0 && (!x || !y || !z || !u || !v || !w)) return SEM_ERR_ARG;
  const size_t need = sem_extract_workspace_bytes(n_elem, order, n_iso, dt);
  if (n_elem > 0 && (!workspace || workspace_bytes < need)) return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_elem == 0) {
    hipError_t e = launch_isosurface(order, dt, *tab, 0, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, n_iso, iso_host, nullptr, 0, nullptr, tri_count,
                                     active_cells, nullptr, IsoWorkspace{}, status_word, s);
    return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
  }
  const ExtractLayout f = extract_layout(n_elem, order, n_iso, dt);
  char* b = static_cast<char*>(workspace);
  if (!q) q = b + f.q_off;
  if (!q_minmax) q_minmax = b + f.mm_off;
  const IsoWorkspace ws = iso_workspace_layout(workspace, n_elem, n_iso);
  hipError_t e = launch_extract(order, dt, *tab, n_elem, x, y, z, u, v, w, q, omega_mag,
                                q_minmax, n_iso, iso_host, tri_xyz, tri_capacity, tri_count,
                                active_cells, ws, status_word, s);
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_extract_noalloc(int64_t n_elem, int order, sem_dtype dt, const void* x, const void* y,
                        const void* z, const void* u, const void* v, const void* w, void* q,
                        void* omega_mag, void* q_minmax, int n_iso, const double* iso_host,
                        void* const* tri_xyz, const int64_t* tri_capacity, int64_t* tri_count,
                        int64_t* active_cells, int32_t* status_word, void* stream) {
  int rc = check_common(n_elem, order, dt);
  if (rc) return rc;
  if (n_iso < 1 || n_iso > SEM_MAX_ISO || !iso_host || !tri_count) return SEM_ERR_ARG;
  if (!tri_xyz || !tri_capacity) return SEM_ERR_ARG;
  for (int k = 0; k < n_iso; ++k)
    if (tri_capacity[k] < 0 || (tri_capacity[k] > 0 && !tri_xyz[k])) return SEM_ERR_ARG;
  if (n_elem > 0 && (!x || !y || !z || !u || !v || !w || !q || !q_minmax)) return SEM_ERR_ARG;
  // the counts, offsets and scan partials must fit the fixed scratch
  if ((int64_t)n_iso * n_elem > SEM_NOALLOC_MAX_COUNTS) return SEM_ERR_WORKSPACE;
  if (iso_workspace_layout(nullptr, n_elem, n_iso).bytes > noalloc_scratch_bytes())
    return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the device address looked up for this GPU by sem_init, never the
  // array's host-side name
  const IsoWorkspace ws =
      n_elem > 0 ? iso_workspace_layout(tab->scratch, n_elem, n_iso) : IsoWorkspace{};
  hipError_t e =
      n_elem == 0
          ? launch_isosurface(order, dt, *tab, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                              n_iso, iso_host, nullptr, 0, nullptr, tri_count, active_cells,
                              nullptr, IsoWorkspace{}, status_word, s)
          : launch_extract(order, dt, *tab, n_elem, x, y, z, u, v, w, q, omega_mag, q_minmax,
                           n_iso, iso_host, tri_xyz, tri_capacity, tri_count, active_cells, ws,
                           status_word, s);
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

size_t sem_isosurface_workspace_bytes(int64_t n_elem, int order, int n_iso) {
  (void)order;
  if (n_elem < 0 || n_iso < 1) return 0;
  return iso_workspace_layout(nullptr, n_elem, n_iso).bytes;
}

int sem_isosurface(int64_t n_elem, int order, sem_dtype dt, const void* x, const void* y,
                   const void* z, const void* field, const void* field_minmax, int n_iso,
                   const double* iso_host, void* tri_xyz, int64_t tri_capacity,
                   uint64_t* tri_edge_key, int64_t* tri_count, int64_t* active_cells,
                   uint8_t* case_idx, void* workspace, size_t workspace_bytes,
                   int32_t* status_word, void* stream) {
  int rc = check_common(n_elem, order, dt, false);
  if (rc) return rc;
  if (mixed_dtype(dt)) dt = SEM_F32;
  if (n_iso < 1 || n_iso > SEM_MAX_ISO || !iso_host || !tri_count) return SEM_ERR_ARG;
  if (n_elem > 0 && (!x || !y || !z || !field)) return SEM_ERR_ARG;
  if (tri_capacity < 0 || (tri_capacity > 0 && !tri_xyz)) return SEM_ERR_ARG;
  if ((int64_t)n_iso * n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  IsoWorkspace ws = iso_workspace_layout(workspace, n_elem, n_iso);
  if (n_elem > 0 && (!workspace || workspace_bytes < ws.bytes)) return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  hipError_t e = launch_isosurface(order, dt, *tab, n_elem, x, y, z, field, field_minmax, n_iso,
                                   iso_host, tri_xyz, tri_capacity, tri_edge_key, tri_count,
                                   active_cells, case_idx, ws, status_word,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

size_t sem_batch_plan_bytes(int n_snap) {
  if (n_snap < 1 || n_snap > kBatchMaxSnap) return 0;
  return batch_plan_bytes(n_snap);
}

int sem_batch_variant(int order, sem_dtype dt) {
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  const int v = tab->tuned_variant[dt == SEM_F64 ? 0 : 1][order] - 1;
  return v >= 0 ? v : batch_default_variant(order, dt);
}

int sem_batch_set_variant(int order, sem_dtype dt, int variant) {
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  if (!batch_variant_ok(order, dt, variant)) return SEM_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SEM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_dev[dev].ready) return SEM_ERR_NOT_INIT;
  g_dev[dev].tab.tuned_variant[dt == SEM_F64 ? 0 : 1][order] = variant + 1;
  return SEM_OK;
}

int sem_batch_plan(int n_snap, const sem_snapshot* snaps, sem_dtype dt, void* plan,
                   size_t plan_bytes, unsigned* launch_code) {
  if (n_snap < 1 || n_snap > kBatchMaxSnap || !snaps) return SEM_ERR_ARG;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  if (!plan || plan_bytes < batch_plan_bytes(n_snap)) return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  for (int i = 0; i < n_snap; ++i) {
    const sem_snapshot& sn = snaps[i];
    if (sn.order < SEM_MIN_ORDER || sn.order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
    if (sn.n_elem < 0 || sn.n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
    if (sn.n_elem > 0 && (!sn.x || !sn.y || !sn.z || !sn.u || !sn.v || !sn.w)) return SEM_ERR_ARG;
    if (sn.n_elem > 0 && !sn.q && !sn.omega_mag && !sn.q_minmax) return SEM_ERR_ARG;
  }
  std::vector<unsigned char> host(batch_plan_bytes(n_snap), 0);
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(host.data());
  BatchSnap* bs = reinterpret_cast<BatchSnap*>(host.data() + 256);
  unsigned code = 0;
  int next = 0;
  // descriptors grouped by order; items numbered within each order
  for (int n = SEM_MIN_ORDER; n <= kMaxOrder; ++n) {
    hdr->snap_begin[n] = next;
    int var = tab->tuned_variant[dt == SEM_F64 ? 0 : 1][n] - 1;
    if (!batch_variant_ok(n, dt, var)) var = batch_default_variant(n, dt);
    const int chunk = batch_variant_chunk(n, dt, var), form = batch_variant_form(var);
    int64_t items = 0;
    for (int i = 0; i < n_snap; ++i) {
      const sem_snapshot& sn = snaps[i];
      if (sn.order != n) continue;
      BatchSnap& b = bs[next++];
      b.n_elem = sn.n_elem;
      b.item_begin = items;
      b.order = n;
      b.chunk = chunk;
      b.form = form;
      b.pad = 0;
      const void* f[6] = {sn.x, sn.y, sn.z, sn.u, sn.v, sn.w};
      for (int k = 0; k < 6; ++k) b.f[k] = f[k];
      b.q = sn.q;
      b.om = sn.omega_mag;
      b.qmm = sn.q_minmax;
      b.dmat = dt == SEM_F32 && f32_line_sums(n) ? (const void*)tab->d32[n]
                                                 : (const void*)tab->d64[n];
      b.eo = tab->eo7;
      items += (sn.n_elem + chunk - 1) / chunk;
    }
    hdr->items[n] = items;
    if (items > 0) code |= (unsigned)(form + 1) << (3 * n);
  }
  hdr->snap_begin[0] = 0;
  hdr->snap_begin[kMaxOrder + 1] = next;
  hdr->n_snap = n_snap;
  hdr->dt = dt;
  if (launch_code) *launch_code = code;
  return hipMemcpy(plan, host.data(), host.size(), hipMemcpyHostToDevice) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_qcrit_batch(const void* plan, unsigned launch_code, sem_dtype dt, int32_t* status_word,
                    void* stream) {
  if (!plan) return SEM_ERR_ARG;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  const PhaseTimer pt = phase_timer(SEM_PHASE_QCRIT);
  const hipError_t e =
      launch_qcrit_batch(dt, plan, launch_code, 8 * tab->cu_count, status_word,
                         static_cast<hipStream_t>(stream), pt.start, pt.stop);
  phase_done(pt);
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

size_t sem_iso_batch_plan_bytes(int n_job) {
  if (n_job < 1 || n_job > kIsoBatchMaxJob) return 0;
  return iso_batch_plan_bytes(n_job);
}

int sem_iso_batch_plan(int n_snap, const sem_snapshot* snaps, int n_job,
                       const sem_iso_job* jobs, sem_dtype dt, void* plan, size_t plan_bytes,
                       sem_iso_batch_info* info) {
  if (n_snap < 1 || n_snap > kBatchMaxSnap || !snaps || !info) return SEM_ERR_ARG;
  if (n_job < 1 || n_job > kIsoBatchMaxJob || !jobs) return SEM_ERR_ARG;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  if (!plan || plan_bytes < iso_batch_plan_bytes(n_job)) return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  for (int i = 0; i < n_snap; ++i) {
    const sem_snapshot& sn = snaps[i];
    if (sn.order < SEM_MIN_ORDER || sn.order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
    if (sn.n_elem < 0 || sn.n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  }
  std::vector<const void*> field(n_job), mm(n_job);
  for (int k = 0; k < n_job; ++k) {
    const sem_iso_job& jb = jobs[k];
    if (jb.snap < 0 || jb.snap >= n_snap) return SEM_ERR_ARG;
    if (jb.n_iso < 1 || jb.n_iso > 4) return SEM_ERR_ARG;
    for (int q = 0; q < jb.n_iso; ++q)
      if (jb.iso[q] != jb.iso[q]) return SEM_ERR_ARG;
    const sem_snapshot& sn = snaps[jb.snap];
    if (jb.field == SEM_JOB_Q) {
      field[k] = sn.q;
      mm[k] = sn.q_minmax;
    } else if (jb.field == SEM_JOB_OMEGA) {
      field[k] = sn.omega_mag;
      mm[k] = nullptr;
    } else if (jb.field == SEM_JOB_SCALAR) {
      field[k] = jb.scalar;
      mm[k] = nullptr;
    } else {
      return SEM_ERR_ARG;
    }
    if (sn.n_elem > 0 && (!field[k] || !sn.x || !sn.y || !sn.z)) return SEM_ERR_ARG;
  }
  std::vector<unsigned char> host(iso_batch_plan_bytes(n_job), 0);
  IsoBatchHeader* hdr = reinterpret_cast<IsoBatchHeader*>(host.data());
  IsoBatchJob* out = reinterpret_cast<IsoBatchJob*>(host.data() + 256);
  // count slots in the caller's job order (the soup's order)
  std::vector<int64_t> slot(n_job);
  int64_t n_slots = 0;
  for (int k = 0; k < n_job; ++k) {
    slot[k] = n_slots;
    n_slots += (int64_t)jobs[k].n_iso * snaps[jobs[k].snap].n_elem;
  }
  unsigned code = 0;
  int next = 0;
  for (int n = SEM_MIN_ORDER; n <= kMaxOrder; ++n) {
    hdr->job_begin[n] = next;
    int64_t items = 0;
    for (int k = 0; k < n_job; ++k) {
      const sem_iso_job& jb = jobs[k];
      const sem_snapshot& sn = snaps[jb.snap];
      if (sn.order != n) continue;
      IsoBatchJob& d = out[next++];
      d.n_elem = sn.n_elem;
      d.item_begin = items;
      d.slot_begin = slot[k];
      d.order = n;
      d.n_iso = jb.n_iso;
      d.job = k;
      d.x = sn.x;
      d.y = sn.y;
      d.z = sn.z;
      d.field = field[k];
      d.mm = mm[k];
      for (int q = 0; q < 4; ++q) {
        const double c = q < jb.n_iso ? jb.iso[q] : 0.0;
        d.isod[q] = c;
        d.isof[q] = (float)c;
      }
      items += sn.n_elem;
    }
    hdr->items[n] = items;
    if (items > 0) code |= 1u << n;
  }
  hdr->job_begin[0] = 0;
  hdr->job_begin[kMaxOrder + 1] = next;
  hdr->n_job = n_job;
  hdr->dt = dt;
  hdr->n_slots = n_slots;
  info->launch_code = code;
  info->dt = dt;
  info->n_job = n_job;
  info->n_slots = n_slots;
  info->workspace_bytes = iso_workspace_layout(nullptr, n_slots, 1).bytes;
  return hipMemcpy(plan, host.data(), host.size(), hipMemcpyHostToDevice) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_isosurface_batch(const void* plan, const sem_iso_batch_info* info, sem_dtype dt,
                         void* tri_xyz, int64_t tri_capacity, int64_t* tri_offset,
                         int64_t* tri_count, int64_t* active_cells, void* workspace,
                         size_t workspace_bytes, int32_t* status_word, void* stream) {
  if (!plan || !info || !tri_count) return SEM_ERR_ARG;
  if ((dt != SEM_F64 && dt != SEM_F32) || dt != info->dt) return SEM_ERR_DTYPE;
  if (info->n_job < 1 || info->n_job > kIsoBatchMaxJob || info->n_slots < 0) return SEM_ERR_ARG;
  if (info->launch_code & ~(((1u << (kMaxOrder + 1)) - 1u) & ~1u)) return SEM_ERR_ARG;
  if (tri_capacity < 0 || (tri_capacity > 0 && !tri_xyz)) return SEM_ERR_ARG;
  IsoWorkspace ws = iso_workspace_layout(workspace, info->n_slots, 1);
  if (!workspace || workspace_bytes < ws.bytes) return SEM_ERR_WORKSPACE;
  const DeviceTables* tab = current_tables();
  if (!tab) return SEM_ERR_NOT_INIT;
  const hipError_t e = launch_iso_batch(dt, *tab, plan, info->launch_code, info->n_job,
                                        info->n_slots, tri_xyz, tri_capacity, tri_offset,
                                        tri_count, active_cells, ws, status_word,
                                        static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_autotune(int order, sem_dtype dt, int* variant_out, float* ms_out) {
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (dt != SEM_F64 && dt != SEM_F32) return SEM_ERR_DTYPE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SEM_ERR_HIP;
  if (!current_tables()) return SEM_ERR_NOT_INIT;
  const int64_t n_elem = 8192;
  const int64_t p = order + 1, pts = n_elem * p * p * p;
  const size_t esz = dt == SEM_F64 ? 8 : 4;
  const size_t fb = (pts * esz + 255) & ~size_t(255);
  const size_t mmb = (2 * n_elem * esz + 255) & ~size_t(255);
  const size_t plan_b = batch_plan_bytes(1);
  void* buf = nullptr;
  if (hipMalloc(&buf, 8 * fb + mmb + plan_b) != hipSuccess) return SEM_ERR_HIP;
  char* b = static_cast<char*>(buf);
  void* f[6];
  for (int k = 0; k < 6; ++k) f[k] = b + k * fb;
  void* plan = b + 8 * fb + mmb;
  sem_snapshot sn{};
  sn.n_elem = n_elem;
  sn.order = order;
  sn.x = f[0]; sn.y = f[1]; sn.z = f[2]; sn.u = f[3]; sn.v = f[4]; sn.w = f[5];
  sn.q = b + 6 * fb;
  sn.omega_mag = b + 7 * fb;
  sn.q_minmax = b + 8 * fb;
  int rc = SEM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best_ms = 0.f;
  int best = -1;
  const int ti = dt == SEM_F64 ? 0 : 1;
  if (launch_tune_fill(dt, order, n_elem, f, nullptr) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = SEM_ERR_HIP;
  for (int var = 0; var < kBatchVariants && rc == SEM_OK; ++var) {
    if (ms_out) ms_out[var] = -1.f;
    if (!batch_variant_ok(order, dt, var)) continue;
    {
      std::lock_guard<std::mutex> lock(g_mutex);
      g_dev[dev].tab.tuned_variant[ti][order] = var + 1;
    }
    unsigned mask = 0;
    rc = sem_batch_plan(1, &sn, dt, plan, plan_b, &mask);
    if (rc != SEM_OK) break;
    const int grid = 8 * current_tables()->cu_count;
    float ms = 0.f;
    if (launch_qcrit_batch(dt, plan, mask, grid, nullptr, nullptr, nullptr, nullptr) !=
            hipSuccess ||
        hipEventRecord(e0, nullptr) != hipSuccess) {
      rc = SEM_ERR_HIP;
      break;
    }
    for (int r = 0; r < 5; ++r)
      (void)launch_qcrit_batch(dt, plan, mask, grid, nullptr, nullptr, nullptr, nullptr);
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = SEM_ERR_HIP;
      break;
    }
    ms /= 5.f;
    if (ms_out) ms_out[var] = ms;
    if (best < 0 || ms < best_ms) {
      best_ms = ms;
      best = var;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipDeviceSynchronize();
  (void)hipFree(buf);
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    g_dev[dev].tab.tuned_variant[ti][order] = (rc == SEM_OK && best >= 0) ? best + 1 : 0;
  }
  if (rc == SEM_OK && variant_out) *variant_out = best;
  return rc;
}

size_t sem_gs_workspace_bytes(int64_t n_elem, int order, int64_t n_global) {
  if (n_elem < 0 || order < SEM_MIN_ORDER || order > SEM_MAX_ORDER || n_global < 0 ||
      n_global >= (int64_t)0xffffffffll)
    return 0;
  const int64_t p = order + 1;
  return gs_layout(nullptr, n_elem * p * p * p, n_global).bytes;
}

int sem_gs_setup(int64_t n_elem, int order, const int64_t* gid, int64_t n_global, void* gs,
                 size_t gs_bytes, int32_t* status_word, void* stream) {
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff || n_global < 0 ||
      n_global >= (int64_t)0xffffffffll)
    return SEM_ERR_ARG;
  if (n_elem > 0 && !gid) return SEM_ERR_ARG;
  const int64_t p = order + 1;
  const GsLayout l = gs_layout(gs, n_elem * p * p * p, n_global);
  if (!gs || gs_bytes < l.bytes) return SEM_ERR_WORKSPACE;
  if (!current_tables()) return SEM_ERR_NOT_INIT;
  const hipError_t e = launch_gs_setup(n_elem * p * p * p, gid, n_global, l, status_word,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_dsavg(int64_t n_elem, int order, sem_dtype dt, const void* gs, int64_t n_global,
              const void* field, void* out, void* stream) {
  const int rc = check_common(n_elem, order, dt, false);
  if (rc) return rc;
  if (n_global < 0 || n_global >= (int64_t)0xffffffffll) return SEM_ERR_ARG;
  if (n_global == 0) return SEM_OK;
  if (!gs || !field || !out) return SEM_ERR_ARG;
  if (!current_tables()) return SEM_ERR_NOT_INIT;
  const int64_t p = order + 1;
  const GsLayout l = gs_layout(const_cast<void*>(gs), n_elem * p * p * p, n_global);
  const hipError_t e = launch_dsavg(dt == SEM_F64 ? SEM_F64 : SEM_F32, n_global, l, field, out,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_global_edge_keys(int64_t n_ref, int order, int64_t n_elem, const uint64_t* local_keys,
                         const int64_t* gid, uint64_t* global_keys, int32_t* status_word,
                         void* stream) {
  if (order < SEM_MIN_ORDER || order > SEM_MAX_ORDER) return SEM_ERR_ORDER;
  if (n_ref < 0 || n_elem < 0) return SEM_ERR_ARG;
  if (n_ref == 0) return SEM_OK;
  if (!local_keys || !gid || !global_keys) return SEM_ERR_ARG;
  if (!current_tables()) return SEM_ERR_NOT_INIT;
  const hipError_t e = launch_global_keys(n_ref, order, n_elem, local_keys, gid, global_keys,
                                          status_word, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

size_t sem_weld_workspace_bytes(int64_t n_ref) {
  if (n_ref < 0 || n_ref > (int64_t)0x3fffffff) return 0;
  return weld_layout(nullptr, n_ref).bytes;
}

int sem_weld(int64_t n_ref, sem_dtype dt, const void* tri_xyz, const uint64_t* keys,
             int64_t* tri_index, void* vert_xyz, int64_t vert_capacity, int64_t* n_vert,
             void* workspace, size_t workspace_bytes, int32_t* status_word, void* stream) {
  if (dt < SEM_F64 || dt > SEM_MIXED_FP16X3) return SEM_ERR_DTYPE;
  if (n_ref < 0 || n_ref % 3 != 0 || n_ref > (int64_t)0x3fffffff || vert_capacity < 0 ||
      !n_vert)
    return SEM_ERR_ARG;
  if (n_ref > 0 && (!tri_xyz || !keys || !tri_index)) return SEM_ERR_ARG;
  if (vert_capacity > 0 && !vert_xyz) return SEM_ERR_ARG;
  const WeldLayout w = weld_layout(workspace, n_ref);
  if (!workspace || workspace_bytes < w.bytes) return SEM_ERR_WORKSPACE;
  if (!current_tables()) return SEM_ERR_NOT_INIT;
  const hipError_t e = launch_weld(n_ref, dt == SEM_F64 ? SEM_F64 : SEM_F32, tri_xyz, keys,
                                   tri_index, vert_xyz, vert_capacity, n_vert, w, status_word,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

const char* sem_phase_name(int phase) {
  switch (phase) {
    case SEM_PHASE_QCRIT: return "qcrit";
    case SEM_PHASE_COUNT: return "count";
    case SEM_PHASE_SCAN: return "scan";
    case SEM_PHASE_EMIT: return "emit";
    default: return "unknown";
  }
}

int sem_timing_begin(int max_spans) {
  if (max_spans < 1 || max_spans > (1 << 20)) return SEM_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SEM_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return SEM_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_tmutex);
  Timing& t = g_timing[dev];
  if (t.on) return SEM_ERR_ARG;
  t = Timing{};
  t.ev.resize((size_t)2 * max_spans);
  for (size_t k = 0; k < t.ev.size(); ++k) {
    if (hipEventCreate(&t.ev[k]) != hipSuccess) {
      for (size_t q = 0; q < k; ++q) (void)hipEventDestroy(t.ev[q]);
      t = Timing{};
      return SEM_ERR_HIP;
    }
  }
  t.on = true;
  return SEM_OK;
}

int sem_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (bytes == 0) return SEM_OK;
  if (!src || !dst || bytes % 16 != 0) return SEM_ERR_ARG;
  if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return SEM_ERR_ARG;
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return SEM_ERR_ARG;
  hipError_t e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int64_t sem_timing_end(double* ms_total, int64_t* spans, int n_phases) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SEM_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices || n_phases < 0) return SEM_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_tmutex);
  Timing& t = g_timing[dev];
  if (!t.on) return SEM_ERR_ARG;
  double tot[SEM_NUM_PHASES] = {0, 0, 0, 0};
  int64_t cnt[SEM_NUM_PHASES] = {0, 0, 0, 0};
  int64_t rc = t.dropped;
  for (const Span& sp : t.spans) {
    float ms = 0.f;
    if (hipEventSynchronize(t.ev[sp.ev1]) != hipSuccess ||
        hipEventElapsedTime(&ms, t.ev[sp.ev0], t.ev[sp.ev1]) != hipSuccess) {
      rc = SEM_ERR_HIP;
      break;
    }
    tot[sp.phase] += ms;
    cnt[sp.phase] += 1;
  }
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t = Timing{};
  for (int q = 0; q < n_phases; ++q) {
    if (ms_total) ms_total[q] = q < SEM_NUM_PHASES ? tot[q] : 0.0;
    if (spans) spans[q] = q < SEM_NUM_PHASES ? cnt[q] : 0;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// learned in-transit compression
// ---------------------------------------------------------------------------

int64_t sem_ae_param_count(void) { return ae_param_count(); }

size_t sem_ae_workspace_bytes(int64_t n) { return n < 1 ? 0 : ae_workspace_bytes(n); }

static bool ae_mask_ok(int m) { return (m & ~SEM_AE_TANH_HIDDEN) == 0; }

int sem_ae_blocks(int64_t n_elem, const float* u, const float* v, const float* w,
                  const float* theta, float* blocks, float* scale, void* stream) {
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  if (n_elem == 0) return SEM_OK;
  if (!u || !v || !w || !theta || !blocks || !scale) return SEM_ERR_ARG;
  const float* f[4] = {u, v, w, theta};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_ae_scales(n_elem, f, scale, nullptr, s);
  if (e == hipSuccess) e = launch_ae_pack(0, n_elem, f, scale, blocks, s);
  return e == hipSuccess ? SEM_OK : SEM_ERR_HIP;
}

int sem_ae_forward(int64_t n, const float* blocks, const float* params, int tanh_mask,
                   float* recon, uint16_t* latent, void* workspace, size_t workspace_bytes,
                   void* stream) {
  if (n < 0 || n > (int64_t)0x7fffffff || !ae_mask_ok(tanh_mask)) return SEM_ERR_ARG;
  if (n == 0) return SEM_OK;
  if (!blocks || !params || (!recon && !latent)) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < ae_workspace_bytes(n)) return SEM_ERR_WORKSPACE;
  return launch_ae_forward(n, blocks, params, tanh_mask, recon, latent, workspace,
                           static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_ae_grad(int64_t n, const float* pool, int64_t n_pool, const int64_t* idx,
                const float* params, int tanh_mask, int loss_kind, float* grad, float* loss,
                void* workspace, size_t workspace_bytes, int32_t* status_word, void* stream) {
  if (n < 1 || n > (int64_t)0x7fffffff || n_pool < 1 || !ae_mask_ok(tanh_mask))
    return SEM_ERR_ARG;
  if (loss_kind != SEM_AE_LOSS_MSE && loss_kind != SEM_AE_LOSS_MAX) return SEM_ERR_ARG;
  if (!idx && n > n_pool) return SEM_ERR_ARG;
  if (!pool || !params || !grad) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < ae_workspace_bytes(n)) return SEM_ERR_WORKSPACE;
  return launch_ae_grad(n, pool, n_pool, idx, params, tanh_mask, loss_kind, grad, loss,
                        workspace, status_word, static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_ae_adam(int64_t n, float* params, const float* grad, float* m, float* v, int step,
                float lr, float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return SEM_ERR_ARG;
  if (n == 0) return SEM_OK;
  if (!params || !grad || !m || !v) return SEM_ERR_ARG;
  return launch_ae_adam(n, params, grad, m, v, step, lr, beta1, beta2, eps,
                        static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

size_t sem_eig_workspace_bytes(int n) {
  return (n < 2 || n > 512 || (n & 1)) ? 0 : eig_workspace_bytes(n);
}

int sem_sym_eig(int n, const double* a, int r, double* lam, float* vec, void* workspace,
                size_t workspace_bytes, int* sweeps, void* stream) {
  if (n < 2 || n > 512 || (n & 1) || r < 1 || r > n || !a || !vec) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < eig_workspace_bytes(n)) return SEM_ERR_WORKSPACE;
  return launch_sym_eig(n, a, r, lam, vec, workspace, sweeps,
                        static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

size_t sem_ae_pca_workspace_bytes(int64_t n_pool) {
  return n_pool < 1 ? 0 : pca_workspace_bytes(n_pool);
}

int sem_ae_pca_init(int64_t n_pool, const float* pool, float* params, double* lam,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (n_pool < 1 || n_pool > ((int64_t)1 << 24) || !pool || !params) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < pca_workspace_bytes(n_pool)) return SEM_ERR_WORKSPACE;
  return launch_ae_pca_init(n_pool, pool, params, lam, workspace,
                            static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

size_t sem_ae_compress_workspace_bytes(int64_t n_elem) {
  return (n_elem < 0 || n_elem > (int64_t)0x7fffffff) ? 0 : compress_workspace_bytes(n_elem);
}

int sem_ae_compress(int64_t n_elem, const float* u, const float* v, const float* w,
                    const float* theta, const float* params, int tanh_mask, uint16_t* latent,
                    float* scale, uint8_t* flags, float* raw, int64_t raw_cap, int64_t* n_raw,
                    void* workspace, size_t workspace_bytes, int32_t* status_word,
                    void* stream) {
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff || raw_cap < 0 || !ae_mask_ok(tanh_mask))
    return SEM_ERR_ARG;
  if (n_elem == 0) return SEM_OK;
  if (!u || !v || !w || !theta || !params || !latent || !scale || !flags || !n_raw)
    return SEM_ERR_ARG;
  if (raw_cap > 0 && !raw) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < compress_workspace_bytes(n_elem)) return SEM_ERR_WORKSPACE;
  const float* f[4] = {u, v, w, theta};
  return launch_ae_compress(n_elem, f, params, tanh_mask, latent, scale, flags, raw, raw_cap,
                            n_raw, workspace, status_word,
                            static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_ae_decompress(int64_t n_elem, const uint16_t* latent, const float* scale,
                      const uint8_t* flags, const float* raw, int64_t raw_count,
                      const float* params, int tanh_mask, float* u, float* v, float* w,
                      float* theta, void* workspace, size_t workspace_bytes,
                      int32_t* status_word, void* stream) {
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff || raw_count < 0 || !ae_mask_ok(tanh_mask))
    return SEM_ERR_ARG;
  if (raw_count > 0 && !raw) return SEM_ERR_ARG;
  if (n_elem == 0) return SEM_OK;
  if (!latent || !scale || !flags || !params || !u || !v || !w || !theta) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < compress_workspace_bytes(n_elem)) return SEM_ERR_WORKSPACE;
  float* f[4] = {u, v, w, theta};
  return launch_ae_decompress(n_elem, latent, scale, flags, raw, raw_count, params, tanh_mask,
                              f, workspace, status_word,
                              static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

int sem_modal_compress(int64_t n_elem, const float* u, const float* v, const float* w,
                       const float* theta, uint16_t* coef, float* scale, uint8_t* flags,
                       float* ru, float* rv, float* rw, float* rtheta, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (n_elem < 0 || n_elem > (int64_t)0x7fffffff) return SEM_ERR_ARG;
  if (n_elem == 0) return SEM_OK;
  if (!u || !v || !w || !theta || !scale || !flags) return SEM_ERR_ARG;
  const bool any_r = ru || rv || rw || rtheta;
  if (any_r && !(ru && rv && rw && rtheta)) return SEM_ERR_ARG;
  if (!workspace || workspace_bytes < compress_workspace_bytes(n_elem)) return SEM_ERR_WORKSPACE;
  double xi[8], wq[8], dm[64];
  if (!gll_basis(7, xi, wq, dm)) return SEM_ERR_ARG;
  const float* f[4] = {u, v, w, theta};
  float* r[4] = {ru, rv, rw, rtheta};
  return launch_modal(n_elem, f, xi, wq, scale, coef, flags, any_r ? r : nullptr, workspace,
                      static_cast<hipStream_t>(stream)) == hipSuccess
             ? SEM_OK
             : SEM_ERR_HIP;
}

}  // extern "C"
