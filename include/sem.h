/*
 * sem.h -- C ABI of libsem: the in situ extraction hot path for
 * spectral-element snapshots on AMD Instinct MI355X (gfx950).
 *
 * Context (the paper, sections 1 and 3): the solver is a spectral-element
 * code whose snapshots sit in GPU memory in the Nek data model -- fields at
 * the Gauss-Lobatto-Legendre (GLL) nodes of order-N hexahedral elements.
 * The paper's analysis copies them to the host for rendering; this library
 * instead extracts Q-criterion / vorticity-magnitude fields and isosurface
 * triangles on the device, so only triangles and counts need to leave HBM.
 * The steps themselves are standard (GLL collocation: Deville, Fischer &
 * Mund 2002; Q-criterion: Hunt, Wray & Moin 1988; marching cubes: Lorensen
 * & Cline 1987); the paper does not print them.
 *
 * Conventions shared by every call
 * --------------------------------
 * Layout      every field argument is a DEVICE pointer to n_elem blocks of
 *             (N+1)^3 contiguous values, element-major, node (i, j, k) of
 *             element e at offset e*(N+1)^3 + i + (N+1)*(j + (N+1)*k)
 *             (i fastest; i, j, k run along the reference directions r, s, t).
 * dtype       SEM_F64: all data and arithmetic in double; SEM_F32: all data
 *             and arithmetic in float.
 * Orders      SEM_MIN_ORDER <= N <= SEM_MAX_ORDER.
 * Streams     `stream` is a hipStream_t passed as void* (NULL = null stream)
 *             on the CURRENT device; every call is asynchronous on it and
 *             never synchronises it.
 * Ownership   the caller owns every buffer; no call allocates or frees
 *             caller memory.  The library owns only its per-device constant
 *             tables (GLL derivative matrices, case table) between sem_init
 *             and sem_finalize.
 * Errors      host-detectable errors are returned synchronously before any
 *             work is queued (SEM_ERR_*).  Conditions found on the device are
 *             OR-ed into *status_word (a DEVICE int32, may be NULL) when the
 *             queued work runs: SEM_FLAG_BAD_JACOBIAN if det J <= 0 at some
 *             node (outputs there are not meaningful), SEM_FLAG_TRI_OVERFLOW
 *             if an isosurface did not fit in the triangle buffer.
 * n_elem == 0 is a valid empty call (isosurface counts are still written).
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Precision of a call.  SEM_F64 / SEM_F32: storage and arithmetic in that
 * type.  SEM_MIXED_*: FP32 storage (every field, output and triangle array
 * is float); the 1-D derivative contractions run on the matrix cores with
 * BF16 or FP16 operands and FP32 accumulation -- plain (one rounded product)
 * or split (x3: hi*hi + lo*hi + hi*lo with x = hi + lo, after Henry, Tang &
 * Heinecke 2019 and, for FP16 with the lo parts scaled by 2^11, Ootomo &
 * Yokota 2022); the Jacobian is inverted in FP64; chain rule, Q and |omega|
 * are FP32.  Mixed modes need N = 7 in sem_derivs, sem_qcrit and
 * sem_extract (SEM_ERR_ORDER otherwise); sem_isosurface, which takes no
 * derivative, treats them as SEM_F32. */
typedef enum {
  SEM_F64 = 0,
  SEM_F32 = 1,
  SEM_MIXED_BF16 = 2,
  SEM_MIXED_FP16 = 3,
  SEM_MIXED_BF16X3 = 4,
  SEM_MIXED_FP16X3 = 5
} sem_dtype;

enum {
  SEM_OK = 0,
  SEM_ERR_ARG = -1,        /* NULL required pointer, negative size, bad count */
  SEM_ERR_ORDER = -2,      /* order outside [SEM_MIN_ORDER, SEM_MAX_ORDER]   */
  SEM_ERR_NOT_INIT = -3,   /* sem_init was not called for the current device */
  SEM_ERR_HIP = -4,        /* a HIP runtime call or kernel launch failed     */
  SEM_ERR_WORKSPACE = -5,  /* isosurface workspace NULL or too small         */
  SEM_ERR_DTYPE = -6       /* dtype is not one of the sem_dtype values       */
};

enum {
  SEM_FLAG_BAD_JACOBIAN = 1,   /* det J <= 0 at some node                         */
  SEM_FLAG_TRI_OVERFLOW = 2,   /* triangles did not fit (counts stay exact)       */
  SEM_FLAG_BAD_ID = 4,         /* a node id or edge key outside its valid range   */
  SEM_FLAG_VERT_OVERFLOW = 8,  /* welded vertices did not fit (count stays exact) */
  SEM_FLAG_RAW_OVERFLOW = 16   /* raw fallback blocks did not fit (count exact)   */
};

#define SEM_MIN_ORDER 1
#define SEM_MAX_ORDER 9
#define SEM_MAX_ISO 64          /* isovalues per sem_isosurface call        */
#define SEM_MC_MAX_TRI 5        /* triangles per marching-cubes case        */

/* Human-readable text for a SEM_* return code (static storage). */
const char* sem_status_str(int status);

/* Build record of this library, for matching a loaded binary to its
 * sources (static storage, never NULL):
 *   "sources_sha256=<64 hex digits>;arch=gfx950;hip=<hipcc's HIP version>"
 * where the digest covers the library's source files as compiled: every
 * file of the kernel source directory (.hip, .cpp, .h) in name order, each
 * as its file name then its bytes, then this header the same way. */
const char* sem_build_info(void);

/* ---------------------------------------------------------------------
 * Host-side basis and table queries (no GPU needed).
 * ------------------------------------------------------------------- */

/* GLL nodes xi[N+1], quadrature weights w[N+1] and collocation derivative
 * matrix D[(N+1)*(N+1)] (row-major, D[i*(N+1)+m] = l_m'(xi_i)) of order N,
 * in FP64, as the library computes them for its kernels.  Nodes: -1, +1 and
 * the roots of the derivative of the Legendre polynomial P_N; weights
 * 2/(N(N+1)P_N(xi)^2); off-diagonal D from the Lagrange-cardinal closed
 * form, diagonal = minus the off-diagonal row sum.  Host pointers, any may
 * be NULL.  Returns SEM_ERR_ORDER for N outside [1, 15]. */
int sem_gll(int order, double* nodes, double* weights, double* dmat);

/* The marching-cubes case table the kernels use: ntri[256] triangles per
 * case and tri[256][SEM_MC_MAX_TRI][3] edge ids (-1 padded).  Corners
 * v = a + 2b + 4c sit at (a, b, c); edges 0-3 run along r, 4-7 along s, 8-11
 * along t, each from its lower to its higher corner.  The table is
 * generated by the face-consistent loop rule: on each face two crossings
 * form one segment and four crossings cut off each above-isovalue corner;
 * segments are oriented with the above side on the left seen from outside,
 * closed into loops, and each loop is fan-triangulated from its smallest
 * edge id that shares no face with a non-adjacent loop vertex.  Host
 * pointers, either may be NULL. */
int sem_mc_table(uint8_t* ntri, int8_t* tri);

/* ---------------------------------------------------------------------
 * Device set-up.
 * ------------------------------------------------------------------- */

/* Upload the constant tables (D of every supported order in FP64 and FP32,
 * the case table) to `device`.  Idempotent; thread-safe; must precede any
 * compute call on that device (and any stream capture).  Leaves the
 * caller's current device unchanged. */
int sem_init(int device);

/* Release the tables on every initialised device. */
void sem_finalize(void);

/* ---------------------------------------------------------------------
 * Hot path.
 * ------------------------------------------------------------------- */

/* Physical gradient of one scalar field on an isoparametric mesh:
 * reference derivatives f_r, f_s, f_t by one D contraction per direction,
 * Jacobian J = d(x,y,z)/d(r,s,t) from the same contractions of the
 * coordinates, and the chain rule df/dx_j = sum_a f_{r_a} (J^-1)_{a j}.
 * x, y, z, f: inputs; dfdx, dfdy, dfdz: outputs (all [n_elem][(N+1)^3]). */
int sem_derivs(int64_t n_elem, int order, sem_dtype dt,
               const void* x, const void* y, const void* z, const void* f,
               void* dfdx, void* dfdy, void* dfdz,
               int32_t* status_word, void* stream);

/* Q-criterion and vorticity magnitude from velocity (u, v, w):
 * A = grad(u) as in sem_derivs, Q = (|Omega|^2 - |S|^2)/2 with
 * S, Omega the symmetric and antisymmetric parts of A, and
 * |omega| = |(A32 - A23, A13 - A31, A21 - A12)|, evaluated at every node of
 * every element (no averaging across elements).
 * q, omega_mag: outputs [n_elem][(N+1)^3] (either may be NULL);
 * q_minmax: optional output [n_elem][2] = (min, max) of Q over each
 * element with NaN counted as -inf, the form sem_isosurface culls with. */
int sem_qcrit(int64_t n_elem, int order, sem_dtype dt,
              const void* x, const void* y, const void* z,
              const void* u, const void* v, const void* w,
              void* q, void* omega_mag, void* q_minmax,
              int32_t* status_word, void* stream);

/* Bytes of device workspace sem_isosurface needs (256-byte aligned start). */
size_t sem_isosurface_workspace_bytes(int64_t n_elem, int order, int n_iso);

/* Marching cubes of `field` over the N^3 sub-hexahedra of every element,
 * for n_iso isovalues, compacted into one triangle soup.
 *   field_minmax  optional [n_elem][2] (min, max) per element as written by
 *                 sem_qcrit; elements whose range does not straddle an
 *                 isovalue are skipped without reading the field (exact).
 *   iso_host      HOST array of n_iso isovalues, rounded to the dtype.
 *   tri_xyz       [tri_capacity][3][3] (triangle, vertex, coordinate), dtype;
 *                 may be NULL when tri_capacity == 0 (count-only call).
 *   tri_edge_key  optional [tri_capacity][3] uint64 vertex keys
 *                 (e*(N+1)^3 + n_lo)*3 + axis of the crossed edge.
 *   tri_count     DEVICE int64[n_iso]: exact triangle count per isovalue,
 *                 even when the buffer overflowed.
 *   active_cells  optional DEVICE int64[n_iso]: cells whose case is neither
 *                 0 nor 255.
 *   case_idx      optional DEVICE uint8[n_iso][n_elem][N^3] case per cell.
 * A node is above the isovalue c when f > c (NaN never is; a vertex on an
 * edge with a NaN end is NaN).  On a crossed
 * edge from its low node (f0, p0) to its high node (f1, p1) the vertex is
 * p0 + t (p1 - p0) with t = (c - f0)/(f1 - f0).  Output order: isovalue,
 * element, cell index i + N(j + N k), case-table slot; triangles whose
 * position is >= tri_capacity are dropped and SEM_FLAG_TRI_OVERFLOW is set. */
int sem_isosurface(int64_t n_elem, int order, sem_dtype dt,
                   const void* x, const void* y, const void* z,
                   const void* field, const void* field_minmax,
                   int n_iso, const double* iso_host,
                   void* tri_xyz, int64_t tri_capacity,
                   uint64_t* tri_edge_key,
                   int64_t* tri_count, int64_t* active_cells,
                   uint8_t* case_idx,
                   void* workspace, size_t workspace_bytes,
                   int32_t* status_word, void* stream);

/* Bytes of device workspace sem_extract needs for this problem and dtype
 * (0 for invalid arguments). */
size_t sem_extract_workspace_bytes(int64_t n_elem, int order, int n_iso, sem_dtype dt);

/* Q-criterion, vorticity magnitude and the isosurfaces of Q in one call:
 * the results of sem_qcrit followed by sem_isosurface on Q (same case
 * table, vertex rule, NaN and tie rules, same triangles in the same order),
 * with Q never re-read for classification.  For N = 7 in FP64 the first
 * kernel stages each element's six tiles in LDS, computes Q and |omega|,
 * and counts every isovalue's triangles from the Q tile; the counts are
 * exclusive-scanned, and a second kernel re-stages the Q and coordinate
 * tiles of the elements that have triangles and emits them.  Other orders
 * and FP32 run sem_qcrit's kernel, then sem_isosurface's count and emission.
 *   q, omega_mag, q_minmax  optional device outputs, as in sem_qcrit (when
 *                 q or q_minmax is NULL the workspace holds them).
 *   iso_host      HOST array of n_iso isovalues.
 *   tri_xyz       HOST array of n_iso DEVICE pointers: isovalue s writes its
 *                 triangles to tri_xyz[s] as [tri_capacity[s]][3][3], in
 *                 (element, cell, slot) order -- isovalue s of
 *                 sem_isosurface's output.
 *   tri_capacity  HOST array of n_iso capacities (a NULL tri_xyz[s] is
 *                 allowed with capacity 0: count only).
 *   tri_count     DEVICE int64[n_iso], exact even on overflow.
 *   active_cells  optional DEVICE int64[n_iso].
 *   workspace     device scratch of sem_extract_workspace_bytes(); its
 *                 contents need no initialisation and are overwritten.
 * Calls sharing a workspace must not overlap (same stream is fine). */
int sem_extract(int64_t n_elem, int order, sem_dtype dt,
                const void* x, const void* y, const void* z,
                const void* u, const void* v, const void* w,
                void* q, void* omega_mag, void* q_minmax,
                int n_iso, const double* iso_host,
                void* const* tri_xyz, const int64_t* tri_capacity,
                int64_t* tri_count, int64_t* active_cells,
                void* workspace, size_t workspace_bytes,
                int32_t* status_word, void* stream);

/* Largest n_iso * n_elem that sem_extract_noalloc accepts. */
#define SEM_NOALLOC_MAX_COUNTS (1 << 20)

/* sem_extract for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, kernels and results as sem_extract, with the
 * per-(isovalue, element) triangle counts, their exclusive prefix and the
 * scan's partial sums held in a fixed scratch array that the library keeps
 * on every initialised GPU (about 12 MiB, resident until the process ends;
 * its address is looked up once per device by sem_init) instead of a
 * caller workspace.  q and q_minmax are required outputs here (sem_extract
 * keeps them in its workspace when they are NULL); omega_mag and
 * active_cells stay optional.  Nothing in the scratch needs clearing: every
 * value is written before it is read in each call.  SEM_ERR_WORKSPACE when
 * n_iso * n_elem > SEM_NOALLOC_MAX_COUNTS; otherwise the arguments and
 * errors of sem_extract.  The call allocates and frees nothing.  All calls
 * on one GPU share its scratch: calls that may overlap in time (different
 * streams, or host threads without ordering) race on it and must not be
 * issued; calls on one stream are ordered and safe. */
int sem_extract_noalloc(int64_t n_elem, int order, sem_dtype dt,
                        const void* x, const void* y, const void* z,
                        const void* u, const void* v, const void* w,
                        void* q, void* omega_mag, void* q_minmax,
                        int n_iso, const double* iso_host,
                        void* const* tri_xyz, const int64_t* tri_capacity,
                        int64_t* tri_count, int64_t* active_cells,
                        int32_t* status_word, void* stream);

/* ---------------------------------------------------------------------
 * Batched snapshots: one persistent launch over many snapshots
 * ---------------------------------------------------------------------
 * Snapshots of different order and size (all in one precision, F64 or F32)
 * go through one persistent kernel per order present (per-order
 * instantiations, each with its own register budget), all launched by one
 * call: its workgroups walk the work items -- one or a few consecutive
 * elements of one snapshot -- of every snapshot of that order, each
 * computing Q, |omega| and the element ranges exactly as sem_qcrit defines
 * them.  How a work item is computed is the variant set for its (order,
 * precision), by default the form sem_qcrit uses, or the one sem_autotune
 * measured fastest on this device:
 *   0, 1, 2  LDS-tile form, 256 threads, 1, 2 or 4 elements per work item
 *            (if the kernel's LDS tile holds them);
 *   3        register-pencil form, 128 threads (256 for N >= 8), one
 *            element (default for FP32, and for FP64 N <= 6);
 *   4        direct-to-LDS form, 256 threads, one element (N = 7, FP64
 *            only; its default);
 *   5        one thread per node, one element (default for FP64 N >= 8).
 * A plan (device buffer) holds the snapshot descriptors, so sem_qcrit_batch
 * takes no host data and can be captured in a HIP graph and replayed. */
typedef struct {
  int64_t n_elem;
  int order;
  const void *x, *y, *z, *u, *v, *w;   /* DEVICE inputs, sem layout      */
  void *q, *omega_mag, *q_minmax;      /* DEVICE outputs, any may be NULL
                                          (not all three)                */
} sem_snapshot;

/* Bytes of a plan for n_snap snapshots (1 <= n_snap <= 4096; else 0). */
size_t sem_batch_plan_bytes(int n_snap);

/* Write the plan of n_snap snapshots (HOST array) into the DEVICE buffer
 * plan, and into *launch_code (may be NULL) the kernels it needs: 3 bits
 * per order N at bit 3N, 0 = no snapshot of that order, else 1 + the form
 * of its work items.  A setup call: it copies synchronously (not
 * capturable).  The plan records the pointers and the variants set at this
 * moment. */
int sem_batch_plan(int n_snap, const sem_snapshot* snaps, sem_dtype dt, void* plan,
                   size_t plan_bytes, unsigned* launch_code);

/* Q, |omega| and element ranges of every snapshot of the plan: one
 * persistent launch per order in launch_code (the code sem_batch_plan
 * returned for this plan), on `stream`; dt must be the plan's.
 * Asynchronous; capturable in a HIP graph. */
int sem_qcrit_batch(const void* plan, unsigned launch_code, sem_dtype dt, int32_t* status_word,
                    void* stream);

/* Time the batched kernel on 8,192 synthetic elements of this order with
 * every variant that applies, keep the fastest for (order, dt) on the
 * current device and return it in *variant_out (may be NULL); ms_out (may
 * be NULL) receives the six timings in ms (-1 = variant not applicable).
 * A setup call: allocates temporary device memory and synchronises the
 * device. */
int sem_autotune(int order, sem_dtype dt, int* variant_out, float* ms_out);

/* Variant the next plans use for (order, dt) on the current device. */
int sem_batch_variant(int order, sem_dtype dt);

/* Set the variant for (order, dt) on the current device without timing
 * (SEM_ERR_ARG if it does not apply to the order). */
int sem_batch_set_variant(int order, sem_dtype dt, int variant);

/* ---------------------------------------------------------------------
 * Batched isosurfaces: persistent count, one scan, persistent emission
 * ---------------------------------------------------------------------
 * The marching-cubes extraction of sem_isosurface (Lorensen & Cline 1987;
 * the cases, order and vertex rule are sem_isosurface's) over many
 * (snapshot, field, isovalue set) jobs at once: one persistent count kernel
 * per order present walks every (job, element) work item, one exclusive
 * scan runs over the counts of every job, and one persistent emission
 * kernel per order writes the triangles.  Every job's triangles go into one
 * soup, ordered by job (the caller's order), isovalue, element, cell and
 * case-table slot; each (job, isovalue) gets its first triangle and count.
 * A job's triangles are bit-identical to those sem_isosurface writes for
 * the same field and isovalues. */
enum { SEM_JOB_Q = 0, SEM_JOB_OMEGA = 1, SEM_JOB_SCALAR = 2 };
typedef struct {
  int snap;              /* index into the snapshot array of the plan call      */
  int field;             /* SEM_JOB_Q: the snapshot's q (its q_minmax, if any,
                            culls elements); SEM_JOB_OMEGA: its omega_mag;
                            SEM_JOB_SCALAR: `scalar`                             */
  const void* scalar;    /* DEVICE field in the sem layout (SEM_JOB_SCALAR)     */
  int n_iso;             /* 1 <= n_iso <= 4                                     */
  double iso[4];         /* isovalues, cast to the plan's precision             */
} sem_iso_job;

typedef struct {
  unsigned launch_code;  /* bit N set when some job has order N                 */
  sem_dtype dt;          /* the plan's precision                                */
  int n_job;
  int64_t n_slots;       /* (job, isovalue, element) count slots                */
  size_t workspace_bytes;/* workspace sem_isosurface_batch needs                */
} sem_iso_batch_info;

/* Bytes of an isosurface plan for n_job jobs (1 <= n_job <= 16384; else 0). */
size_t sem_iso_batch_plan_bytes(int n_job);

/* Write the plan of n_job jobs (HOST array) over n_snap snapshots (HOST
 * array; only their order, element count, coordinates, q, omega_mag and
 * q_minmax are used) into the DEVICE buffer plan, and its launch facts into
 * *info (HOST).  SEM_ERR_ARG for a job naming a snapshot outside
 * [0, n_snap), an unknown field, a NULL field the job needs, n_iso outside
 * [1, 4] or a NaN isovalue; SEM_ERR_ORDER for a snapshot order outside
 * [SEM_MIN_ORDER, SEM_MAX_ORDER].  A setup call: it copies synchronously
 * (not capturable); the plan records the pointers given now. */
int sem_iso_batch_plan(int n_snap, const sem_snapshot* snaps, int n_job,
                       const sem_iso_job* jobs, sem_dtype dt, void* plan, size_t plan_bytes,
                       sem_iso_batch_info* info);

/* Isosurfaces of every job of the plan into tri_xyz (DEVICE
 * [tri_capacity][3][3], dt), on `stream`; info is the plan call's and dt
 * its precision (SEM_ERR_DTYPE otherwise): tri_offset (DEVICE [4 * n_job],
 * may be NULL) receives the first triangle of (job j, isovalue s) at
 * 4j + s, tri_count (DEVICE [4 * n_job]) its count (0 for s >= the job's
 * n_iso), active_cells (DEVICE [4 * n_job], may be NULL) its active cells.
 * Counts are exact when the soup does not fit; triangles past tri_capacity
 * are not written and SEM_FLAG_TRI_OVERFLOW is set.  workspace (DEVICE,
 * >= info->workspace_bytes) needs no clearing.  Asynchronous; capturable in
 * a HIP graph (no host data is read at launch time). */
int sem_isosurface_batch(const void* plan, const sem_iso_batch_info* info, sem_dtype dt,
                         void* tri_xyz, int64_t tri_capacity, int64_t* tri_offset,
                         int64_t* tri_count, int64_t* active_cells, void* workspace,
                         size_t workspace_bytes, int32_t* status_word, void* stream);

/* ---------------------------------------------------------------------
 * C0 averaging over shared GLL nodes and welded isosurface output
 * ---------------------------------------------------------------------
 * Elements store their own copy of every node.  gid[e][node] (DEVICE int64,
 * the field layout) gives each stored node a global id in [0, n_global);
 * coincident copies share an id (NekRS keeps such ids for its gather-
 * scatter).  Derived fields computed per element differ between copies; the
 * direct-stiffness average (Deville, Fischer & Mund 2002, ch. 4: the
 * gather-scatter sum divided by the multiplicity) replaces every copy by the
 * mean over all copies of its node, so isosurfaces close across element
 * faces. */

/* Bytes of the buffer sem_gs_setup fills (0 for invalid arguments). */
size_t sem_gs_workspace_bytes(int64_t n_elem, int order, int64_t n_global);

/* Build the gather-scatter structure of gid into the caller's DEVICE buffer
 * gs (the copies of every global node, in increasing storage order).  The
 * buffer is read by sem_dsavg until the caller frees or rebuilds it.  Ids
 * outside [0, n_global) set SEM_FLAG_BAD_ID and are left out.  Requires
 * n_global < 2^32 - 1. */
int sem_gs_setup(int64_t n_elem, int order, const int64_t* gid, int64_t n_global, void* gs,
                 size_t gs_bytes, int32_t* status_word, void* stream);

/* out = direct-stiffness average of field (both [n_elem][(N+1)^3] of dtype
 * dt; mixed dtypes mean FP32): for each global node, the copies' values are
 * summed one at a time in increasing storage order in dt, divided by their
 * number, and written to every copy.  out may equal field. */
int sem_dsavg(int64_t n_elem, int order, sem_dtype dt, const void* gs, int64_t n_global,
              const void* field, void* out, void* stream);

/* Global keys of n_ref element-local edge keys (as written by
 * sem_isosurface: (e (N+1)^3 + n_lo) * 3 + axis):
 *   key = (min(gid_lo, gid_hi) << 32) | max(gid_lo, gid_hi).
 * Vertices on the same global edge get the same key in every element.  A
 * local key outside the n_elem elements, or ids outside [0, 2^32 - 1), give
 * the key 0xffff...ff and set SEM_FLAG_BAD_ID. */
int sem_global_edge_keys(int64_t n_ref, int order, int64_t n_elem, const uint64_t* local_keys,
                         const int64_t* gid, uint64_t* global_keys, int32_t* status_word,
                         void* stream);

/* Bytes of device workspace sem_weld needs for n_ref = 3 * triangles. */
size_t sem_weld_workspace_bytes(int64_t n_ref);

/* Weld a triangle soup (tri_xyz [n_ref / 3][3][3] of dtype dt, keys [n_ref]
 * global edge keys): the distinct keys, numbered in order of first
 * occurrence (corner r = 3 * triangle + corner), are the vertices; vertex v
 * gets the coordinates of its first occurrence (vert_xyz [vert_capacity][3]),
 * and tri_index[r] (DEVICE int64 [n_ref]) the index of corner r's key.
 * *n_vert (DEVICE int64) is exact even when vertices beyond vert_capacity are
 * dropped (SEM_FLAG_VERT_OVERFLOW).  A key of all ones sets SEM_FLAG_BAD_ID
 * and gets index -1.  The result does not depend on scheduling. */
int sem_weld(int64_t n_ref, sem_dtype dt, const void* tri_xyz, const uint64_t* keys,
             int64_t* tri_index, void* vert_xyz, int64_t vert_capacity, int64_t* n_vert,
             void* workspace, size_t workspace_bytes, int32_t* status_word, void* stream);

/* ---------------------------------------------------------------------
 * Kernel-phase timing (a tracing aid, not part of the method)
 * ------------------------------------------------------------------- */

/* Phases the timing reports: the Q / |omega| kernel (which also counts
 * triangles in sem_extract's N = 7 FP64 path), the separate classify-and-
 * count kernel, the exclusive scan with the totals, and triangle emission. */
enum { SEM_PHASE_QCRIT = 0, SEM_PHASE_COUNT = 1, SEM_PHASE_SCAN = 2, SEM_PHASE_EMIT = 3,
       SEM_NUM_PHASES = 4 };

/* Name of a phase ("qcrit", "count", "scan", "emit"), or "unknown". */
const char* sem_phase_name(int phase);

/* Start timing on the CURRENT device: every later sem_qcrit, sem_isosurface
 * and sem_extract on this device records a HIP event on its stream before
 * and after each phase, for at most max_spans phase executions (later ones
 * are counted as dropped).  The library creates the 2*max_spans events
 * here (host-side runtime objects; no device memory).  Returns SEM_ERR_ARG
 * when max_spans is outside [1, 1<<20] or timing is already on for this
 * device, SEM_ERR_HIP when event creation fails. */
int sem_timing_begin(int max_spans);

/* Stop timing on the current device: waits for the recorded events, writes
 * for phases 0..n_phases-1 the summed duration in milliseconds (ms_total)
 * and the number of timed executions (spans) -- either array may be NULL --
 * releases the events, and returns the number of dropped spans (>= 0), or
 * SEM_ERR_ARG when timing was not on, SEM_ERR_HIP on a runtime error. */
int64_t sem_timing_end(double* ms_total, int64_t* spans, int n_phases);

/* Copy `bytes` from src to dst (both DEVICE, 16-byte aligned, not
 * overlapping; bytes a multiple of 16) with a plain streaming kernel: each
 * 16-byte chunk read once and written once, consecutive lanes on
 * consecutive chunks.  It is the reference for the HBM bandwidth this GPU
 * sustains, beside which the extraction kernels' rates are reported.
 * SEM_ERR_ARG for NULL pointers with bytes > 0, misaligned pointers or a
 * size that is not a multiple of 16; bytes == 0 does nothing.  Needs no
 * sem_init. */
int sem_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* ---------------------------------------------------------------------
 * Learned in-transit compression (order 7, FP32 fields u, v, w, theta)
 * ---------------------------------------------------------------------
 * The in-transit workflow (section 4.2) ships every snapshot from the
 * simulation nodes to visualisation nodes; this compressor cuts the bytes.
 * Per element, each channel is divided by its element maximum s_ec and the
 * 4 x 8^3 block goes through a convolutional autoencoder: three
 * kernel-2 stride-2 convolutions 4 -> 32 -> 64 -> 32 channels (8^3 -> 4^3
 * -> 2^3 -> 1: the 32-value latent, stored as IEEE binary16) and three
 * kernel-2 stride-2 transposed convolutions 32 -> 64 -> 32 -> 4 back.  Layers
 * are linear; tanh_mask (bits 0, 1, 3, 4 only: SEM_AE_TANH_HIDDEN) adds tanh
 * after hidden layers.  An element whose reconstruction misses
 * max |f - f_hat| <= 1e-3 max(s_ec, 1e-3 max_e s_ec) on any channel is
 * shipped raw instead.
 *
 * Parameters (FP32, sem_ae_param_count() values): for each layer, weights
 * then biases; a convolution's weight (d, i, o) at (d Cin + i) Cout + o, a
 * transposed one's at (i 8 + d) Cout + o, d = dx + 2 dy + 4 dz.
 * Blocks (the network's input layout, FP32 [E][512][4]): value (i, j, k) of
 * channel c at [e][m][c], m the Morton index (bits i0 j0 k0 i1 j1 k1 i2 j2 k2
 * from the least significant).  Every pointer is DEVICE memory; workspace
 * sizes come from the matching *_workspace_bytes call. */
#define SEM_AE_LATENT 32
#define SEM_AE_TANH_HIDDEN 0x1B

int64_t sem_ae_param_count(void);

/* Workspace of sem_ae_forward / sem_ae_grad for a batch of n elements. */
size_t sem_ae_workspace_bytes(int64_t n);

/* Normalised blocks [E][512][4] and element maxima scale[E][4] of four
 * fields [E][8][8][8] (GLL layout). */
int sem_ae_blocks(int64_t n_elem, const float* u, const float* v, const float* w,
                  const float* theta, float* blocks, float* scale, void* stream);

/* Network on n blocks: reconstruction [n][512][4] (normalised, may be NULL)
 * and binary16 latent [n][32] (may be NULL). */
int sem_ae_forward(int64_t n, const float* blocks, const float* params, int tanh_mask,
                   float* recon, uint16_t* latent, void* workspace, size_t workspace_bytes,
                   void* stream);

/* Loss (*loss, device float, may be NULL) and its gradient
 * grad[sem_ae_param_count()] on the batch pool[idx[r]], r < n (idx NULL:
 * the first n blocks of the pool).  loss_kind SEM_AE_LOSS_MSE: mean squared
 * error over every value; SEM_AE_LOSS_MAX: mean over (block, channel) of
 * the squared largest absolute error over the block's nodes (the squared
 * form of the relative L-inf bound of the raw fallback), whose gradient
 * 2 m sign(y - x) / (4 n) sits at the node(s) of the maximum m, shared
 * equally by ties; any other value is SEM_ERR_ARG.  The latent is rounded
 * to binary16 in the forward pass and its gradient passed through
 * unchanged.  An index outside [0, n_pool) sets SEM_FLAG_BAD_ID and
 * contributes a zero block. */
#define SEM_AE_LOSS_MSE 0
#define SEM_AE_LOSS_MAX 1
int sem_ae_grad(int64_t n, const float* pool, int64_t n_pool, const int64_t* idx,
                const float* params, int tanh_mask, int loss_kind, float* grad, float* loss,
                void* workspace, size_t workspace_bytes, int32_t* status_word, void* stream);

/* One Adam step (Kingma & Ba 2015) on n values; step counts from 1. */
int sem_ae_adam(int64_t n, float* params, const float* grad, float* m, float* v, int step,
                float lr, float beta1, float beta2, float eps, void* stream);

/* Symmetric eigenproblem of the n x n FP64 matrix a (n even, 2 <= n <= 512),
 * cyclic Jacobi (Golub & Van Loan, Matrix Computations, section 8.5, with
 * the round-robin parallel ordering): the r largest eigenvalues in
 * decreasing order into lam[r] (may be NULL) and their eigenvectors into
 * vec[n][r] (FP32, each signed so that its largest-magnitude entry is
 * positive); *sweeps (device int, may be NULL) receives the sweeps used.
 * Each round of rotations runs over the whole GPU; the call synchronises
 * `stream` once per sweep to read the convergence test (a setup call, not
 * capturable). */
size_t sem_eig_workspace_bytes(int n);
int sem_sym_eig(int n, const double* a, int r, double* lam, float* vec, void* workspace,
                size_t workspace_bytes, int* sweeps, void* stream);

/* Parameters from layer-wise principal components of n_pool blocks
 * (1 <= n_pool <= 2^24): layer
 * 0 the identity on each 2^3 patch, layers 1 and 2 the 64 and 32 leading
 * eigenvectors of the second-moment matrices of their inputs, decoder
 * layers the transposes, biases zero; lam (may be NULL) receives the 64 +
 * 32 eigenvalues.  Synchronises `stream` (the eigensolver's convergence
 * tests). */
size_t sem_ae_pca_workspace_bytes(int64_t n_pool);
int sem_ae_pca_init(int64_t n_pool, const float* pool, float* params, double* lam,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Compress E elements: binary16 latent [E][32], scale [E][4], flags [E]
 * (1 = raw), the raw elements' fields packed in element order into
 * raw[raw_cap][4][512] and their count into *n_raw (device int64; exact even
 * when raw_cap is too small, which sets SEM_FLAG_RAW_OVERFLOW). */
size_t sem_ae_compress_workspace_bytes(int64_t n_elem);
int sem_ae_compress(int64_t n_elem, const float* u, const float* v, const float* w,
                    const float* theta, const float* params, int tanh_mask, uint16_t* latent,
                    float* scale, uint8_t* flags, float* raw, int64_t raw_cap, int64_t* n_raw,
                    void* workspace, size_t workspace_bytes, int32_t* status_word,
                    void* stream);

/* Fields [E][8][8][8] from a compressed snapshot (workspace: the
 * compression's size for E).  raw holds raw_count blocks (raw may be NULL
 * when raw_count is 0); a flagged element past them decodes from its latent
 * and sets SEM_FLAG_RAW_OVERFLOW. */
int sem_ae_decompress(int64_t n_elem, const uint16_t* latent, const float* scale,
                      const uint8_t* flags, const float* raw, int64_t raw_count,
                      const float* params, int tanh_mask, float* u, float* v, float* w,
                      float* theta, void* workspace, size_t workspace_bytes,
                      int32_t* status_word, void* stream);

/* Non-learned baseline at the same bytes: per channel the eight Legendre
 * coefficients with degrees in {0, 1}^3 of the element's interpolant (GLL
 * quadrature), stored as binary16 of c / s_ec into coef[E][4][8]; scale,
 * fallback flags by the same rule, reconstructions (may be NULL). */
int sem_modal_compress(int64_t n_elem, const float* u, const float* v, const float* w,
                       const float* theta, uint16_t* coef, float* scale, uint8_t* flags,
                       float* ru, float* rv, float* rw, float* rtheta, void* workspace,
                       size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
