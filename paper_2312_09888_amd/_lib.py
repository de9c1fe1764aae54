"""ctypes binding of libsem.so: the C ABI declared in include/sem.h.

Argument marshalling only -- every step of the extraction runs in the HIP
kernels behind these calls.  Device buffers are torch tensors (used for
memory and streams); the library is launched on the current torch stream of
the tensors' device.  There is no fallback: if libsem.so is missing or
fails to load, every entry point raises.
"""

import ctypes
import math
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsem.so")

SEM_F64, SEM_F32 = 0, 1
SEM_MIXED_BF16, SEM_MIXED_FP16, SEM_MIXED_BF16X3, SEM_MIXED_FP16X3 = 2, 3, 4, 5
# precision names of the mixed modes (FP32 storage, MFMA derivative contractions)
MIXED = {"bf16": SEM_MIXED_BF16, "fp16": SEM_MIXED_FP16, "bf16x3": SEM_MIXED_BF16X3,
         "fp16x3": SEM_MIXED_FP16X3}
SEM_OK = 0
SEM_ERR_ARG, SEM_ERR_ORDER, SEM_ERR_NOT_INIT = -1, -2, -3
SEM_ERR_HIP, SEM_ERR_WORKSPACE, SEM_ERR_DTYPE = -4, -5, -6
SEM_FLAG_BAD_JACOBIAN, SEM_FLAG_TRI_OVERFLOW, SEM_FLAG_BAD_ID, SEM_FLAG_VERT_OVERFLOW = 1, 2, 4, 8
SEM_MIN_ORDER, SEM_MAX_ORDER = 1, 9
SEM_MAX_ISO = 64
SEM_NOALLOC_MAX_COUNTS = 1 << 20   # n_iso * n_elem of sem_extract_noalloc
SEM_FLAG_RAW_OVERFLOW = 16
SEM_AE_LATENT = 32
SEM_AE_TANH_HIDDEN = 0x1B
SEM_AE_LOSS_MSE, SEM_AE_LOSS_MAX = 0, 1
BATCH_VARIANTS = 6          # variants of the batched kernel (sem_autotune)
SEM_MC_MAX_TRI = 5
SEM_PHASE_QCRIT, SEM_PHASE_COUNT, SEM_PHASE_SCAN, SEM_PHASE_EMIT = 0, 1, 2, 3
SEM_NUM_PHASES = 4

EXPORTS = (
    "sem_status_str", "sem_build_info", "sem_gll", "sem_mc_table", "sem_init", "sem_finalize",
    "sem_derivs", "sem_qcrit", "sem_isosurface_workspace_bytes", "sem_isosurface",
    "sem_extract_workspace_bytes", "sem_extract", "sem_extract_noalloc",
    "sem_phase_name", "sem_timing_begin", "sem_timing_end", "sem_stream_copy",
    "sem_gs_workspace_bytes", "sem_gs_setup", "sem_dsavg", "sem_global_edge_keys",
    "sem_weld_workspace_bytes", "sem_weld",
    "sem_batch_plan_bytes", "sem_batch_plan", "sem_qcrit_batch", "sem_autotune",
    "sem_batch_variant", "sem_batch_set_variant",
    "sem_iso_batch_plan_bytes", "sem_iso_batch_plan", "sem_isosurface_batch",
    "sem_ae_param_count", "sem_ae_workspace_bytes", "sem_ae_blocks", "sem_ae_forward",
    "sem_ae_grad", "sem_ae_adam", "sem_eig_workspace_bytes", "sem_sym_eig",
    "sem_ae_pca_workspace_bytes", "sem_ae_pca_init", "sem_ae_compress_workspace_bytes",
    "sem_ae_compress", "sem_ae_decompress", "sem_modal_compress",
)


class _Snapshot(ctypes.Structure):
    """sem_snapshot of include/sem.h."""
    _fields_ = [("n_elem", ctypes.c_int64), ("order", ctypes.c_int)] + [
        (k, ctypes.c_void_p) for k in ("x", "y", "z", "u", "v", "w", "q", "omega_mag",
                                       "q_minmax")]


class _IsoJob(ctypes.Structure):
    """sem_iso_job of include/sem.h."""
    _fields_ = [("snap", ctypes.c_int), ("field", ctypes.c_int), ("scalar", ctypes.c_void_p),
                ("n_iso", ctypes.c_int), ("iso", ctypes.c_double * 4)]


class _IsoBatchInfo(ctypes.Structure):
    """sem_iso_batch_info of include/sem.h."""
    _fields_ = [("launch_code", ctypes.c_uint), ("dt", ctypes.c_int), ("n_job", ctypes.c_int),
                ("n_slots", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


SEM_JOB_Q, SEM_JOB_OMEGA, SEM_JOB_SCALAR = 0, 1, 2


class SemError(RuntimeError):
    """A SEM_* error code returned by the library."""

    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {status_str(code)} (code {code})")


_lib = None


def lib():
    """Load libsem.so once; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libsem.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2312_09888_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.sem_status_str.restype = ctypes.c_char_p
        L.sem_status_str.argtypes = [i32]
        L.sem_build_info.restype = ctypes.c_char_p
        L.sem_build_info.argtypes = []
        L.sem_gll.restype = i32
        L.sem_gll.argtypes = [i32, vp, vp, vp]
        L.sem_mc_table.restype = i32
        L.sem_mc_table.argtypes = [vp, vp]
        L.sem_init.restype = i32
        L.sem_init.argtypes = [i32]
        L.sem_finalize.restype = None
        L.sem_finalize.argtypes = []
        L.sem_derivs.restype = i32
        L.sem_derivs.argtypes = [i64, i32, i32] + [vp] * 7 + [vp, vp]
        L.sem_qcrit.restype = i32
        L.sem_qcrit.argtypes = [i64, i32, i32] + [vp] * 9 + [vp, vp]
        L.sem_isosurface_workspace_bytes.restype = ctypes.c_size_t
        L.sem_isosurface_workspace_bytes.argtypes = [i64, i32, i32]
        L.sem_isosurface.restype = i32
        L.sem_isosurface.argtypes = ([i64, i32, i32] + [vp] * 5 + [i32, vp, vp, i64]
                                     + [vp] * 5 + [ctypes.c_size_t, vp, vp])
        L.sem_extract_workspace_bytes.restype = ctypes.c_size_t
        L.sem_extract_workspace_bytes.argtypes = [i64, i32, i32, i32]
        L.sem_extract.restype = i32
        L.sem_extract.argtypes = ([i64, i32, i32] + [vp] * 9 + [i32, vp, vp, vp, vp, vp,
                                                                vp, ctypes.c_size_t, vp, vp])
        L.sem_extract_noalloc.restype = i32
        L.sem_extract_noalloc.argtypes = ([i64, i32, i32] + [vp] * 9 + [i32, vp, vp, vp, vp, vp,
                                                                        vp, vp])
        L.sem_phase_name.restype = ctypes.c_char_p
        L.sem_phase_name.argtypes = [i32]
        L.sem_timing_begin.restype = i32
        L.sem_timing_begin.argtypes = [i32]
        L.sem_timing_end.restype = i64
        L.sem_timing_end.argtypes = [vp, vp, i32]
        L.sem_stream_copy.restype = i32
        L.sem_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.sem_gs_workspace_bytes.restype = ctypes.c_size_t
        L.sem_gs_workspace_bytes.argtypes = [i64, i32, i64]
        L.sem_gs_setup.restype = i32
        L.sem_gs_setup.argtypes = [i64, i32, vp, i64, vp, ctypes.c_size_t, vp, vp]
        L.sem_dsavg.restype = i32
        L.sem_dsavg.argtypes = [i64, i32, i32, vp, i64, vp, vp, vp]
        L.sem_global_edge_keys.restype = i32
        L.sem_global_edge_keys.argtypes = [i64, i32, i64, vp, vp, vp, vp, vp]
        L.sem_weld_workspace_bytes.restype = ctypes.c_size_t
        L.sem_weld_workspace_bytes.argtypes = [i64]
        L.sem_weld.restype = i32
        L.sem_weld.argtypes = [i64, i32, vp, vp, vp, vp, i64, vp, vp, ctypes.c_size_t, vp, vp]
        L.sem_batch_plan_bytes.restype = ctypes.c_size_t
        L.sem_batch_plan_bytes.argtypes = [i32]
        L.sem_batch_plan.restype = i32
        L.sem_batch_plan.argtypes = [i32, vp, i32, vp, ctypes.c_size_t, vp]
        L.sem_qcrit_batch.restype = i32
        L.sem_qcrit_batch.argtypes = [vp, ctypes.c_uint, i32, vp, vp]
        L.sem_autotune.restype = i32
        L.sem_autotune.argtypes = [i32, i32, vp, vp]
        L.sem_batch_variant.restype = i32
        L.sem_batch_variant.argtypes = [i32, i32]
        L.sem_batch_set_variant.restype = i32
        L.sem_batch_set_variant.argtypes = [i32, i32, i32]
        L.sem_iso_batch_plan_bytes.restype = ctypes.c_size_t
        L.sem_iso_batch_plan_bytes.argtypes = [i32]
        L.sem_iso_batch_plan.restype = i32
        L.sem_iso_batch_plan.argtypes = [i32, vp, i32, vp, i32, vp, ctypes.c_size_t, vp]
        L.sem_isosurface_batch.restype = i32
        L.sem_isosurface_batch.argtypes = [vp, vp, i32, vp, i64, vp, vp, vp, vp,
                                           ctypes.c_size_t, vp, vp]
        sz, flt = ctypes.c_size_t, ctypes.c_float
        L.sem_ae_param_count.restype = i64
        L.sem_ae_param_count.argtypes = []
        L.sem_ae_workspace_bytes.restype = sz
        L.sem_ae_workspace_bytes.argtypes = [i64]
        L.sem_ae_blocks.restype = i32
        L.sem_ae_blocks.argtypes = [i64] + [vp] * 7
        L.sem_ae_forward.restype = i32
        L.sem_ae_forward.argtypes = [i64, vp, vp, i32, vp, vp, vp, sz, vp]
        L.sem_ae_grad.restype = i32
        L.sem_ae_grad.argtypes = [i64, vp, i64, vp, vp, i32, i32, vp, vp, vp, sz, vp, vp]
        L.sem_ae_adam.restype = i32
        L.sem_ae_adam.argtypes = [i64, vp, vp, vp, vp, i32, flt, flt, flt, flt, vp]
        L.sem_eig_workspace_bytes.restype = sz
        L.sem_eig_workspace_bytes.argtypes = [i32]
        L.sem_sym_eig.restype = i32
        L.sem_sym_eig.argtypes = [i32, vp, i32, vp, vp, vp, sz, vp, vp]
        L.sem_ae_pca_workspace_bytes.restype = sz
        L.sem_ae_pca_workspace_bytes.argtypes = [i64]
        L.sem_ae_pca_init.restype = i32
        L.sem_ae_pca_init.argtypes = [i64, vp, vp, vp, vp, sz, vp]
        L.sem_ae_compress_workspace_bytes.restype = sz
        L.sem_ae_compress_workspace_bytes.argtypes = [i64]
        L.sem_ae_compress.restype = i32
        L.sem_ae_compress.argtypes = [i64] + [vp] * 5 + [i32, vp, vp, vp, vp, i64, vp, vp, sz,
                                                        vp, vp]
        L.sem_ae_decompress.restype = i32
        L.sem_ae_decompress.argtypes = [i64] + [vp] * 4 + [i64, vp, i32] + [vp] * 5 + [sz, vp, vp]
        L.sem_modal_compress.restype = i32
        L.sem_modal_compress.argtypes = [i64] + [vp] * 12 + [sz, vp]
        del dbl
        _lib = L
    return _lib


def status_str(code):
    return lib().sem_status_str(int(code)).decode()


def build_info():
    """The loaded library's build record (sem_build_info) as a dict:
    sources_sha256, arch, hip."""
    text = lib().sem_build_info().decode()
    return dict(item.split("=", 1) for item in text.split(";"))


def _check(code, where):
    if code != SEM_OK:
        raise SemError(code, where)


# ---------------------------------------------------------------------------
# host-side queries
# ---------------------------------------------------------------------------

def gll(order):
    """(nodes, weights, D) of order N as the library computes them."""
    p = order + 1
    nodes = np.zeros(p)
    weights = np.zeros(p)
    d = np.zeros((p, p))
    _check(lib().sem_gll(order, nodes.ctypes.data, weights.ctypes.data, d.ctypes.data),
           "sem_gll")
    return nodes, weights, d


def mc_table():
    """(ntri[256] uint8, tri[256, 5, 3] int8) as the kernels use it."""
    ntri = np.zeros(256, dtype=np.uint8)
    tri = np.zeros((256, SEM_MC_MAX_TRI, 3), dtype=np.int8)
    _check(lib().sem_mc_table(ntri.ctypes.data, tri.ctypes.data), "sem_mc_table")
    return ntri, tri


# ---------------------------------------------------------------------------
# device calls (torch tensors)
# ---------------------------------------------------------------------------

_ready = set()


def _torch():
    import torch
    return torch


def init(device=None):
    """sem_init for a device index (default: the current torch device)."""
    torch = _torch()
    if device is None:
        device = torch.cuda.current_device()
    device = int(device)
    if device not in _ready:
        _check(lib().sem_init(device), "sem_init")
        _ready.add(device)
    return device


def _dtype_code(t, precision=None):
    """SEM_F64 / SEM_F32 from the tensor dtype, or a mixed mode by name
    (float32 tensors only)."""
    torch = _torch()
    if precision is not None:
        if precision not in MIXED:
            raise ValueError(f"precision must be one of {sorted(MIXED)}")
        if t.dtype != torch.float32:
            raise TypeError("mixed precision takes float32 fields")
        return MIXED[precision]
    if t.dtype == torch.float64:
        return SEM_F64
    if t.dtype == torch.float32:
        return SEM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _field_check(ref, *ts):
    """All tensors on ref's device, same dtype and shape, contiguous."""
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda or t.device != ref.device:
            raise ValueError("all fields must be on the same GPU device")
        if t.dtype != ref.dtype or t.shape != ref.shape:
            raise ValueError("fields must share dtype and shape")
        if not t.is_contiguous():
            raise ValueError("fields must be contiguous")


def _order_of(t):
    if t.dim() != 4 or not (t.shape[1] == t.shape[2] == t.shape[3]):
        raise ValueError("fields must have shape (E, N+1, N+1, N+1)")
    return t.shape[1] - 1


def _ptr(t):
    return None if t is None else t.data_ptr()


def _status_check(status, ref):
    torch = _torch()
    if status is not None and (status.dtype != torch.int32 or status.numel() < 1
                               or status.device != ref.device):
        raise ValueError("status must be an int32 tensor on the fields' device")


def _stream(t):
    torch = _torch()
    return torch.cuda.current_stream(t.device).cuda_stream


def derivs(x, y, z, f, status=None, precision=None):
    """Physical gradient (df/dx, df/dy, df/dz) of one field.  `precision`
    names a mixed mode ("bf16", "fp16", "bf16x3", "fp16x3") for float32
    fields; None computes in the fields' own dtype."""
    torch = _torch()
    _field_check(x, y, z, f)
    _status_check(status, x)
    init(x.device.index)
    _order_of(x)
    out = [torch.empty_like(f) for _ in range(3)]
    with torch.cuda.device(x.device):
        _check(lib().sem_derivs(x.shape[0], _order_of(x), _dtype_code(x, precision), _ptr(x),
                                _ptr(y),
                                _ptr(z), _ptr(f), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                                _ptr(status), _stream(x)), "sem_derivs")
    return tuple(out)


def qcrit(x, y, z, u, v, w, status=None, q=None, omega_mag=None, minmax=None,
          want=("q", "omega", "minmax"), precision=None):
    """Q-criterion, vorticity magnitude and per-element (min, max) of Q
    (`precision` as in derivs)."""
    torch = _torch()
    _field_check(x, y, z, u, v, w)
    _field_check(x, q, omega_mag)
    _status_check(status, x)
    _order_of(x)
    init(x.device.index)
    e = x.shape[0]
    if minmax is not None and (minmax.numel() < 2 * e or minmax.dtype != x.dtype
                               or not minmax.is_contiguous() or minmax.device != x.device):
        raise ValueError("minmax must be a contiguous (E, 2) tensor of the field dtype")
    if q is None and "q" in want:
        q = torch.empty_like(u)
    if omega_mag is None and "omega" in want:
        omega_mag = torch.empty_like(u)
    if minmax is None and "minmax" in want:
        minmax = torch.empty((e, 2), dtype=u.dtype, device=u.device)
    with torch.cuda.device(x.device):
        _check(lib().sem_qcrit(e, _order_of(x), _dtype_code(x, precision), _ptr(x), _ptr(y),
                               _ptr(z),
                               _ptr(u), _ptr(v), _ptr(w), _ptr(q), _ptr(omega_mag),
                               _ptr(minmax), _ptr(status), _stream(x)), "sem_qcrit")
    return q, omega_mag, minmax


def workspace_bytes(n_elem, order, n_iso):
    return int(lib().sem_isosurface_workspace_bytes(n_elem, order, n_iso))


def isosurface_into(x, y, z, field, isovalues, tri_xyz, tri_count, workspace,
                    minmax=None, edge_keys=None, active=None, case_idx=None, status=None):
    """Raw call: write into caller-provided buffers (no allocation, no sync)."""
    torch = _torch()
    _field_check(x, y, z, field)
    _status_check(status, x)
    _order_of(x)
    init(x.device.index)
    iso = np.ascontiguousarray(np.asarray(isovalues, dtype=np.float64))
    cap = 0 if tri_xyz is None else tri_xyz.shape[0]
    e, n, k = x.shape[0], _order_of(x), len(iso)

    def need(t, numel, dtypes, what):
        if t is None:
            return
        if not t.is_cuda or t.device != x.device or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous tensor on {x.device}")
        if t.dtype not in dtypes:
            raise ValueError(f"{what} has dtype {t.dtype}")
        if t.numel() < numel:
            raise ValueError(f"{what} holds {t.numel()} values, needs {numel}")

    if tri_count is None:
        raise ValueError("tri_count is required")
    need(tri_count, k, (torch.int64,), "tri_count")
    need(active, k, (torch.int64,), "active")
    need(tri_xyz, cap * 9, (x.dtype,), "tri_xyz")
    need(edge_keys, cap * 3, (torch.int64,), "edge_keys")
    need(case_idx, k * e * n ** 3, (torch.uint8,), "case_idx")
    need(minmax, 2 * e, (x.dtype,), "minmax")
    if e > 0:
        need(workspace, workspace_bytes(e, n, k), (torch.uint8,), "workspace")
    with torch.cuda.device(x.device):
        _check(lib().sem_isosurface(
            x.shape[0], _order_of(x), _dtype_code(x), _ptr(x), _ptr(y), _ptr(z),
            _ptr(field), _ptr(minmax), len(iso), iso.ctypes.data, _ptr(tri_xyz), cap,
            _ptr(edge_keys), _ptr(tri_count), _ptr(active), _ptr(case_idx),
            _ptr(workspace), 0 if workspace is None else workspace.numel(),
            _ptr(status), _stream(x)), "sem_isosurface")


def isosurface(x, y, z, field, isovalues, minmax=None, edge_keys=False, cases=False,
               status=None):
    """Two-phase extraction: count, synchronise, allocate exactly, emit.

    Returns a dict with tri_xyz (T, 3, 3), tri_count (n_iso,), active
    (n_iso,), and optionally edge_key (T, 3) and cases (n_iso, E, N^3).
    """
    torch = _torch()
    dev = x.device
    n_iso = len(isovalues)
    e = x.shape[0]
    n = _order_of(x)
    ws = torch.empty(max(workspace_bytes(e, n, n_iso), 1), dtype=torch.uint8, device=dev)
    tri_count = torch.zeros(n_iso, dtype=torch.int64, device=dev)
    active = torch.zeros(n_iso, dtype=torch.int64, device=dev)
    # count-only phase: its capacity is 0, so it must not touch the caller's
    # status word (the overflow flag would be set by design)
    isosurface_into(x, y, z, field, isovalues, None, tri_count, ws, minmax=minmax,
                    active=active, status=None)
    total = int(tri_count.sum().item())
    tri = torch.empty((total, 3, 3), dtype=x.dtype, device=dev)
    keys = torch.empty((total, 3), dtype=torch.int64, device=dev) if edge_keys else None
    cidx = (torch.empty((n_iso, e, n ** 3), dtype=torch.uint8, device=dev)
            if cases else None)
    isosurface_into(x, y, z, field, isovalues, tri if total else None, tri_count, ws,
                    minmax=minmax, edge_keys=keys, active=active, case_idx=cidx,
                    status=status)
    out = {"tri_xyz": tri, "tri_count": tri_count, "active": active}
    if edge_keys:
        out["edge_key"] = keys
    if cases:
        out["cases"] = cidx
    return out


def extract_workspace_bytes(n_elem, order, n_iso, dtype_code=SEM_F64):
    return int(lib().sem_extract_workspace_bytes(n_elem, order, n_iso, dtype_code))


def extract_into(x, y, z, u, v, w, isovalues, tri_list, tri_count, workspace, q=None,
                 omega_mag=None, minmax=None, active=None, status=None, precision=None):
    """Raw fused call: tri_list[s] is a (cap_s, 3, 3) tensor or None (count
    only); `precision` as in derivs."""
    torch = _torch()
    _field_check(x, y, z, u, v, w)
    _field_check(x, q, omega_mag)
    _status_check(status, x)
    n = _order_of(x)
    init(x.device.index)
    iso = np.ascontiguousarray(np.asarray(isovalues, dtype=np.float64))
    k, e = len(iso), x.shape[0]
    if len(tri_list) != k:
        raise ValueError("one triangle buffer (or None) per isovalue")
    caps = np.zeros(k, dtype=np.int64)
    ptrs = (ctypes.c_void_p * k)()
    for s, t in enumerate(tri_list):
        if t is None:
            continue
        if (not t.is_cuda or t.device != x.device or t.dtype != x.dtype
                or not t.is_contiguous() or t.dim() != 3 or tuple(t.shape[1:]) != (3, 3)):
            raise ValueError("triangle buffers must be contiguous (cap, 3, 3) tensors")
        caps[s] = t.shape[0]
        ptrs[s] = t.data_ptr() if t.shape[0] else None
    for t, numel, what in ((tri_count, k, "tri_count"), (active, k, "active")):
        if t is not None and (t.dtype != torch.int64 or t.numel() < numel
                              or t.device != x.device or not t.is_contiguous()):
            raise ValueError(f"{what} must be an int64 tensor of >= {numel} values")
    if tri_count is None:
        raise ValueError("tri_count is required")
    if minmax is not None and (minmax.numel() < 2 * e or minmax.dtype != x.dtype
                               or not minmax.is_contiguous() or minmax.device != x.device):
        raise ValueError("minmax must be a contiguous (E, 2) tensor of the field dtype")
    code = _dtype_code(x, precision)
    need = extract_workspace_bytes(e, n, k, code)
    if e > 0 and (workspace is None or workspace.dtype != torch.uint8
                  or workspace.numel() < need or workspace.device != x.device):
        raise ValueError(f"workspace must be a uint8 tensor of >= {need} bytes")
    with torch.cuda.device(x.device):
        _check(lib().sem_extract(
            e, n, code, _ptr(x), _ptr(y), _ptr(z), _ptr(u), _ptr(v), _ptr(w),
            _ptr(q), _ptr(omega_mag), _ptr(minmax), k, iso.ctypes.data,
            ctypes.cast(ptrs, ctypes.c_void_p), caps.ctypes.data, _ptr(tri_count),
            _ptr(active), _ptr(workspace), 0 if workspace is None else workspace.numel(),
            _ptr(status), _stream(x)), "sem_extract")


def extract_noalloc_into(x, y, z, u, v, w, isovalues, tri_list, tri_count, q, minmax,
                         omega_mag=None, active=None, status=None, precision=None):
    """sem_extract_noalloc: as extract_into, with the library's fixed device
    scratch in place of a workspace (q and minmax are required outputs;
    n_iso * n_elem <= SEM_NOALLOC_MAX_COUNTS)."""
    torch = _torch()
    _field_check(x, y, z, u, v, w)
    _field_check(x, q, omega_mag)
    _status_check(status, x)
    n = _order_of(x)
    init(x.device.index)
    iso = np.ascontiguousarray(np.asarray(isovalues, dtype=np.float64))
    k, e = len(iso), x.shape[0]
    if len(tri_list) != k:
        raise ValueError("one triangle buffer (or None) per isovalue")
    caps = np.zeros(k, dtype=np.int64)
    ptrs = (ctypes.c_void_p * k)()
    for s, t in enumerate(tri_list):
        if t is None:
            continue
        if (not t.is_cuda or t.device != x.device or t.dtype != x.dtype
                or not t.is_contiguous() or t.dim() != 3 or tuple(t.shape[1:]) != (3, 3)):
            raise ValueError("triangle buffers must be contiguous (cap, 3, 3) tensors")
        caps[s] = t.shape[0]
        ptrs[s] = t.data_ptr() if t.shape[0] else None
    for t, numel, what in ((tri_count, k, "tri_count"), (active, k, "active")):
        if t is not None and (t.dtype != torch.int64 or t.numel() < numel
                              or t.device != x.device or not t.is_contiguous()):
            raise ValueError(f"{what} must be an int64 tensor of >= {numel} values")
    if tri_count is None or q is None or minmax is None:
        raise ValueError("tri_count, q and minmax are required")
    if (minmax.numel() < 2 * e or minmax.dtype != x.dtype or not minmax.is_contiguous()
            or minmax.device != x.device):
        raise ValueError("minmax must be a contiguous (E, 2) tensor of the field dtype")
    code = _dtype_code(x, precision)
    with torch.cuda.device(x.device):
        _check(lib().sem_extract_noalloc(
            e, n, code, _ptr(x), _ptr(y), _ptr(z), _ptr(u), _ptr(v), _ptr(w),
            _ptr(q), _ptr(omega_mag), _ptr(minmax), k, iso.ctypes.data,
            ctypes.cast(ptrs, ctypes.c_void_p), caps.ctypes.data, _ptr(tri_count),
            _ptr(active), _ptr(status), _stream(x)), "sem_extract_noalloc")


def extract(x, y, z, u, v, w, isovalues, status=None, want_fields=True, precision=None):
    """Fused Q / |omega| / isosurfaces with exact allocation (two calls).

    Returns a dict: q, omega_mag, minmax (when want_fields), tri (list of
    (T_s, 3, 3) tensors, one per isovalue), tri_count, active.
    """
    torch = _torch()
    dev = x.device
    k, e, n = len(isovalues), x.shape[0], _order_of(x)
    ws = torch.empty(max(extract_workspace_bytes(e, n, k, _dtype_code(x, precision)), 1),
                     dtype=torch.uint8, device=dev)
    cnt = torch.zeros(k, dtype=torch.int64, device=dev)
    act = torch.zeros(k, dtype=torch.int64, device=dev)
    extract_into(x, y, z, u, v, w, isovalues, [None] * k, cnt, ws, precision=precision)
    counts = cnt.cpu().tolist()
    tris = [torch.empty((c, 3, 3), dtype=x.dtype, device=dev) for c in counts]
    q = torch.empty_like(u) if want_fields else None
    om = torch.empty_like(u) if want_fields else None
    mm = torch.empty((e, 2), dtype=u.dtype, device=dev) if want_fields else None
    extract_into(x, y, z, u, v, w, isovalues, tris, cnt, ws, q=q, omega_mag=om, minmax=mm,
                 active=act, status=status, precision=precision)
    return {"q": q, "omega_mag": om, "minmax": mm, "tri": tris, "tri_count": cnt,
            "active": act}


# ---------------------------------------------------------------------------
# kernel-phase timing
# ---------------------------------------------------------------------------

def phase_name(phase):
    return lib().sem_phase_name(int(phase)).decode()


def timing_begin(max_spans=4096):
    """Start recording HIP events around every kernel phase of later calls on
    the current device (sem_timing_begin)."""
    init()
    _check(lib().sem_timing_begin(int(max_spans)), "sem_timing_begin")


def timing_end():
    """Stop timing; returns ({phase name: (total ms, spans)}, dropped spans)."""
    tot = np.zeros(SEM_NUM_PHASES)
    cnt = np.zeros(SEM_NUM_PHASES, dtype=np.int64)
    rc = lib().sem_timing_end(tot.ctypes.data, cnt.ctypes.data, SEM_NUM_PHASES)
    if rc < 0:
        raise SemError(int(rc), "sem_timing_end")
    return ({phase_name(k): (float(tot[k]), int(cnt[k])) for k in range(SEM_NUM_PHASES)},
            int(rc))


def stream_copy(src, dst):
    """Plain device copy of src into dst (sem_stream_copy): the bandwidth
    reference kernel.  Both contiguous tensors on one device, same number of
    bytes (a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if (not src.is_cuda or src.device != dst.device or not src.is_contiguous()
            or not dst.is_contiguous() or dst.numel() * dst.element_size() != nbytes):
        raise ValueError("src and dst must be contiguous tensors of equal size on one device")
    with _torch().cuda.device(src.device):
        _check(lib().sem_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(src)),
               "sem_stream_copy")


# ---------------------------------------------------------------------------
# C0 averaging and welded output
# ---------------------------------------------------------------------------

class GatherScatter:
    """Device gather-scatter structure of a global node numbering
    (sem_gs_setup); keeps the buffer it was built in."""

    def __init__(self, gid, n_global=None, status=None):
        torch = _torch()
        if gid.dtype != torch.int64 or not gid.is_cuda or not gid.is_contiguous():
            raise ValueError("gid must be a contiguous int64 tensor on a GPU")
        self.order = _order_of(gid)
        self.n_elem = gid.shape[0]
        self.device = gid.device
        if n_global is None:
            n_global = int(gid.max().item()) + 1 if gid.numel() else 0
        self.n_global = int(n_global)
        init(gid.device.index)
        nb = int(lib().sem_gs_workspace_bytes(self.n_elem, self.order, self.n_global))
        if nb == 0 and self.n_elem > 0:
            raise SemError(SEM_ERR_ARG, "sem_gs_workspace_bytes")
        self.buf = torch.empty(max(nb, 1), dtype=torch.uint8, device=gid.device)
        _status_check(status, gid)
        with torch.cuda.device(gid.device):
            _check(lib().sem_gs_setup(self.n_elem, self.order, _ptr(gid), self.n_global,
                                      _ptr(self.buf), self.buf.numel(), _ptr(status),
                                      _stream(gid)), "sem_gs_setup")


def dsavg(field, gs, out=None):
    """Direct-stiffness average of a field over the gather-scatter's nodes."""
    torch = _torch()
    _field_check(field, out)
    if tuple(field.shape) != (gs.n_elem,) + (gs.order + 1,) * 3 or field.device != gs.device:
        raise ValueError("field does not match the gather-scatter's mesh")
    if out is None:
        out = torch.empty_like(field)
    with torch.cuda.device(field.device):
        _check(lib().sem_dsavg(gs.n_elem, gs.order, _dtype_code(field), _ptr(gs.buf),
                               gs.n_global, _ptr(field), _ptr(out), _stream(field)),
               "sem_dsavg")
    return out


def global_edge_keys(local_keys, gid, status=None):
    """Global keys (uint64 stored as int64) of element-local edge keys."""
    torch = _torch()
    order = _order_of(gid)
    out = torch.empty_like(local_keys)
    with torch.cuda.device(gid.device):
        _check(lib().sem_global_edge_keys(local_keys.numel(), order, gid.shape[0],
                                          _ptr(local_keys), _ptr(gid), _ptr(out),
                                          _ptr(status), _stream(gid)),
               "sem_global_edge_keys")
    return out


def weld(tri_xyz, keys, status=None):
    """(vertices (V, 3), indices (T, 3) int64) of a soup with global keys."""
    torch = _torch()
    n_ref = keys.numel()
    if tri_xyz.numel() != 3 * n_ref:
        raise ValueError("tri_xyz must hold 3 coordinates per key")
    dev = keys.device
    init(dev.index)
    ws = torch.empty(max(int(lib().sem_weld_workspace_bytes(n_ref)), 1), dtype=torch.uint8,
                     device=dev)
    idx = torch.empty((n_ref // 3, 3), dtype=torch.int64, device=dev)
    verts = torch.empty((max(n_ref, 1), 3), dtype=tri_xyz.dtype, device=dev)
    n_vert = torch.zeros(1, dtype=torch.int64, device=dev)
    code = SEM_F64 if tri_xyz.dtype == torch.float64 else SEM_F32
    with torch.cuda.device(dev):
        _check(lib().sem_weld(n_ref, code, _ptr(tri_xyz), _ptr(keys), _ptr(idx), _ptr(verts),
                              n_ref, _ptr(n_vert), _ptr(ws), ws.numel(), _ptr(status),
                              _stream(keys)), "sem_weld")
    return verts[:int(n_vert.item())], idx


# ---------------------------------------------------------------------------
# batched snapshots
# ---------------------------------------------------------------------------

class BatchPlan:
    """Device plan of several snapshots (sem_batch_plan).  Each snapshot is a
    dict with x, y, z, u, v, w and the outputs q, omega_mag, minmax (any may
    be None but not all); all tensors share one precision and device.  The
    plan keeps references to the tensors it points at."""

    def __init__(self, snapshots):
        torch = _torch()
        if not snapshots:
            raise ValueError("no snapshots")
        ref = snapshots[0]["x"]
        self.dtype_code = _dtype_code(ref)
        self.device = ref.device
        init(ref.device.index)
        arr = (_Snapshot * len(snapshots))()
        self._keep = []
        for i, sn in enumerate(snapshots):
            x = sn["x"]
            _field_check(x, sn["y"], sn["z"], sn["u"], sn["v"], sn["w"])
            _field_check(x, sn.get("q"), sn.get("omega_mag"))
            if x.dtype != ref.dtype or x.device != ref.device:
                raise ValueError("all snapshots share one dtype and device")
            mm = sn.get("minmax")
            if mm is not None and (mm.numel() < 2 * x.shape[0] or mm.dtype != x.dtype):
                raise ValueError("minmax must hold (E, 2) values of the field dtype")
            arr[i].n_elem = x.shape[0]
            arr[i].order = _order_of(x)
            for k in ("x", "y", "z", "u", "v", "w"):
                setattr(arr[i], k, _ptr(sn[k]))
            arr[i].q = _ptr(sn.get("q"))
            arr[i].omega_mag = _ptr(sn.get("omega_mag"))
            arr[i].q_minmax = _ptr(mm)
            self._keep.append(sn)
        nb = int(lib().sem_batch_plan_bytes(len(snapshots)))
        if nb == 0:
            raise SemError(SEM_ERR_ARG, "sem_batch_plan_bytes")
        self.buf = torch.empty(nb, dtype=torch.uint8, device=ref.device)
        code = ctypes.c_uint(0)
        with torch.cuda.device(ref.device):
            torch.cuda.current_stream(ref.device).synchronize()
            _check(lib().sem_batch_plan(len(snapshots), ctypes.addressof(arr), self.dtype_code,
                                        _ptr(self.buf), nb, ctypes.addressof(code)),
                   "sem_batch_plan")
        self.launch_code = code.value


def qcrit_batch(plan, status=None):
    """One persistent launch per order over every snapshot of the plan
    (capturable)."""
    torch = _torch()
    with torch.cuda.device(plan.device):
        _check(lib().sem_qcrit_batch(_ptr(plan.buf), plan.launch_code, plan.dtype_code,
                                     _ptr(status),
                                     torch.cuda.current_stream(plan.device).cuda_stream),
               "sem_qcrit_batch")


def autotune(order, dtype_code=SEM_F64, device=None):
    """Measure the batched kernel's variants for (order, dtype); returns
    (chosen variant, [ms of variants 0..5], -1 where not applicable).
    Variants 0, 1, 2: LDS-tile form with 1, 2, 4 elements per work item;
    3: register-pencil form (several elements per item at low orders);
    4: direct-to-LDS form (N = 7, FP64);
    5: one thread per node."""
    init(device)
    var = ctypes.c_int(0)
    ms = (ctypes.c_float * BATCH_VARIANTS)()
    _check(lib().sem_autotune(int(order), int(dtype_code), ctypes.addressof(var),
                              ctypes.addressof(ms)), "sem_autotune")
    return var.value, [float(v) for v in ms]


def batch_variant(order, dtype_code=SEM_F64):
    rc = lib().sem_batch_variant(int(order), int(dtype_code))
    if rc < 0:
        raise SemError(rc, "sem_batch_variant")
    return rc


def batch_set_variant(order, dtype_code, variant, device=None):
    init(device)
    _check(lib().sem_batch_set_variant(int(order), int(dtype_code), int(variant)),
           "sem_batch_set_variant")


def _snapshot_array(snapshots):
    arr = (_Snapshot * len(snapshots))()
    for i, sn in enumerate(snapshots):
        x = sn["x"]
        arr[i].n_elem = x.shape[0]
        arr[i].order = _order_of(x)
        for k in ("x", "y", "z", "u", "v", "w"):
            setattr(arr[i], k, _ptr(sn.get(k)))
        arr[i].q = _ptr(sn.get("q"))
        arr[i].omega_mag = _ptr(sn.get("omega_mag"))
        arr[i].q_minmax = _ptr(sn.get("minmax"))
    return arr


class IsoBatchPlan:
    """Device plan of batched isosurfaces (sem_iso_batch_plan).  `snapshots`
    are dicts as for BatchPlan (x, y, z and the fields the jobs use: q,
    omega_mag, minmax); each job is a dict with "snap" (index), "field"
    ("q", "omega_mag" or a scalar tensor of the snapshot's shape) and
    "isovalues" (1 to 4 floats).  Holds references to every tensor it points
    at."""

    def __init__(self, snapshots, jobs):
        torch = _torch()
        if not snapshots or not jobs:
            raise ValueError("no snapshots or no jobs")
        ref = snapshots[0]["x"]
        self.dtype_code = _dtype_code(ref)
        self.device = ref.device
        init(ref.device.index)
        for sn in snapshots:
            x = sn["x"]
            _field_check(x, sn["y"], sn["z"], sn.get("q"), sn.get("omega_mag"))
            if x.dtype != ref.dtype or x.device != ref.device:
                raise ValueError("all snapshots share one dtype and device")
            mm = sn.get("minmax")
            if mm is not None and (mm.numel() < 2 * x.shape[0] or mm.dtype != x.dtype):
                raise ValueError("minmax must hold (E, 2) values of the field dtype")
        arr = _snapshot_array(snapshots)
        jarr = (_IsoJob * len(jobs))()
        self._keep = [snapshots]
        for k, jb in enumerate(jobs):
            f = jb["field"]
            jarr[k].snap = int(jb["snap"])       # range checked by the library
            if isinstance(f, str):
                jarr[k].field = {"q": SEM_JOB_Q, "omega_mag": SEM_JOB_OMEGA}[f]
                jarr[k].scalar = None
            else:
                if 0 <= jb["snap"] < len(snapshots):
                    _field_check(snapshots[jb["snap"]]["x"], f)
                jarr[k].field = SEM_JOB_SCALAR
                jarr[k].scalar = _ptr(f)
                self._keep.append(f)
            iv = [float(c) for c in jb["isovalues"]]
            jarr[k].n_iso = len(iv)              # 1..4, checked by the library
            for q, c in enumerate(iv[:4]):
                jarr[k].iso[q] = c
        nb = int(lib().sem_iso_batch_plan_bytes(len(jobs)))
        if nb == 0:
            raise SemError(SEM_ERR_ARG, "sem_iso_batch_plan_bytes")
        self.buf = torch.empty(nb, dtype=torch.uint8, device=ref.device)
        self.info = _IsoBatchInfo()
        with torch.cuda.device(ref.device):
            torch.cuda.current_stream(ref.device).synchronize()
            _check(lib().sem_iso_batch_plan(len(snapshots), ctypes.addressof(arr), len(jobs),
                                            ctypes.addressof(jarr), self.dtype_code,
                                            _ptr(self.buf), nb, ctypes.addressof(self.info)),
                   "sem_iso_batch_plan")
        self.n_job = len(jobs)
        self.workspace = torch.empty(max(int(self.info.workspace_bytes), 1), dtype=torch.uint8,
                                     device=ref.device)
        self.dtype = ref.dtype


def isosurface_batch_into(plan, tri_xyz, tri_count, tri_offset=None, active=None, status=None):
    """Isosurfaces of every job of the plan into tri_xyz ((cap, 3, 3), the
    plan's dtype): tri_count and tri_offset ((4 * n_job,) int64) receive the
    count and first triangle of (job j, isovalue s) at 4j + s.  Asynchronous
    and capturable; the counts are exact when the soup overflows."""
    torch = _torch()
    cap = 0 if tri_xyz is None else tri_xyz.shape[0]
    for t in (tri_count, tri_offset, active):
        if t is not None and (t.dtype != torch.int64 or t.numel() < 4 * plan.n_job):
            raise ValueError("per-(job, isovalue) arrays hold 4 * n_job int64")
    if tri_xyz is not None and tri_xyz.dtype != plan.dtype:
        raise ValueError("tri_xyz must have the plan's dtype")
    with torch.cuda.device(plan.device):
        _check(lib().sem_isosurface_batch(
            _ptr(plan.buf), ctypes.addressof(plan.info), plan.dtype_code,
            _ptr(tri_xyz) if cap else None, cap, _ptr(tri_offset), _ptr(tri_count),
            _ptr(active), _ptr(plan.workspace), plan.workspace.numel(), _ptr(status),
            torch.cuda.current_stream(plan.device).cuda_stream), "sem_isosurface_batch")


def isosurface_batch(plan, status=None, active=False):
    """Counts, then a soup of exactly that size: returns a dict with tri_xyz
    (T, 3, 3), tri_count and tri_offset ((n_job, 4) int64) and, if asked,
    active ((n_job, 4))."""
    torch = _torch()
    dev = plan.device
    cnt = torch.zeros(4 * plan.n_job, dtype=torch.int64, device=dev)
    off = torch.zeros(4 * plan.n_job, dtype=torch.int64, device=dev)
    act = torch.zeros(4 * plan.n_job, dtype=torch.int64, device=dev) if active else None
    # count-only call: with no capacity the overflow flag is set by design,
    # so it does not touch the caller's status word
    isosurface_batch_into(plan, None, cnt, off, act, None)
    total = int(cnt.sum().item())
    tri = torch.empty((max(total, 1), 3, 3), dtype=plan.dtype, device=dev)
    isosurface_batch_into(plan, tri, cnt, off, act, status)
    out = {"tri_xyz": tri[:total], "tri_count": cnt.view(plan.n_job, 4).cpu(),
           "tri_offset": off.view(plan.n_job, 4).cpu()}
    if active:
        out["active"] = act.view(plan.n_job, 4).cpu()
    return out


# ---------------------------------------------------------------------------
# learned in-transit compression (order 7, FP32 u, v, w, theta)
# ---------------------------------------------------------------------------

def _ae_fields(fields):
    torch = _torch()
    if len(fields) != 4:
        raise ValueError("four fields (u, v, w, theta)")
    ref = fields[0]
    if ref.dtype != torch.float32 or _order_of(ref) != 7:
        raise TypeError("compression takes float32 order-7 fields")
    _field_check(ref, *fields)
    init(ref.device.index)
    return ref


def _ws(nbytes, ref):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=ref.device)


def ae_param_count():
    return int(lib().sem_ae_param_count())


def ae_blocks(fields):
    """(blocks [E, 512, 4] Morton order, scale [E, 4]) of (u, v, w, theta)."""
    torch = _torch()
    ref = _ae_fields(fields)
    e = ref.shape[0]
    blocks = torch.empty((e, 512, 4), dtype=torch.float32, device=ref.device)
    scale = torch.empty((e, 4), dtype=torch.float32, device=ref.device)
    _check(lib().sem_ae_blocks(e, *(f.data_ptr() for f in fields), blocks.data_ptr(),
                               scale.data_ptr(), _stream(ref)), "sem_ae_blocks")
    return blocks, scale


def ae_forward(blocks, params, tanh_mask=0):
    """(reconstruction [n, 512, 4], binary16 latent [n, 32]) of n blocks."""
    torch = _torch()
    n = blocks.shape[0]
    recon = torch.empty_like(blocks)
    latent = torch.empty((n, SEM_AE_LATENT), dtype=torch.float16, device=blocks.device)
    ws = _ws(lib().sem_ae_workspace_bytes(n), blocks)
    _check(lib().sem_ae_forward(n, blocks.data_ptr(), params.data_ptr(), int(tanh_mask),
                                recon.data_ptr(), latent.data_ptr(), ws.data_ptr(), ws.numel(),
                                _stream(blocks)), "sem_ae_forward")
    return recon, latent


def ae_grad(pool, params, idx=None, n=None, tanh_mask=0, grad=None, workspace=None,
            status=None, loss_kind=SEM_AE_LOSS_MSE):
    """(loss [1] float32, grad) of the batch pool[idx] (or the first n);
    loss_kind SEM_AE_LOSS_MSE or SEM_AE_LOSS_MAX."""
    torch = _torch()
    if idx is not None:
        if idx.dtype != torch.int64 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 tensor")
        n = idx.numel()
    elif n is None:
        n = pool.shape[0]
    if grad is None:
        grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=pool.device)
    if workspace is None:
        workspace = _ws(lib().sem_ae_workspace_bytes(n), pool)
    _check(lib().sem_ae_grad(n, pool.data_ptr(), pool.shape[0], _ptr(idx), params.data_ptr(),
                             int(tanh_mask), int(loss_kind), grad.data_ptr(), loss.data_ptr(),
                             workspace.data_ptr(), workspace.numel(), _ptr(status),
                             _stream(pool)), "sem_ae_grad")
    return loss, grad


def ae_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().sem_ae_adam(params.numel(), params.data_ptr(), grad.data_ptr(), m.data_ptr(),
                             v.data_ptr(), int(step), float(lr), float(beta1), float(beta2),
                             float(eps), _stream(params)), "sem_ae_adam")


def sym_eig(a, r):
    """(r leading eigenvalues, eigenvectors [n, r] float32, sweeps) of the
    symmetric float64 matrix a [n, n] (n even, <= 512)."""
    torch = _torch()
    n = a.shape[0]
    init(a.device.index)
    lam = torch.empty(r, dtype=torch.float64, device=a.device)
    vec = torch.empty((n, r), dtype=torch.float32, device=a.device)
    sweeps = torch.zeros(1, dtype=torch.int32, device=a.device)
    ws = _ws(lib().sem_eig_workspace_bytes(n), a)
    _check(lib().sem_sym_eig(n, a.contiguous().data_ptr(), int(r), lam.data_ptr(),
                             vec.data_ptr(), ws.data_ptr(), ws.numel(), sweeps.data_ptr(),
                             _stream(a)), "sem_sym_eig")
    return lam, vec, sweeps


def ae_pca_init(pool):
    """(params, eigenvalues [96]) from layer-wise principal components of the
    blocks pool [n, 512, 4]."""
    torch = _torch()
    init(pool.device.index)
    params = torch.empty(ae_param_count(), dtype=torch.float32, device=pool.device)
    lam = torch.empty(96, dtype=torch.float64, device=pool.device)
    ws = _ws(lib().sem_ae_pca_workspace_bytes(pool.shape[0]), pool)
    _check(lib().sem_ae_pca_init(pool.shape[0], pool.data_ptr(), params.data_ptr(),
                                 lam.data_ptr(), ws.data_ptr(), ws.numel(), _stream(pool)),
           "sem_ae_pca_init")
    return params, lam


def ae_train(pool, params, steps, batch=2048, lr=1e-4, seed=0, tanh_mask=0, m=None, v=None,
             step0=0, loss_every=0, loss_kind=SEM_AE_LOSS_MSE, warmup=0, cosine=False):
    """Adam on the loss of random batches of the pool (indices drawn on the
    device from a seeded generator), the library's gradient and Adam
    kernels; learning rate lr, optionally ramped up linearly over `warmup`
    steps and decayed along a half cosine to 0 at `steps`; returns (m, v,
    losses)."""
    torch = _torch()
    if m is None:
        m = torch.zeros_like(params)
    if v is None:
        v = torch.zeros_like(params)
    gen = torch.Generator(device=pool.device).manual_seed(seed)
    ws = _ws(lib().sem_ae_workspace_bytes(batch), pool)
    grad = torch.empty_like(params)
    losses = []
    for t in range(1, steps + 1):
        idx = torch.randint(0, pool.shape[0], (batch,), device=pool.device, generator=gen)
        loss, _ = ae_grad(pool, params, idx=idx, tanh_mask=tanh_mask, grad=grad, workspace=ws,
                          loss_kind=loss_kind)
        rate = lr * (min(1.0, t / warmup) if warmup else 1.0)
        if cosine:
            rate *= 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps))
        ae_adam(params, grad, m, v, step0 + t, rate)
        if loss_every and (t % loss_every == 0 or t == steps):
            losses.append((t, float(loss.item())))
    return m, v, losses


def ae_compress(fields, params, tanh_mask=0, raw_cap=None, status=None):
    """Compressed snapshot: dict(latent [E, 32] float16, scale [E, 4],
    flags [E] uint8, raw [n_raw, 4, 512], n_raw)."""
    torch = _torch()
    ref = _ae_fields(fields)
    e = ref.shape[0]
    dev = ref.device
    latent = torch.empty((e, SEM_AE_LATENT), dtype=torch.float16, device=dev)
    scale = torch.empty((e, 4), dtype=torch.float32, device=dev)
    flags = torch.empty(e, dtype=torch.uint8, device=dev)
    n_raw = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _ws(lib().sem_ae_compress_workspace_bytes(e), ref)
    cap = e if raw_cap is None else int(raw_cap)
    raw = torch.empty((max(cap, 1), 4, 512), dtype=torch.float32, device=dev)
    _check(lib().sem_ae_compress(e, *(f.data_ptr() for f in fields), params.data_ptr(),
                                 int(tanh_mask), latent.data_ptr(), scale.data_ptr(),
                                 flags.data_ptr(), raw.data_ptr(), cap, n_raw.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _ptr(status), _stream(ref)),
           "sem_ae_compress")
    k = int(n_raw.item())
    return {"latent": latent, "scale": scale, "flags": flags, "raw": raw[:min(k, cap)],
            "n_raw": k}


def ae_decompress(packet, params, tanh_mask=0, status=None):
    """(u, v, w, theta) [E, 8, 8, 8] from a compressed snapshot."""
    torch = _torch()
    latent = packet["latent"]
    e = latent.shape[0]
    dev = latent.device
    init(dev.index)
    out = [torch.empty((e, 8, 8, 8), dtype=torch.float32, device=dev) for _ in range(4)]
    ws = _ws(lib().sem_ae_compress_workspace_bytes(e), latent)
    raw = packet["raw"]
    _check(lib().sem_ae_decompress(e, latent.data_ptr(), packet["scale"].data_ptr(),
                                   packet["flags"].data_ptr(),
                                   raw.data_ptr() if raw.numel() else None, raw.shape[0],
                                   params.data_ptr(), int(tanh_mask),
                                   *(t.data_ptr() for t in out), ws.data_ptr(), ws.numel(),
                                   _ptr(status), _stream(latent)), "sem_ae_decompress")
    return tuple(out)


def modal_compress(fields, recon=True):
    """Legendre modal truncation baseline: dict(coef [E, 4, 8] float16,
    scale, flags, recon (u, v, w, theta) or None)."""
    torch = _torch()
    ref = _ae_fields(fields)
    e = ref.shape[0]
    dev = ref.device
    coef = torch.empty((e, 4, 8), dtype=torch.float16, device=dev)
    scale = torch.empty((e, 4), dtype=torch.float32, device=dev)
    flags = torch.empty(e, dtype=torch.uint8, device=dev)
    r = [torch.empty_like(ref) for _ in range(4)] if recon else [None] * 4
    ws = _ws(lib().sem_ae_compress_workspace_bytes(e), ref)
    _check(lib().sem_modal_compress(e, *(f.data_ptr() for f in fields), coef.data_ptr(),
                                    scale.data_ptr(), flags.data_ptr(), *(_ptr(t) for t in r),
                                    ws.data_ptr(), ws.numel(), _stream(ref)),
           "sem_modal_compress")
    return {"coef": coef, "scale": scale, "flags": flags, "recon": tuple(r) if recon else None}


def compressed_bytes(n_elem, n_raw):
    """Bytes shipped for a compressed snapshot: binary16 latent, FP32 scales
    and a flag byte per element, and the raw elements' 4 x 512 FP32 values."""
    return n_elem * (SEM_AE_LATENT * 2 + 4 * 4 + 1) + n_raw * 4 * 512 * 4
