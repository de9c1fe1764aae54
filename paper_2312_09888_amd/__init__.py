"""MI355X-native in situ extraction for spectral-element snapshots.

Q-criterion / vorticity magnitude and marching-cubes isosurfaces of fields
stored at the GLL nodes of order-N hexahedral elements, computed by
hand-written HIP kernels (gfx950) behind the C ABI of ``include/sem.h``.
This package is the thin ctypes binding (``_lib``) and the build script
(``build``); it has no CPU fallback.
"""

from ._lib import (  # noqa: F401
    MIXED, SEM_F32, SEM_F64, SEM_FLAG_BAD_JACOBIAN, SEM_FLAG_TRI_OVERFLOW, SEM_MAX_ORDER,
    SEM_MIN_ORDER, SemError, derivs, extract, extract_into, extract_workspace_bytes, gll,
    init, isosurface, isosurface_into, lib, mc_table, phase_name, qcrit, status_str,
    timing_begin, timing_end, workspace_bytes, GatherScatter, dsavg, global_edge_keys, weld,
    SEM_FLAG_BAD_ID, SEM_FLAG_VERT_OVERFLOW, BatchPlan, qcrit_batch, autotune, batch_variant,
    batch_set_variant, BATCH_VARIANTS, SEM_FLAG_RAW_OVERFLOW, SEM_AE_LATENT, SEM_AE_TANH_HIDDEN, SEM_AE_LOSS_MSE, SEM_AE_LOSS_MAX,
    ae_param_count, ae_blocks, ae_forward, ae_grad, ae_adam, sym_eig, ae_pca_init, ae_train,
    ae_compress, ae_decompress, modal_compress, compressed_bytes, stream_copy,
    extract_noalloc_into, SEM_NOALLOC_MAX_COUNTS, IsoBatchPlan, isosurface_batch,
    isosurface_batch_into, SEM_JOB_Q, SEM_JOB_OMEGA, SEM_JOB_SCALAR, build_info,
)
