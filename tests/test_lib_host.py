"""CPU tests of libsem: it loads, exports every declared symbol, its host-side
basis and case table agree with the oracle's independent computations, and
host-detectable argument errors are returned before any device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2312_09888_amd as sem
from paper_2312_09888_amd import _lib
from oracle import gll, mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 9
    lib = sem.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    for name, val in (("SEM_MAX_ORDER", _lib.SEM_MAX_ORDER), ("SEM_MAX_ISO", _lib.SEM_MAX_ISO),
                      ("SEM_MC_MAX_TRI", _lib.SEM_MC_MAX_TRI),
                      ("SEM_MIN_ORDER", _lib.SEM_MIN_ORDER)):
        assert re.search(rf"#define {name} {val}\b", text), name


@pytest.mark.parametrize("n", range(1, 16))
def test_library_basis_matches_oracle(n):
    xi, w, d = sem.gll(n)
    np.testing.assert_allclose(xi, gll.gll_nodes(n), rtol=0, atol=2.3e-16)
    np.testing.assert_allclose(w, gll.gll_weights(n), rtol=0, atol=4e-16)
    np.testing.assert_allclose(d, gll.diff_matrix(n), rtol=0, atol=1e-14 * n * n)


def test_library_case_table_equals_oracle_entry_by_entry():
    ntri, tri = sem.mc_table()
    o_ntri, o_tri = mc.case_table()
    assert o_tri.shape == tri.shape
    np.testing.assert_array_equal(ntri, o_ntri)
    np.testing.assert_array_equal(tri, o_tri)


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert sem.status_str(code)
    assert sem.status_str(123) == "unknown status"


def test_build_record_matches_the_sources():
    from paper_2312_09888_amd import build as B
    rec = sem.build_info()
    assert rec["arch"] == "gfx950" and rec["hip"]
    # the library in the tree was built from the sources in the tree
    assert rec["sources_sha256"] == B.source_sha256()


def test_gll_rejects_bad_order():
    L = sem.lib()
    assert L.sem_gll(0, None, None, None) == _lib.SEM_ERR_ORDER
    assert L.sem_gll(16, None, None, None) == _lib.SEM_ERR_ORDER


# Fake, never-dereferenced addresses: every call below must fail validation.
FAKE = ctypes.c_void_p(0x1000)


def _qcrit(**kw):
    a = dict(n=4, order=7, dt=0, x=FAKE, y=FAKE, z=FAKE, u=FAKE, v=FAKE, w=FAKE,
             q=FAKE, om=FAKE, mm=None)
    a.update(kw)
    return sem.lib().sem_qcrit(a["n"], a["order"], a["dt"], a["x"], a["y"], a["z"], a["u"],
                               a["v"], a["w"], a["q"], a["om"], a["mm"], None, None)


def test_qcrit_argument_errors():
    assert _qcrit(order=0) == _lib.SEM_ERR_ORDER
    assert _qcrit(order=10) == _lib.SEM_ERR_ORDER
    assert _qcrit(dt=7) == _lib.SEM_ERR_DTYPE
    assert _qcrit(n=-1) == _lib.SEM_ERR_ARG
    assert _qcrit(x=None) == _lib.SEM_ERR_ARG
    assert _qcrit(w=None) == _lib.SEM_ERR_ARG
    assert _qcrit(q=None, om=None, mm=None) == _lib.SEM_ERR_ARG
    assert _qcrit(n=0) == _lib.SEM_OK            # empty call is a no-op


def test_derivs_argument_errors():
    L = sem.lib()
    f = FAKE
    assert L.sem_derivs(4, 0, 0, f, f, f, f, f, f, f, None, None) == _lib.SEM_ERR_ORDER
    assert L.sem_derivs(4, 7, 9, f, f, f, f, f, f, f, None, None) == _lib.SEM_ERR_DTYPE
    assert L.sem_derivs(4, 7, 0, f, f, f, None, f, f, f, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_derivs(4, 7, 0, f, f, f, f, f, f, None, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_derivs(0, 7, 0, f, f, f, f, f, f, f, None, None) == _lib.SEM_OK


def _iso(**kw):
    iso = np.array([0.1, 0.2])
    a = dict(n=4, order=7, dt=0, field=FAKE, n_iso=2, iso=iso.ctypes.data, tri=FAKE, cap=10,
             count=FAKE, ws=FAKE, ws_bytes=1 << 30)
    a.update(kw)
    return sem.lib().sem_isosurface(a["n"], a["order"], a["dt"], FAKE, FAKE, FAKE, a["field"],
                                    None, a["n_iso"], a["iso"], a["tri"], a["cap"], None,
                                    a["count"], None, None, a["ws"], a["ws_bytes"], None, None)


def test_isosurface_argument_errors():
    assert _iso(order=0) == _lib.SEM_ERR_ORDER
    assert _iso(dt=9) == _lib.SEM_ERR_DTYPE
    assert _iso(n_iso=0) == _lib.SEM_ERR_ARG
    assert _iso(n_iso=_lib.SEM_MAX_ISO + 1) == _lib.SEM_ERR_ARG
    assert _iso(iso=None) == _lib.SEM_ERR_ARG
    assert _iso(count=None) == _lib.SEM_ERR_ARG
    assert _iso(field=None) == _lib.SEM_ERR_ARG
    assert _iso(cap=-1) == _lib.SEM_ERR_ARG
    assert _iso(tri=None) == _lib.SEM_ERR_ARG          # capacity > 0 needs a buffer
    assert _iso(ws=None) == _lib.SEM_ERR_WORKSPACE
    need = sem.workspace_bytes(4, 7, 2)
    assert _iso(ws_bytes=need - 1) == _lib.SEM_ERR_WORKSPACE


def test_workspace_size_grows_with_problem():
    a = sem.workspace_bytes(1000, 7, 1)
    b = sem.workspace_bytes(1000, 7, 3)
    c = sem.workspace_bytes(100000, 7, 3)
    assert 0 < a < b < c
    assert c >= 100000 * 3 * (4 + 8)
    assert sem.workspace_bytes(10, 7, 0) == 0


def test_workspace_size_never_shrinks_across_the_scan_tile_change():
    # the scan's tiles grow from 1,024 to 4,096 counts above 2^20 counts, so
    # the tile count drops there; the workspaces reserve tile sums that never
    # shrink, so a workspace sized for a problem also fits every smaller one
    for n_iso in (1, 4):
        lo = (1 << 20) // n_iso - 3
        sizes = [sem.workspace_bytes(e, 7, n_iso) for e in range(lo, lo + 8)]
        assert sizes == sorted(sizes)
        sizes = [sem.extract_workspace_bytes(e, 7, n_iso) for e in range(lo, lo + 8)]
        assert sizes == sorted(sizes)
    big = [sem.workspace_bytes(e, 7, 1) for e in ((1 << 22) - 1, 1 << 22, (1 << 22) + 1)]
    assert big == sorted(big)


def _no_gpu():
    try:
        import torch
        return torch.cuda.device_count() == 0
    except Exception:  # pragma: no cover
        return True


@pytest.mark.skipif(not _no_gpu(), reason="only meaningful where no device exists")
def test_compute_without_device_reports_not_initialised():
    assert _qcrit() == _lib.SEM_ERR_NOT_INIT
    assert sem.lib().sem_init(0) in (_lib.SEM_ERR_HIP, _lib.SEM_ERR_ARG)


def _extract(**kw):
    iso = np.array([0.1, 0.2])
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    caps = np.array([10, 10], dtype=np.int64)
    a = dict(n=4, order=7, dt=0, u=FAKE, n_iso=2, iso=iso.ctypes.data,
             ptrs=ctypes.cast(ptrs, ctypes.c_void_p), caps=caps.ctypes.data, count=FAKE,
             ws=FAKE, ws_bytes=1 << 30)
    a.update(kw)
    return sem.lib().sem_extract(a["n"], a["order"], a["dt"], FAKE, FAKE, FAKE, a["u"], FAKE,
                                 FAKE, None, None, None, a["n_iso"], a["iso"], a["ptrs"],
                                 a["caps"], a["count"], None, a["ws"], a["ws_bytes"], None,
                                 None)


def test_extract_argument_errors():
    assert _extract(order=0) == _lib.SEM_ERR_ORDER
    assert _extract(dt=9) == _lib.SEM_ERR_DTYPE
    assert _extract(n=-3) == _lib.SEM_ERR_ARG
    assert _extract(u=None) == _lib.SEM_ERR_ARG
    assert _extract(n_iso=0) == _lib.SEM_ERR_ARG
    assert _extract(iso=None) == _lib.SEM_ERR_ARG
    assert _extract(ptrs=None) == _lib.SEM_ERR_ARG
    assert _extract(caps=None) == _lib.SEM_ERR_ARG
    assert _extract(count=None) == _lib.SEM_ERR_ARG
    bad_caps = np.array([10, -1], dtype=np.int64)
    assert _extract(caps=bad_caps.ctypes.data) == _lib.SEM_ERR_ARG
    nullp = (ctypes.c_void_p * 2)(0x1000, None)
    assert _extract(ptrs=ctypes.cast(nullp, ctypes.c_void_p)) == _lib.SEM_ERR_ARG
    assert _extract(ws=None) == _lib.SEM_ERR_WORKSPACE
    need = sem.extract_workspace_bytes(4, 7, 2)
    assert _extract(ws_bytes=need - 1) == _lib.SEM_ERR_WORKSPACE


def test_extract_workspace_sizes():
    a = sem.extract_workspace_bytes(1000, 7, 3)
    assert a >= 1000 * 3 * 8
    # higher orders also hold Q and its element ranges
    b = sem.extract_workspace_bytes(1000, 9, 3, _lib.SEM_F64)
    assert b >= 1000 * 1000 * 8
    assert sem.extract_workspace_bytes(1000, 9, 3, _lib.SEM_F32) < b
    assert sem.extract_workspace_bytes(10, 0, 1) == 0


def test_timing_argument_errors_and_phase_names():
    L = sem.lib()
    assert L.sem_timing_begin(0) == _lib.SEM_ERR_ARG
    assert L.sem_timing_begin((1 << 20) + 1) == _lib.SEM_ERR_ARG
    assert [sem.phase_name(k) for k in range(_lib.SEM_NUM_PHASES)] == [
        "qcrit", "count", "scan", "emit"]
    assert sem.phase_name(9) == "unknown"
    text = open(HEADER).read()
    assert re.search(rf"SEM_NUM_PHASES = {_lib.SEM_NUM_PHASES}\b", text)


def test_extract_noalloc_argument_errors():
    L = sem.lib()
    iso = (ctypes.c_double * 2)(0.1, 0.2)
    caps = (ctypes.c_int64 * 2)(0, 0)
    ptrs = (ctypes.c_void_p * 2)(None, None)

    def call(n, n_iso=1, q=FAKE, mm=FAKE, order=7):
        return L.sem_extract_noalloc(n, order, 0, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, q, None,
                                     mm, n_iso, iso, ptrs, caps, FAKE, None, None, None)

    # the scratch holds SEM_NOALLOC_MAX_COUNTS (isovalue, element) counts
    assert call(_lib.SEM_NOALLOC_MAX_COUNTS + 1) == _lib.SEM_ERR_WORKSPACE
    assert call(_lib.SEM_NOALLOC_MAX_COUNTS // 2 + 1, n_iso=2) == _lib.SEM_ERR_WORKSPACE
    # Q and its element ranges are required outputs
    assert call(4, q=None) == _lib.SEM_ERR_ARG
    assert call(4, mm=None) == _lib.SEM_ERR_ARG
    assert call(4, order=0) == _lib.SEM_ERR_ORDER
    assert call(4, n_iso=0) == _lib.SEM_ERR_ARG
    text = open(HEADER).read()
    assert re.search(r"#define SEM_NOALLOC_MAX_COUNTS \(1 << 20\)", text)
    assert _lib.SEM_NOALLOC_MAX_COUNTS == 1 << 20


def test_stream_copy_argument_errors():
    L = sem.lib()
    assert L.sem_stream_copy(None, None, 0, None) == _lib.SEM_OK
    assert L.sem_stream_copy(None, FAKE, 16, None) == _lib.SEM_ERR_ARG
    assert L.sem_stream_copy(FAKE, FAKE, 24, None) == _lib.SEM_ERR_ARG        # not 16 x k
    assert L.sem_stream_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x8000), 16,
                             None) == _lib.SEM_ERR_ARG                       # misaligned
    assert L.sem_stream_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1010), 32,
                             None) == _lib.SEM_ERR_ARG                       # overlapping


@pytest.mark.skipif(not _no_gpu(), reason="only meaningful where no device exists")
def test_timing_end_without_device_or_begin_fails():
    assert sem.lib().sem_timing_end(None, None, 4) < 0


def test_mixed_modes_need_order_7_where_they_differentiate():
    L = sem.lib()
    f = FAKE
    for dt in (_lib.SEM_MIXED_BF16, _lib.SEM_MIXED_FP16, _lib.SEM_MIXED_BF16X3,
               _lib.SEM_MIXED_FP16X3):
        assert _qcrit(order=5, dt=dt) == _lib.SEM_ERR_ORDER
        assert L.sem_derivs(4, 6, dt, f, f, f, f, f, f, f, None, None) == _lib.SEM_ERR_ORDER
        assert _extract(order=8, dt=dt) == _lib.SEM_ERR_ORDER
        assert _qcrit(dt=dt, x=None) == _lib.SEM_ERR_ARG
        # the isosurface takes no derivative: any order, FP32 storage
        assert _iso(order=5, dt=dt, ws=None) == _lib.SEM_ERR_WORKSPACE
        assert (sem.extract_workspace_bytes(1000, 7, 3, dt)
                == sem.extract_workspace_bytes(1000, 7, 3, _lib.SEM_F32))
        assert sem.extract_workspace_bytes(1000, 5, 3, dt) == 0
    assert set(_lib.MIXED.values()) == {2, 3, 4, 5}
    text = open(HEADER).read()
    for name, val in (("SEM_MIXED_BF16", 2), ("SEM_MIXED_FP16", 3), ("SEM_MIXED_BF16X3", 4),
                      ("SEM_MIXED_FP16X3", 5)):
        assert re.search(rf"{name} = {val}\b", text), name


def test_c0_argument_errors():
    L = sem.lib()
    f = FAKE
    assert L.sem_gs_setup(4, 0, f, 10, f, 1 << 20, None, None) == _lib.SEM_ERR_ORDER
    assert L.sem_gs_setup(4, 3, None, 10, f, 1 << 20, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_gs_setup(4, 3, f, -1, f, 1 << 20, None, None) == _lib.SEM_ERR_ARG
    need = L.sem_gs_workspace_bytes(4, 3, 100)
    assert need >= 4 * 64 * 8 + 100 * 12
    assert L.sem_gs_setup(4, 3, f, 100, f, need - 1, None, None) == _lib.SEM_ERR_WORKSPACE
    assert L.sem_gs_workspace_bytes(4, 3, 1 << 33) == 0
    assert L.sem_dsavg(4, 3, 9, f, 100, f, f, None) == _lib.SEM_ERR_DTYPE
    assert L.sem_dsavg(4, 3, 0, None, 100, f, f, None) == _lib.SEM_ERR_ARG
    assert L.sem_dsavg(4, 3, 0, f, 0, f, f, None) == _lib.SEM_OK      # nothing to average
    assert L.sem_global_edge_keys(6, 0, 4, f, f, f, None, None) == _lib.SEM_ERR_ORDER
    assert L.sem_global_edge_keys(6, 3, 4, None, f, f, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_global_edge_keys(0, 3, 4, None, None, None, None, None) == _lib.SEM_OK
    wb = L.sem_weld_workspace_bytes(300)
    assert wb >= 300 * (4 + 4 + 8) + 2 * 600 * 8
    n = ctypes.c_void_p(0x2000)
    assert L.sem_weld(301, 0, f, f, f, f, 10, n, f, wb, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_weld(300, 9, f, f, f, f, 10, n, f, wb, None, None) == _lib.SEM_ERR_DTYPE
    assert L.sem_weld(300, 0, f, f, f, None, 10, n, f, wb, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_weld(300, 0, f, f, f, f, 10, None, f, wb, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_weld(300, 0, f, f, f, f, 10, n, f, wb - 1, None, None) == _lib.SEM_ERR_WORKSPACE


def test_batch_argument_errors_and_struct_layout():
    L = sem.lib()
    assert L.sem_batch_plan_bytes(0) == 0 and L.sem_batch_plan_bytes(5000) == 0
    assert L.sem_batch_plan_bytes(3) >= 256 + 3 * ctypes.sizeof(_lib._Snapshot)
    # sem_snapshot: int64 n_elem, int order, then nine pointers
    assert ctypes.sizeof(_lib._Snapshot) == 8 + 8 + 9 * 8
    assert _lib._Snapshot.x.offset == 16
    arr = (_lib._Snapshot * 1)()
    assert L.sem_batch_plan(0, ctypes.addressof(arr), 0, FAKE, 1 << 20, None) == _lib.SEM_ERR_ARG
    assert L.sem_batch_plan(1, ctypes.addressof(arr), 2, FAKE, 1 << 20, None) == \
        _lib.SEM_ERR_DTYPE
    assert L.sem_batch_plan(1, ctypes.addressof(arr), 0, FAKE, 10, None) == \
        _lib.SEM_ERR_WORKSPACE
    assert L.sem_qcrit_batch(None, 0, 0, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_qcrit_batch(FAKE, 0, 7, None, None) == _lib.SEM_ERR_DTYPE
    assert L.sem_autotune(0, 0, None, None) == _lib.SEM_ERR_ORDER
    assert L.sem_autotune(5, 3, None, None) == _lib.SEM_ERR_DTYPE
    assert L.sem_batch_variant(10, 0) == _lib.SEM_ERR_ORDER
    assert L.sem_batch_set_variant(9, 1, 4) == _lib.SEM_ERR_ARG     # direct-to-LDS: N = 7 FP64
    assert L.sem_batch_set_variant(7, 1, 4) == _lib.SEM_ERR_ARG
    assert L.sem_batch_set_variant(9, 0, 1) == _lib.SEM_ERR_ARG     # 2 x 1000 nodes > tile
    assert L.sem_batch_set_variant(5, 1, 7) == _lib.SEM_ERR_ARG


def test_compression_entry_points_reject_bad_arguments():
    L = _lib.lib()
    FAKE = ctypes.c_void_p(16)
    assert L.sem_ae_param_count() == 67812
    assert L.sem_ae_workspace_bytes(0) == 0 and L.sem_ae_workspace_bytes(8) > 8 * 2048 * 4
    assert L.sem_eig_workspace_bytes(3) == 0 and L.sem_eig_workspace_bytes(514) == 0
    assert L.sem_eig_workspace_bytes(512) >= 2 * 512 * 512 * 8
    assert L.sem_ae_pca_workspace_bytes(0) == 0
    assert L.sem_ae_compress_workspace_bytes(-1) == 0
    # tanh only after hidden layers
    assert L.sem_ae_forward(4, FAKE, FAKE, 0x04, FAKE, None, FAKE, 1 << 30, None) == \
        _lib.SEM_ERR_ARG
    assert L.sem_ae_forward(4, FAKE, FAKE, 0x20, FAKE, None, FAKE, 1 << 30, None) == \
        _lib.SEM_ERR_ARG
    assert L.sem_ae_forward(4, FAKE, FAKE, 0, None, None, FAKE, 1 << 30, None) == \
        _lib.SEM_ERR_ARG
    assert L.sem_ae_forward(4, FAKE, FAKE, 0, FAKE, None, FAKE, 16, None) == \
        _lib.SEM_ERR_WORKSPACE
    assert L.sem_ae_forward(0, None, None, 0, None, None, None, 0, None) == _lib.SEM_OK
    assert L.sem_ae_grad(0, FAKE, 1, None, FAKE, 0, 0, FAKE, None, FAKE, 1 << 30, None,
                         None) == _lib.SEM_ERR_ARG
    assert L.sem_ae_grad(5, FAKE, 4, None, FAKE, 0, 0, FAKE, None, FAKE, 1 << 30, None,
                         None) == _lib.SEM_ERR_ARG          # first n > pool without indices
    assert L.sem_ae_grad(4, FAKE, 4, None, FAKE, 0, 2, FAKE, None, FAKE, 1 << 30, None,
                         None) == _lib.SEM_ERR_ARG          # unknown loss
    assert L.sem_ae_grad(4, FAKE, 4, None, FAKE, 0, -1, FAKE, None, FAKE, 1 << 30, None,
                         None) == _lib.SEM_ERR_ARG
    assert L.sem_ae_adam(10, FAKE, FAKE, FAKE, FAKE, 0, 1e-3, 0.9, 0.999, 1e-8, None) == \
        _lib.SEM_ERR_ARG                                     # steps count from 1
    assert L.sem_ae_adam(10, FAKE, FAKE, FAKE, FAKE, 1, 1e-3, 1.0, 0.999, 1e-8, None) == \
        _lib.SEM_ERR_ARG
    assert L.sem_sym_eig(5, FAKE, 2, None, FAKE, FAKE, 1 << 30, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_sym_eig(8, FAKE, 9, None, FAKE, FAKE, 1 << 30, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_sym_eig(8, FAKE, 2, None, FAKE, FAKE, 8, None, None) == _lib.SEM_ERR_WORKSPACE
    assert L.sem_ae_compress(4, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, FAKE, -1,
                             FAKE, FAKE, 1 << 30, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_ae_compress(4, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, None, 4,
                             FAKE, FAKE, 1 << 30, None, None) == _lib.SEM_ERR_ARG
    assert L.sem_ae_compress(4, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, FAKE, 4,
                             FAKE, FAKE, 8, None, None) == _lib.SEM_ERR_WORKSPACE
    assert L.sem_modal_compress(4, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, FAKE, None, None,
                                None, FAKE, 1 << 30, None) == _lib.SEM_ERR_ARG   # some recon


def test_bench_finds_committed_profile_summaries():
    # bench.py reads the traffic and matrix-core summaries it reports from
    # profiles/, named for the kernel without its template arguments
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    path = bench.traffic_file(bench.q_kernel_name("f64"), "f64")
    assert os.path.basename(path) == "qcount_dma7_channel65536_f64_traffic.json"
    assert os.path.exists(path)
    assert os.path.exists(bench.MFMA_FILE)
