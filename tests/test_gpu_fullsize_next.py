"""Parity of the batched, compression and C0 paths at the benchmark's full
sizes and launch configurations, on outputs the oracle computes one by one.

* Batched: the 16 uneven FP32 snapshots of the benchmark (orders 5/7/9,
  342.9 M points) in one batched call with the autotuned forms; Q and
  |omega| of sampled elements of every snapshot within 1e-5 normwise of the
  oracle, element ranges exact.
* Compression: the 262,144-element held-out snapshot, PCA-initialised
  network as the benchmark trains it; for sampled elements the binary16
  latent within one step (plus FP32 rounding) of the oracle's encoder, the
  fallback flags equal to the oracle's rule (FP32) on the kernel's
  reconstruction, raw blocks bit-exact.
* C0: the channel snapshot's Q averaged over shared nodes (bit-exact on
  every node: both sides sum a node's copies in storage order) and the
  welded isosurface at the 90th percentile (keys, vertex numbering, indices
  and coordinates exact against the oracle's weld of the same soup).
"""

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import ae, c0, gll
from oracle import sem as osem

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batched_full_size_fp32():
    snaps, keep = [], []
    for seed in range(16):
        spec, arrs = W.batch_snapshot(seed, DEV, dtype=torch.float32)
        x, y, z, u, v, w, _ = arrs
        e = x.shape[0]
        snaps.append({"x": x, "y": y, "z": z, "u": u, "v": v, "w": w,
                      "q": torch.empty_like(u), "omega_mag": torch.empty_like(u),
                      "minmax": torch.empty((e, 2), dtype=torch.float32, device=DEV)})
        keep.append(spec[0])
    assert sum(s["x"].numel() for s in snaps) == 342931224
    for n in (5, 7, 9):
        sem.autotune(n, sem.SEM_F32)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.qcrit_batch(sem.BatchPlan(snaps), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rng = np.random.default_rng(5)
    for sn, n in zip(snaps, keep):
        e = sn["x"].shape[0]
        els = np.unique(np.concatenate([[0, e - 1], rng.choice(e, 6, replace=False)]))
        idx = torch.from_numpy(els).to(DEV)
        arrs = [sn[k].index_select(0, idx).double().cpu().numpy()
                for k in ("x", "y", "z", "u", "v", "w")]
        oq, oom, bad = osem.qcrit(*arrs, gll.diff_matrix(n))
        assert not bad.any()
        gq = sn["q"].index_select(0, idx).cpu().numpy().astype(np.float64)
        gom = sn["omega_mag"].index_select(0, idx).cpu().numpy().astype(np.float64)
        assert np.abs(gq - oq).max() / np.abs(oq).max() < 1e-5, n
        assert np.abs(gom - oom).max() / np.abs(oom).max() < 1e-5, n
        gq32 = sn["q"].index_select(0, idx).cpu().numpy()
        np.testing.assert_array_equal(sn["minmax"].index_select(0, idx).cpu().numpy(),
                                      osem.elem_minmax(gq32))


def test_compression_full_size():
    ph, el = W.ae_training_elements(0, 16384)
    pools = []
    for p in np.unique(ph):
        f = W.ae_fields(int(p), DEV, elements=el[ph == p], dtype=torch.float32)
        pools.append(sem.ae_blocks(list(f))[0])
    params, _ = sem.ae_pca_init(torch.cat(pools))
    del pools
    fields = list(W.ae_fields(63.5, DEV, dtype=torch.float32))
    e = fields[0].shape[0]
    assert e == 262144
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    pk = sem.ae_compress(fields, params, status=st)
    pure = dict(pk, flags=torch.zeros_like(pk["flags"]), raw=pk["raw"][:0])
    rec = sem.ae_decompress(pure, params)
    out = sem.ae_decompress(pk, params)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    flags = pk["flags"].cpu().numpy().astype(bool)
    assert pk["n_raw"] == int(flags.sum())
    # global channel maxima from the fields themselves (the oracle's own)
    gmax = np.array([float(f.abs().max().item()) for f in fields], dtype=np.float32)
    rng = np.random.default_rng(8)
    els = np.unique(np.concatenate([[0, e - 1], rng.choice(e, 2046, replace=False),
                                    np.flatnonzero(flags)[:64]]))
    idx = torch.from_numpy(els).to(DEV)
    hf = [f.index_select(0, idx).cpu().numpy() for f in fields]
    hr = [f.index_select(0, idx).cpu().numpy() for f in rec]
    ho = [f.index_select(0, idx).cpu().numpy() for f in out]
    np.testing.assert_array_equal(ae.fallback(hf, hr, gmax), flags[els])
    for c in range(4):
        np.testing.assert_array_equal(ho[c][flags[els]], hf[c][flags[els]])
    assert not ae.fallback(hf, ho, gmax).any()
    # latent of the sampled elements: within one binary16 step of the encoder,
    # plus the FP32 encoder's own rounding (normwise 2e-6 of the element's
    # latent; its small components have binary16 steps below that)
    x, _ = ae.blocks(hf)
    layers = ae.unpack(params.cpu().numpy())
    a = x.astype(np.float64)
    for l in range(3):
        a = ae.conv(a, *layers[l])
    enc = a.reshape(-1, 32)
    z = pk["latent"].index_select(0, idx).float().cpu().numpy().astype(np.float64)
    step = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(enc), 2.0 ** -14))) - 10)
    fp32 = 2e-6 * np.abs(enc).max(axis=1, keepdims=True)
    assert np.all(np.abs(z - enc) <= step * 1.0001 + fp32)


def test_c0_and_weld_full_size_channel():
    n = 7
    with open(os.path.join(ROOT, "tests", "golden", "channel_isovalues.json")) as fh:
        iso = json.load(fh)["isovalues"][0]
    fields = [f.contiguous() for f in W.channel_config(n, device=DEV)]
    x, y, z = fields[:3]
    q, _, _ = sem.qcrit(*fields)
    gid_np = W.lattice_gid(W.CHANNEL_SHAPE, n)
    gid = torch.from_numpy(gid_np).to(DEV)
    gs = sem.GatherScatter(gid)
    qa = sem.dsavg(q, gs)
    # averages: the oracle over the whole field, compared on every node
    qh = q.cpu().numpy()
    np.testing.assert_array_equal(qa.cpu().numpy(), c0.dsavg(qh, gid_np))
    r = sem.isosurface(x, y, z, qa, [iso], edge_keys=True)
    keys = sem.global_edge_keys(r["edge_key"], gid)
    verts, idxs = sem.weld(r["tri_xyz"], keys)
    okeys = c0.global_edge_keys(r["edge_key"].cpu().numpy().astype(np.uint64), gid_np, n)
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint64), okeys)
    ov, oi = c0.weld(r["tri_xyz"].cpu().numpy(), okeys)
    np.testing.assert_array_equal(idxs.cpu().numpy(), oi)
    np.testing.assert_array_equal(verts.cpu().numpy(), ov)
    assert ov.shape[0] < 3 * oi.shape[0]
