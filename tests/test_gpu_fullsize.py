"""Parity at the benchmark's full size and launch configuration.

The turbulent-channel snapshot (65,536 order-7 elements, 33,554,432 GLL
points, Q isovalues at its 90/95/99th percentiles) is generated on the GPU
and run through sem_extract -- the fused call bench.py times -- in FP64 and
in FP32 (the FP64 inputs rounded).  The CPU oracle computes Q and |omega| of
every element from the same inputs (FP32 inputs widened exactly), and:

  * Q and |omega| agree everywhere, normwise, within 1e-10 (FP64) / 1e-5
    (FP32); the per-element ranges are exactly those of the kernel's own Q;
  * stage-isolated: the kernel's case of every cell (sem_isosurface's case
    dump of the kernel's Q) equals the oracle's classification of that same
    Q, and sem_extract's triangle and active-cell counts equal the oracle's
    counts of it; sem_extract and sem_isosurface emit identical triangles;
  * end to end (GPU Q -> cases against oracle Q -> cases): a cell's case may
    differ only where one of its nodes lies within the band
    max |Q_gpu - Q_oracle| + |c_dt - c| of the isovalue (c_dt: the isovalue
    rounded to the working precision); counts must then be equal whenever no
    cell differs;
  * the triangles of sampled elements equal the oracle's extraction of the
    kernel's Q within the precision's bound, and -- where every cell of the
    element has the same case on both sides -- the oracle's extraction of
    the oracle's Q within the conditioning-aware bound
    |dp| <= tol L + |dt| |x1 - x0|, with |dt| bounded from the two ends'
    field errors and |f1 - f0| (a vertex moves along its edge as t does).
"""

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import gll, mc
from oracle import sem as osem

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEV = "cuda:0"
N = 7
P = N + 1
TOL = {np.float64: 1e-10, np.float32: 1e-5}
TDT = {np.float64: torch.float64, np.float32: torch.float32}
CHUNK = 4096


def _isovalues():
    with open(os.path.join(ROOT, "tests", "golden", "channel_isovalues.json")) as fh:
        return json.load(fh)["isovalues"]


@pytest.fixture(scope="module")
def channel():
    """The FP64 channel snapshot on the GPU and its inputs on the host."""
    fields = [f.contiguous() for f in W.channel_config(N, device=DEV)]
    assert fields[0].shape[0] == 65536
    host = [f.cpu().numpy() for f in fields]
    return fields, host


def _oracle_q(host):
    """Oracle Q and |omega| of every element (chunks of CHUNK elements)."""
    d = gll.diff_matrix(N)
    e_tot = host[0].shape[0]
    oq = np.empty(host[0].shape, dtype=np.float64)
    oom = np.empty_like(oq)
    for a in range(0, e_tot, CHUNK):
        sl = slice(a, min(a + CHUNK, e_tot))
        q, om, bad = osem.qcrit(*(h[sl].astype(np.float64) for h in host), d)
        assert not bad.any()
        oq[sl], oom[sl] = q, om
    return oq, oom


def _band_cells(q_ref, c_ref, band):
    """(E, N^3) bool: cells with a node within `band` of the isovalue."""
    e_cnt = q_ref.shape[0]
    near = (np.abs(q_ref - c_ref) <= band).reshape(e_cnt, P, P, P)
    cell = np.zeros((e_cnt, N, N, N), dtype=bool)
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                cell |= near[:, cc:cc + N, b:b + N, a:a + N]
    return cell.reshape(e_cnt, -1)


def _vertex_bound(keys, q_gpu, q_ref, dc, tol_abs, coords):
    """Per-vertex bound of |p_gpu - p_oracle| (vertices of the oracle's
    extraction of q_ref, identified by their edge keys), shape (T, 3, 1)."""
    keys = keys.astype(np.int64)
    axis = keys % 3
    node = keys // 3
    lo = node
    hi = node + np.array([1, P, P * P])[axis]
    qg, qr = q_gpu.reshape(-1), q_ref.reshape(-1)
    df0 = np.abs(qg[lo] - qr[lo])
    df1 = np.abs(qg[hi] - qr[hi])
    den = np.minimum(np.abs(qr[hi] - qr[lo]), np.abs(qg[hi] - qg[lo]))
    dt = np.minimum(1.0, (dc + 2.0 * (df0 + df1)) / den)
    span = np.stack([np.abs(c.reshape(-1)[hi] - c.reshape(-1)[lo]) for c in coords], axis=-1)
    return tol_abs + dt[..., None] * span


def _end_to_end(fields_dev, host, dt):
    isos = _isovalues()
    tol = TOL[dt]
    e_tot = host[0].shape[0]
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    r = sem.extract(*fields_dev, isos, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    q, om, mm = r["q"], r["omega_mag"], r["minmax"]

    # 1. Q and |omega| of every element against the oracle
    h64 = [h.astype(np.float64) for h in host]
    oq, oom = _oracle_q(h64)
    qh = q.cpu().numpy()
    q64 = qh.astype(np.float64)
    dq = np.abs(q64 - oq)
    errq = dq.max() / np.abs(oq).max()
    errw = np.abs(om.cpu().numpy().astype(np.float64) - oom).max() / np.abs(oom).max()
    print(f"[{np.dtype(dt).name}] Q normwise {errq:.3e}, |omega| normwise {errw:.3e}")
    assert errq < tol and errw < tol
    np.testing.assert_array_equal(mm.cpu().numpy(), osem.elem_minmax(qh))
    band_q = float(dq.max())
    del om

    # 2. stage-isolated: kernel cases of the kernel's Q, counts, triangles
    ri = sem.isosurface(fields_dev[0], fields_dev[1], fields_dev[2], q, isos, minmax=mm,
                        cases=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ri["tri_count"].cpu().numpy(), r["tri_count"].cpu().numpy())
    np.testing.assert_array_equal(ri["active"].cpu().numpy(), r["active"].cpu().numpy())
    off = 0
    for s in range(len(isos)):
        cnt = int(r["tri_count"][s])
        assert torch.equal(ri["tri_xyz"][off:off + cnt], r["tri"][s])
        off += cnt
    gcases = ri["cases"].cpu().numpy()
    del ri
    ntri_tab, _ = mc.case_table()
    per_elem = []
    for s, c in enumerate(isos):
        cs = mc.classify(qh, c).reshape(e_tot, -1)
        np.testing.assert_array_equal(gcases[s], cs)
        cnt = ntri_tab[cs].astype(np.int64).sum(axis=1)
        assert int(r["tri_count"][s]) == int(cnt.sum())
        assert int(r["active"][s]) == int(np.count_nonzero((cs != 0) & (cs != 255)))
        per_elem.append(cnt)

    # 3. end to end: oracle Q classified against the exact isovalue
    agree_elems = []
    for s, c in enumerate(isos):
        c_dt = float(dt(c))
        band = band_q + abs(c_dt - c)
        oc = mc.classify(oq, c).reshape(e_tot, -1)
        bad = gcases[s] != oc
        near = _band_cells(oq, c, band)
        n_bad = int(bad.sum())
        outside = int((bad & ~near).sum())
        margin = float(np.abs(oq - c).min())
        o_cnt = int(ntri_tab[oc].astype(np.int64).sum())
        print(f"[{np.dtype(dt).name}] iso {c:.6f}: band {band:.3e}, margin {margin:.3e}, "
              f"{n_bad} of {oc.size} cells differ ({int(near.sum())} in the band), "
              f"triangles gpu {int(r['tri_count'][s])} oracle {o_cnt}")
        assert outside == 0
        if n_bad == 0:
            assert int(r["tri_count"][s]) == o_cnt
        if margin > 1e3 * band:
            assert n_bad == 0
        agree_elems.append(~bad.any(axis=1))
        del oc, bad, near

    # 4. triangles of sampled elements
    per_elem = np.stack(per_elem)
    flat = per_elem.ravel()
    offs = (np.cumsum(flat) - flat).reshape(per_elem.shape)
    rng = np.random.default_rng(7)
    scale = max(np.abs(h).max() for h in h64[:3])
    worst_iso = worst_e2e = 0.0
    for s, c in enumerate(isos):
        cand = np.nonzero(per_elem[s] > 0)[0]
        els = np.unique(np.concatenate([cand[:1], cand[-1:],
                                        rng.choice(cand, 48, replace=False)]))
        tri = r["tri"][s]
        base = int(offs[s, 0])
        for e in els:
            nt = int(per_elem[s, e])
            sl = slice(e, e + 1)
            got = tri[int(offs[s, e]) - base:int(offs[s, e]) - base + nt].cpu().numpy()
            o = mc.extract(host[0][sl], host[1][sl], host[2][sl], qh[sl], [c])
            assert int(o["tri_count"][0]) == nt
            err = np.abs(got.astype(np.float64) - o["tri_xyz"]).max()
            worst_iso = max(worst_iso, err / scale)
            assert err <= tol * scale
            if not agree_elems[s][e]:
                continue
            oe = mc.extract(h64[0][sl], h64[1][sl], h64[2][sl], oq[sl], [c], edge_keys=True)
            assert int(oe["tri_count"][0]) == nt
            bound = _vertex_bound(oe["edge_key"], q64[sl], oq[sl], abs(float(dt(c)) - c),
                                  tol * scale, [h[sl] for h in h64[:3]])
            diff = np.abs(got.astype(np.float64) - oe["tri_xyz"])
            worst_e2e = max(worst_e2e, float(diff.max()) / scale)
            assert np.all(diff <= bound)
    print(f"[{np.dtype(dt).name}] vertices: stage-isolated {worst_iso:.3e}, end to end "
          f"{worst_e2e:.3e} (relative to the largest coordinate)")


def test_channel_full_size_fp64(channel):
    fields, host = channel
    _end_to_end(fields, host, np.float64)


def test_channel_full_size_fp32(channel):
    fields, host = channel
    f32 = [f.to(torch.float32).contiguous() for f in fields]
    h32 = [h.astype(np.float32) for h in host]
    _end_to_end(f32, h32, np.float32)
