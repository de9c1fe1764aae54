"""GPU parity: every C-ABI entry point against the CPU FP64 oracle.

Bars: case indices, active-cell and triangle counts, edge keys bit-exact;
fields and vertex positions within 1e-10 (FP64) / 1e-5 (FP32) normwise
relative error (max |a - b| / max |b|; vertices relative to the largest
coordinate magnitude).  FP32 runs give the oracle the same FP32 inputs,
widened exactly to FP64, and classify in FP32 like the kernel.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gll, mc, sem as osem

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {np.float64: 1e-10, np.float32: 1e-5}
TDT = {np.float64: torch.float64, np.float32: torch.float32}


def dev(a, dt=np.float64):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dt))).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def status_word():
    return torch.zeros(1, dtype=torch.int32, device=DEV)


def warped_mesh(n, shape, amp=0.06, seed=0):
    x, y, z = W.box_mesh(shape, n, ((0.0, 1.7), (-0.4, 0.9), (0.2, 1.4)))
    return W.warp(x, y, z, amp=amp)


def smooth_velocity(x, y, z, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(3):
        k = rng.uniform(0.5, 3.0, size=(3, 3))
        ph = rng.uniform(0, 6.28, size=3)
        out.append(sum(np.sin(k[m, 0] * x + k[m, 1] * y + k[m, 2] * z + ph[m])
                       for m in range(3)))
    return out


# --------------------------------------------------------------------------
# sem_derivs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", list(range(1, 10)))
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_derivs_matches_oracle(n, dt):
    for shape in ((1, 1, 1), (7, 1, 1), (4, 4, 4)):
        x, y, z = warped_mesh(n, shape)
        f = np.sin(1.3 * x) * np.cos(0.7 * y) + z * z * x
        xs, ys, zs, fs = (a.astype(dt) for a in (x, y, z, f))
        st = status_word()
        g = sem.derivs(dev(xs, dt), dev(ys, dt), dev(zs, dt), dev(fs, dt), status=st)
        (ox, oy, oz), bad = osem.derivs(*(a.astype(np.float64) for a in (xs, ys, zs, fs)),
                                        gll.diff_matrix(n))
        assert not bad.any() and int(st.item()) == 0
        for got, want in zip(g, (ox, oy, oz)):
            assert relerr(host(got), want) < TOL[dt], (shape, relerr(host(got), want))


def test_derivs_exact_on_polynomials_fp64():
    n = 6
    x, y, z = W.box_mesh((3, 2, 2), n, ((0.0, 1.5), (0.5, 1.3), (-1.0, 0.2)))
    f = x ** 6 * y ** 2 * z ** 5 + 3 * x * y * z
    g = sem.derivs(dev(x), dev(y), dev(z), dev(f))
    want = (6 * x ** 5 * y ** 2 * z ** 5 + 3 * y * z,
            2 * x ** 6 * y * z ** 5 + 3 * x * z,
            5 * x ** 6 * y ** 2 * z ** 4 + 3 * x * y)
    for got, w in zip(g, want):
        assert relerr(host(got), w) < 1e-11


# --------------------------------------------------------------------------
# sem_qcrit
# --------------------------------------------------------------------------

def _check_qcrit(x, y, z, u, v, w, n, dt):
    arrs = [a.astype(dt) for a in (x, y, z, u, v, w)]
    st = status_word()
    q, om, mm = sem.qcrit(*(dev(a, dt) for a in arrs), status=st)
    oq, oom, bad = osem.qcrit(*(a.astype(np.float64) for a in arrs), gll.diff_matrix(n))
    assert int(st.item()) == int(bad.any())
    hq, hom, hmm = host(q), host(om), host(mm)
    assert relerr(hq, oq) < TOL[dt], relerr(hq, oq)
    assert relerr(hom, oom) < TOL[dt], relerr(hom, oom)
    # the per-element range is exactly that of the kernel's own Q
    np.testing.assert_array_equal(hmm, osem.elem_minmax(hq).astype(dt))
    return hq, oq


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_qcrit_taylor_green(dt):
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    _check_qcrit(x, y, z, u, v, w, n, dt)


@pytest.mark.parametrize("n", list(range(1, 10)))
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_qcrit_warped_random(n, dt):
    for shape, seed in (((1, 1, 1), 1), ((7, 1, 1), 2), ((4, 4, 4), 3)):
        x, y, z = warped_mesh(n, shape)
        u, v, w = smooth_velocity(x, y, z, seed)
        _check_qcrit(x, y, z, u, v, w, n, dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_qcrit_channel_sample(dt):
    els = np.arange(0, 65536, 331)
    x, y, z, u, v, w = W.channel_config(7, elements=els)
    _check_qcrit(x, y, z, u, v, w, 7, dt)


def test_qcrit_optional_outputs_and_bad_jacobian():
    n = 3
    x, y, z = warped_mesh(n, (3, 1, 1))
    x = x.copy()
    x[1] = x[1, :, :, ::-1]
    u, v, w = smooth_velocity(x, y, z)
    st = status_word()
    q, _, _ = sem.qcrit(*(dev(a) for a in (x, y, z, u, v, w)), status=st, want=("q",))
    assert int(st.item()) & sem.SEM_FLAG_BAD_JACOBIAN
    oq, _, bad = osem.qcrit(x, y, z, u, v, w, gll.diff_matrix(n))
    assert bad[1].all() and not bad[0].any()
    good = ~bad.reshape(3, -1).any(axis=1)
    assert relerr(host(q)[good], oq[good]) < 1e-10


@pytest.mark.parametrize("scale", [2.0 ** -500, 2.0 ** 505])
def test_qcrit_fp64_far_scales(scale):
    """Order 7, FP64: the Taylor-Green velocity scaled so that the root's
    argument in the kernel (|omega|^2 times det J^2) leaves [2^-1000, 2^1000]
    at some or all nodes, where the kernel takes the library root instead of
    its refined hardware estimate; Q and |omega| still within 1e-10
    normwise (relative errors do not depend on the scale)."""
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    u, v, w = (scale * a for a in (u, v, w))
    _check_qcrit(x, y, z, u, v, w, n, np.float64)


def test_qcrit_linear_field_exact():
    n = 5
    x, y, z = warped_mesh(n, (2, 2, 2))
    q, om, _ = sem.qcrit(*(dev(a) for a in (x, y, z, -y, x, 0 * x)))
    np.testing.assert_allclose(host(q), 1.0, atol=1e-11)
    np.testing.assert_allclose(host(om), 2.0, atol=1e-11)


# --------------------------------------------------------------------------
# sem_isosurface, stage-isolated (same field on both sides)
# --------------------------------------------------------------------------

def _compare_iso(x, y, z, f, isos, dt, use_minmax=True):
    arrs = [a.astype(dt) for a in (x, y, z, f)]
    t = [dev(a, dt) for a in arrs]
    mm = dev(osem.elem_minmax(arrs[3]), dt) if use_minmax else None
    st = status_word()
    r = sem.isosurface(*t, isos, minmax=mm, edge_keys=True, cases=True, status=st)
    o = mc.extract(*arrs, isos, edge_keys=True)
    assert int(st.item()) == 0
    np.testing.assert_array_equal(host(r["cases"]), o["cases"])
    np.testing.assert_array_equal(host(r["tri_count"]), o["tri_count"])
    np.testing.assert_array_equal(host(r["active"]), o["active"])
    np.testing.assert_array_equal(host(r["edge_key"]).astype(np.uint64), o["edge_key"])
    scale = max(np.abs(a).max() for a in arrs[:3])
    got = host(r["tri_xyz"]).astype(np.float64)
    # a vertex on an edge with a NaN end is NaN on both sides
    np.testing.assert_array_equal(np.isnan(got), np.isnan(o["tri_xyz"]))
    ok = ~np.isnan(got)
    err = np.abs(got[ok] - o["tri_xyz"][ok])
    assert (err.max() if err.size else 0.0) <= TOL[dt] * scale
    return r, o


@pytest.mark.parametrize("n", list(range(1, 10)))
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_isosurface_matches_oracle(n, dt):
    for shape, seed in (((1, 1, 1), 4), ((7, 1, 1), 5), ((3, 3, 3), 6)):
        x, y, z = warped_mesh(n, shape)
        f = smooth_velocity(x, y, z, seed)[0]
        _compare_iso(x, y, z, f, [-0.7, 0.1, 0.55], dt)


def test_isosurface_cull_does_not_change_output():
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    q, _, _ = osem.qcrit(x, y, z, u, v, w, gll.diff_matrix(n))
    r1, _ = _compare_iso(x, y, z, q, [0.1, -0.2], np.float64, use_minmax=True)
    r2, _ = _compare_iso(x, y, z, q, [0.1, -0.2], np.float64, use_minmax=False)
    assert torch.equal(r1["tri_xyz"], r2["tri_xyz"])
    assert torch.equal(r1["edge_key"], r2["edge_key"])


def test_isosurface_nan_and_ties():
    n = 2
    x, y, z = W.box_mesh((2, 1, 1), n, ((0, 2.0), (0, 1.0), (0, 1.0)))
    f = np.round(np.sin(3 * x + y) * 4) / 4          # many exact ties with 0.25
    f[0, 1, 1, 1] = np.nan
    _compare_iso(x, y, z, f, [0.25, 0.0], np.float64, use_minmax=True)
    _compare_iso(x, y, z, f, [0.25, 0.0], np.float64, use_minmax=False)


def test_isosurface_brute_force_sign_patterns():
    """All 2^12 patterns of a 1x1x2 grid (order-1 elements) on the GPU."""
    pats = np.arange(2 ** 12, dtype=np.int64)
    bits = (pats[:, None] >> np.arange(12)) & 1
    vals = np.where(bits == 1, 1.0, -1.0).reshape(-1, 3, 2, 2)
    o = np.array([0, 1])
    kk, jj, ii = np.meshgrid(o, o, o, indexing="ij")
    f = np.concatenate([vals[:, None, c:c + 2] for c in range(2)], axis=1).reshape(-1, 2, 2, 2)
    cz = np.tile([0, 1], pats.size)
    x = np.broadcast_to(ii.astype(float), f.shape).copy()
    y = np.broadcast_to(jj.astype(float), f.shape).copy()
    z = (kk[None] + cz[:, None, None, None]).astype(float)
    _compare_iso(x, y, z, f, [0.0], np.float64)


def test_isosurface_overflow_and_exact_counts():
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    q, _, _ = osem.qcrit(x, y, z, u, v, w, gll.diff_matrix(n))
    o = mc.extract(x, y, z, q, [0.1], edge_keys=True)
    total = int(o["tri_count"][0])
    t = [dev(a) for a in (x, y, z, q)]
    for cap in (0, 1000, total - 1, total):
        ws = torch.empty(sem.workspace_bytes(512, n, 1), dtype=torch.uint8, device=DEV)
        tri = torch.full((max(cap, 1), 3, 3), -7.0, dtype=torch.float64, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
        st = status_word()
        sem.isosurface_into(*t, [0.1], tri if cap else None, cnt, ws, status=st)
        assert int(cnt.item()) == total
        assert bool(int(st.item()) & sem.SEM_FLAG_TRI_OVERFLOW) == (cap < total)
        if cap:
            np.testing.assert_array_equal(host(tri)[:cap], o["tri_xyz"][:cap])


@pytest.mark.parametrize("n_elem", [65536, 65537])
def test_isosurface_scan_tile_boundary(n_elem):
    # 64 isovalues x n_elem counts make 1,024 scan tiles of 4,096 (the tile
    # offsets folded into the apply kernel) or 1,025 (a separate scan of the
    # tile sums); order-1 elements, one cell each, random node values
    rng = np.random.default_rng(n_elem)
    o = np.array([0.0, 1.0])
    kk, jj, ii = np.meshgrid(o, o, o, indexing="ij")
    e = np.arange(n_elem, dtype=np.float64)[:, None, None, None]
    x = ii[None] + 2.0 * (e % 256)
    y = jj[None] + 2.0 * (e // 256)
    z = np.broadcast_to(kk[None], (n_elem, 2, 2, 2)).copy()
    f = rng.uniform(-1.0, 1.0, size=(n_elem, 2, 2, 2))
    isos = [float(c) for c in np.linspace(-0.9, 0.9, 64)]
    st = status_word()
    r = sem.isosurface(*(dev(a) for a in (x, y, z, f)), isos, status=st)
    assert int(st.item()) == 0
    ntri, _ = mc.case_table()
    per = np.stack([ntri[mc.classify(f, c).reshape(n_elem, -1)[:, 0]].astype(np.int64)
                    for c in isos])                       # (isovalue, element)
    np.testing.assert_array_equal(host(r["tri_count"]), per.sum(axis=1))
    # the soup is isovalue-major: triangles of elements at tile edges
    first = np.concatenate([[0], np.cumsum(per.ravel())])
    scale = float(np.abs(x).max())
    for s, el in ((0, 0), (0, 4095), (0, 4096), (15, 65535), (31, 12345), (63, n_elem - 1),
                  (63, n_elem - 2)):
        k = s * n_elem + el
        c = int(per[s, el])
        got = host(r["tri_xyz"][int(first[k]):int(first[k]) + c])
        want = mc.extract(x[el:el + 1], y[el:el + 1], z[el:el + 1], f[el:el + 1],
                          [isos[s]])["tri_xyz"]
        assert got.shape == want.shape
        if c:
            assert np.abs(got - want).max() <= TOL[np.float64] * scale


def test_isosurface_empty_input():
    e = torch.empty((0, 8, 8, 8), dtype=torch.float64, device=DEV)
    cnt = torch.full((2,), 99, dtype=torch.int64, device=DEV)
    act = torch.full((2,), 99, dtype=torch.int64, device=DEV)
    sem.isosurface_into(e, e, e, e, [0.1, 0.2], None, cnt, None, active=act)
    assert host(cnt).tolist() == [0, 0] and host(act).tolist() == [0, 0]


def test_isosurface_deterministic():
    n = 7
    x, y, z = warped_mesh(n, (5, 4, 3))
    f = smooth_velocity(x, y, z, 9)[1]
    t = [dev(a) for a in (x, y, z, f)]
    r1 = sem.isosurface(*t, [0.0, 0.4, -0.4], edge_keys=True)
    r2 = sem.isosurface(*t, [0.0, 0.4, -0.4], edge_keys=True)
    assert torch.equal(r1["tri_xyz"], r2["tri_xyz"])
    assert torch.equal(r1["edge_key"], r2["edge_key"])


# --------------------------------------------------------------------------
# end to end: Q on the GPU, then its isosurface
# --------------------------------------------------------------------------

def _band_check(cases_gpu, cases_ref, q_ref, c_ref, band, n):
    """Cells may differ only where a node lies within `band` of the isovalue."""
    p = n + 1
    e_cnt = q_ref.shape[0]
    near = (np.abs(q_ref - c_ref) <= band).reshape(e_cnt, p, p, p)
    cell_near = np.zeros((e_cnt, n, n, n), dtype=bool)
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                cell_near |= near[:, cc:cc + n, b:b + n, a:a + n]
    bad = cases_gpu.reshape(e_cnt, -1) != cases_ref.reshape(e_cnt, -1)
    assert not np.any(bad & ~cell_near.reshape(e_cnt, -1))
    return int(bad.sum())


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_taylor_green_end_to_end_counts_bit_exact(dt):
    n, c = 7, 0.1
    arrs = [a.astype(dt) for a in W.tgv_config(n)]
    t = [dev(a, dt) for a in arrs]
    q, _, mm = sem.qcrit(*t)
    r = sem.isosurface(t[0], t[1], t[2], q, [c], minmax=mm, cases=True)
    oq, _, _ = osem.qcrit(*(a.astype(np.float64) for a in arrs), gll.diff_matrix(n))
    o = mc.extract(*(a.astype(np.float64) for a in arrs[:3]), oq, [c])
    diff = np.abs(host(q).astype(np.float64) - oq).max()
    c_dt = float(dt(c))
    band = diff + abs(c_dt - c)
    margin = np.abs(oq - c).min()
    mism = _band_check(host(r["cases"])[0], o["cases"][0], oq, c, band, n)
    # the closed-form margin of this snapshot (3.1e-4) exceeds the band
    assert margin > band, (margin, band)
    assert mism == 0
    np.testing.assert_array_equal(host(r["tri_count"]), o["tri_count"])
    np.testing.assert_array_equal(host(r["active"]), o["active"])
    np.testing.assert_array_equal(host(r["cases"]), o["cases"])
    assert int(o["tri_count"][0]) == 37184 and int(o["active"][0]) == 18624


def test_stream_copy_copies_every_byte():
    """The bandwidth reference kernel: an exact copy, ragged grid tail
    included (sizes that are not multiples of the grid's stride)."""
    for nbytes in (16, 4096 + 48, (1 << 24) + 16 * 1234):
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=DEV)
        dst = torch.zeros_like(src)
        sem.stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), nbytes
