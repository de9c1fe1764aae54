"""GPU: sem_extract_noalloc (fixed library scratch instead of a workspace)
gives exactly sem_extract's results -- Q, |omega|, element ranges, triangle
and active-cell counts and every triangle, bit for bit -- on consecutive
calls that reuse the scratch, the second one smaller than the first, in
FP64 at order 7 (the direct-load kernels) and FP32 at order 5 (pencil
kernels and the two-pass isosurface)."""

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _fields(n, shape, dt):
    if n == 7:
        arrs = W.tgv_config(n, shape=shape)
    else:
        x, y, z = W.box_mesh(shape, n, ((0.0, 1.7), (-0.4, 0.9), (0.2, 1.4)))
        x, y, z = W.warp(x, y, z, amp=0.05)
        arrs = (x, y, z, np.sin(2 * x + y) * z, np.cos(x - 3 * z), x * y - np.sin(z))
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(DEV) for a in arrs]


def _reference(f, isos):
    r = sem.extract(*f, isos)
    torch.cuda.synchronize()
    return r


def _noalloc(f, isos, counts):
    e = f[0].shape[0]
    tris = [torch.full((c, 3, 3), float("nan"), dtype=f[0].dtype, device=DEV) for c in counts]
    q = torch.full_like(f[3], float("nan"))
    om = torch.full_like(f[3], float("nan"))
    mm = torch.full((e, 2), float("nan"), dtype=f[0].dtype, device=DEV)
    cnt = torch.full((len(isos),), -1, dtype=torch.int64, device=DEV)
    act = torch.full((len(isos),), -1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.extract_noalloc_into(*f, isos, tris, cnt, q, mm, omega_mag=om, active=act, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"q": q, "omega_mag": om, "minmax": mm, "tri": tris, "tri_count": cnt,
            "active": act}


def _same(a, b):
    for k in ("q", "omega_mag", "minmax", "tri_count", "active"):
        assert torch.equal(a[k], b[k]), k
    assert len(a["tri"]) == len(b["tri"])
    for s, (ta, tb) in enumerate(zip(a["tri"], b["tri"])):
        assert torch.equal(ta, tb), s


@pytest.mark.parametrize("n, dt, big, small", [
    (7, np.float64, (8, 8, 8), (4, 4, 2)),
    (5, np.float32, (6, 5, 4), (3, 1, 1)),
])
def test_noalloc_matches_extract_on_consecutive_calls(n, dt, big, small):
    for shape, isos in ((big, [0.1, -0.2, 0.35]), (small, [0.05])):
        f = _fields(n, shape, dt)
        ref = _reference(f, isos)
        counts = ref["tri_count"].cpu().tolist()
        assert sum(counts) > 0
        _same(_noalloc(f, isos, counts), ref)


def test_noalloc_overflow_keeps_counts_exact_and_rejects_too_large():
    f = _fields(7, (4, 4, 4), np.float64)
    ref = _reference(f, [0.1])
    total = int(ref["tri_count"][0])
    tri = torch.zeros((total // 2, 3, 3), dtype=torch.float64, device=DEV)
    q = torch.empty_like(f[3])
    mm = torch.empty((f[0].shape[0], 2), dtype=torch.float64, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.extract_noalloc_into(*f, [0.1], [tri], cnt, q, mm, status=st)
    torch.cuda.synchronize()
    assert int(cnt.item()) == total
    assert int(st.item()) & sem.SEM_FLAG_TRI_OVERFLOW
    assert torch.equal(tri, ref["tri"][0][:total // 2])
    # more (isovalue, element) counts than the scratch holds: refused on the
    # host before any work is queued
    isos = list(np.linspace(-0.5, 0.5, 64))
    big = [torch.empty((sem.SEM_NOALLOC_MAX_COUNTS // 64 + 1, 8, 8, 8), dtype=torch.float64,
                       device=DEV)] * 6
    with pytest.raises(sem.SemError):
        sem.extract_noalloc_into(*big, isos, [None] * 64, torch.zeros(64, dtype=torch.int64,
                                                                      device=DEV),
                                 big[0], torch.empty((big[0].shape[0], 2), dtype=torch.float64,
                                                     device=DEV))
