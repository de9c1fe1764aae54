"""GPU: batched isosurfaces (persistent count, one scan, persistent emission).

Jobs -- (snapshot, field, up to four isovalues) over snapshots of mixed order
and uneven size -- must give exactly what the marching-cubes definition gives
for each job's field: counts and active cells bit-exact against the CPU
oracle's classification of the same field values (stage-isolated), vertices
within 1e-10 (FP64) / 1e-5 (FP32) of the largest coordinate, soup order job,
isovalue, element, cell, slot.  Against sem_isosurface on the same field the
soup is bit-identical.  At the batched-snapshot benchmark's full size the
batch is compared bit for bit with per-job sem_isosurface calls, and the
triangles of sampled elements of every job with the oracle.
"""

import numpy as np
import pytest

import workloads as W
from oracle import mc

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


def _snapshot(n, shape, seed, tdt):
    x, y, z = W.box_mesh(shape, n, ((0.0, 1.7), (-0.4, 0.9), (0.2, 1.4)))
    x, y, z = W.warp(x, y, z, amp=0.05)
    rng = np.random.default_rng(seed)
    f = []
    for _ in range(4):                       # u, v, w, theta
        k = rng.uniform(0.5, 4.0, size=(3, 3))
        ph = rng.uniform(0, 6.28, size=3)
        f.append(sum(np.sin(k[m, 0] * x + k[m, 1] * y + k[m, 2] * z + ph[m])
                     for m in range(3)))
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(tdt) for a in (x, y, z, *f)]
    e = t[0].shape[0]
    return {"x": t[0], "y": t[1], "z": t[2], "u": t[3], "v": t[4], "w": t[5],
            "theta": t[6], "q": torch.empty_like(t[3]), "omega_mag": torch.empty_like(t[3]),
            "minmax": torch.empty((e, 2), dtype=tdt, device=DEV)}


# mixed odd and even orders, ragged sizes, one empty snapshot
SPECS = [(7, (3, 2, 2), 1), (2, (3, 2, 1), 2), (5, (4, 3, 2), 3), (9, (2, 2, 1), 4),
         (6, (2, 1, 2), 5), (1, (5, 1, 1), 6), (8, (1, 2, 1), 7), (3, (2, 2, 2), 8),
         (4, (1, 1, 3), 9)]


def _snaps(tdt):
    snaps = [_snapshot(n, shape, seed, tdt) for n, shape, seed in SPECS]
    # an empty snapshot of order 5 (no elements)
    e0 = {k: v[:0] for k, v in _snapshot(5, (1, 1, 1), 0, tdt).items()}
    snaps.insert(3, e0)
    sem.qcrit_batch(sem.BatchPlan([s for s in snaps if s["x"].shape[0] > 0]))
    return snaps


def _quantiles(f, qs):
    v = f.double().reshape(-1)
    return [float(c) for c in torch.quantile(v, torch.tensor(qs, dtype=torch.float64,
                                                             device=DEV)).cpu()]


def _jobs(snaps):
    jobs = []
    for i, sn in enumerate(snaps):
        if sn["x"].shape[0] == 0:
            jobs.append({"snap": i, "field": "q", "isovalues": [0.0, 1.0]})
            continue
        jobs.append({"snap": i, "field": "q",
                     "isovalues": _quantiles(sn["q"], [0.5, 0.9, 0.99])})
        jobs.append({"snap": i, "field": "omega_mag",
                     "isovalues": _quantiles(sn["omega_mag"], [0.3, 0.7])})
        # four isovalues, one below and one above the whole field
        lo, hi = float(sn["theta"].min()), float(sn["theta"].max())
        jobs.append({"snap": i, "field": sn["theta"],
                     "isovalues": [lo - 1.0, -0.2, 0.4, hi + 1.0]})
    return jobs


def _field(sn, job):
    f = job["field"]
    return sn[f] if isinstance(f, str) else f


@pytest.mark.parametrize("tdt", [torch.float64, torch.float32])
def test_batch_isosurfaces_match_oracle_and_single_calls(tdt):
    snaps = _snaps(tdt)
    jobs = _jobs(snaps)
    plan = sem.IsoBatchPlan(snaps, jobs)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    res = sem.isosurface_batch(plan, status=st, active=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    tri = res["tri_xyz"].cpu().numpy().astype(np.float64)
    cnt, off, act = res["tri_count"].numpy(), res["tri_offset"].numpy(), res["active"].numpy()
    running = 0
    for j, job in enumerate(jobs):
        sn = snaps[job["snap"]]
        iv = job["isovalues"]
        m = len(iv)
        assert (cnt[j, m:] == 0).all()
        if sn["x"].shape[0] == 0:
            assert (cnt[j] == 0).all() and (act[j] == 0).all()
            assert (off[j] == running).all()
            continue
        field = _field(sn, job)
        host = [sn[k].cpu().numpy() for k in ("x", "y", "z")]
        o = mc.extract(*host, field.cpu().numpy(), iv)
        np.testing.assert_array_equal(cnt[j, :m], o["tri_count"], err_msg=str(j))
        np.testing.assert_array_equal(act[j, :m], o["active"], err_msg=str(j))
        lo = off[j, 0]
        assert lo == running
        np.testing.assert_array_equal(off[j, :m], lo + np.concatenate(
            [[0], np.cumsum(o["tri_count"])[:-1]]))
        got = tri[lo:lo + int(cnt[j].sum())]
        scale = max(float(np.abs(h).max()) for h in host)
        if got.size:
            assert np.abs(got - o["tri_xyz"]).max() <= TOL[tdt] * scale, j
        # bit-identical to the single-call path on the same field
        single = sem.isosurface(sn["x"], sn["y"], sn["z"], field, iv)
        np.testing.assert_array_equal(single["tri_count"].cpu().numpy(), cnt[j, :m])
        assert torch.equal(single["tri_xyz"], res["tri_xyz"][lo:lo + int(cnt[j].sum())])
        running += int(cnt[j].sum())
    assert running == tri.shape[0]


def test_batch_isosurfaces_overflow_keeps_counts_exact():
    tdt = torch.float64
    snaps = _snaps(tdt)
    jobs = _jobs(snaps)
    plan = sem.IsoBatchPlan(snaps, jobs)
    full = sem.isosurface_batch(plan)
    total = int(full["tri_count"].sum())
    assert total > 100
    cap = total // 3
    tri = torch.full((cap, 3, 3), float("nan"), dtype=tdt, device=DEV)
    cnt = torch.zeros(4 * len(jobs), dtype=torch.int64, device=DEV)
    off = torch.zeros_like(cnt)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.isosurface_batch_into(plan, tri, cnt, off, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) & sem.SEM_FLAG_TRI_OVERFLOW
    np.testing.assert_array_equal(cnt.view(-1, 4).cpu().numpy(), full["tri_count"].numpy())
    np.testing.assert_array_equal(off.view(-1, 4).cpu().numpy(), full["tri_offset"].numpy())
    assert torch.equal(tri, full["tri_xyz"][:cap])


def test_batch_isosurfaces_graph_replays_match_eager():
    tdt = torch.float32
    snaps = _snaps(tdt)
    live = [s for s in snaps if s["x"].shape[0] > 0]
    qplan = sem.BatchPlan(live)
    jobs = _jobs(snaps)
    plan = sem.IsoBatchPlan(snaps, jobs)
    eager = sem.isosurface_batch(plan)
    total = eager["tri_xyz"].shape[0]
    tri = torch.empty((total, 3, 3), dtype=tdt, device=DEV)
    cnt = torch.zeros(4 * len(jobs), dtype=torch.int64, device=DEV)
    off = torch.zeros_like(cnt)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            sem.qcrit_batch(qplan)
            sem.isosurface_batch_into(plan, tri, cnt, off)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    q_ref = [s["q"].clone() for s in live]
    for rep in range(3):
        for s in live:                       # eager work between the replays
            s["q"].fill_(float("nan"))
            s["omega_mag"].zero_()
        tri.fill_(float("nan"))
        cnt.fill_(-1)
        off.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for s, q in zip(live, q_ref):
            assert torch.equal(s["q"], q), rep
        assert torch.equal(tri, eager["tri_xyz"]), rep
        assert torch.equal(cnt.view(-1, 4).cpu(), eager["tri_count"]), rep
        assert torch.equal(off.view(-1, 4).cpu(), eager["tri_offset"]), rep


def test_batch_isosurface_plan_rejects_bad_jobs():
    tdt = torch.float64
    snaps = _snaps(tdt)[:2]
    bad = [
        [{"snap": 2, "field": "q", "isovalues": [0.1]}],              # no such snapshot
        [{"snap": 0, "field": "q", "isovalues": []}],                 # no isovalue
        [{"snap": 0, "field": "q", "isovalues": [0, 1, 2, 3, 4]}],    # five isovalues
        [{"snap": 0, "field": "q", "isovalues": [float("nan")]}],     # NaN isovalue
    ]
    for jobs in bad:
        with pytest.raises(sem.SemError):
            sem.IsoBatchPlan(snaps, jobs)
    # a field the snapshot does not have
    nq = dict(snaps[0])
    nq["q"] = None
    with pytest.raises(sem.SemError):
        sem.IsoBatchPlan([nq], [{"snap": 0, "field": "q", "isovalues": [0.1]}])
    # precision of the call different from the plan's
    plan = sem.IsoBatchPlan(snaps, [{"snap": 0, "field": "q", "isovalues": [0.1]}])
    plan.dtype_code = sem.SEM_F32
    with pytest.raises(sem.SemError):
        sem.isosurface_batch_into(plan, None, torch.zeros(4, dtype=torch.int64, device=DEV))


def test_batch_isosurfaces_full_size_benchmark_snapshots():
    """The 16 FP32 snapshots of the batched benchmark (orders 5, 7, 9, 4,913
    to 122,451 elements), Q, |omega| and theta at four isovalues each: the
    batched soup equals 48 sem_isosurface calls bit for bit, and the
    triangles of 24 sampled elements of every job equal the oracle's on the
    same field values."""
    snaps, theta = [], []
    for seed in range(16):
        _, arrs = W.batch_snapshot(seed, DEV, dtype=torch.float32)
        x, y, z, u, v, w, th = arrs
        e = x.shape[0]
        snaps.append({"x": x, "y": y, "z": z, "u": u, "v": v, "w": w,
                      "q": torch.empty_like(u), "omega_mag": torch.empty_like(u),
                      "minmax": torch.empty((e, 2), dtype=torch.float32, device=DEV)})
        theta.append(th)
    sem.qcrit_batch(sem.BatchPlan(snaps))
    gen = torch.Generator(device=DEV).manual_seed(0)
    jobs = []
    for i, sn in enumerate(snaps):
        for f in ("q", "omega_mag", theta[i]):
            flat = (sn[f] if isinstance(f, str) else f).reshape(-1)
            idx = torch.randint(0, flat.numel(), (1 << 20,), device=DEV, generator=gen)
            qs = torch.quantile(flat[idx].double(), torch.tensor(
                [0.9, 0.95, 0.99, 0.999], dtype=torch.float64, device=DEV))
            jobs.append({"snap": i, "field": f, "isovalues": [float(c) for c in qs.cpu()]})
    plan = sem.IsoBatchPlan(snaps, jobs)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    res = sem.isosurface_batch(plan, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    cnt, off = res["tri_count"].numpy(), res["tri_offset"].numpy()
    rng = np.random.default_rng(5)
    compared = 0
    for j, job in enumerate(jobs):
        sn = snaps[job["snap"]]
        field = _field(sn, job)
        iv = job["isovalues"]
        single = sem.isosurface(sn["x"], sn["y"], sn["z"], field, iv, edge_keys=True)
        n_j = int(cnt[j].sum())
        np.testing.assert_array_equal(single["tri_count"].cpu().numpy(), cnt[j])
        lo = int(off[j, 0])
        assert torch.equal(single["tri_xyz"], res["tri_xyz"][lo:lo + n_j]), j
        # sampled elements against the oracle: the element of each triangle
        # from its edge keys ((e (N+1)^3 + node) * 3 + axis)
        e_cnt, p = sn["x"].shape[0], sn["x"].shape[1]
        elem = (single["edge_key"][:, 0] // (3 * p ** 3)).cpu().numpy()
        iso_of = np.repeat(np.arange(4), cnt[j])
        pick = np.sort(rng.choice(e_cnt, size=24, replace=False))
        sub = torch.from_numpy(pick).to(DEV)
        host = [sn[k][sub].cpu().numpy() for k in ("x", "y", "z")]
        o = mc.extract(*host, field[sub].cpu().numpy(), iv)
        tri = single["tri_xyz"].cpu().numpy().astype(np.float64)
        for s in range(4):
            mine = tri[(iso_of == s) & np.isin(elem, pick)]
            theirs = o["tri_xyz"][int(o["tri_count"][:s].sum()):int(o["tri_count"][:s + 1].sum())]
            assert mine.shape == theirs.shape, (j, s)
            compared += mine.shape[0]
            if mine.size:
                scale = max(float(np.abs(h).max()) for h in host)
                assert np.abs(mine - theirs).max() <= 1e-5 * scale, (j, s)
    assert compared > 10000, compared
