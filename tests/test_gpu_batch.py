"""GPU: batched snapshots (one persistent launch per order over many snapshots).

Every snapshot of a batch -- different orders, uneven element counts --
must give sem_qcrit's definition: Q and |omega| within 1e-10 (FP64) / 1e-5
(FP32) normwise of the CPU oracle, element ranges exactly those of the
kernel's own Q.  The plan can be captured in a HIP graph: every replay, with
eager work between replays, must reproduce the eager result bit for bit.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gll
from oracle import sem as osem

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {np.float64: 1e-10, np.float32: 1e-5}
TDT = {np.float64: torch.float64, np.float32: torch.float32}


def _snapshot(n, shape, seed, dt):
    x, y, z = W.box_mesh(shape, n, ((0.0, 1.7), (-0.4, 0.9), (0.2, 1.4)))
    x, y, z = W.warp(x, y, z, amp=0.05)
    rng = np.random.default_rng(seed)
    vel = []
    for _ in range(3):
        k = rng.uniform(0.5, 3.0, size=(3, 3))
        ph = rng.uniform(0, 6.28, size=3)
        vel.append(sum(np.sin(k[m, 0] * x + k[m, 1] * y + k[m, 2] * z + ph[m])
                       for m in range(3)))
    return [np.asarray(a, dtype=dt) for a in (x, y, z, *vel)]


def _batch(dt, specs):
    snaps, host = [], []
    for n, shape, seed in specs:
        arrs = _snapshot(n, shape, seed, dt)
        t = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]
        e = t[0].shape[0]
        snaps.append({"x": t[0], "y": t[1], "z": t[2], "u": t[3], "v": t[4], "w": t[5],
                      "q": torch.full_like(t[3], np.nan), "omega_mag": torch.empty_like(t[3]),
                      "minmax": torch.empty((e, 2), dtype=TDT[dt], device=DEV)})
        host.append((n, arrs))
    return snaps, host


SPECS = [(2, (3, 2, 1), 1), (5, (4, 3, 3), 2), (7, (3, 3, 1), 3), (9, (2, 2, 2), 4),
         (1, (5, 1, 1), 5), (6, (1, 1, 1), 6)]


def _check(snaps, host, dt):
    for sn, (n, arrs) in zip(snaps, host):
        a64 = [a.astype(np.float64) for a in arrs]
        oq, oom, _ = osem.qcrit(*a64, gll.diff_matrix(n))
        hq = sn["q"].cpu().numpy().astype(np.float64)
        assert np.abs(hq - oq).max() / np.abs(oq).max() < TOL[dt], n
        hom = sn["omega_mag"].cpu().numpy().astype(np.float64)
        assert np.abs(hom - oom).max() / np.abs(oom).max() < TOL[dt], n
        np.testing.assert_array_equal(sn["minmax"].cpu().numpy(),
                                      osem.elem_minmax(sn["q"].cpu().numpy()))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_batch_matches_oracle_mixed_orders(dt):
    snaps, host = _batch(dt, SPECS)
    plan = sem.BatchPlan(snaps)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.qcrit_batch(plan, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _check(snaps, host, dt)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_autotune_then_ragged_chunks(dt):
    code = sem.SEM_F64 if dt == np.float64 else sem.SEM_F32
    for n in (3, 5, 7, 9):
        var, ms = sem.autotune(n, code)
        assert 0 <= var < sem.BATCH_VARIANTS and ms[var] > 0
        assert ms[var] == min(m for m in ms if m > 0)
        assert ms[0] > 0 and ms[3] > 0 and ms[5] > 0
        assert (ms[4] > 0) == (n == 7 and dt == np.float64)
        assert sem.batch_variant(n, code) == var
    # element counts that are not multiples of any chunk
    snaps, host = _batch(dt, [(3, (7, 1, 1), 11), (5, (3, 3, 1), 12), (7, (5, 1, 1), 13)])
    plan = sem.BatchPlan(snaps)
    sem.qcrit_batch(plan)
    torch.cuda.synchronize()
    _check(snaps, host, dt)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_every_variant_matches_oracle(dt, variant):
    code = sem.SEM_F64 if dt == np.float64 else sem.SEM_F32
    # the last snapshot is one order-9 element spanning the whole box, the
    # largest element (and the largest FP32 rounding of its line sums) here
    specs = [(2, (5, 1, 1), 31), (4, (3, 2, 1), 32), (5, (3, 1, 1), 33), (7, (3, 1, 1), 34),
             (8, (2, 1, 1), 35), (9, (2, 2, 1), 36), (9, (1, 1, 1), 37)]
    default = {n: sem.batch_variant(n, code) for n, _, _ in specs}
    for n, _, _ in specs:
        try:
            sem.batch_set_variant(n, code, variant)
        except sem.SemError:
            sem.batch_set_variant(n, code, 0)      # not applicable to this order
    try:
        snaps, host = _batch(dt, specs)
        plan = sem.BatchPlan(snaps)
        st = torch.zeros(1, dtype=torch.int32, device=DEV)
        sem.qcrit_batch(plan, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        _check(snaps, host, dt)
    finally:
        for n, v in default.items():
            sem.batch_set_variant(n, code, v)


@pytest.mark.parametrize("n", [4, 7, 9])
def test_empty_snapshot_and_bad_jacobian(n):
    dt = np.float64
    snaps, host = _batch(dt, [(n, (2, 1, 1), 21), (n, (2, 2, 1), 22), (3, (1, 1, 1), 23)])
    empty = {k: (v[:0] if v is not None else None) for k, v in snaps[0].items()}
    x = snaps[1]["x"]
    x[1] = torch.flip(x[1], dims=[2])        # inverted element in the second snapshot
    plan = sem.BatchPlan([snaps[0], empty, snaps[1], snaps[2]])
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.qcrit_batch(plan, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) & sem.SEM_FLAG_BAD_JACOBIAN
    _check([snaps[0], snaps[2]], [host[0], host[2]], dt)


def test_batch_equals_per_snapshot_kernels_bitwise():
    """With the default forms the batch runs the per-element bodies of
    sem_qcrit's own kernels: results are identical bit for bit."""
    for dt in (np.float64, np.float32):
        code = sem.SEM_F64 if dt == np.float64 else sem.SEM_F32
        specs = [(5, (3, 2, 1), 41), (7, (3, 3, 1), 42), (9, (2, 2, 1), 43), (7, (1, 2, 1), 44)]
        default = {n: sem.batch_variant(n, code) for n, _, _ in specs}
        try:
            for n in default:
                sem.batch_set_variant(n, code, 4 if (n == 7 and dt == np.float64)
                                      else 3 if (n <= 7 or dt == np.float32) else 5)
            snaps, _ = _batch(dt, specs)
            sem.qcrit_batch(sem.BatchPlan(snaps))
            for sn in snaps:
                q, om, mm = sem.qcrit(sn["x"], sn["y"], sn["z"], sn["u"], sn["v"], sn["w"])
                assert torch.equal(q, sn["q"]) and torch.equal(om, sn["omega_mag"])
                assert torch.equal(mm, sn["minmax"])
        finally:
            for n, v in default.items():
                sem.batch_set_variant(n, code, v)


def test_batch_graph_replays_match_eager():
    dt = np.float32
    snaps, host = _batch(dt, SPECS)
    plan = sem.BatchPlan(snaps)
    sem.qcrit_batch(plan)
    torch.cuda.synchronize()
    eager = [(s["q"].clone(), s["omega_mag"].clone(), s["minmax"].clone()) for s in snaps]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            sem.qcrit_batch(plan)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for s in snaps:                      # eager work between the replays
            s["q"].fill_(float("nan"))
            s["omega_mag"].zero_()
            s["minmax"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for s, (q, om, mm) in zip(snaps, eager):
            assert torch.equal(s["q"], q), rep
            assert torch.equal(s["omega_mag"], om), rep
            assert torch.equal(s["minmax"], mm), rep
    _check(snaps, host, dt)
