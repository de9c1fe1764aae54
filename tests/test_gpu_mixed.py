"""GPU: mixed-precision modes (FP32 storage, BF16/FP16 matrix-core contractions).

Error bars follow from the operand formats.  Rounding to a p-bit significand
has unit roundoff u = 2^-p (BF16: p = 8, FP16: p = 11), so a product of two
rounded operands is off by at most about 2u relative.  The split forms write
x = hi + lo and keep hi*hi, lo*hi and hi*lo, leaving about 3u^2; FP32
accumulation and the FP32 chain rule add about 2^-22.  A line derivative
sums eight products D_im (f_m - f_0); on these smooth fields the sum of
their magnitudes stays within 32x the derivative's scale, so derivatives are
checked normwise against 32 u_eff and Q (quadratic in the gradient) against
64 u_eff.  The oracle gets the same FP32 inputs widened exactly to FP64, so
only the method's rounding is measured.  Errors are printed for the record.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gll, mc, sem as osem

torch = pytest.importorskip("torch")
import paper_2312_09888_amd as sem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
F32_FLOOR = 2.0 ** -22
U_EFF = {
    "bf16": 2 * 2.0 ** -8 + F32_FLOOR,
    "fp16": 2 * 2.0 ** -11 + F32_FLOOR,
    "bf16x3": 3 * 2.0 ** -16 + F32_FLOOR,
    "fp16x3": 3 * 2.0 ** -22 + F32_FLOOR,
}
MODES = list(U_EFF)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(DEV)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _f32(arrs):
    return [np.asarray(a, dtype=np.float32) for a in arrs]


def _oracle_q(arrs32, n=7):
    return osem.qcrit(*(a.astype(np.float64) for a in arrs32), gll.diff_matrix(n))


def _mixed_q(arrs32, mode):
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    q, om, mm = sem.qcrit(*(dev(a) for a in arrs32), status=st, precision=mode)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return q, om, mm


@pytest.mark.parametrize("mode", MODES)
def test_mixed_qcrit_taylor_green_within_bound(mode):
    arrs = _f32(W.tgv_config(7))
    oq, oom, _ = _oracle_q(arrs)
    q, om, mm = _mixed_q(arrs, mode)
    hq, hom = host(q), host(om)
    eq, eom = normwise(hq, oq), normwise(hom, oom)
    print(f"\n[{mode}] TGV Q: max-abs {np.abs(hq - oq).max():.3e} normwise {eq:.3e} "
          f"rel-L2 {rel_l2(hq, oq):.3e}; |omega|: max-abs {np.abs(hom - oom).max():.3e} "
          f"normwise {eom:.3e} rel-L2 {rel_l2(hom, oom):.3e}")
    assert eq <= 64 * U_EFF[mode], eq
    assert eom <= 64 * U_EFF[mode], eom
    # element ranges are those of the kernel's own Q, exactly
    np.testing.assert_array_equal(host(mm), osem.elem_minmax(hq))


@pytest.mark.parametrize("mode", MODES)
def test_mixed_qcrit_channel_sample_within_bound(mode):
    els = np.arange(0, 65536, 331)
    arrs = _f32(W.channel_config(7, elements=els))
    oq, oom, _ = _oracle_q(arrs)
    q, om, _ = _mixed_q(arrs, mode)
    eq, eom = normwise(host(q), oq), normwise(host(om), oom)
    print(f"\n[{mode}] channel sample Q normwise {eq:.3e} rel-L2 {rel_l2(host(q), oq):.3e}; "
          f"|omega| normwise {eom:.3e}")
    assert eq <= 64 * U_EFF[mode], eq
    assert eom <= 64 * U_EFF[mode], eom


@pytest.mark.parametrize("mode", MODES)
def test_mixed_derivs_polynomial_within_bound(mode):
    n = 7
    x, y, z = W.box_mesh((3, 2, 2), n, ((0.0, 1.5), (0.5, 1.3), (-1.0, 0.2)))
    x, y, z = _f32((x, y, z))
    X, Y, Z = (a.astype(np.float64) for a in (x, y, z))
    f = (X ** 7 * Y ** 2 * Z ** 5 + 3 * X * Y * Z).astype(np.float32)
    g = sem.derivs(dev(x), dev(y), dev(z), dev(f), precision=mode)
    want = (7 * X ** 6 * Y ** 2 * Z ** 5 + 3 * Y * Z,
            2 * X ** 7 * Y * Z ** 5 + 3 * X * Z,
            5 * X ** 7 * Y ** 2 * Z ** 4 + 3 * X * Y)
    # the oracle differentiates the FP32-rounded samples exactly as well
    od, _ = osem.derivs(X, Y, Z, f.astype(np.float64), gll.diff_matrix(n))
    for got, w, o in zip(g, want, od):
        e = normwise(host(got), o)
        assert e <= 32 * U_EFF[mode], (mode, e)
        assert normwise(o, w) < 1e-5     # FP32 sampling of a degree-7 polynomial


def test_mixed_error_ordering():
    arrs = _f32(W.tgv_config(7))
    oq, _, _ = _oracle_q(arrs)
    err = {m: rel_l2(host(_mixed_q(arrs, m)[0]), oq) for m in MODES}
    print("\nrel-L2 error of Q by mode:", {k: f"{v:.2e}" for k, v in err.items()})
    assert err["fp16x3"] < err["bf16x3"] < err["fp16"] < err["bf16"]


def _band_mismatch(cases_gpu, cases_ref, q_ref, c, band, n=7):
    p = n + 1
    e = q_ref.shape[0]
    near = (np.abs(q_ref - c) <= band).reshape(e, p, p, p)
    cell_near = np.zeros((e, n, n, n), dtype=bool)
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                cell_near |= near[:, cc:cc + n, b:b + n, a:a + n]
    bad = cases_gpu.reshape(e, -1) != cases_ref.reshape(e, -1)
    assert not np.any(bad & ~cell_near.reshape(e, -1))
    return int(bad.sum())


@pytest.mark.parametrize("mode", MODES)
def test_mixed_taylor_green_case_and_count_mismatch(mode):
    c = 0.1
    arrs = _f32(W.tgv_config(7))
    oq, _, _ = _oracle_q(arrs)
    t = [dev(a) for a in arrs]
    q, _, mm = sem.qcrit(*t, precision=mode)
    r = sem.isosurface(t[0], t[1], t[2], q, [c], minmax=mm, cases=True)
    o = mc.extract(*(a.astype(np.float64) for a in arrs[:3]), oq, [c])
    hq = host(q)
    band = np.abs(hq - oq).max() + abs(float(np.float32(c)) - c)
    mism = _band_mismatch(host(r["cases"])[0], o["cases"][0], oq, c, band)
    cells = o["cases"][0].size
    tri_g, tri_o = int(host(r["tri_count"])[0]), int(o["tri_count"][0])
    print(f"\n[{mode}] case mismatches {mism} of {cells} cells ({mism / cells:.2e}); "
          f"triangles {tri_g} vs {tri_o} ({abs(tri_g - tri_o) / tri_o:.2e})")
    margin = np.abs(oq - c).min()
    if margin > band:       # no node near enough to the isovalue to flip
        assert mism == 0 and tri_g == tri_o
    # stage-isolated: the isosurface of the kernel's own Q is exact
    o2 = mc.extract(*(a.astype(np.float64) for a in arrs[:3]), hq.astype(np.float32), [c])
    np.testing.assert_array_equal(host(r["cases"])[0], o2["cases"][0])
    assert int(host(r["tri_count"])[0]) == int(o2["tri_count"][0])


@pytest.mark.parametrize("mode", ["bf16x3", "fp16"])
def test_mixed_extract_equals_qcrit_then_isosurface(mode):
    arrs = _f32(W.tgv_config(7, shape=(4, 3, 2)))
    t = [dev(a) for a in arrs]
    isos = [0.02, 0.05, 0.1, 0.2, 0.3, 0.4]   # counted four at a time: 4 + 2
    r = sem.extract(*t, isos, precision=mode)
    q, _, mm = sem.qcrit(*t, precision=mode)
    assert torch.equal(r["q"], q)
    for s, c in enumerate(isos):
        one = sem.isosurface(t[0], t[1], t[2], q, [c], minmax=mm)
        assert torch.equal(r["tri"][s], one["tri_xyz"])


def test_mixed_flags_inverted_element():
    arrs = _f32(W.tgv_config(7, shape=(2, 2, 2)))
    x = arrs[0].copy()
    x[3] = x[3][:, :, ::-1]          # mirror one element: det J < 0
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    sem.qcrit(dev(x), *(dev(a) for a in arrs[1:]), status=st, precision="bf16x3")
    assert int(st.item()) & sem.SEM_FLAG_BAD_JACOBIAN


def test_mixed_rejects_other_orders_and_dtypes():
    x = torch.zeros((2, 6, 6, 6), dtype=torch.float32, device=DEV)
    with pytest.raises(sem.SemError):
        sem.qcrit(x, x, x, x, x, x, precision="bf16")
    xd = torch.zeros((2, 8, 8, 8), dtype=torch.float64, device=DEV)
    with pytest.raises(TypeError):
        sem.qcrit(xd, xd, xd, xd, xd, xd, precision="bf16")
