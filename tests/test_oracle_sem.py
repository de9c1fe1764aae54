"""Pins for the oracle's derivatives, geometry, Q-criterion and |omega|.

Fixed by mathematics: exact differentiation of tensor-product polynomials of
degree <= N, the gradient of the coordinates being the identity on any
isoparametric mesh, exact Q and |omega| of linear fields, algebraic
identities of the velocity-gradient invariants, the closed-form Taylor-Green
vorticity and Q, and spectral convergence in N.
"""

import numpy as np
import pytest

import workloads as W
from oracle import gll, sem


def _affine_box(n, e_shape=(2, 3, 2), lo=(-0.3, 0.2, 1.0), h=(0.7, 0.4, 1.3)):
    b = tuple((lo[a], lo[a] + h[a] * e_shape[a]) for a in range(3))
    return W.box_mesh(e_shape, n, b)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 9])
def test_exact_derivative_of_tensor_polynomials(n):
    x, y, z = _affine_box(n)
    d = gll.diff_matrix(n)
    jinv, det, bad = sem.geometry(x, y, z, d)
    assert not bad.any()
    rng = np.random.default_rng(n)
    for _ in range(6):
        a, b, c = rng.integers(0, n + 1, size=3)
        f = x ** a * y ** b * z ** c
        gx, gy, gz = sem.physical_gradient(f, jinv, d)
        ex = a * x ** max(a - 1, 0) * y ** b * z ** c if a else 0 * x
        ey = b * x ** a * y ** max(b - 1, 0) * z ** c if b else 0 * x
        ez = c * x ** a * y ** b * z ** max(c - 1, 0) if c else 0 * x
        scale = 1 + np.abs(f).max() * n * n
        for got, want in ((gx, ex), (gy, ey), (gz, ez)):
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * scale)


def test_degree_above_n_is_not_exact():
    n = 3
    x, y, z = _affine_box(n)
    (gx, _, _), _ = sem.derivs(x, y, z, x ** (n + 1), gll.diff_matrix(n))
    assert np.max(np.abs(gx - (n + 1) * x ** n)) > 1e-4


@pytest.mark.parametrize("mesh", ["warp", "channel"])
def test_coordinate_gradient_is_identity(mesh):
    n = 7
    if mesh == "warp":
        x, y, z = W.warp(*W.box_mesh((3, 3, 3), n, ((0, 2.0),) * 3), amp=0.1)
    else:
        x, y, z = W.channel_config(n, elements=np.arange(0, 65536, 4093))[:3]
    d = gll.diff_matrix(n)
    jinv, _, bad = sem.geometry(x, y, z, d)
    assert not bad.any()
    for i, c in enumerate((x, y, z)):
        g = sem.physical_gradient(c, jinv, d)
        for j in range(3):
            np.testing.assert_allclose(g[j], 1.0 if i == j else 0.0,
                                       rtol=0, atol=1e-11)


def test_linear_fields_exact_q_and_vorticity():
    n = 5
    x, y, z = W.warp(*W.box_mesh((2, 2, 2), n, ((0, 1.5),) * 3), amp=0.08)
    d = gll.diff_matrix(n)
    # solid-body rotation about z: Q = 1, |omega| = 2
    q, om, bad = sem.qcrit(x, y, z, -y, x, 0 * x, d)
    assert not bad.any()
    np.testing.assert_allclose(q, 1.0, atol=1e-11)
    np.testing.assert_allclose(om, 2.0, atol=1e-11)
    # planar pure strain: Q = -1, |omega| = 0
    q, om, _ = sem.qcrit(x, y, z, x, -y, 0 * x, d)
    np.testing.assert_allclose(q, -1.0, atol=1e-11)
    np.testing.assert_allclose(om, 0.0, atol=1e-6)   # sqrt of rounding noise
    # simple shear u = (y, 0, 0): Q = 0, |omega| = 1
    q, om, _ = sem.qcrit(x, y, z, y, 0 * x, 0 * x, d)
    np.testing.assert_allclose(q, 0.0, atol=1e-11)
    np.testing.assert_allclose(om, 1.0, atol=1e-11)


def test_general_linear_field_invariants():
    """Q = -tr(A^2)/2 and |omega|^2 = |A|_F^2 - tr(A^2) for constant A."""
    n = 4
    x, y, z = W.warp(*W.box_mesh((2, 1, 2), n, ((0, 1.0),) * 3), amp=0.05)
    d = gll.diff_matrix(n)
    rng = np.random.default_rng(7)
    for _ in range(5):
        a = rng.normal(size=(3, 3))
        u, v, w = (a[i, 0] * x + a[i, 1] * y + a[i, 2] * z for i in range(3))
        q, om, _ = sem.qcrit(x, y, z, u, v, w, d)
        tr_a2 = np.trace(a @ a)
        np.testing.assert_allclose(q, -0.5 * tr_a2, atol=1e-10)
        np.testing.assert_allclose(om ** 2, np.sum(a * a) - tr_a2, atol=1e-9)


def _tgv_closed(x, y, z):
    q = -0.5 * np.cos(z) ** 2 * (np.cos(2 * x) + np.cos(2 * y))
    w1 = -np.cos(x) * np.sin(y) * np.sin(z)
    w2 = -np.sin(x) * np.cos(y) * np.sin(z)
    w3 = 2 * np.sin(x) * np.sin(y) * np.cos(z)
    return q, np.sqrt(w1 * w1 + w2 * w2 + w3 * w3)


def test_taylor_green_closed_form_and_spectral_convergence():
    errs = {}
    for n in (5, 7, 9):
        x, y, z, u, v, w = W.tgv_config(n)
        q, om, bad = sem.qcrit(x, y, z, u, v, w, gll.diff_matrix(n))
        assert not bad.any()
        qc, omc = _tgv_closed(x, y, z)
        errs[n] = (np.abs(q - qc).max(), np.abs(om - omc).max())
    assert errs[7][0] < 1e-6 and errs[7][1] < 1e-6
    for a, b in ((5, 7), (7, 9)):
        assert errs[a][0] / errs[b][0] > 100
        assert errs[a][1] / errs[b][1] > 100


def test_taylor_green_is_divergence_free_and_q_symmetric():
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    a, _ = sem.velocity_gradient(x, y, z, u, v, w, gll.diff_matrix(n))
    assert np.abs(a[0, 0] + a[1, 1] + a[2, 2]).max() < 1e-7


def test_inverted_element_is_flagged():
    n = 3
    x, y, z = _affine_box(n, e_shape=(2, 1, 1))
    x = x.copy()
    x[1] = x[1, :, :, ::-1]          # mirror element 1 along r: det J < 0
    _, det, bad = sem.geometry(x, y, z, gll.diff_matrix(n))
    assert not bad[0].any() and bad[1].all()
    assert (det[1] < 0).all()


def test_elem_minmax_treats_nan_as_below():
    f = np.arange(16.0).reshape(2, 2, 2, 2)
    f[0, 0, 0, 0] = np.nan
    mm = sem.elem_minmax(f)
    assert mm[0, 0] == -np.inf and mm[0, 1] == 7.0
    assert mm[1, 0] == 8.0 and mm[1, 1] == 15.0
