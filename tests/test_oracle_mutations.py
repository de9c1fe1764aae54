"""Planted mistakes: each plausible error in the oracle must fail a pin.

Every case patches one oracle function with a realistic slip (transposed
operand, dropped term, wrong sign or index, inconsistent face rule), runs
the relevant pin check on the CPU and expects it to fail.  The patches are
undone after each case.
"""

import contextlib

import numpy as np
import pytest

import workloads as W
from oracle import gll, mc, sem


@contextlib.contextmanager
def patched(mod, name, fn):
    old = getattr(mod, name)
    setattr(mod, name, fn)
    try:
        yield
    finally:
        setattr(mod, name, old)


def _fails(check):
    with pytest.raises(AssertionError):
        check()


# --------------------------------------------------------------------------
# pin checks (the same statements as the pin tests, at small sizes)
# --------------------------------------------------------------------------

def pin_polynomial():
    n = 4
    x, y, z = W.box_mesh((2, 1, 2), n, ((0.0, 1.3), (0.2, 0.9), (-0.5, 0.7)))
    d = gll.diff_matrix(n)
    f = x ** 3 * y ** 2 * z ** 4
    (gx, gy, gz), _ = sem.derivs(x, y, z, f, d)
    assert np.allclose(gx, 3 * x ** 2 * y ** 2 * z ** 4, atol=1e-10)
    assert np.allclose(gy, 2 * x ** 3 * y * z ** 4, atol=1e-10)
    assert np.allclose(gz, 4 * x ** 3 * y ** 2 * z ** 3, atol=1e-10)


def pin_coordinate_identity():
    n = 5
    x, y, z = W.warp(*W.box_mesh((2, 2, 2), n, ((0, 2.0),) * 3), amp=0.1)
    d = gll.diff_matrix(n)
    jinv, _, _ = sem.geometry(x, y, z, d)
    for i, c in enumerate((x, y, z)):
        g = sem.physical_gradient(c, jinv, d)
        for j in range(3):
            assert np.allclose(g[j], 1.0 if i == j else 0.0, atol=1e-10)


def pin_linear_fields():
    n = 3
    x, y, z = W.warp(*W.box_mesh((2, 1, 1), n, ((0, 1.5),) * 3), amp=0.08)
    d = gll.diff_matrix(n)
    q, om, _ = sem.qcrit(x, y, z, -y, x, 0 * x, d)
    assert np.allclose(q, 1.0, atol=1e-10) and np.allclose(om, 2.0, atol=1e-10)
    q, om, _ = sem.qcrit(x, y, z, y, 0 * x, 0 * x, d)
    assert np.allclose(q, 0.0, atol=1e-10) and np.allclose(om, 1.0, atol=1e-10)
    rng = np.random.default_rng(0)
    a = rng.normal(size=(3, 3))
    u, v, w = (a[i, 0] * x + a[i, 1] * y + a[i, 2] * z for i in range(3))
    q, om, _ = sem.qcrit(x, y, z, u, v, w, d)
    assert np.allclose(q, -0.5 * np.trace(a @ a), atol=1e-9)
    assert np.allclose(om ** 2, np.sum(a * a) - np.trace(a @ a), atol=1e-8)


def pin_case_table():
    mc._TABLE = None
    ntri, table = mc.case_table()
    for c in range(256):
        bit = [(c >> v) & 1 for v in range(8)]
        crossed = sum(bit[mc.EDGE_CORNERS[e][0]] != bit[mc.EDGE_CORNERS[e][1]]
                      for e in range(12))
        assert ntri[c] == crossed - 2 * len(mc.case_loops(c))


def pin_watertight_1x1x2():
    import test_oracle_mc as T
    mc._TABLE = None
    dims = (1, 1, 2)
    pats = np.arange(2 ** 12, dtype=np.int64)
    bits = (pats[:, None] >> np.arange(12)) & 1
    vals = np.where(bits == 1, 1.0, -1.0).reshape(-1, 3, 2, 2)
    x, y, z, f, origin = T._grid_elements(dims, vals)
    r = mc.extract(x, y, z, f, [0.0], edge_keys=True)
    gid, _ = T._global_vertex_ids(r["edge_key"].astype(np.int64), origin, dims, 2)
    T._check_watertight(gid, T._boundary_fn(T._planes_factory(dims, 1)))


def pin_sphere_outward():
    import test_oracle_mc as T
    mc._TABLE = None
    r, _ = T._sphere(4)
    p = r["tri_xyz"]
    vol = np.sum(np.einsum("ti,ti->t", p[:, 0], np.cross(p[:, 1], p[:, 2]))) / 6.0
    assert vol > 0


def pin_ties():
    f = np.zeros((1, 2, 2, 2))
    f[0, 0, 0, 0] = 0.5
    assert mc.classify(f, 0.5)[0, 0, 0, 0] == 0      # f == c is not above


@pytest.fixture(autouse=True)
def _fresh_table():
    mc._TABLE = None
    yield
    mc._TABLE = None


def test_pins_pass_unmutated():
    for check in (pin_polynomial, pin_coordinate_identity, pin_linear_fields, pin_case_table,
                  pin_watertight_1x1x2, pin_sphere_outward, pin_ties):
        check()


def test_transposed_derivative_matrix_is_caught():
    orig = gll.diff_matrix
    with patched(gll, "diff_matrix", lambda n, xi=None: orig(n, xi).T.copy()):
        _fails(pin_polynomial)


def test_wrong_contraction_index_is_caught():
    orig = sem.ref_derivs

    def bad(f, d):
        fr, _, ft = orig(f, d)
        fs = np.einsum("mj,ekmi->ekji", d, f)   # contracts D's first index
        return fr, fs, ft
    with patched(sem, "ref_derivs", bad):
        _fails(pin_polynomial)
    # (swapping s and t everywhere is a relabelling of the reference
    # coordinates and leaves every physical result unchanged -- not a slip)


def test_transposed_jacobian_inverse_is_caught():
    orig = sem.inverse3

    def bad(m):
        inv, det = orig(m)
        return np.swapaxes(inv, 0, 1), det
    with patched(sem, "inverse3", bad):
        _fails(pin_coordinate_identity)


def test_dropped_chain_rule_term_is_caught():
    def bad(f, jinv, d):
        fr, fs, ft = sem.ref_derivs(f, d)
        return tuple(fr * jinv[0, b] + fs * jinv[1, b] for b in range(3))
    with patched(sem, "physical_gradient", bad):
        _fails(pin_coordinate_identity)


def test_q_sign_and_vorticity_index_are_caught():
    def bad_sign(a):
        q, om = (lambda qq: qq)(orig(a))
        return -q, om
    orig = sem.q_and_vorticity
    with patched(sem, "q_and_vorticity", bad_sign):
        _fails(pin_linear_fields)

    def bad_omega(a):
        q, _ = orig(a)
        w1 = a[2, 1] - a[1, 2]
        w2 = a[0, 2] - a[2, 0]
        w3 = a[1, 0] + a[0, 1]      # wrong sign
        return q, np.sqrt(w1 * w1 + w2 * w2 + w3 * w3)
    with patched(sem, "q_and_vorticity", bad_omega):
        _fails(pin_linear_fields)

    def bad_q(a):
        at = np.swapaxes(a, 0, 1)
        s = 0.5 * (a + at)
        om = 0.5 * (a - a)          # rotation part lost
        q = 0.5 * (np.sum(om * om, axis=(0, 1)) - np.sum(s * s, axis=(0, 1)))
        return q, orig(a)[1]
    with patched(sem, "q_and_vorticity", bad_q):
        _fails(pin_linear_fields)


def test_smallest_edge_fan_start_is_caught():
    with patched(mc, "fan_start", lambda loop: 0):
        _fails(pin_watertight_1x1x2)


def test_face_inconsistent_ambiguity_is_caught():
    orig = mc.face_segments

    def bad(case):
        segs = orig(case)
        # resolve ambiguous faces the other way on the z = 1 face only
        bit = [(case >> v) & 1 for v in range(8)]
        _, _, corners, edges, normal = mc.FACES[5]
        crossed = [e for e in edges if bit[mc.EDGE_CORNERS[e][0]] != bit[mc.EDGE_CORNERS[e][1]]]
        if len(crossed) != 4:
            return segs
        segs = [sg for sg in segs if not (sg[0] in edges and sg[1] in edges)]
        below = [v for v in corners if not bit[v]]
        for v in below:
            inc = [e for e in crossed if v in mc.EDGE_CORNERS[e]]
            p1, p2 = mc._edge_mid(inc[0]), mc._edge_mid(inc[1])
            left = np.cross(normal, p2 - p1)
            side = np.dot(left, mc.CORNER_POS[v] - p1)
            segs.append((inc[1], inc[0]) if side > 0 else (inc[0], inc[1]))
        return segs
    with patched(mc, "face_segments", bad):
        _fails(pin_watertight_1x1x2)


def test_reversed_orientation_is_caught():
    orig = mc.case_triangles

    def bad(case):
        return [(a, c, b) for a, b, c in orig(case)]
    with patched(mc, "case_triangles", bad):
        _fails(pin_sphere_outward)


def test_non_strict_comparison_is_caught():
    def bad(field, iso):
        field = np.asarray(field)
        return field >= field.dtype.type(iso)
    with patched(mc, "above", bad):
        _fails(pin_ties)


# --------------------------------------------------------------------------
# C0 averaging and welding (oracle/c0.py)
# --------------------------------------------------------------------------

def test_vertex_measured_from_the_high_end_is_caught():
    import test_oracle_mc as T

    def from_high(x0, x1, f0, f1, c):
        t = (c - f0) / (f1 - f0)
        return x1 + t * (x0 - x1)              # t taken from the high corner
    with patched(mc, "edge_vertex", from_high):
        _fails(T._plane_pin)


def test_c0_sum_without_division_is_caught():
    import test_oracle_c0 as T
    from oracle import c0

    def bad(field, gid):
        f = np.asarray(field)
        g = np.asarray(gid).ravel()
        s = np.zeros(int(g.max()) + 1, dtype=f.dtype)
        np.add.at(s, g, f.ravel())
        return s[g].reshape(f.shape)             # dssum, not the average
    with patched(c0, "dsavg", bad):
        _fails(T.test_two_element_example_exact)


def test_element_local_keys_break_the_weld():
    import test_oracle_c0 as T
    from oracle import c0

    def bad(local_keys, gid, order):
        return np.asarray(local_keys, dtype=np.uint64)   # ids of the element copy
    with patched(c0, "global_edge_keys", bad):
        _fails(T.test_welded_sphere_is_closed_manifold_across_elements)


def test_last_occurrence_weld_is_caught():
    import test_oracle_c0 as T
    from oracle import c0
    orig = c0.weld

    def bad(tri_xyz, keys):
        v, i = orig(tri_xyz, keys)
        return v[::-1].copy(), (v.shape[0] - 1 - i)      # reversed vertex order
    with patched(c0, "weld", bad):
        _fails(T.test_welded_sphere_is_closed_manifold_across_elements)


# --------------------------------------------------------------------------
# compression network, optimiser, fallback and baseline (oracle/ae.py)
# --------------------------------------------------------------------------

def test_wrong_tanh_derivative_is_caught():
    import test_oracle_ae as T
    from oracle import ae
    orig = ae.gradient

    def bad(params, x, quantize=True, tanh_mask=ae.TANH_NONE):
        # 1 - y instead of 1 - y^2 in the backward pass
        x = np.asarray(x, dtype=np.float64)
        acts = ae.forward(params, x, quantize, tanh_mask)
        layers = ae.unpack(params)
        g = 2.0 * (acts[-1] - x) / x.size
        grads = [None] * len(ae.ARCH)
        for l in range(len(ae.ARCH) - 1, -1, -1):
            kind = ae.ARCH[l][0]
            if (tanh_mask >> l) & 1:
                g = g * (1.0 - acts[l + 1])
            gx, gw, gb = (ae.conv_grads if kind == "conv" else ae.conv_t_grads)(
                acts[l], layers[l][0], g)
            grads[l] = (gw, gb)
            g = gx
        return ae.loss(acts[-1], x), ae.pack(grads)
    assert orig is not bad
    with patched(ae, "gradient", bad):
        _fails(lambda: T.test_gradient_matches_central_differences(ae.TANH_HIDDEN))


def test_flipped_kernel_offset_in_conv_t_is_caught():
    import test_oracle_ae as T
    from oracle import ae

    def bad(x, w, b):
        y = np.empty((x.shape[0], w.shape[1]) + tuple(2 * s for s in x.shape[2:]))
        for dz, dy, dx in ae._delta():
            # kernel tap (dx, dy, dz) instead of (dz, dy, dx)
            y[:, :, dz::2, dy::2, dx::2] = np.einsum("io,bizyx->bozyx", w[:, :, dx, dy, dz], x)
        return y + b[None, :, None, None, None]
    with patched(ae, "conv_t", bad):
        _fails(T.test_conv_t_impulse_response)
        _fails(T.test_conv_t_is_the_adjoint_of_conv)


def test_adam_without_bias_correction_is_caught():
    import test_oracle_ae as T
    from oracle import ae

    def bad(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        g = np.asarray(grad, dtype=np.float64)
        m = beta1 * np.asarray(m) + (1.0 - beta1) * g
        v = beta2 * np.asarray(v) + (1.0 - beta2) * g * g
        return np.asarray(params) - lr * m / (np.sqrt(v) + eps), m, v
    with patched(ae, "adam", bad):
        _fails(T.test_adam_constant_gradient_closed_form)


def test_fallback_without_floor_is_caught():
    import test_oracle_ae as T
    from oracle import ae

    def bad(fields, recon, gmax):
        f = np.stack([np.asarray(a) for a in fields], axis=1)
        r = np.stack([np.asarray(a) for a in recon], axis=1)
        s = np.abs(f).max(axis=(2, 3, 4))
        err = np.abs(f - r).max(axis=(2, 3, 4))
        return np.any(err > 1e-3 * s, axis=1)          # no floor
    with patched(ae, "fallback", bad):
        _fails(T.test_fallback_rule_at_its_boundary)


def test_total_degree_truncation_is_caught():
    import test_oracle_ae as T
    from oracle import ae
    orig = ae.modal_truncate

    def bad(fields, quantize=True):
        r, keep = orig(fields, quantize)
        # total degree <= 1 (4 modes) instead of every degree <= 1 (8 modes)
        k = keep.copy()
        k[:, :, 1, 1, :] = 0
        k[:, :, 1, :, 1] = 0
        k[:, :, :, 1, 1] = 0
        v2 = ae.legendre_vandermonde()[:, :2]
        return np.einsum("ka,lb,mc,xyabc->xyklm", v2, v2, v2, k), k
    with patched(ae, "modal_truncate", bad):
        _fails(T.test_modal_truncation_keeps_its_span_and_drops_higher_modes)


def test_pca_init_with_trailing_eigenvectors_is_caught():
    import test_oracle_ae as T
    from oracle import ae

    def bad(c, r):
        lam, u = np.linalg.eigh(c)
        return lam[:r], u[:, :r]                        # smallest, not largest
    with patched(ae, "_leading_eigvecs", bad):
        _fails(T.test_pca_init_is_exact_on_data_of_low_rank)


def _max_loss_gradient(factor, split):
    """The max-error loss gradient with a planted slip: a scale `factor`
    on 2 m sign(d), and tied maxima either shared (`split`) or each given
    the full amount."""
    from oracle import ae

    def bad(out, x, kind=ae.LOSS_MSE):
        d = out - np.asarray(x, dtype=np.float64)
        if kind != ae.LOSS_MAX:
            return 2.0 * d / d.size
        a = np.abs(d).reshape(d.shape[0], ae.CHANNELS, -1)
        m = a.max(axis=2, keepdims=True)
        top = (a == m) & (m > 0)
        ties = np.maximum(top.sum(axis=2, keepdims=True), 1) if split else 1
        g = np.where(top, factor * m * np.sign(d.reshape(a.shape))
                     / (d.shape[0] * ae.CHANNELS) / ties, 0.0)
        return g.reshape(d.shape)
    return bad


def test_max_loss_gradient_without_the_factor_two_is_caught():
    import test_oracle_ae as T
    from oracle import ae
    with patched(ae, "loss_gradient", _max_loss_gradient(1.0, True)):
        _fails(T.test_max_loss_gradient_matches_central_differences)


def test_max_loss_gradient_with_flipped_sign_is_caught():
    import test_oracle_ae as T
    from oracle import ae
    with patched(ae, "loss_gradient", _max_loss_gradient(-2.0, True)):
        _fails(T.test_max_loss_gradient_matches_central_differences)


def test_max_loss_gradient_without_the_tie_split_is_caught():
    import test_oracle_ae as T
    from oracle import ae
    with patched(ae, "loss_gradient", _max_loss_gradient(2.0, False)):
        _fails(T.test_max_loss_closed_form_and_tie_split)
    # the unplanted form passes both pins
    with patched(ae, "loss_gradient", _max_loss_gradient(2.0, True)):
        T.test_max_loss_closed_form_and_tie_split()
        T.test_max_loss_gradient_matches_central_differences()
