"""Pins of the compression oracle (oracle/ae.py) against facts that do not
come from the oracle itself: impulse responses and adjointness of the
(transposed) convolutions, central finite differences of the loss, the
closed form of Adam under a constant gradient, binary16 rounding of values
whose correct rounding is known, exactness of the modal truncation on its
own span and its orthogonality to higher Legendre modes, and the fallback
rule at its boundary."""

import numpy as np
import pytest

from oracle import ae, gll

RNG = np.random.default_rng(2024)


def _one_layer(kind, cin, cout):
    shape = (cout, cin, 2, 2, 2) if kind == "conv" else (cin, cout, 2, 2, 2)
    return RNG.normal(size=shape), RNG.normal(size=cout)


def test_parameter_count_and_layout():
    assert ae.param_count() == (4 * 32 * 8 + 32) + (32 * 64 * 8 + 64) + (64 * 32 * 8 + 32) \
        + (32 * 64 * 8 + 64) + (64 * 32 * 8 + 32) + (32 * 4 * 8 + 4) == 67812
    p = np.zeros(ae.param_count())
    # layer 0 (conv 4 -> 32): d = 5 -> (dz, dy, dx) = (1, 0, 1), i = 2, o = 7
    p[(5 * 4 + 2) * 32 + 7] = 1.0
    # layer 3 (convT 32 -> 64) starts after layers 0..2; i = 3, d = 6 (1, 1, 0), o = 9
    off = sum(w + b for w, b in ae.layer_sizes()[:3])
    p[off + (3 * 8 + 6) * 64 + 9] = 2.0
    layers = ae.unpack(p)
    w0, w3 = layers[0][0], layers[3][0]
    assert w0[7, 2, 1, 0, 1] == 1.0 and np.count_nonzero(w0) == 1
    assert w3[3, 9, 1, 1, 0] == 2.0 and np.count_nonzero(w3) == 1
    q = RNG.normal(size=ae.param_count())
    np.testing.assert_array_equal(ae.pack(ae.unpack(q)), q)


def test_conv_impulse_response():
    w, b = _one_layer("conv", 3, 5)
    x = np.zeros((1, 3, 4, 4, 4))
    x[0, 1, 3, 0, 2] = 1.0                     # z = 3, y = 0, x = 2
    y = ae.conv(x, w, b)
    want = np.broadcast_to(b[None, :, None, None, None], y.shape).copy()
    want[0, :, 1, 0, 1] += w[:, 1, 1, 0, 0]     # dz = 1, dy = 0, dx = 0
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-15)


def test_conv_t_impulse_response():
    w, b = _one_layer("convT", 3, 5)
    x = np.zeros((1, 3, 2, 2, 2))
    x[0, 2, 1, 0, 1] = 1.0
    y = ae.conv_t(x, w, b)
    want = np.broadcast_to(b[None, :, None, None, None], y.shape).copy()
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                want[0, :, 2 + dz, dy, 2 + dx] += w[2, :, dz, dy, dx]
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-15)


def test_conv_t_is_the_adjoint_of_conv():
    w, _ = _one_layer("conv", 4, 6)
    x = RNG.normal(size=(2, 4, 8, 8, 8))
    y = RNG.normal(size=(2, 6, 4, 4, 4))
    lhs = np.sum(ae.conv(x, w, np.zeros(6)) * y)
    # conv_t takes W[in, out]: the conv's W[out, in] read as is
    rhs = np.sum(x * ae.conv_t(y, w, np.zeros(4)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _small_params(seed):
    p = ae.init_params(seed).astype(np.float64)
    # non-zero biases so that every bias gradient is exercised
    at = 0
    for w, b in ae.layer_sizes():
        at += w
        p[at:at + b] = np.random.default_rng(seed + 1).normal(scale=0.1, size=b)
        at += b
    return p


@pytest.mark.parametrize("mask", [ae.TANH_NONE, ae.TANH_HIDDEN])
def test_gradient_matches_central_differences(mask):
    p = _small_params(3)
    x = RNG.uniform(-1, 1, size=(2, 4, 8, 8, 8))
    _, g = ae.gradient(p, x, quantize=False, tanh_mask=mask)
    # loss ~0.3: central differences carry ~1e-16 * 0.3 / h of rounding and
    # ~h^2 of truncation; h = 1e-5 keeps both near 1e-11
    h = 1e-5
    idx = np.concatenate([RNG.choice(p.size, 40, replace=False),
                          np.cumsum([0] + [w + b for w, b in ae.layer_sizes()][:-1])
                          + np.array([w for w, _ in ae.layer_sizes()])])   # first biases
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (ae.loss(ae.forward(p + e, x, False, mask)[-1], x)
              - ae.loss(ae.forward(p - e, x, False, mask)[-1], x)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * abs(fd) + 1e-10, k
    d = RNG.normal(size=p.size)
    fd = (ae.loss(ae.forward(p + h * d, x, False, mask)[-1], x)
          - ae.loss(ae.forward(p - h * d, x, False, mask)[-1], x)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * abs(fd)


def test_max_loss_gradient_matches_central_differences():
    """Away from ties (random data has none) the max-error loss is smooth,
    so central differences pin its gradient, bias terms included."""
    p = _small_params(5)
    x = RNG.uniform(-1, 1, size=(3, 4, 8, 8, 8))
    _, g = ae.gradient(p, x, quantize=False, loss_kind=ae.LOSS_MAX)

    def lf(q):
        return ae.loss(ae.forward(q, x, False)[-1], x, ae.LOSS_MAX)

    h = 1e-6
    idx = np.concatenate([RNG.choice(p.size, 40, replace=False),
                          np.cumsum([0] + [w + b for w, b in ae.layer_sizes()][:-1])
                          + np.array([w for w, _ in ae.layer_sizes()])])
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (lf(p + e) - lf(p - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * abs(fd) + 1e-9, k
    d = RNG.normal(size=p.size)
    fd = (lf(p + h * d) - lf(p - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-5 * abs(fd)


def test_max_loss_closed_form_and_tie_split():
    """One block, two channels with errors: the loss is the mean over the
    four channels of the squared maxima; two tied maxima share the gradient
    equally, so moving both outward by eps raises the loss by the
    directional derivative 2 m eps / 4 to first order."""
    x = np.zeros((1, 4, 8, 8, 8))
    out = np.zeros_like(x)
    out[0, 0, 1, 2, 3] = 0.3
    out[0, 0, 4, 4, 4] = -0.1
    out[0, 2, 0, 0, 0] = -0.5
    out[0, 2, 7, 7, 7] = 0.5          # tie with the node above at |d| = 0.5
    assert ae.loss(out, x, ae.LOSS_MAX) == pytest.approx((0.3 ** 2 + 0.5 ** 2) / 4)
    g = ae.loss_gradient(out, x, ae.LOSS_MAX)
    assert g[0, 0, 1, 2, 3] == pytest.approx(2 * 0.3 / 4)
    assert g[0, 0, 4, 4, 4] == 0.0
    assert g[0, 2, 0, 0, 0] == pytest.approx(-2 * 0.5 / 4 / 2)
    assert g[0, 2, 7, 7, 7] == pytest.approx(2 * 0.5 / 4 / 2)
    assert np.count_nonzero(g) == 3
    eps = 1e-7
    moved = out.copy()
    moved[0, 2, 0, 0, 0] -= eps
    moved[0, 2, 7, 7, 7] += eps
    rise = ae.loss(moved, x, ae.LOSS_MAX) - ae.loss(out, x, ae.LOSS_MAX)
    assert rise == pytest.approx(-g[0, 2, 0, 0, 0] * eps + g[0, 2, 7, 7, 7] * eps, rel=1e-5)
    # a block without error has zero gradient
    assert not ae.loss_gradient(x, x, ae.LOSS_MAX).any()


def test_straight_through_gradient_when_rounding_is_exact():
    p = _small_params(5)
    # latent layer: zero weights, biases exactly representable in binary16
    off = sum(w + b for w, b in ae.layer_sizes()[:2])
    w2, b2 = ae.layer_sizes()[2]
    p[off:off + w2] = 0.0
    p[off + w2:off + w2 + b2] = np.arange(b2) / 64.0 - 0.25
    x = RNG.uniform(-1, 1, size=(2, 4, 8, 8, 8))
    l1, g1 = ae.gradient(p, x, quantize=True)
    l0, g0 = ae.gradient(p, x, quantize=False)
    assert l1 == l0
    np.testing.assert_array_equal(g1, g0)


def test_binary16_rounding_is_nearest_even():
    assert ae.to_half(1 + 2.0 ** -11) == 1.0                     # tie -> even
    assert ae.to_half(1 + 3 * 2.0 ** -11) == 1 + 2.0 ** -9       # tie -> even
    assert ae.to_half(1 + 2.0 ** -11 + 2.0 ** -20) == 1 + 2.0 ** -10
    assert ae.to_half(2.0 ** -25) == 0.0                         # half the least subnormal
    assert ae.to_half(3 * 2.0 ** -25) == 2.0 ** -23
    assert np.isinf(ae.to_half(65520.0)) and ae.to_half(65519.0) == 65504.0


def test_adam_constant_gradient_closed_form():
    p0 = RNG.normal(size=50)
    g = RNG.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = p0
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        p, m, v = ae.adam(p, g, m, v, t, lr, eps=eps)
        # bias correction makes every step exactly lr g / (|g| + eps)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)


@pytest.mark.parametrize("mask", [ae.TANH_NONE, ae.TANH_HIDDEN])
def test_training_decreases_the_loss(mask):
    p = _small_params(7)
    x = np.stack([np.stack([np.cos(k * np.linspace(-1, 1, 512)).reshape(8, 8, 8)
                            for k in (1, 2, 3, 0)]) * (0.5 + 0.1 * b) for b in range(3)])
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, g = ae.gradient(p, x, tanh_mask=mask)
    assert ae.loss(ae.forward(p - 1e-3 * g, x, True, mask)[-1], x) < l0   # descent
    for t in range(1, 41):
        _, g = ae.gradient(p, x, tanh_mask=mask)
        p, m, v = ae.adam(p, g, m, v, t, 3e-3)
    assert ae.loss(ae.forward(p, x, True, mask)[-1], x) < 0.2 * l0


def test_blocks_normalise_each_channel():
    f = [RNG.normal(size=(3, 8, 8, 8)) * s for s in (1.0, 5.0, 0.0, 1e-3)]
    x, s = ae.blocks(f)
    np.testing.assert_array_equal(s[:, 2], 0.0)
    np.testing.assert_array_equal(x[:, 2], 0.0)
    for c in (0, 1, 3):
        np.testing.assert_allclose(np.abs(x[:, c]).max(axis=(1, 2, 3)), 1.0, rtol=0, atol=0)
        np.testing.assert_allclose(x[:, c] * s[:, c, None, None, None], f[c], rtol=1e-15)


def test_fallback_rule_at_its_boundary():
    f = [RNG.normal(size=(4, 8, 8, 8)) for _ in range(3)] + [np.zeros((4, 8, 8, 8))]
    s = np.abs(np.stack(f, 1)).max(axis=(2, 3, 4))
    gmax = s.max(axis=0)
    r = [a.copy() for a in f]
    assert not ae.fallback(f, r, gmax).any()                       # exact: kept
    r[1][0, 3, 3, 3] += 0.99e-3 * s[0, 1]                         # just inside
    r[1][1, 0, 0, 0] -= 1.01e-3 * s[1, 1]                         # just outside
    r[3][2, 5, 5, 5] = 1e-12                                      # zero channel, any error
    flags = ae.fallback(f, r, gmax)
    np.testing.assert_array_equal(flags, [False, True, True, False])
    # the floor: a channel small on one element is judged against 1e-3 of its global max
    g = [a.copy() for a in f]
    g[0][3] *= 1e-5
    s2 = np.abs(np.stack(g, 1)).max(axis=(2, 3, 4))
    r2 = [a.copy() for a in g]
    r2[0][3, 1, 2, 3] += 0.9e-6 * s2[:, 0].max()
    assert not ae.fallback(g, r2, s2.max(axis=0))[3]
    r2[0][3, 1, 2, 3] += 0.2e-6 * s2[:, 0].max()
    assert ae.fallback(g, r2, s2.max(axis=0))[3]


def _ref_coords():
    xi = gll.gll_nodes(7)
    z, y, x = np.meshgrid(xi, xi, xi, indexing="ij")
    return x, y, z


def test_modal_truncation_keeps_its_span_and_drops_higher_modes():
    x, y, z = _ref_coords()
    tri = 1 + 2 * x - y + 0.5 * x * z + 0.25 * x * y * z - 0.75 * y * z
    p2 = (3 * x ** 2 - 1) / 2                                    # Legendre P_2(x)
    p5yz = (63 * y ** 5 - 70 * y ** 3 + 15 * y) / 8 * z          # P_5(y) P_1(z)
    f = [tri[None], p2[None], (tri + p2 + p5yz)[None], np.zeros((1, 8, 8, 8))]
    r, _ = ae.modal_truncate(f, quantize=False)
    np.testing.assert_allclose(r[0, 0], tri, atol=1e-13)
    np.testing.assert_allclose(r[0, 1], 0.0, atol=1e-13)
    np.testing.assert_allclose(r[0, 2], tri, atol=1e-12)
    np.testing.assert_array_equal(r[0, 3], 0.0)
    r2, _ = ae.modal_truncate([r[:, c] for c in range(4)], quantize=False)
    np.testing.assert_allclose(r2, r, atol=1e-13)                # a projection
    rq, _ = ae.modal_truncate(f, quantize=True)
    s = np.abs(tri).max()
    assert np.abs(rq[0, 0] - tri).max() <= 8 * 2.0 ** -11 * s     # binary16 coefficients


def test_compressed_bytes():
    assert ae.compressed_bytes(1, 0) == 32 * 2 + 4 * 4 + 1
    assert ae.compressed_bytes(10, 3) == 10 * 81 + 3 * 4 * 512 * 4
    raw = 4 * 512 * 4
    assert raw / ae.compressed_bytes(1, 0) == pytest.approx(101.14, abs=0.01)


def _low_rank_blocks(b, rank, seed, noise=0.0):
    """Blocks spanned by `rank` fixed patterns (plus optional noise).  Each
    pattern is, on every 4^3 octant, a multiple of one of 8 octant patterns,
    so the octant vectors span at most 8 dimensions and the blocks `rank`."""
    r = np.random.default_rng(seed)
    q = r.normal(size=(8, 4, 4, 4, 4))
    basis = np.zeros((rank, 4, 8, 8, 8))
    for k in range(rank):
        for oz in range(2):
            for oy in range(2):
                for ox in range(2):
                    basis[k, :, 4 * oz:4 * oz + 4, 4 * oy:4 * oy + 4, 4 * ox:4 * ox + 4] = \
                        r.normal() * q[k % 8]
    coef = r.normal(size=(b, rank)) * np.geomspace(1, 0.1, rank)
    x = coef @ basis.reshape(rank, -1) + noise * r.normal(size=(b, 4 * 512))
    return x.reshape(b, 4, 8, 8, 8)


def test_pca_init_is_exact_on_data_of_low_rank():
    # data of rank 20 <= 32: octant and global projections keep all of it
    x = _low_rank_blocks(64, 20, 11)
    p, lams = ae.pca_init(x)
    out = ae.forward(p, x, quantize=False)[-1]
    np.testing.assert_allclose(out, x, atol=1e-10 * np.abs(x).max())
    # eigenvalues decrease; beyond the data's rank the global ones vanish
    assert np.all(np.diff(lams[0]) <= 0) and np.all(np.diff(lams[1]) <= 0)
    assert lams[1][19] > 1e-6 * lams[1][0] and np.all(lams[1][20:] <= 1e-9 * lams[1][0])


def test_pca_init_layers_are_orthonormal_projections():
    x = _low_rank_blocks(96, 48, 12, noise=1e-3)
    p, _ = ae.pca_init(x)
    flat = p
    sizes = ae.layer_sizes()
    off = sizes[0][0] + sizes[0][1]
    w1 = flat[off:off + sizes[1][0]].reshape(256, 64)       # [k][o]
    np.testing.assert_allclose(w1.T @ w1, np.eye(64), atol=1e-12)
    off += sizes[1][0] + sizes[1][1]
    w2 = flat[off:off + sizes[2][0]].reshape(512, 32)
    np.testing.assert_allclose(w2.T @ w2, np.eye(32), atol=1e-12)
    # the decoder is the transpose: encoding a reconstruction changes nothing
    z = ae.forward(p, x, quantize=False)[3]
    out = ae.forward(p, x, quantize=False)[-1]
    np.testing.assert_allclose(ae.forward(p, out, quantize=False)[3], z, atol=1e-10)
    # and the 32-dim code is optimal among the octant codes: the residual is
    # orthogonal to the reconstruction
    assert abs(np.sum((x - out) * out)) <= 1e-9 * np.sum(x * x)
