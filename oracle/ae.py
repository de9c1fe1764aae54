"""Per-element convolutional autoencoder for in-transit compression (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Context: in the paper's in-transit workflow (section 4.2) simulation nodes
hand every snapshot to separate visualisation nodes over the network
(ADIOS2/SST), so the bytes per snapshot set the cost of the hand-off.  The
paper does not compress; the compressor here is the project's growth
direction, and every step below is a textbook definition:

* Block: the four fields (u, v, w, theta) of one order-7 element, 4 x 8^3
  values, each channel divided by its own element maximum
  s_ec = max |f_c| over the element (0 -> block channel 0).
* Network: three strided convolutions (kernel 2, stride 2; 8^3 -> 4^3 ->
  2^3 -> 1) down to a 32-value latent, and three transposed convolutions
  (kernel 2, stride 2) back up.  Convolution and its transpose follow the
  usual deep-learning definitions (Dumoulin & Visin 2016, "A guide to
  convolution arithmetic", sections 2 and 4):
      conv:   y[o, z, y, x] = b[o] + sum_{i, dz, dy, dx}
                              W[o, i, dz, dy, dx] x[i, 2z+dz, 2y+dy, 2x+dx]
      convT:  y[o, 2z+dz, 2y+dy, 2x+dx] = b[o] + sum_i W[i, o, dz, dy, dx]
                                          x[i, z, y, x]
  Every layer is linear by default; a mask selects tanh after chosen
  layers (bit l: layer l), so both forms have a definition here.
* Latent stored in IEEE binary16 (round to nearest even); training passes
  the rounded latent forward and its gradient through unchanged (the
  straight-through estimator, Bengio, Leonard & Courville 2013).
* Loss: mean squared error over every value of the batch's blocks; or the
  max-error loss, the mean over (block, channel) of the squared largest
  absolute error over the block's 512 nodes, the smooth-in-the-square form
  of the relative L-inf bound that decides the raw fallback below.  Its
  gradient at a (block, channel) is 2 m sign(y - x) / (blocks x channels)
  at the node(s) where |y - x| reaches the maximum m, shared equally when
  several nodes tie (a subgradient, independent of the node order), and 0
  elsewhere.
* Gradients by the chain rule (reverse mode), written out per layer.
* Optimiser: Adam (Kingma & Ba 2015, algorithm 1).
* Initialisation by layer-wise principal components (uncentred; in the
  spirit of PCANet, Chan et al. 2015): layer 0 is the identity on each
  2^3 patch (32 in, 32 out); layer 1 keeps the 64 leading eigenvectors of
  the second-moment matrix of its 256-value inputs (one per 4^3 octant of
  every block), layer 2 the 32 leading ones of its 512-value inputs; each
  decoder layer is the transpose of its encoder layer; biases are zero.
* Raw fallback: an element is shipped raw if for any channel
  max |f - f_hat| > 1e-3 * max(s_ec, 1e-3 * max_e s_ec) (relative L-inf
  with a floor for channels that vanish on an element, e.g. w of
  Taylor-Green).
* Non-learned baseline at the same bytes: per channel, the Legendre
  coefficients of the element's interpolant with degrees (a, b, c) in
  {0, 1}^3 (eight per channel, 32 per element, stored in binary16 after
  division by s_ec), from the modal expansion of Deville, Fischer & Mund
  (2002), section 2.4; everything else dropped.

Parameter vector (the library's layout, shared as an interface): for each
layer in order, its weights then its biases.  Weights of a convolution
layer are stored at ((d * Cin + i) * Cout + o), of a transposed one at
((i * 8 + d) * Cout + o), where d = dx + 2 dy + 4 dz.

All arithmetic is FP64 unless a function says otherwise.
"""

import numpy as np

from . import gll

N = 7
P = N + 1
CHANNELS = 4
LATENT = 32
# (kind, Cin, Cout)
ARCH = (("conv", 4, 32), ("conv", 32, 64), ("conv", 64, 32),
        ("convT", 32, 64), ("convT", 64, 32), ("convT", 32, 4))
LATENT_LAYER = 2
LOSS_MSE = 0            # mean squared error
LOSS_MAX = 1            # mean squared per-(block, channel) maximum error
TANH_NONE = 0           # the library's network: every layer linear
TANH_HIDDEN = 0b011011  # tanh after layers 0, 1, 3, 4 (not the latent or output)
REL_BOUND = 1e-3
FLOOR = 1e-3


def layer_sizes():
    """(weight count, bias count) of each layer."""
    return [(cin * cout * 8, cout) for _, cin, cout in ARCH]


def param_count():
    return sum(w + b for w, b in layer_sizes())


def _delta():
    """(dz, dy, dx) of d = dx + 2 dy + 4 dz, for d = 0..7."""
    return [((d >> 2) & 1, (d >> 1) & 1, d & 1) for d in range(8)]


def unpack(params):
    """Flat parameter vector -> [(W, b)] in the conv conventions above:
    conv W[o, i, dz, dy, dx], convT W[i, o, dz, dy, dx]."""
    p = np.asarray(params, dtype=np.float64)
    out, at = [], 0
    for kind, cin, cout in ARCH:
        flat = p[at:at + cin * cout * 8]
        at += cin * cout * 8
        b = p[at:at + cout].copy()
        at += cout
        if kind == "conv":
            w = np.empty((cout, cin, 2, 2, 2))
            f = flat.reshape(8, cin, cout)                 # [d][i][o]
            for d, (dz, dy, dx) in enumerate(_delta()):
                w[:, :, dz, dy, dx] = f[d].T
        else:
            w = np.empty((cin, cout, 2, 2, 2))
            f = flat.reshape(cin, 8, cout)                 # [i][d][o]
            for d, (dz, dy, dx) in enumerate(_delta()):
                w[:, :, dz, dy, dx] = f[:, d, :]
        out.append((w, b))
    assert at == p.size
    return out


def pack(layers):
    """Inverse of ``unpack``."""
    chunks = []
    for (kind, cin, cout), (w, b) in zip(ARCH, layers):
        if kind == "conv":
            f = np.empty((8, cin, cout))
            for d, (dz, dy, dx) in enumerate(_delta()):
                f[d] = w[:, :, dz, dy, dx].T
        else:
            f = np.empty((cin, 8, cout))
            for d, (dz, dy, dx) in enumerate(_delta()):
                f[:, d, :] = w[:, :, dz, dy, dx]
        chunks += [f.ravel(), np.asarray(b, dtype=np.float64).ravel()]
    return np.concatenate(chunks)


def init_params(seed):
    """Glorot-uniform weights (fan in + fan out over the 2^3 kernel), zero
    biases (Glorot & Bengio 2010)."""
    rng = np.random.default_rng(seed)
    layers = []
    for kind, cin, cout in ARCH:
        lim = np.sqrt(6.0 / (8 * cin + 8 * cout))
        shape = (cout, cin, 2, 2, 2) if kind == "conv" else (cin, cout, 2, 2, 2)
        layers.append((rng.uniform(-lim, lim, size=shape), np.zeros(cout)))
    return pack(layers).astype(np.float32)


# --------------------------------------------------------------------------
# layers (batched over elements: x[B, C, n, n, n], spatial [z][y][x])
# --------------------------------------------------------------------------

def conv(x, w, b):
    y = np.zeros((x.shape[0], w.shape[0]) + tuple(s // 2 for s in x.shape[2:]))
    for dz, dy, dx in _delta():
        y += np.einsum("oi,bizyx->bozyx", w[:, :, dz, dy, dx], x[:, :, dz::2, dy::2, dx::2])
    return y + b[None, :, None, None, None]


def conv_t(x, w, b):
    y = np.empty((x.shape[0], w.shape[1]) + tuple(2 * s for s in x.shape[2:]))
    for dz, dy, dx in _delta():
        y[:, :, dz::2, dy::2, dx::2] = np.einsum("io,bizyx->bozyx", w[:, :, dz, dy, dx], x)
    return y + b[None, :, None, None, None]


def conv_grads(x, w, g):
    """Gradients of conv(x, w, b) given g = dL/dy: (dL/dx, dL/dw, dL/db)."""
    dx_ = np.zeros_like(x)
    dw = np.empty_like(w)
    for dz, dy, dx in _delta():
        xs = x[:, :, dz::2, dy::2, dx::2]
        dw[:, :, dz, dy, dx] = np.einsum("bozyx,bizyx->oi", g, xs)
        dx_[:, :, dz::2, dy::2, dx::2] = np.einsum("oi,bozyx->bizyx", w[:, :, dz, dy, dx], g)
    return dx_, dw, g.sum(axis=(0, 2, 3, 4))


def conv_t_grads(x, w, g):
    """Gradients of conv_t(x, w, b) given g = dL/dy: (dL/dx, dL/dw, dL/db)."""
    dx_ = np.zeros_like(x)
    dw = np.empty_like(w)
    for dz, dy, dx in _delta():
        gs = g[:, :, dz::2, dy::2, dx::2]
        dw[:, :, dz, dy, dx] = np.einsum("bozyx,bizyx->io", gs, x)
        dx_ += np.einsum("io,bozyx->bizyx", w[:, :, dz, dy, dx], gs)
    return dx_, dw, g.sum(axis=(0, 2, 3, 4))


def to_half(z):
    """Round to IEEE binary16 (nearest, ties to even; overflow to inf) and back."""
    with np.errstate(over="ignore"):
        return np.asarray(z, dtype=np.float64).astype(np.float16).astype(np.float64)


def forward(params, x, quantize=True, tanh_mask=TANH_NONE):
    """Activations [x, a1, ..., a6] of a batch of blocks x[B, 4, 8, 8, 8];
    a3 is the latent (binary16-rounded if ``quantize``), a6 the output."""
    acts = [np.asarray(x, dtype=np.float64)]
    for l, ((kind, _, _), (w, b)) in enumerate(zip(ARCH, unpack(params))):
        y = (conv if kind == "conv" else conv_t)(acts[-1], w, b)
        if (tanh_mask >> l) & 1:
            y = np.tanh(y)
        if l == LATENT_LAYER and quantize:
            y = to_half(y)
        acts.append(y)
    return acts


def loss(out, x, kind=LOSS_MSE):
    d = out - np.asarray(x, dtype=np.float64)
    if kind == LOSS_MAX:
        m = np.abs(d).reshape(d.shape[0], CHANNELS, -1).max(axis=2)
        return float(np.mean(m ** 2))
    return float(np.mean(d ** 2))


def loss_gradient(out, x, kind=LOSS_MSE):
    """dL/d(out) of ``loss``."""
    d = out - np.asarray(x, dtype=np.float64)
    if kind != LOSS_MAX:
        return 2.0 * d / d.size
    a = np.abs(d).reshape(d.shape[0], CHANNELS, -1)
    m = a.max(axis=2, keepdims=True)
    top = (a == m) & (m > 0)
    ties = np.maximum(top.sum(axis=2, keepdims=True), 1)
    g = np.where(top, 2.0 * m * np.sign(d.reshape(a.shape)) / (d.shape[0] * CHANNELS) / ties,
                 0.0)
    return g.reshape(d.shape)


def gradient(params, x, quantize=True, tanh_mask=TANH_NONE, loss_kind=LOSS_MSE):
    """(loss, dL/dparams) for the batch x, by reverse mode."""
    x = np.asarray(x, dtype=np.float64)
    acts = forward(params, x, quantize, tanh_mask)
    layers = unpack(params)
    g = loss_gradient(acts[-1], x, loss_kind)
    grads = [None] * len(ARCH)
    for l in range(len(ARCH) - 1, -1, -1):
        kind = ARCH[l][0]
        if (tanh_mask >> l) & 1:
            g = g * (1.0 - acts[l + 1] ** 2)
        w, _ = layers[l]
        gx, gw, gb = (conv_grads if kind == "conv" else conv_t_grads)(acts[l], w, g)
        grads[l] = (gw, gb)
        g = gx                     # straight through the latent rounding
    return loss(acts[-1], x, loss_kind), pack(grads)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def _leading_eigvecs(c, r):
    """The r leading eigenvectors of the symmetric matrix c (columns, by
    decreasing eigenvalue; numpy's symmetric eigensolver)."""
    lam, u = np.linalg.eigh(c)
    order = np.argsort(lam)[::-1][:r]
    return lam[order], u[:, order]


def pca_init(x):
    """Parameters from layer-wise principal components of the blocks
    x[B, 4, 8, 8, 8] (see the module text), with the eigenvalues kept by
    layers 1 and 2."""
    x = np.asarray(x, dtype=np.float64)
    layers = []
    # layer 0: identity on each patch, flat k = d * 4 + i -> channel o = k
    w0 = np.zeros((32, 4, 2, 2, 2))
    for d, (dz, dy, dx) in enumerate(_delta()):
        for i in range(4):
            w0[d * 4 + i, i, dz, dy, dx] = 1.0
    layers.append((w0, np.zeros(32)))
    a = conv(x, w0, np.zeros(32))
    lams = []
    for cin, cout in ((32, 64), (64, 32)):
        # inputs of one output position, ordered k = d * cin + i
        v = np.stack([a[:, :, dz::2, dy::2, dx::2] for dz, dy, dx in _delta()], axis=1)
        v = v.transpose(0, 3, 4, 5, 1, 2).reshape(-1, 8 * cin)
        lam, u = _leading_eigvecs(v.T @ v, cout)
        lams.append(lam)
        w = np.empty((cout, cin, 2, 2, 2))
        uk = u.reshape(8, cin, cout)
        for d, (dz, dy, dx) in enumerate(_delta()):
            w[:, :, dz, dy, dx] = uk[d].T
        layers.append((w, np.zeros(cout)))
        a = conv(a, w, np.zeros(cout))
    # decoder: transposes (convT takes W[in, out] = the conv's W[out, in])
    for l in (2, 1, 0):
        w = layers[l][0]
        layers.append((w, np.zeros(w.shape[1])))
    return pack(layers), lams


# --------------------------------------------------------------------------
# blocks, fallback, compression
# --------------------------------------------------------------------------

def blocks(fields):
    """(x[E, 4, 8, 8, 8], s[E, 4]) from four fields f[E][8][8][8] (GLL
    layout [k][j][i], so the spatial axes are z, y, x).  Computed in the
    fields' dtype."""
    f = np.stack([np.asarray(a) for a in fields], axis=1)
    s = np.abs(f).max(axis=(2, 3, 4))
    safe = np.where(s > 0, s, 1).astype(f.dtype)
    x = np.where(s[:, :, None, None, None] > 0, f / safe[:, :, None, None, None], 0)
    return x.astype(f.dtype), s


def fallback(fields, recon, gmax):
    """Per-element raw-fallback flags: any channel with
    max |f - f_hat| > 1e-3 max(s_ec, 1e-3 gmax_c).  Decided in the inputs'
    dtype (FP32 inputs -> FP32 comparisons)."""
    f = np.stack([np.asarray(a) for a in fields], axis=1)
    r = np.stack([np.asarray(a) for a in recon], axis=1)
    dt = f.dtype.type
    s = np.abs(f).max(axis=(2, 3, 4))
    err = np.abs(f - r).max(axis=(2, 3, 4))
    gm = np.asarray(gmax, dtype=f.dtype)
    bound = dt(REL_BOUND) * np.maximum(s, dt(FLOOR) * gm[None, :])
    return np.any(err > bound, axis=1)


def reconstruct(params, x, s, tanh_mask=TANH_NONE):
    """Decoded fields f_hat[E, 4, 8, 8, 8] = s * network(x) (binary16 latent)."""
    out = forward(params, x, True, tanh_mask)[-1]
    return out * np.asarray(s, dtype=np.float64)[:, :, None, None, None]


def compressed_bytes(n_elem, n_raw):
    """Bytes of a compressed snapshot: binary16 latent + FP32 scales + one
    flag byte per element, and 4 x 8^3 FP32 values per raw element."""
    return n_elem * (LATENT * 2 + CHANNELS * 4 + 1) + n_raw * CHANNELS * P ** 3 * 4


# --------------------------------------------------------------------------
# non-learned baseline: Legendre modal truncation at the same bytes
# --------------------------------------------------------------------------

def legendre_vandermonde():
    """V[n, a] = P_a(xi_n) on the order-7 GLL nodes."""
    xi = gll.gll_nodes(N)
    return np.stack([gll.legendre_value(a, xi) for a in range(P)], axis=1)


def modal_truncate(fields, quantize=True):
    """(f_hat[E, 4, 8, 8, 8], coefficients[E, 4, 2, 2, 2]): modal
    coefficients c = V^-1 f along each axis, modes with every degree <= 1
    kept (stored as binary16 of c / s_ec if ``quantize``), the rest
    dropped."""
    f = np.stack([np.asarray(a, dtype=np.float64) for a in fields], axis=1)
    vinv = np.linalg.inv(legendre_vandermonde())           # [mode, node]
    # axes: x element, y channel; k, l, m nodes along z, y, x; a, b, c modes
    c = np.einsum("ak,bl,cm,xyklm->xyabc", vinv, vinv, vinv, f)
    keep = c[:, :, :2, :2, :2]
    s = np.abs(f).max(axis=(2, 3, 4))
    if quantize:
        safe = np.where(s > 0, s, 1.0)[:, :, None, None, None]
        keep = np.where(s[:, :, None, None, None] > 0, to_half(keep / safe) * safe, 0.0)
    v2 = legendre_vandermonde()[:, :2]                      # [node, mode <= 1]
    r = np.einsum("ka,lb,mc,xyabc->xyklm", v2, v2, v2, keep)
    return r, keep
