"""Seeded synthetic snapshots for the extraction path (inputs only).

This module plays the role of the solver that hands snapshots to the in situ
stage (the paper's section 3: a mesh plus point arrays at the GLL nodes of
each element).  It holds none of the extraction arithmetic: it places mesh
nodes and samples closed-form or random-mode velocity fields there.  Both the
CPU oracle and the HIP library consume exactly the arrays produced here.

Layout: arrays of shape (E, N+1, N+1, N+1), index [e, k, j, i], i fastest;
elements of a box mesh are numbered e = ex + Ex (ey + Ey ez).

Node placement: GLL points of order N on every element edge, taken from
numpy's Legendre root finder (a library routine; the oracle and the library
each compute the nodes independently).  Coordinates come from per-axis 1-D
global lattices, X[ex N + i], so nodes shared by neighbouring elements are
bitwise identical.

Arrays are numpy float64 by default; pass ``device=`` (a torch device) to
build them with torch on that device (used for the large channel snapshot,
whose random-mode sum is too slow for a single host core).
"""

import math

import numpy as np

__all__ = [
    "gll_points", "axis_lattice", "box_mesh", "element_axes", "tgv_velocity",
    "channel_modes", "channel_velocity", "warp", "tgv_config", "channel_config",
    "lattice_gid", "batch_spec", "batch_snapshot", "CHANNEL_SHAPE", "TGV_SHAPE",
    "ae_fields", "ae_mesh", "ae_training_elements", "AE_SHAPE", "AE_PHASES",
]

TGV_SHAPE = (8, 8, 8)          # Taylor-Green box [0, 2 pi]^3, 512 elements
CHANNEL_SHAPE = (64, 32, 32)   # channel [0, 4 pi] x [-1, 1] x [0, 2 pi]
CHANNEL_SEED = 2312


def gll_points(n):
    """GLL points of order n on [-1, 1] (numpy Legendre roots of P_n')."""
    if n < 1:
        raise ValueError("order must be >= 1")
    inner = np.sort(np.polynomial.legendre.Legendre.basis(n).deriv().roots().real) \
        if n > 1 else np.zeros(0)
    return np.concatenate(([-1.0], inner, [1.0]))


def axis_lattice(n_el, n, lo, hi, stretch=None):
    """1-D global lattice of n_el * n + 1 points on [lo, hi].

    Elements are uniform in the computational coordinate eta in [-1, 1];
    ``stretch`` = beta applies y = tanh(beta eta) / tanh(beta) pointwise
    (wall-normal channel clustering), then the result is mapped to [lo, hi].
    """
    xi = gll_points(n)
    g = np.empty(n_el * n + 1)
    for e in range(n_el):
        g[e * n:e * n + n + 1] = -1.0 + (2.0 * e + (xi + 1.0)) / n_el
    g[0], g[-1] = -1.0, 1.0
    if stretch is not None:
        g = np.tanh(stretch * g) / math.tanh(stretch)
    return lo + (hi - lo) * 0.5 * (g + 1.0)


def element_axes(shape, elements=None):
    """(ex, ey, ez) index arrays for the selected elements (default: all)."""
    ex_n, ey_n, ez_n = shape
    e = np.arange(ex_n * ey_n * ez_n) if elements is None else np.asarray(elements)
    return e % ex_n, (e // ex_n) % ey_n, e // (ex_n * ey_n)


def box_mesh(shape, n, bounds, stretch=(None, None, None), elements=None,
             device=None):
    """Coordinates (x, y, z) of a tensor-product box mesh of order n."""
    lat = [axis_lattice(shape[a], n, bounds[a][0], bounds[a][1], stretch[a])
           for a in range(3)]
    ex, ey, ez = element_axes(shape, elements)
    p = n + 1
    loc = np.arange(p)
    xs = lat[0][ex[:, None] * n + loc[None, :]]      # (E, P) along i
    ys = lat[1][ey[:, None] * n + loc[None, :]]      # along j
    zs = lat[2][ez[:, None] * n + loc[None, :]]      # along k
    e_cnt = xs.shape[0]
    x = np.broadcast_to(xs[:, None, None, :], (e_cnt, p, p, p))
    y = np.broadcast_to(ys[:, None, :, None], (e_cnt, p, p, p))
    z = np.broadcast_to(zs[:, :, None, None], (e_cnt, p, p, p))
    out = [np.ascontiguousarray(c) for c in (x, y, z)]
    if device is not None:
        import torch
        out = [torch.from_numpy(c).to(device) for c in out]
    return tuple(out)


def lattice_gid(shape, n, elements=None):
    """Global node ids of the box meshes above (int64, shape (E, P, P, P)):
    stored node (i, j, k) of element (ex, ey, ez) is lattice point
    (gx, gy, gz) = (ex n + i, ey n + j, ez n + k), numbered
    gx + Lx (gy + Ly gz) with L = shape * n + 1.  Coincident copies on
    element faces, edges and corners get equal ids."""
    ex, ey, ez = element_axes(shape, elements)
    p = n + 1
    lx, ly = shape[0] * n + 1, shape[1] * n + 1
    loc = np.arange(p)
    gx = (ex[:, None] * n + loc[None, :])[:, None, None, :]
    gy = (ey[:, None] * n + loc[None, :])[:, None, :, None]
    gz = (ez[:, None] * n + loc[None, :])[:, :, None, None]
    return np.ascontiguousarray((gx + lx * (gy + ly * gz)).astype(np.int64))


def _lib(a):
    if isinstance(a, np.ndarray):
        return np
    import torch
    return torch


def tgv_velocity(x, y, z):
    """Taylor-Green vortex u = sin x cos y cos z, v = -cos x sin y cos z, w = 0."""
    xp = _lib(x)
    u = xp.sin(x) * xp.cos(y) * xp.cos(z)
    v = -xp.cos(x) * xp.sin(y) * xp.cos(z)
    w = xp.zeros_like(x)
    return u, v, w


def warp(x, y, z, amp=0.05):
    """Smooth non-affine warp of a box mesh (exercises every Jacobian entry).

    x' = x + a sin(y) sin(z), y' = y + a sin(z) sin(x), z' = z + a sin(x) sin(y)
    with a small enough that the map stays orientation preserving.
    """
    xp = _lib(x)
    return (x + amp * xp.sin(y) * xp.sin(z),
            y + amp * xp.sin(z) * xp.sin(x),
            z + amp * xp.sin(x) * xp.sin(y))


def channel_modes(seed=CHANNEL_SEED, shells=32, per_shell=8, rms=0.1):
    """Random solenoidal Fourier modes with a k^-5/3 shell spectrum.

    Shell n = 1..shells has wavenumber magnitude k = n and ``per_shell``
    random unit directions d; each mode gets a random unit polarisation
    sigma orthogonal to d (so the field is divergence free), a random phase
    and an amplitude proportional to sqrt(E(k) / per_shell) with
    E(k) = k^-5/3; all amplitudes are then scaled so that the mean square of
    one velocity component is rms^2.  Returns (kvec (M,3), sigma (M,3),
    phase (M,), amp (M,)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kv, sg, ph, am = [], [], [], []
    for n in range(1, shells + 1):
        for _ in range(per_shell):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            r = rng.normal(size=3)
            s = r - np.dot(r, d) * d
            s /= np.linalg.norm(s)
            kv.append(n * d)
            sg.append(s)
            ph.append(rng.uniform(0.0, 2.0 * np.pi))
            am.append(math.sqrt(n ** (-5.0 / 3.0) / per_shell))
    kv, sg, ph, am = map(np.asarray, (kv, sg, ph, am))
    # mean square of one component of sum a sigma cos(.) is sum a^2 |sigma_c|^2 / 2
    ms = np.sum(am ** 2) / 2.0 / 3.0
    am = am * (rms / math.sqrt(ms))
    return kv, sg, ph, am


def channel_velocity(x, y, z, modes=None):
    """Parabolic mean (1 - y^2, 0, 0) plus the random-mode fluctuation."""
    xp = _lib(x)
    kv, sg, ph, am = channel_modes() if modes is None else modes
    u = 1.0 - y * y
    v = xp.zeros_like(x)
    w = xp.zeros_like(x)
    for m in range(kv.shape[0]):
        arg = kv[m, 0] * x + kv[m, 1] * y + kv[m, 2] * z + ph[m]
        c = am[m] * xp.cos(arg)
        u = u + sg[m, 0] * c
        v = v + sg[m, 1] * c
        w = w + sg[m, 2] * c
    return u, v, w


def tgv_config(n=7, shape=TGV_SHAPE, elements=None, device=None):
    """Taylor-Green snapshot on the uniform [0, 2 pi]^3 box: (x, y, z, u, v, w)."""
    b = ((0.0, 2 * np.pi),) * 3
    x, y, z = box_mesh(shape, n, b, elements=elements, device=device)
    return (x, y, z) + tgv_velocity(x, y, z)


def channel_config(n=7, shape=CHANNEL_SHAPE, elements=None, device=None,
                   beta=2.0, seed=CHANNEL_SEED, dtype=None):
    """Turbulent-channel-like snapshot: (x, y, z, u, v, w).

    Domain [0, 4 pi] x [-1, 1] x [0, 2 pi], tanh wall-normal stretching
    (beta = 2) applied pointwise to the GLL node coordinates, so the
    Jacobian varies from node to node.
    """
    b = ((0.0, 4 * np.pi), (-1.0, 1.0), (0.0, 2 * np.pi))
    x, y, z = box_mesh(shape, n, b, stretch=(None, beta, None),
                       elements=elements, device=device)
    vel = channel_velocity(x, y, z, channel_modes(seed))
    out = (x, y, z) + tuple(vel)
    if dtype is not None:
        out = tuple(a.astype(dtype) if isinstance(a, np.ndarray) else a.to(dtype)
                    for a in out)
    return out


# --------------------------------------------------------------------------
# batched uneven snapshots
# --------------------------------------------------------------------------

def batch_spec(seed, orders=(5, 7, 9), e_min=4096, e_max=200000):
    """(order, shape, stretch) of batch snapshot `seed`: order drawn from
    `orders`, element count log-uniform in [e_min, e_max] arranged as a
    near-cubic box, per-axis tanh stretching beta uniform in [1, 3]."""
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.choice(orders))
    e = int(round(math.exp(rng.uniform(math.log(e_min), math.log(e_max)))))
    a = max(1, int(round(e ** (1.0 / 3.0))))
    shape = (a, a, max(1, int(math.ceil(e / (a * a)))))
    beta = tuple(float(b) for b in rng.uniform(1.0, 3.0, size=3))
    return n, shape, beta


def batch_snapshot(seed, device, dtype=None, features=256, chunk=1 << 22, e_min=4096,
                   e_max=200000):
    """Batch snapshot `seed` on `device` (torch): unit box mesh with the
    spec's order, shape and stretching; velocity = channel-style random
    solenoidal modes (8 shells x 4 directions, seeded); scalar theta = a
    Gaussian random field by random Fourier features (Rahimi & Recht 2007):
    theta = sqrt(2 / F) sum_f cos(k_f . x + b_f), k_f ~ N(0, 1 / l^2),
    l = 0.1 of the domain, b_f ~ U(0, 2 pi).  Returns (spec, (x, y, z, u,
    v, w, theta)).  e_min, e_max: range of the element count."""
    import torch
    n, shape, beta = batch_spec(seed, e_min=e_min, e_max=e_max)
    lat = [torch.from_numpy(axis_lattice(shape[a], n, 0.0, 1.0, beta[a])).to(device)
           for a in range(3)]
    ex, ey, ez = (torch.from_numpy(c).to(device) for c in element_axes(shape))
    loc = torch.arange(n + 1, device=device)
    p = n + 1
    e_cnt = ex.shape[0]
    xs = lat[0][ex[:, None] * n + loc[None, :]]
    ys = lat[1][ey[:, None] * n + loc[None, :]]
    zs = lat[2][ez[:, None] * n + loc[None, :]]
    x = xs[:, None, None, :].expand(e_cnt, p, p, p).contiguous()
    y = ys[:, None, :, None].expand(e_cnt, p, p, p).contiguous()
    z = zs[:, :, None, None].expand(e_cnt, p, p, p).contiguous()
    u, v, w = channel_velocity(x, y, z, channel_modes(seed, shells=8, per_shell=4))
    rng = np.random.default_rng(20_000 + seed)
    kf = torch.from_numpy(rng.normal(0.0, 1.0 / 0.1, size=(features, 3))).to(device)
    bf = torch.from_numpy(rng.uniform(0.0, 2.0 * np.pi, size=features)).to(device)
    pts = torch.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], dim=1)
    theta = torch.empty(pts.shape[0], dtype=x.dtype, device=device)
    for c0 in range(0, pts.shape[0], chunk):
        ph = pts[c0:c0 + chunk] @ kf.T + bf
        theta[c0:c0 + chunk] = torch.cos(ph).sum(dim=1) * math.sqrt(2.0 / features)
    out = (x, y, z, u, v, w, theta.reshape(x.shape))
    if dtype is not None:
        out = tuple(t.to(dtype).contiguous() for t in out)
    return (n, shape, beta), out


# --------------------------------------------------------------------------
# compression snapshots: Taylor-Green velocity and a random scalar, advected
# --------------------------------------------------------------------------

AE_SHAPE = (64, 64, 64)          # 262,144 order-7 elements on [0, 2 pi]^3
AE_PHASES = 64
AE_DRIFT = (1.0, 0.5, 0.25)      # translation direction of the advected fields
AE_THETA_SEED = 4096


def ae_fields(phase, device, shape=AE_SHAPE, elements=None, dtype=None, features=256,
              chunk=1 << 22):
    """(u, v, w, theta) of compression snapshot `phase` (0 <= phase < 64) on
    `device` (torch), order 7, uniform box [0, 2 pi]^3 of `shape` elements
    (or the subset `elements`, numbered as in element_axes).

    Every field is a fixed pattern translated by t = 2 pi phase / 64 along
    AE_DRIFT, f(x - t d): the Taylor-Green velocity and a Gaussian random
    scalar theta by random Fourier features (Rahimi & Recht 2007; 256
    features, k ~ N(0, 1 / l^2) with l = 0.1 of the domain, seeded).  The
    phase may be fractional (a held-out time between training phases)."""
    import torch
    n, p = 7, 8
    lat = [torch.from_numpy(axis_lattice(shape[a], n, 0.0, 2 * np.pi)).to(device)
           for a in range(3)]
    ex, ey, ez = (torch.from_numpy(np.asarray(c)).to(device)
                  for c in element_axes(shape, elements))
    loc = torch.arange(p, device=device)
    t = 2 * np.pi * float(phase) / AE_PHASES
    xs = lat[0][ex[:, None] * n + loc[None, :]] - t * AE_DRIFT[0]
    ys = lat[1][ey[:, None] * n + loc[None, :]] - t * AE_DRIFT[1]
    zs = lat[2][ez[:, None] * n + loc[None, :]] - t * AE_DRIFT[2]
    e_cnt = xs.shape[0]
    x = xs[:, None, None, :].expand(e_cnt, p, p, p)
    y = ys[:, None, :, None].expand(e_cnt, p, p, p)
    z = zs[:, :, None, None].expand(e_cnt, p, p, p)
    u, v, w = tgv_velocity(x, y, z)
    rng = np.random.default_rng(AE_THETA_SEED)
    ell = 0.1 * 2 * np.pi
    kf = torch.from_numpy(rng.normal(0.0, 1.0 / ell, size=(features, 3))).to(device)
    bf = torch.from_numpy(rng.uniform(0.0, 2.0 * np.pi, size=features)).to(device)
    pts = torch.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], dim=1)
    theta = torch.empty(pts.shape[0], dtype=pts.dtype, device=device)
    for c0 in range(0, pts.shape[0], chunk):
        ph = pts[c0:c0 + chunk] @ kf.T + bf
        theta[c0:c0 + chunk] = torch.cos(ph).sum(dim=1) * math.sqrt(2.0 / features)
    out = (u.contiguous(), v.contiguous(), w.contiguous(), theta.reshape(e_cnt, p, p, p))
    if dtype is not None:
        out = tuple(f.to(dtype).contiguous() for f in out)
    return out


def ae_mesh(device, shape=AE_SHAPE, elements=None, dtype=None):
    """(x, y, z) of the compression snapshots' uniform [0, 2 pi]^3 mesh on
    `device` (torch), order 7 (the fields of ae_fields sit at these nodes)."""
    import torch
    n, p = 7, 8
    lat = [torch.from_numpy(axis_lattice(shape[a], n, 0.0, 2 * np.pi)).to(device)
           for a in range(3)]
    ex, ey, ez = (torch.from_numpy(np.asarray(c)).to(device)
                  for c in element_axes(shape, elements))
    loc = torch.arange(p, device=device)
    e_cnt = ex.shape[0]
    xs = lat[0][ex[:, None] * n + loc[None, :]]
    ys = lat[1][ey[:, None] * n + loc[None, :]]
    zs = lat[2][ez[:, None] * n + loc[None, :]]
    out = (xs[:, None, None, :].expand(e_cnt, p, p, p), ys[:, None, :, None].expand(e_cnt, p, p, p),
           zs[:, :, None, None].expand(e_cnt, p, p, p))
    return tuple((c.to(dtype) if dtype is not None else c).contiguous() for c in out)


def ae_training_elements(seed, count, shape=AE_SHAPE, phases=AE_PHASES):
    """(phase, element) pairs of a training sample: `count` elements drawn
    uniformly from the integer phases and the mesh, seeded."""
    rng = np.random.default_rng(30_000 + seed)
    n_el = shape[0] * shape[1] * shape[2]
    return rng.integers(0, phases, size=count), rng.integers(0, n_el, size=count)
