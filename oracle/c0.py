"""C0 averaging over shared GLL nodes, global edge keys, welding (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Elements store their own copy of every node, so a node on an element face,
edge or corner is stored once per element that touches it.  A global id per
stored node (``gid``, equal for coincident nodes) identifies the copies.
Fields derived per element (Q, |omega|) differ between the copies; the
direct-stiffness average -- the gather-scatter sum of spectral-element codes
(Deville, Fischer & Mund 2002, ch. 4) divided by the multiplicity --
replaces every copy by the mean over all copies of its node:

  s_g = f_{n_1} + f_{n_2} + ... + f_{n_m}   (copies of g in increasing
                                            storage order, summed left to
                                            right in the field's precision)
  avg_g = s_g / m_g,    out_n = avg_{gid[n]}.

Global edge key of a triangle vertex lying on the edge between stored nodes
a and b:  (min(gid_a, gid_b) << 32) | max(gid_a, gid_b)  (ids < 2^32).

Welding a triangle soup: the distinct keys, in order of first occurrence
(corner r = 3 * triangle + corner index), are the vertices; a vertex takes
the coordinates of its first occurrence, and every triangle corner gets the
index of its key.
"""

import numpy as np


def multiplicity(gid):
    """Number of stored copies of each node, per stored node."""
    g = np.asarray(gid).ravel()
    cnt = np.bincount(g)
    return cnt[g].reshape(np.shape(gid))


def dsavg(field, gid):
    """Direct-stiffness average of ``field`` over nodes with equal ``gid``.

    The sums run over the copies in increasing storage order, one addition
    at a time, in the field's own dtype (``np.add.at`` is unbuffered and
    sequential); the result has the field's dtype.
    """
    f = np.asarray(field)
    g = np.asarray(gid).ravel()
    n_global = int(g.max()) + 1 if g.size else 0
    s = np.zeros(n_global, dtype=f.dtype)
    np.add.at(s, g, f.ravel())
    m = np.bincount(g, minlength=n_global).astype(f.dtype)
    avg = np.zeros_like(s)
    np.divide(s, m, out=avg, where=m > 0)
    return avg[g].reshape(f.shape)


def edge_nodes(local_keys, order):
    """(element, low node, high node) of element-local edge keys
    (e (N+1)^3 + n_lo) * 3 + axis."""
    p = order + 1
    k = np.asarray(local_keys, dtype=np.uint64).astype(np.int64)
    axis = k % 3
    flat = k // 3
    e, n_lo = flat // p ** 3, flat % p ** 3
    step = np.array([1, p, p * p], dtype=np.int64)[axis]
    return e, n_lo, n_lo + step


def global_edge_keys(local_keys, gid, order):
    """Global keys of element-local edge keys, given the node ids."""
    p = order + 1
    e, lo, hi = edge_nodes(local_keys, order)
    g = np.asarray(gid, dtype=np.int64).reshape(-1, p ** 3)
    a, b = g[e, lo], g[e, hi]
    mn, mx = np.minimum(a, b), np.maximum(a, b)
    return ((mn.astype(np.uint64) << np.uint64(32)) | mx.astype(np.uint64)).reshape(
        np.shape(local_keys))


def weld(tri_xyz, keys):
    """(vertices (V, 3), indices (T, 3) int64) of a soup with global keys."""
    k = np.asarray(keys, dtype=np.uint64).ravel()
    xyz = np.asarray(tri_xyz).reshape(-1, 3)
    if k.size == 0:
        return xyz[:0].copy(), np.zeros((0, 3), dtype=np.int64)
    uniq, first, inverse = np.unique(k, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")      # distinct keys by first occurrence
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    idx = rank[inverse.ravel()].reshape(-1, 3).astype(np.int64)
    return xyz[first[order]].copy(), idx
