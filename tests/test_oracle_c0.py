"""Pins of the C0-averaging and welding oracle (oracle/c0.py).

The statements checked are fixed by the definitions, not by re-typing them:
multiplicities of a lattice (1 inside, 2 on faces, 4 on edges, 8 at
corners), a two-element example with exact dyadic averages, C0 inputs left
unchanged, a C0 result, conservation of the total, idempotence, and -- for
welding -- that the isosurface of a smooth closed level set, welded over a
multi-element lattice, is a closed oriented 2-manifold of Euler
characteristic 2 whose vertices are exactly the distinct crossed lattice
edges.
"""

import numpy as np

import workloads as W
from oracle import c0, mc


def test_lattice_multiplicities():
    n = 3
    gid = W.lattice_gid((2, 2, 2), n)
    m = c0.multiplicity(gid)
    p = n + 1
    # stored node (i, j, k) of an element: each coordinate on the shared
    # middle plane doubles the count
    e_axes = W.element_axes((2, 2, 2))
    for e in range(8):
        ex, ey, ez = e_axes[0][e], e_axes[1][e], e_axes[2][e]
        for k in range(p):
            for j in range(p):
                for i in range(p):
                    shared = sum(((ex == 0 and i == n) or (ex == 1 and i == 0),
                                  (ey == 0 and j == n) or (ey == 1 and j == 0),
                                  (ez == 0 and k == n) or (ez == 1 and k == 0)))
                    assert m[e, k, j, i] == 2 ** shared
    assert int(gid.max()) + 1 == (2 * n + 1) ** 3


def test_two_element_example_exact():
    n = 1
    gid = W.lattice_gid((2, 1, 1), n)           # 12 lattice nodes, 4 shared
    f = np.zeros((2, 2, 2, 2))
    f[0] = 1.0
    f[1] = 2.0
    f[1, :, :, 1] = 5.0                          # the far face of element 1
    out = c0.dsavg(f, gid)
    # shared face (element 0 at i = 1, element 1 at i = 0): (1 + 2) / 2
    assert np.all(out[0, :, :, 1] == 1.5) and np.all(out[1, :, :, 0] == 1.5)
    assert np.all(out[0, :, :, 0] == 1.0) and np.all(out[1, :, :, 1] == 5.0)


def _c0_field(shape, n, seed=0):
    x, y, z = W.box_mesh(shape, n, ((0, 1.0), (0, 1.3), (0, 0.8)))
    rng = np.random.default_rng(seed)
    a = rng.normal(size=4)
    return np.sin(3 * x + a[0]) * np.cos(2 * y + a[1]) + a[2] * z * x + a[3]


def test_c0_input_is_kept_and_output_is_c0():
    shape, n = (3, 2, 2), 4
    gid = W.lattice_gid(shape, n)
    f = _c0_field(shape, n)
    out = c0.dsavg(f, gid)
    # copies of a C0 field are identical: the mean is the value to rounding
    np.testing.assert_allclose(out, f, rtol=4e-16, atol=4e-16)
    rng = np.random.default_rng(3)
    g = rng.normal(size=f.shape)                 # discontinuous across faces
    out = c0.dsavg(g, gid)
    flat_g, flat_o = gid.ravel(), out.ravel()
    order = np.argsort(flat_g, kind="stable")
    sg, so = flat_g[order], flat_o[order]
    same = sg[1:] == sg[:-1]
    assert np.array_equal(so[1:][same], so[:-1][same])     # bitwise C0
    # conservation: sum of the copies is unchanged (to rounding)
    assert abs(out.sum() - g.sum()) < 1e-12 * np.abs(g).sum()
    # idempotent
    np.testing.assert_allclose(c0.dsavg(out, gid), out, rtol=4e-16, atol=4e-16)
    # interior nodes (multiplicity 1) untouched, bit for bit
    inner = c0.multiplicity(gid) == 1
    assert np.array_equal(out[inner], g[inner])


def test_dsavg_fp32_sums_in_fp32():
    gid = W.lattice_gid((2, 1, 1), 2)
    g = np.random.default_rng(1).normal(size=gid.shape).astype(np.float32)
    out = c0.dsavg(g, gid)
    assert out.dtype == np.float32


def _sphere_soup(shape, n, r=0.31, center=(0.5, 0.52, 0.47)):
    x, y, z = W.box_mesh(shape, n, ((0, 1.0), (0, 1.0), (0, 1.0)))
    f = r * r - ((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    gid = W.lattice_gid(shape, n)
    res = mc.extract(x, y, z, f, [0.0], edge_keys=True)
    keys = c0.global_edge_keys(res["edge_key"].astype(np.uint64), gid, n)
    return res, keys, gid, f


def test_welded_sphere_is_closed_manifold_across_elements():
    shape, n = (3, 3, 3), 3
    res, keys, gid, f = _sphere_soup(shape, n)
    verts, idx = c0.weld(res["tri_xyz"], keys)
    t = idx.shape[0]
    assert t > 200
    # every directed edge once, its reverse once: closed and oriented
    directed = np.concatenate([idx[:, [0, 1]], idx[:, [1, 2]], idx[:, [2, 0]]])
    d = {}
    for a, b in map(tuple, directed):
        d[(a, b)] = d.get((a, b), 0) + 1
    assert all(v == 1 for v in d.values())
    assert all((b, a) in d for (a, b) in d)
    n_edges = len(d) // 2
    assert verts.shape[0] - n_edges + t == 2                 # Euler characteristic
    # vertices = distinct crossed lattice edges (an edge between lattice
    # points with the field above at exactly one end)
    assert verts.shape[0] == np.unique(keys).size
    # vertices are numbered in order of first occurrence: reading the
    # corners in order, each new index is the next integer
    seen, nxt = set(), 0
    for v in idx.ravel():
        if v not in seen:
            assert v == nxt
            seen.add(v)
            nxt += 1
    # each vertex position is the first occurrence's
    flat = res["tri_xyz"].reshape(-1, 3)
    first = {}
    for r, k in enumerate(np.asarray(keys).ravel()):
        first.setdefault(int(k), r)
    for v in range(0, verts.shape[0], 97):
        k = int(np.asarray(keys).ravel()[np.argmax(idx.ravel() == v)])
        assert np.array_equal(verts[v], flat[first[k]])


def test_global_keys_agree_across_shared_faces():
    shape, n = (2, 2, 2), 3
    res, keys, gid, _ = _sphere_soup(shape, n, r=0.4, center=(0.5, 0.5, 0.5))
    flat = res["tri_xyz"].reshape(-1, 3)
    k = np.asarray(keys).ravel()
    # equal global keys <=> the same lattice edge: the positions agree bit
    # for bit (the lattice coordinates and field are identical copies)
    order = np.argsort(k, kind="stable")
    ks, ps = k[order], flat[order]
    same = ks[1:] == ks[:-1]
    assert same.any()
    assert np.array_equal(ps[1:][same], ps[:-1][same])
    # and distinct keys are distinct points
    uniq_pts = np.unique(flat, axis=0).shape[0]
    assert uniq_pts == np.unique(k).size


def test_weld_of_empty_soup():
    v, i = c0.weld(np.zeros((0, 3, 3)), np.zeros((0, 3), dtype=np.uint64))
    assert v.shape == (0, 3) and i.shape == (0, 3)
