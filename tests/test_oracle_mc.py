"""Pins for the oracle's marching-cubes case table, extraction and compaction.

Fixed by combinatorics and geometry: triangle count = crossed edges - 2 loops,
invariance of the loop structure under the 48 symmetries of the cube (23 case
orbits under rotations, 22 under rotations and reflections), brute-force
watertightness over every sign pattern of small cell grids, the Euler
characteristic, enclosed volume and area of an extracted sphere, and the
exact symmetry of the Taylor-Green Q isosurface.
"""

import itertools

import numpy as np
import pytest

import workloads as W
from oracle import gll, mc, sem


# --------------------------------------------------------------------------
# case table
# --------------------------------------------------------------------------

def _crossed(case):
    bit = [(case >> v) & 1 for v in range(8)]
    return [e for e in range(12)
            if bit[mc.EDGE_CORNERS[e][0]] != bit[mc.EDGE_CORNERS[e][1]]]


def test_triangle_count_is_crossed_minus_two_loops():
    ntri, table = mc.case_table()
    assert ntri[0] == 0 and ntri[255] == 0
    for c in range(256):
        loops = mc.case_loops(c)
        crossed = _crossed(c)
        assert sorted(e for lp in loops for e in lp) == crossed
        assert all(len(lp) >= 3 for lp in loops)
        assert ntri[c] == len(crossed) - 2 * len(loops)
        tris = table[c, :ntri[c]]
        assert (table[c, ntri[c]:] == -1).all()
        # every triangle uses crossed edges only, all three distinct
        for t in tris:
            assert len(set(t.tolist())) == 3 and set(t.tolist()) <= set(crossed)


def test_single_corner_cases_are_one_triangle():
    ntri, _ = mc.case_table()
    for v in range(8):
        assert ntri[1 << v] == 1
        assert ntri[255 ^ (1 << v)] == 1


def _symmetries():
    """The 48 cube symmetries as corner permutations, with their determinant."""
    out = []
    for perm in itertools.permutations(range(3)):
        sgn = np.linalg.det(np.eye(3)[list(perm)])
        for flips in itertools.product((0, 1), repeat=3):
            det = sgn * (-1) ** sum(flips)
            mapping = []
            for v in range(8):
                a = mc.CORNER_POS[v]
                b = [a[perm[d]] ^ flips[d] for d in range(3)]
                mapping.append(b[0] + 2 * b[1] + 4 * b[2])
            out.append((mapping, det))
    return out


def _apply(case, mapping):
    return sum(((case >> v) & 1) << mapping[v] for v in range(8))


def test_loop_structure_invariant_under_cube_symmetries():
    syms = _symmetries()
    assert len(syms) == 48
    ntri, _ = mc.case_table()
    shape = {c: sorted(len(lp) for lp in mc.case_loops(c)) for c in range(256)}
    for c in range(256):
        for mapping, _ in syms:
            c2 = _apply(c, mapping)
            assert shape[c2] == shape[c]
            assert ntri[c2] == ntri[c]


def _orbit_count(group):
    seen, orbits = set(), 0
    for c in range(256):
        if c in seen:
            continue
        orbits += 1
        for mapping, _ in group:
            seen.add(_apply(c, mapping))
    return orbits


def test_orbit_counts_match_burnside():
    syms = _symmetries()
    rot = [s for s in syms if s[1] > 0]
    assert len(rot) == 24
    assert _orbit_count(rot) == 23
    assert _orbit_count(syms) == 22


def test_complement_symmetry_fails_only_on_ambiguous_faces():
    # corners 0 and 3 above: the z=0 face is ambiguous -> above corners are
    # separated (two loops); the complement connects them (one loop)
    case = (1 << 0) | (1 << 3)
    assert len(mc.case_loops(case)) == 2
    assert len(mc.case_loops(255 ^ case)) == 1
    # without ambiguous faces complementing keeps the loop structure
    for c in range(256):
        bit = [(c >> v) & 1 for v in range(8)]
        ambiguous = any(
            len([e for e in edges if bit[mc.EDGE_CORNERS[e][0]] != bit[mc.EDGE_CORNERS[e][1]]]) == 4
            for _, _, _, edges, _ in mc.FACES)
        if not ambiguous:
            assert (sorted(map(len, mc.case_loops(c)))
                    == sorted(map(len, mc.case_loops(255 ^ c))))


# --------------------------------------------------------------------------
# brute-force watertightness on small grids
# --------------------------------------------------------------------------

def _grid_elements(dims, node_vals):
    """Order-1 elements (one cell each) of patterns on a dims-cell lattice.

    node_vals: (patterns, nz+1, ny+1, nx+1).  Returns x, y, z, f with shape
    (patterns * nx*ny*nz, 2, 2, 2) and the (pattern, cx, cy, cz) of each.
    """
    nx, ny, nz = dims
    pats = node_vals.shape[0]
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    pe = np.repeat(np.arange(pats), cx.size)
    ex, ey, ez = np.tile(cx, pats), np.tile(cy, pats), np.tile(cz, pats)
    o = np.array([0, 1])
    kk, jj, ii = np.meshgrid(o, o, o, indexing="ij")
    gx = ex[:, None, None, None] + ii
    gy = ey[:, None, None, None] + jj
    gz = ez[:, None, None, None] + kk
    f = node_vals[pe[:, None, None, None], gz, gy, gx]
    return (gx.astype(float), gy.astype(float), gz.astype(float), f,
            (pe, ex, ey, ez))


def _global_vertex_ids(keys, origin, dims, p):
    """Map element-local edge keys to ids of global lattice edges."""
    pe, ex, ey, ez = origin
    axis = keys % 3
    rest = keys // 3
    e = rest // (p ** 3)
    n_lo = rest % (p ** 3)
    i, j, k = n_lo % p, (n_lo // p) % p, n_lo // (p * p)
    n = p - 1
    gx = ex[e] * n + i
    gy = ey[e] * n + j
    gz = ez[e] * n + k
    nx, ny, nz = (d * n + 1 for d in dims)
    gid = (((pe[e] * nz + gz) * ny + gy) * nx + gx) * 3 + axis
    return gid.astype(np.int64), (gx, gy, gz, axis)


def _check_watertight(tri_gid, on_boundary_plane):
    """Interior sides used once each way; boundary sides used exactly once."""
    a = tri_gid
    src = np.concatenate([a[:, 0], a[:, 1], a[:, 2]])
    dst = np.concatenate([a[:, 1], a[:, 2], a[:, 0]])
    assert np.all(src != dst)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    fwd = src < dst
    key = lo * (np.int64(1) << np.int64(31)) + hi
    order = np.argsort(key, kind="stable")
    key, fwd = key[order], fwd[order]
    uniq, start, count = np.unique(key, return_index=True, return_counts=True)
    nf = np.add.reduceat(fwd.astype(np.int64), start)
    bnd = on_boundary_plane(src[order][start], dst[order][start])
    # interior: exactly two uses, opposite directions
    assert np.all(count[~bnd] == 2)
    assert np.all(nf[~bnd] == 1)
    # boundary: exactly one use
    assert np.all(count[bnd] == 1)
    return uniq.size


def _boundary_fn(planes_of):
    def on_plane(s, d):
        ps, pd = planes_of(s), planes_of(d)
        return np.any(ps & pd, axis=1)
    return on_plane


def _planes_factory(dims, n):
    nx, ny, nz = (d * n for d in dims)
    lat = (nx + 1, ny + 1, nz + 1)

    def planes_of(gid):
        axis = gid % 3
        r = gid // 3
        gx = r % lat[0]
        gy = (r // lat[0]) % lat[1]
        gz = (r // (lat[0] * lat[1])) % lat[2]
        out = np.zeros((gid.size, 6), dtype=bool)
        for d, (g, m) in enumerate(((gx, nx), (gy, ny), (gz, nz))):
            off = axis != d          # edge lies in planes normal to d
            out[:, 2 * d] = off & (g == 0)
            out[:, 2 * d + 1] = off & (g == m)
        return out
    return planes_of


@pytest.mark.parametrize("dims", [(1, 1, 2), (2, 1, 1), (1, 2, 1), (2, 2, 1)])
def test_watertight_all_sign_patterns(dims):
    nx, ny, nz = dims
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    pats = np.arange(2 ** nodes, dtype=np.int64)
    bits = (pats[:, None] >> np.arange(nodes)) & 1
    vals = np.where(bits == 1, 1.0, -1.0).reshape(-1, nz + 1, ny + 1, nx + 1)
    x, y, z, f, origin = _grid_elements(dims, vals)
    r = mc.extract(x, y, z, f, [0.0], edge_keys=True)
    gid, _ = _global_vertex_ids(r["edge_key"].astype(np.int64), origin, dims, 2)
    _check_watertight(gid, _boundary_fn(_planes_factory(dims, 1)))
    # vertices sit at edge midpoints for +-1 data at isovalue 0
    assert np.all((r["tri_xyz"] * 2) == np.round(r["tri_xyz"] * 2))


def test_watertight_random_real_values_3x3x3():
    dims = (3, 3, 3)
    rng = np.random.default_rng(11)
    vals = rng.normal(size=(400, 4, 4, 4))
    x, y, z, f, origin = _grid_elements(dims, vals)
    for iso in (-0.3, 0.0, 0.8):
        r = mc.extract(x, y, z, f, [iso], edge_keys=True)
        gid, _ = _global_vertex_ids(r["edge_key"].astype(np.int64), origin, dims, 2)
        _check_watertight(gid, _boundary_fn(_planes_factory(dims, 1)))


def test_watertight_inside_element_of_high_order():
    """Within one order-N element every interior side is shared twice."""
    n = 4
    rng = np.random.default_rng(3)
    f = rng.normal(size=(30, n + 1, n + 1, n + 1))
    x, y, z = (np.broadcast_to(a, f.shape).astype(float) for a in
               np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1),
                           indexing="ij")[::-1])
    r = mc.extract(x, y, z, f, [0.1], edge_keys=True)
    keys = r["edge_key"].astype(np.int64)
    dims = (1, 1, 1)
    # treat every element as its own pattern on a 1x1x1 element lattice
    origin = (np.arange(30), np.zeros(30, int), np.zeros(30, int), np.zeros(30, int))
    gid, _ = _global_vertex_ids(keys, origin, dims, n + 1)
    _check_watertight(gid, _boundary_fn(_planes_factory(dims, n)))


# --------------------------------------------------------------------------
# sphere: topology and geometry
# --------------------------------------------------------------------------

def _sphere(n, shape=(3, 3, 3), centre=(1.52, 1.47, 1.55), radius=0.9):
    x, y, z = W.box_mesh(shape, n, ((0.0, 3.0),) * 3)
    f = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    r = mc.extract(x, y, z, f, [radius ** 2], edge_keys=True)
    ex, ey, ez = W.element_axes(shape)
    origin = (np.zeros(ex.size, dtype=np.int64), ex, ey, ez)
    gid, _ = _global_vertex_ids(r["edge_key"].astype(np.int64), origin, shape, n + 1)
    return r, gid


@pytest.mark.parametrize("n", [2, 4, 7])
def test_sphere_is_closed_genus_zero_outward(n):
    radius = 0.9
    r, gid = _sphere(n, radius=radius)
    n_sides = _check_watertight(gid, lambda s, d: np.zeros(s.size, dtype=bool))
    v = np.unique(gid).size
    f = gid.shape[0]
    assert v - n_sides + f == 2
    p = r["tri_xyz"]
    # signed volume (divergence theorem): positive => normals point outward,
    # i.e. towards f > R^2
    vol = np.sum(np.einsum("ti,ti->t", p[:, 0], np.cross(p[:, 1], p[:, 2]))) / 6.0
    exact = 4.0 / 3.0 * np.pi * radius ** 3
    assert vol > 0
    assert abs(vol / exact - 1.0) < {2: 0.3, 4: 0.1, 7: 0.04}[n]


def _plane_pin(n=3):
    """Vertices of a linear field's isosurfaces on an affine box mesh (straight
    edges): linear interpolation along an edge is exact for a linear field,
    so every vertex lies on the plane a.p + b = c and between its edge's
    endpoints (the vertex rule; the plane is the closed form)."""
    x, y, z = W.box_mesh((3, 2, 2), n, ((0.0, 1.9), (-0.7, 0.6), (0.3, 1.5)))
    a = np.array([0.7, -1.3, 0.4])
    b = 0.2
    f = a[0] * x + a[1] * y + a[2] * z + b
    isos = [float(np.quantile(f, q)) for q in (0.21, 0.5, 0.83)]
    r = mc.extract(x, y, z, f, isos, edge_keys=True)
    p = r["tri_xyz"].reshape(-1, 3)
    cvals = np.repeat(np.repeat(isos, r["tri_count"]), 3)
    assert p.shape[0] > 100
    resid = np.abs(p @ a + b - cvals)
    scale = np.abs(a).sum() * np.abs(p).max() + abs(b)
    assert resid.max() <= 1e-13 * scale, resid.max()
    # between the endpoints of its edge (keys: element, low node, axis)
    keys = r["edge_key"].astype(np.int64).reshape(-1)
    axis = keys % 3
    node = keys // 3
    pp = n + 1
    hi = node + np.array([1, pp, pp * pp])[axis]
    for c, coord in enumerate((x, y, z)):
        lo_c, hi_c = coord.reshape(-1)[node], coord.reshape(-1)[hi]
        assert np.all(p[:, c] >= np.minimum(lo_c, hi_c) - 1e-12)
        assert np.all(p[:, c] <= np.maximum(lo_c, hi_c) + 1e-12)


def test_vertices_of_linear_field_lie_on_its_plane():
    _plane_pin()


def test_sphere_area_converges():
    radius = 0.9
    errs = []
    for n in (2, 4, 8):
        r, _ = _sphere(n, radius=radius)
        p = r["tri_xyz"]
        area = 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]),
                                    axis=1).sum()
        errs.append(abs(area / (4 * np.pi * radius ** 2) - 1.0))
    # linear interpolation on a quadratic field: second-order convergence
    assert errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3
    assert errs[2] < 0.02


# --------------------------------------------------------------------------
# classification, cull and compaction
# --------------------------------------------------------------------------

def test_fp32_classification_uses_fp32_isovalue():
    iso = 0.1                                  # not representable in FP32
    f32 = np.full((1, 2, 2, 2), np.float32(iso), dtype=np.float32)
    f32[0, 0, 0, 0] = np.nextafter(np.float32(iso), np.float32(1))
    cases = mc.classify(f32, iso)
    assert cases[0, 0, 0, 0] == 1              # only corner 0 is above
    f64 = f32.astype(np.float64)
    assert mc.classify(f64, iso)[0, 0, 0, 0] == 255   # float(0.1f) > 0.1


def test_nan_nodes_are_below():
    f = np.zeros((1, 2, 2, 2))
    f[0, 0, 0, 0] = np.nan
    f[0, 1, 1, 1] = 1.0
    assert mc.classify(f, 0.5)[0, 0, 0, 0] == 128


def test_cull_by_minmax_is_exact():
    """Elements rejected by min/max hold no active cell (and vice versa)."""
    rng = np.random.default_rng(5)
    f = rng.normal(size=(500, 4, 4, 4)) * rng.uniform(0.1, 2, size=(500, 1, 1, 1)) \
        + rng.normal(size=(500, 1, 1, 1)) * 2
    f[3, 0, 0, 0] = np.nan
    mm = sem.elem_minmax(f)
    for iso in (-1.0, 0.0, 0.7, 3.0):
        cases = mc.classify(f, iso).reshape(500, -1)
        has_active = np.any((cases != 0) & (cases != 255), axis=1)
        straddle = (mm[:, 1] > iso) & ~(mm[:, 0] > iso)
        # some node above and some node not above <=> some active cell
        # (the node lattice is connected through cell edges)
        np.testing.assert_array_equal(straddle, has_active)


def test_compaction_offsets_and_order():
    n = 3
    x, y, z = W.box_mesh((2, 2, 1), n, ((0, 1.0),) * 3)
    f = np.sin(5 * x) * np.cos(4 * y) + z
    r = mc.extract(x, y, z, f, [0.2, 0.6], edge_keys=True)
    cnt, off = r["cell_ntri"], r["cell_offset"]
    flat_c, flat_o = cnt.ravel(), off.ravel()
    assert flat_o[0] == 0
    np.testing.assert_array_equal(flat_o[1:], np.cumsum(flat_c)[:-1])
    assert r["tri_count"].sum() == flat_c.sum() == r["tri_xyz"].shape[0]
    # triangles of each cell sit at [offset, offset + count) and their edge
    # keys belong to that element and cell
    keys = r["edge_key"].astype(np.int64)
    p = n + 1
    e_of = (keys // 3) // p ** 3
    iso_cells = cnt.shape[1] * cnt.shape[2]
    for flat in np.nonzero(flat_c)[0][::7]:
        e = (flat % iso_cells) // cnt.shape[2]
        o, c = flat_o[flat], flat_c[flat]
        assert np.all(e_of[o:o + c] == e)


def test_taylor_green_octants_and_xy_swap_symmetry():
    n = 7
    x, y, z, u, v, w = W.tgv_config(n)
    q, _, _ = sem.qcrit(x, y, z, u, v, w, gll.diff_matrix(n))
    r = mc.extract(x, y, z, q, [0.1])
    ntri = r["cell_ntri"][0].sum(axis=1).reshape(8, 8, 8)      # [ez, ey, ex]
    act = ((r["cases"][0] != 0) & (r["cases"][0] != 255)).sum(axis=1).reshape(8, 8, 8)
    octs = [ntri[a:a + 4, b:b + 4, c:c + 4].sum() for a in (0, 4) for b in (0, 4)
            for c in (0, 4)]
    assert len(set(octs)) == 1
    np.testing.assert_array_equal(ntri, np.swapaxes(ntri, 1, 2))
    np.testing.assert_array_equal(act, np.swapaxes(act, 1, 2))
    mm = sem.elem_minmax(q)
    assert int(((mm[:, 1] > 0.1) & ~(mm[:, 0] > 0.1)).sum()) == 384
