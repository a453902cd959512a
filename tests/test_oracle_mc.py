"""Pins of the oracle of the paper's own update (Sec. 4.3, Algorithm 1; oracle/mc.py).

The level-set extraction (standard Marching Cubes, the paper's method) is pinned by:
  * a linear field, whose level set is a plane: every vertex on the plane, every face
    vector along the descending gradient, and the total area equal to the plane's
    cross-section of the box, computed independently by clipping in 2D;
  * a ball field w = 1 - |x|^2: a closed (every mesh edge shared by two faces wound
    oppositely), genus-0 (Euler characteristic 2) surface with outward faces whose area
    converges to 4 pi r^2;
  * a noisy field with many ambiguous faces: still closed;
  * every one of the 256 corner configurations against the topology the face rule
    implies: the loops use each cut edge once, and their number is A + B - 1 with A the
    edge-connected groups of above corners and B the groups of below corners joined by
    edges and by the diagonals of faces whose above corners are diagonal;
  * hand-worked cubes (one corner, an edge, an ambiguous face and its complement).
The marching-tetrahedra option keeps the ball pin; the grid is checked against a
brute-force cell list, and the update's fixed point on a sphere with exact normals."""
import math

import numpy as np
import pytest

from oracle import mc
from paper_2405_13839_amd import synth


def _ball_field(depth, r=0.7):
    s = synth.fibonacci_sphere(4000, R=r)
    P = np.concatenate([s.P, np.array([[-1.0, 1.0], [-1.0, 1.0], [-1.0, 1.0]])], axis=1)  # frame [-1, 1]^3
    cells, lo, side = mc.grid_cells(P, depth, dilate=1)
    cells = cells[np.linalg.norm((cells + 0.5) * side / 2 ** depth + lo - 0.0, axis=1) < 1.2]
    _, pos, cidx = mc.corners(cells, lo, side, depth)
    w = 1.0 - np.sum(np.asarray(pos, np.float64) ** 2, axis=0)
    return cells, cidx, pos, w, 1.0 - r * r


def _box_grid(G, side=1.0):
    """Every cell of a G^3 box over [0, side]^3."""
    c = np.stack(np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij"), axis=-1).reshape(-1, 3)
    depth = int(round(math.log2(G)))
    _, pos, cidx = mc.corners(c, np.zeros(3), side, depth)
    return c, cidx, pos


def _mesh_edges(tris):
    """Directed edges of the triangle soup as pairs of vertex keys (exact coordinates: a
    crossing is computed from the same corner values in both cubes sharing its edge)."""
    keys = {}

    def key(p):
        return keys.setdefault(tuple(p.tolist()), len(keys))

    out = []
    for t in tris:
        a, b, c = key(t[0]), key(t[1]), key(t[2])
        out += [(a, b), (b, c), (c, a)]
    return out, len(keys)


def _assert_closed(tris):
    edges, nv = _mesh_edges(tris)
    directed = {}
    for e in edges:
        directed[e] = directed.get(e, 0) + 1
    assert max(directed.values()) == 1, "a directed edge is used twice (inconsistent winding)"
    for (a, b) in directed:
        assert (b, a) in directed, "an edge with one face only (a hole)"
    return nv, len(directed) // 2


@pytest.mark.parametrize("surface", ["cubes", "tets"])
def test_level_set_of_a_ball_is_closed_outward_and_converges(surface):
    areas = []
    for depth in (4, 5, 6):
        cells, cidx, pos, w, iso = _ball_field(depth)
        tris, vecs = mc.extract(cells, cidx, pos, w, iso, surface)
        cen = tris.mean(axis=1)
        area = 0.5 * np.linalg.norm(vecs, axis=1).sum()
        assert np.linalg.norm(vecs.sum(axis=0)) <= 1e-9 * area  # closed surface
        assert np.all(np.sum(vecs * cen, axis=1) > 0)  # every face points away from w > iso
        np.testing.assert_allclose(np.linalg.norm(cen, axis=1), 0.7, atol=2.0 / 2 ** depth)
        if surface == "cubes":
            nv, ne = _assert_closed(tris)
            assert nv - ne + len(tris) == 2  # a sphere
            np.testing.assert_allclose(vecs, np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]))
        areas.append(area)
    err = [abs(a - 4 * math.pi * 0.49) / (4 * math.pi * 0.49) for a in areas]
    assert err[2] < err[1] < err[0] and err[2] < 0.01, err


def _clip(poly, a, b, c):
    """Sutherland-Hodgman: the part of polygon `poly` where a x + b y <= c."""
    out = []
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        fp, fq = a * p[0] + b * p[1] - c, a * q[0] + b * q[1] - c
        if fp <= 0:
            out.append(p)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def _shoelace(poly):
    return 0.5 * abs(sum(p[0] * q[1] - q[0] * p[1] for p, q in zip(poly, poly[1:] + poly[:1])))


@pytest.mark.parametrize("g,iso", [((1.0, 2.0, 3.0), 2.9), ((-0.3, 0.5, 1.1), 0.2), ((2.0, -1.0, 0.7), 0.45)])
def test_level_set_of_a_linear_field_is_its_plane(g, iso):
    """w = g . x on the box [0, 1]^3 (8^3 cells): linear interpolation on an edge is exact,
    so the level set is the plane g . x = iso clipped to the box."""
    g = np.array(g)
    cells, cidx, pos = _box_grid(8)
    P = np.asarray(pos, np.float64)
    w = g @ P
    tris, vecs = mc.marching_cubes(cells, cidx, pos, w, iso)
    assert len(tris) > 0
    np.testing.assert_allclose(tris.reshape(-1, 3) @ g, iso, atol=1e-12)
    gh = g / np.linalg.norm(g)
    nv = np.linalg.norm(vecs, axis=1)
    keep = nv > 1e-14
    np.testing.assert_allclose(vecs[keep] / nv[keep, None], np.tile(-gh, (keep.sum(), 1)), atol=1e-9)
    # the cross-section's area: its projection on the plane of the two axes least aligned
    # with g, clipped to the square by 0 <= x_k <= 1 along the third axis, over |g_k|/|g|
    k = int(np.argmax(np.abs(g)))
    i, j = [a for a in range(3) if a != k]
    # x_k = (iso - g_i x_i - g_j x_j) / g_k in [0, 1]
    poly = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    s = np.sign(g[k])
    poly = _clip(poly, s * g[i], s * g[j], s * iso)  # x_k >= 0
    poly = _clip(poly, -s * g[i], -s * g[j], s * g[k] - s * iso)  # x_k <= 1
    want = _shoelace(poly) / abs(gh[k])
    np.testing.assert_allclose(0.5 * nv.sum(), want, rtol=1e-12)


def test_level_set_with_ambiguous_faces_is_closed():
    """A random field below the iso-value on the box's boundary: many ambiguous faces, and
    the surface is still closed with consistent winding."""
    rng = np.random.default_rng(7)
    cells, cidx, pos = _box_grid(8)
    P = np.asarray(pos, np.float64)
    w = rng.uniform(-1, 1, P.shape[1])
    edge = np.any((P <= 1e-12) | (P >= 1 - 1e-12), axis=0)
    w[edge] = -1.0
    iso = 0.0
    tris, vecs = mc.marching_cubes(cells, cidx, pos, w, iso)
    amb = 0
    for ci in range(len(cells)):
        ab = w[cidx[ci]] > iso
        for walk in mc.FACE_WALKS:
            s = [ab[k] for k in walk]
            amb += int(s[0] == s[2] and s[1] == s[3] and s[0] != s[1])
    assert amb > 100  # an interior ambiguous face counts once from each of its two cubes
    _assert_closed(tris)
    assert np.linalg.norm(vecs.sum(axis=0)) <= 1e-12 * np.abs(vecs).sum()


def _components(nodes, links):
    parent = {v: v for v in nodes}

    def root(v):
        while parent[v] != v:
            v = parent[v]
        return v

    for a, b in links:
        if a in parent and b in parent:
            parent[root(a)] = root(b)
    return len({root(v) for v in nodes})


def test_every_cube_configuration_has_the_face_rule_topology():
    edges = [(u, u | (1 << a)) for u in range(8) for a in range(3) if not (u >> a) & 1]
    faces = [[k for k in range(8) if ((k >> a) & 1) == s] for a in range(3) for s in (0, 1)]
    for case in range(256):
        ab = [bool((case >> k) & 1) for k in range(8)]
        loops = mc.cube_loops(ab)
        cut = sorted(mc.EDGE_INDEX[e] for e in edges if ab[e[0]] != ab[e[1]])
        assert sorted(e for lp in loops for e in lp) == cut  # each cut edge once
        assert all(len(lp) >= 3 for lp in loops)
        assert all(lp[0] == min(lp) for lp in loops) and [lp[0] for lp in loops] == sorted(lp[0] for lp in loops)
        up = [k for k in range(8) if ab[k]]
        down = [k for k in range(8) if not ab[k]]
        A = _components(up, edges)
        diag = []
        for f in faces:  # corners of a face: f[0], f[3] and f[1], f[2] are the diagonals
            if ab[f[0]] == ab[f[3]] and ab[f[1]] == ab[f[2]] and ab[f[0]] != ab[f[1]]:
                diag += [(f[0], f[3]), (f[1], f[2])]
        B = _components(down, edges + diag)
        want = 0 if not up or not down else A + B - 1
        assert len(loops) == want, (case, loops, A, B)


def _face_above_area(ab, wv, iso, face_corners, xy):
    """Area of the part of a unit face on the above side of its segments: for every run of
    above corners along the face's boundary cycle, the polygon of the entry crossing, the run's
    corners and the exit crossing (shoelace in the face's own 2D coordinates)."""
    cyc = face_corners
    if all(ab[k] for k in cyc):
        return 1.0
    out = 0.0
    for i in range(4):
        a, b = cyc[i], cyc[(i + 1) % 4]
        if ab[a] or not ab[b]:
            continue
        pts = []

        def cross(u, v):
            t = (iso - wv[u]) / (wv[v] - wv[u])
            return xy[u] + t * (xy[v] - xy[u])

        pts.append(cross(a, b))
        j = (i + 1) % 4
        while ab[cyc[j]]:
            pts.append(xy[cyc[j]])
            j = (j + 1) % 4
        pts.append(cross(cyc[(j - 1) % 4], cyc[j]))
        out += _shoelace([tuple(p) for p in pts])
    return out



def test_every_cube_configuration_winds_away_from_its_above_corners():
    """Divergence theorem on the above region U of one cube: its boundary is the extracted
    surface plus the above parts of the six faces, so the surface's vector area is
    -sum_faces f * area(U on f) (f the outward face normal), and the triangles' cross
    products add up to twice that. Random corner values, every configuration."""
    rng = np.random.default_rng(11)
    cells = np.zeros((1, 3), np.int64)
    _, pos, cidx = mc.corners(cells, np.zeros(3), 1.0, 0)
    off = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], np.float64)
    for case in range(1, 255):
        ab = [bool((case >> k) & 1) for k in range(8)]
        wv = np.where(ab, rng.uniform(0.55, 1.0, 8), rng.uniform(0.0, 0.45, 8))
        w = np.empty(8)
        w[cidx[0]] = wv
        t, v = mc.marching_cubes(cells, cidx, pos, w, 0.5)
        want = np.zeros(3)
        for axis in range(3):
            for side in (0, 1):
                a1, a2 = (axis + 1) % 3, (axis + 2) % 3
                ring = [k for k in range(8) if ((k >> axis) & 1) == side]
                # the face's corners in cyclic order (any direction: the area is unsigned)
                ring = sorted(ring, key=lambda k: np.arctan2(off[k, a2] - 0.5, off[k, a1] - 0.5))
                area = _face_above_area(ab, wv, 0.5, ring, {k: off[k, [a1, a2]] for k in ring})
                want[axis] += (2 * side - 1) * area
        np.testing.assert_allclose(v.sum(axis=0), -2.0 * want, atol=1e-12, err_msg=str(case))


def _one_cube(above, lo=0.0, hi=1.0):
    cells = np.zeros((1, 3), np.int64)
    _, pos, cidx = mc.corners(cells, np.zeros(3), 1.0, 0)
    w = np.empty(8)
    w[cidx[0]] = np.where(np.array(above, bool), hi, lo)  # corner k of the cell is lattice point cidx[0, k]
    return mc.marching_cubes(cells, cidx, pos, w, 0.5 * (lo + hi))


def test_hand_worked_cubes():
    # one corner (0) above: the triangle of the three edge midpoints, wound away from it
    t, v = _one_cube([1, 0, 0, 0, 0, 0, 0, 0])
    assert t.shape == (1, 3, 3)
    assert sorted(map(tuple, t[0].tolist())) == [(0, 0, 0.5), (0, 0.5, 0), (0.5, 0, 0)]
    np.testing.assert_allclose(v[0], [0.25, 0.25, 0.25])
    # an edge (corners 0, 1) above: the quad y + z = 0.5 around it (area 1/sqrt(2)), two
    # triangles whose cross products add up to twice its vector area
    t, v = _one_cube([1, 1, 0, 0, 0, 0, 0, 0])
    assert t.shape == (2, 3, 3)
    np.testing.assert_allclose(v.sum(axis=0), [0, 1.0, 1.0])
    # corners 0 and 3 (a diagonal of the face z = 0) above: separated, two triangles
    t, v = _one_cube([1, 0, 0, 1, 0, 0, 0, 0])
    assert t.shape == (2, 3, 3)
    np.testing.assert_allclose(sorted(np.round(v, 12).tolist()), sorted([[0.25, 0.25, 0.25], [-0.25, -0.25, 0.25]]))
    # its complement: the below corners 0 and 3 are joined across that face: one hexagon;
    # the above part of the faces is 1/4 of z = 0, all of z = 1, 7/8 of the four sides, so
    # the cross products add up to -2 (0, 0, 1 - 1/4)
    t, v = _one_cube([0, 1, 1, 0, 1, 1, 1, 1])
    assert t.shape == (4, 3, 3)
    np.testing.assert_allclose(v.sum(axis=0), [0, 0, -1.5], atol=1e-15)
    # corners 0 and 7 (a body diagonal) above: two separate triangles
    t, v = _one_cube([1, 0, 0, 0, 0, 0, 0, 1])
    assert t.shape == (2, 3, 3)
    np.testing.assert_allclose(v.sum(axis=0), [0, 0, 0], atol=1e-15)


def test_grid_cells_match_brute_force():
    rng = np.random.default_rng(2)
    P = rng.uniform(-1, 2, (3, 500)).astype(np.float32)
    for depth, dil in [(3, 0), (4, 1), (6, 1)]:
        cells, lo, side = mc.grid_cells(P, depth, dil)
        G = 2 ** depth
        h = side / G
        occ = set()
        for i in range(P.shape[1]):
            c = tuple(int(min(max(math.floor((float(P[d, i]) - lo[d]) / h), 0), G - 1)) for d in range(3))
            occ.add(c)
        want = set()
        for c in occ:
            for dx in range(-dil, dil + 1):
                for dy in range(-dil, dil + 1):
                    for dz in range(-dil, dil + 1):
                        q = (c[0] + dx, c[1] + dy, c[2] + dz)
                        if all(0 <= v < G for v in q):
                            want.add(q)
        assert set(map(tuple, cells.tolist())) == want
        codes = mc.morton(cells)
        assert np.all(np.diff(codes.astype(np.float64)) > 0)  # Morton order, no duplicates


@pytest.mark.parametrize("surface", ["cubes", "tets"])
def test_update_fixed_point_on_a_sphere(surface):
    """Exact outward normals: the level set is close to the sphere and the update returns
    normals within a few degrees of radial, all outward."""
    s = synth.sphere(3000, 0.0, 3)
    N1, iso, nf, cnt = mc.update(s.P, s.N_true, s.area, None, depth=5, dilate=1, surface=surface)
    cos = np.sum(N1 * s.N_true, axis=0)
    assert 0.4 < iso < 0.6 and nf > 1000
    assert np.mean(cnt > 0) > 0.95
    assert np.all(cos[cnt > 0] > 0.95)
