"""Pins of the oracle of the paper's own update (Sec. 4.3, Algorithm 1; oracle/mc.py): the
level-set extraction on an analytic field whose iso-surface is a known sphere (closed, so
the face vectors sum to zero; outward; area converging to 4 pi r^2), the grid against a
brute-force cell list, and the update's fixed point on a sphere with exact normals."""
import math

import numpy as np

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


def test_level_set_of_a_ball_is_closed_outward_and_converges():
    areas = []
    for depth in (4, 5, 6):
        cells, cidx, pos, w, iso = _ball_field(depth)
        tris, vecs = mc.marching_tets(cells, cidx, pos, w, iso)
        cen = tris.mean(axis=1)
        area = 0.5 * np.linalg.norm(vecs, axis=1).sum()
        assert np.linalg.norm(vecs.sum(axis=0)) <= 1e-9 * area  # closed surface
        assert np.all(np.sum(vecs * cen, axis=1) > 0)  # every face points away from w > iso
        np.testing.assert_allclose(np.linalg.norm(cen, axis=1), 0.7, atol=2.0 / 2 ** depth)
        areas.append(area)
    err = [abs(a - 4 * math.pi * 0.49) / (4 * math.pi * 0.49) for a in areas]
    assert err[2] < err[1] < err[0] and err[2] < 0.01, err


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


def test_update_fixed_point_on_a_sphere():
    """Exact outward normals: the level set is close to the sphere and the update returns
    normals within a few degrees of radial, all outward."""
    s = synth.sphere(3000, 0.0, 3)
    N1, iso, nf, cnt = mc.update(s.P, s.N_true, s.area, None, depth=5, dilate=1)
    cos = np.sum(N1 * s.N_true, axis=0)
    assert 0.4 < iso < 0.6 and nf > 1000
    assert np.mean(cnt > 0) > 0.95
    assert np.all(cos[cnt > 0] > 0.95)
