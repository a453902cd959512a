"""Pins of the area-weight and windowed-radius oracles (Sec. 5.1 "Computing Area Weights",
Sec. 5.2 "Poisson Kernels") against closed forms and an independent Voronoi diagram."""
import math

import numpy as np

import oracle


def _tilt(P):
    """Rotate a planar cloud off the axes and translate it (the area is invariant)."""
    a, b = 0.4, -0.7
    Rx = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    return Ry @ Rx @ P + np.array([[0.3], [-0.2], [0.5]])


def test_square_lattice_cells_are_h_squared():
    h = 0.01
    g = np.arange(12) * h
    X, Y = np.meshgrid(g, g)
    P = _tilt(np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)]))
    a = oracle.voronoi_area(P, 15)
    inner = ((X.ravel() >= 3 * h) & (X.ravel() <= 8 * h) & (Y.ravel() >= 3 * h) & (Y.ravel() <= 8 * h))
    np.testing.assert_allclose(a[inner], h * h, rtol=1e-9)
    assert np.all(a[~inner] >= h * h * (1 - 1e-9))  # boundary cells reach the bounding square


def test_hexagonal_lattice_cells():
    h = 0.02
    pts = [(i * h + (j % 2) * h / 2, j * h * math.sqrt(3) / 2) for j in range(14) for i in range(14)]
    x, y = np.array(pts).T
    P = _tilt(np.stack([x, y, np.zeros_like(x)]))
    a = oracle.voronoi_area(P, 15)
    inner = (x > 4 * h) & (x < 9 * h) & (y > 4 * h) & (y < 8 * h)
    np.testing.assert_allclose(a[inner], math.sqrt(3) / 2 * h * h, rtol=1e-9)


def test_planar_random_cells_match_full_voronoi_diagram():
    """Interior points of a random planar set: the 15-NN cell equals the cell of the full
    2D Voronoi diagram (scipy.spatial.Voronoi) exactly when all of the point's Voronoi
    neighbours are among its 15 nearest (true for ~90% of points); otherwise it can only
    be larger (fewer half-planes)."""
    from scipy.spatial import ConvexHull, Voronoi
    rng = np.random.default_rng(4)
    xy = rng.uniform(0, 1, (2, 3000))
    P = _tilt(np.stack([xy[0], xy[1], np.zeros(3000)]))
    a = oracle.voronoi_area(P, 15)
    idx, _ = oracle.knn_self(P, 15)
    vor = Voronoi(xy.T)
    nbrs = [set() for _ in range(3000)]
    for p, q in vor.ridge_points:
        nbrs[p].add(q)
        nbrs[q].add(p)
    full, partial = 0, 0
    for i in range(3000):
        reg = vor.regions[vor.point_region[i]]
        if -1 in reg or len(reg) == 0:
            continue
        V = vor.vertices[reg]
        if V.min() < 0.1 or V.max() > 0.9:
            continue
        ref = ConvexHull(V).volume
        if nbrs[i].issubset(set(idx[i].tolist())):
            assert abs(a[i] - ref) <= 1e-9 * ref
            full += 1
        else:
            assert a[i] >= ref * (1 - 1e-9)
            partial += 1
    assert full > 1500 and partial < 0.15 * (full + partial)


def test_sphere_areas_sum_to_surface():
    from paper_2405_13839_amd import synth
    s = synth.fibonacci_sphere(4000)
    a = oracle.voronoi_area(s.P, 15)
    assert abs(a.sum() - 4 * math.pi) < 0.01 * 4 * math.pi
    assert a.std() / a.mean() < 0.05  # near-uniform sampling, near-uniform cells


def test_delta_window():
    """Points on a line with spacings 0.001, 0.004, 0.02: only the distances in the window
    [0.0015, 0.015] enter the mean; a point with none inside gets the clamped mean."""
    x = np.array([0.0, 0.001, 0.005, 0.025, 1.0, 1.001])
    P = np.stack([x, np.zeros(6), np.zeros(6)])
    d = oracle.delta_knn_window(P, 2, 0.0015, 0.015)
    # point 0: neighbours at 0.001 (out), 0.005 (in) -> 0.005
    assert abs(d[0] - 0.005) < 1e-12
    # point 3 (0.025): neighbours at 0.02, 0.024 -> none inside -> mean 0.022 clamped to 0.015
    assert abs(d[3] - 0.015) < 1e-12
    # point 5 (1.001): neighbours at 0.001 (out), 0.976 (out) -> mean 0.4885 clamped
    assert abs(d[5] - 0.015) < 1e-12


def _nonuniform_sphere(n, seed):
    """Unit sphere sampled with density proportional to 1 + 8 z^2 (rejection), exact normals."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < n:
        u = rng.standard_normal((4 * n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        keep = rng.uniform(0, 9, 4 * n) < 1 + 8 * u[:, 2] ** 2
        out.append(u[keep])
    u = np.concatenate(out)[:n]
    return np.ascontiguousarray(u.T)


def test_voronoi_weights_fix_nonuniform_sampling():
    """Why the weights matter (Sec. 5.1): on an unevenly sampled sphere with exact normals the
    GWN at interior points is 1 with Voronoi weights (to 3%: the tangent-plane cells
    overestimate the curved surface by ~2.4% at 6,000 points, 1.6% at 20,000), while uniform
    weights 4 pi / n miss by ~23% away from the centre."""
    P = _nonuniform_sphere(6000, 5)
    a = oracle.voronoi_area(P, 15)
    Q = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.5], [0.4, 0.0, 0.0]]).T
    w_vor, _, _ = oracle.gwn(P, P, a, None, Q, grad=False)
    w_uni, _, _ = oracle.gwn(P, P, np.full(P.shape[1], 4 * math.pi / P.shape[1]), None, Q, grad=False)
    assert np.abs(w_vor - 1).max() < 0.03
    assert np.abs(w_uni - 1).max() > 0.1
