"""CPU reference of the paper's own normal update (Sec. 4.3, Algorithm 1): the GWN at grid
nodes, the iso-value w_bar, the w_bar level set, a gradient per face from the cross product,
and every face's gradient added to its k nearest input points, then normalised.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy, float64, loops over
cells and tetrahedra; shares no code with the GPU library.

Definitions (the readings are listed with the design notes):
  * grid: the cube of the octree (lo = per-axis minimum of the points, side = the largest
    extent) cut into 2^depth cells per axis. A point's cell is its level-21 octree cell
    floor((x - lo) * 2^21 / side) shifted down to `depth`. The evaluated cells are the cells
    holding points, grown by `dilate` rings of neighbours (inside the cube), in Morton order.
  * nodes: the corners of those cells, at lo + c * side / 2^depth (FP64, then FP32); w at
    every corner with the current normals; w_bar = the mean of w over the input points
    (iso='points', the abstract's wording) or over the corners (iso='corners', Eq. 6 over
    the grid nodes).
  * level set: each cube is cut into 6 tetrahedra around its diagonal from corner (0,0,0)
    to (1,1,1), one per order (a, b, c) of the axes: corners 0, e_a, e_a + e_b, 7 (corner
    index = x + 2y + 4z; the orders are (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y),
    (z,y,x)). A corner is inside when w > w_bar. One inside (or one outside) vertex L gives
    the triangle of the crossings on the edges from L to the other three, in tetrahedron
    order; two inside vertices A < B with outside C < D give the quad e(A,C), e(A,D),
    e(B,D), e(B,C), split into (e(A,C), e(A,D), e(B,D)) and (e(A,C), e(B,D), e(B,C)).
    The crossing on edge (u, v) is p_u + (w_bar - w_u) / (w_v - w_u) (p_v - p_u).
  * face gradient: the cross product (q1 - q0) x (q2 - q0), turned to point away from the
    inside vertices of its tetrahedron (towards decreasing w, i.e. the outward normal; q1 and
    q2 are swapped when it is turned, so triangles are wound outwards); faces are assigned
    to the k nearest input points of their centroid.
  * update: n_j = normalize(sum of its faces' vectors); a point with no face, or a zero sum,
    keeps its normal.
"""
from __future__ import annotations

import numpy as np

import oracle

TREE_DEPTH = 21
ORDERS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
TETS = [(0, 1 << a, (1 << a) | (1 << b), 7) for a, b, _ in ORDERS]


def _spread(v):
    out = np.zeros_like(v, dtype=np.uint64)
    for b in range(TREE_DEPTH):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def morton(c):
    c = np.asarray(c, np.uint64)
    return (_spread(c[:, 0]) << np.uint64(2)) | (_spread(c[:, 1]) << np.uint64(1)) | _spread(c[:, 2])


def frame(P):
    P = np.asarray(P, np.float64)
    lo = P.min(axis=1)
    side = float((P.max(axis=1) - lo).max())
    return lo, side


def grid_cells(P, depth, dilate=1):
    """Evaluated cells [c, 3] (int64, Morton order), lo [3], side."""
    P = np.asarray(P, np.float64)
    lo, side = frame(P)
    G = 1 << depth
    if side > 0:
        scale = 2.0 ** TREE_DEPTH / side
        c21 = np.floor((P.T - lo) * scale)
        c21 = np.clip(c21, 0, 2.0 ** TREE_DEPTH - 1).astype(np.int64)
        c = c21 >> (TREE_DEPTH - depth)
    else:
        c = np.zeros((P.shape[1], 3), np.int64)
    cells = np.unique(c, axis=0)
    if dilate > 0:
        r = np.arange(-dilate, dilate + 1)
        off = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
        cells = (cells[:, None, :] + off[None, :, :]).reshape(-1, 3)
        cells = cells[np.all((cells >= 0) & (cells < G), axis=1)]
        cells = np.unique(cells, axis=0)
    order = np.argsort(morton(cells), kind="stable")
    return cells[order], lo, side


def corners(cells, lo, side, depth):
    """Unique corner lattice points [m, 3], their FP32 positions [3, m], and per cell the
    index of each of its 8 corners [c, 8] (corner k = x + 2y + 4z)."""
    offs = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)])
    allc = (cells[:, None, :] + offs[None]).reshape(-1, 3)
    uniq, inv = np.unique(allc, axis=0, return_inverse=True)
    h = side / float(1 << depth)
    pos = (lo[None, :] + uniq.astype(np.float64) * h).astype(np.float32).T
    return uniq, np.ascontiguousarray(pos), inv.reshape(-1, 8)


def marching_tets(cells, cidx, pos, w, iso):
    """Triangles [F, 3, 3] (float64) and oriented face vectors [F, 3]."""
    P = np.asarray(pos, np.float64).T
    tris, vecs = [], []
    for ci in range(len(cells)):
        cw = w[cidx[ci]]
        cp = P[cidx[ci]]
        for tv in TETS:
            wv = cw[list(tv)]
            pv = cp[list(tv)]
            ins = [bool(x > iso) for x in wv]
            k = sum(ins)
            if k == 0 or k == 4:
                continue

            def cross_pt(u, v):
                return pv[u] + (iso - wv[u]) / (wv[v] - wv[u]) * (pv[v] - pv[u])

            if k in (1, 3):
                lone = [t for t in range(4) if ins[t] == (k == 1)][0]
                others = [t for t in range(4) if t != lone]
                faces = [[cross_pt(lone, o) for o in others]]
            else:
                A, B = [t for t in range(4) if ins[t]]
                C, D = [t for t in range(4) if not ins[t]]
                eAC, eAD, eBD, eBC = cross_pt(A, C), cross_pt(A, D), cross_pt(B, D), cross_pt(B, C)
                faces = [[eAC, eAD, eBD], [eAC, eBD, eBC]]
            cin = pv[[t for t in range(4) if ins[t]]].mean(axis=0)
            for f in faces:
                q0, q1, q2 = f
                v = np.cross(q1 - q0, q2 - q0)
                cen = (q0 + q1 + q2) / 3.0
                if np.dot(v, cin - cen) > 0:
                    v = -v
                    q1, q2 = q2, q1  # wound the way the vector points
                tris.append(np.stack([q0, q1, q2]))
                vecs.append(v)
    if not tris:
        return np.zeros((0, 3, 3)), np.zeros((0, 3))
    return np.array(tris), np.array(vecs)


def _field(P, N, area, delta, Q, lam, eps, beta, leaf):
    if beta > 0:
        w, _, _ = oracle.tree_gwn(P, N, area, delta, Q, lam=lam, eps=eps, beta=beta, leaf=leaf, grad=False)
    else:
        w, _, _ = oracle.gwn(P, N, area, delta, Q, lam=lam, eps=eps, grad=False)
    return w


def level_set(P, N, area, delta, lam=0.0, eps=0.0, depth=8, dilate=1, beta=0.0, leaf=32, iso="points"):
    """(triangles [F,3,3], face vectors [F,3], w_bar, corner positions [3,m], corner w [m])."""
    cells, lo, side = grid_cells(P, depth, dilate)
    _, pos, cidx = corners(cells, lo, side, depth)
    w = _field(P, N, area, delta, pos, lam, eps, beta, leaf)
    if iso == "points":
        iso = float(np.mean(_field(P, N, area, delta, P, lam, eps, beta, leaf)))
    else:
        iso = float(np.mean(w))
    tris, vecs = marching_tets(cells, cidx, pos, w, iso)
    return tris, vecs, iso, pos, w


def update(P, N, area, delta, lam=0.0, eps=0.0, depth=8, dilate=1, k=10, beta=0.0, leaf=32, iso="points"):
    """One iteration of the paper's update: (N_new [3,n], iso, number of faces, faces per
    point [n])."""
    tris, vecs, iso, _, _ = level_set(P, N, area, delta, lam, eps, depth, dilate, beta, leaf, iso)
    N = np.asarray(N, np.float64)
    n = N.shape[1]
    acc = np.zeros((3, n))
    cnt = np.zeros(n, np.int64)
    if len(tris):
        cen = tris.mean(axis=1).T  # [3, F]
        idx, _ = oracle.knn(P, cen, k)
        for f in range(len(tris)):
            acc[:, idx[f]] += vecs[f][:, None]
            cnt[idx[f]] += 1
    norm = np.linalg.norm(acc, axis=0)
    out = N.copy()
    ok = norm > 0
    out[:, ok] = acc[:, ok] / norm[ok]
    return out, iso, len(tris), cnt
