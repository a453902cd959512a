"""CPU reference of the paper's own normal update (Sec. 4.3, Algorithm 1): the GWN at grid
nodes, the iso-value w_bar, the w_bar level set, a gradient per face from the cross product,
and every face's gradient added to its k nearest input points, then normalised.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain NumPy, float64, loops over
cells; shares no code with the GPU library.

Definitions (the readings are listed with the design notes):
  * grid: the cube of the octree (lo = per-axis minimum of the points, side = the largest
    extent) cut into 2^depth cells per axis. A point's cell is its level-21 octree cell
    floor((x - lo) * 2^21 / side) shifted down to `depth`. The evaluated cells are the cells
    holding points, grown by `dilate` rings of neighbours (inside the cube), in Morton order.
  * nodes: the corners of those cells, at lo + c * side / 2^depth (FP64, then FP32); w at
    every corner with the current normals; w_bar = the mean of w over the input points
    (iso='points', the abstract's wording) or over the corners (iso='corners', Eq. 6 over
    the grid nodes).
  * level set, Marching Cubes (the paper's method; Lorensen & Cline 1987), cube by cube.
    Corner index k = x + 2y + 4z; a corner is above when w > w_bar; an edge (u, v), u < v,
    is cut when exactly one end is above, at p_u + (w_bar - w_u) / (w_v - w_u) (p_v - p_u).
    Edges are numbered 0..11 in the lexicographic order of (u, v). On every face of the
    cube, walked counter-clockwise as seen from outside, each maximal run of above corners
    gives one segment, from the cut edge where the walk enters the run to the cut edge
    where it leaves it. A face whose two above corners are diagonal therefore gets two
    segments, one cutting off each above corner (the ambiguous face is resolved by
    separating the above corners; the rule depends on the face's four signs only, so the
    two cubes sharing a face draw the same segments and the surface is closed). The
    segments chain into closed loops on the cube's surface; a loop is written from its
    smallest edge index on, loops in the order of that index, and each loop of L vertices
    is cut into the fan of triangles (v_0, v_i, v_{i+1}), i = 1 .. L-2. The walking
    direction winds every loop so that (q1 - q0) x (q2 - q0) points away from the above
    corners (towards decreasing w: outwards for outward normals).
    With at most four corners above, the loops are the polygons of Lorensen & Cline's
    cases (each of their triangulations is one fan per loop); with more, the complement of
    a case is not reused (that is what opens holes next to an ambiguous face), the same
    face rule is applied instead.
  * level set, marching tetrahedra (a named option, not the paper's): each cube is cut into
    6 tetrahedra around its diagonal from corner 0 to corner 7, one per order (a, b, c) of
    the axes: corners 0, e_a, e_a + e_b, 7 (orders (x,y,z), (x,z,y), (y,x,z), (y,z,x),
    (z,x,y), (z,y,x)). One inside (or one outside) vertex L gives the triangle of the
    crossings on the edges from L to the other three, in tetrahedron order; two inside
    vertices A < B with outside C < D give the quad e(A,C), e(A,D), e(B,D), e(B,C), split
    into (e(A,C), e(A,D), e(B,D)) and (e(A,C), e(B,D), e(B,C)), each turned to point away
    from the inside vertices.
  * face gradient: the cross product (q1 - q0) x (q2 - q0) of the triangle as wound above;
    faces are assigned to the k nearest input points of their centroid.
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


# Corner k of a cube sits at offset (k & 1, (k >> 1) & 1, (k >> 2) & 1) cells.
CORNER_OFFSET = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], np.float64)
# The 12 cube edges (u, v), u < v, v = u plus one axis step, in lexicographic order.
CUBE_EDGES = sorted((u, u | (1 << a)) for u in range(8) for a in range(3) if not (u >> a) & 1)
EDGE_INDEX = {e: i for i, e in enumerate(CUBE_EDGES)}


def _face_walks():
    """The 6 faces' corners in counter-clockwise order about the outward face normal (found
    geometrically: sorted by the angle around the face centre in a right-handed (u, v) frame
    of the face plane, u x v = the outward normal)."""
    walks = []
    for axis in range(3):
        for side in (0, 1):
            f = np.zeros(3)
            f[axis] = 2.0 * side - 1.0
            cs = [k for k in range(8) if ((k >> axis) & 1) == side]
            u = np.zeros(3)
            u[(axis + 1) % 3] = 1.0
            v = np.cross(f, u)
            c = CORNER_OFFSET[cs].mean(axis=0)
            ang = [np.arctan2((CORNER_OFFSET[k] - c) @ v, (CORNER_OFFSET[k] - c) @ u) for k in cs]
            walks.append([cs[i] for i in np.argsort(ang)])
    return walks


FACE_WALKS = _face_walks()


def _edge(a, b):
    return EDGE_INDEX[(min(a, b), max(a, b))]


def cube_loops(above):
    """Loops of cut-edge indices for one cube with the corners above w_bar flagged in
    `above` (8 bools): face segments, chained, each loop from its smallest edge on."""
    nxt = {}
    for walk in FACE_WALKS:
        for i in range(4):
            a, b = walk[i], walk[(i + 1) % 4]
            if above[a] or not above[b]:
                continue  # not where the walk enters a run of above corners
            j = (i + 1) % 4
            while above[walk[(j + 1) % 4]]:
                j = (j + 1) % 4
            nxt[_edge(a, b)] = _edge(walk[j], walk[(j + 1) % 4])
    loops, seen = [], set()
    for e in sorted(nxt):
        if e in seen:
            continue
        loop, x = [e], nxt[e]
        seen.add(e)
        while x != e:
            seen.add(x)
            loop.append(x)
            x = nxt[x]
        loops.append(loop)
    return loops


def marching_cubes(cells, cidx, pos, w, iso):
    """Triangles [F, 3, 3] (float64, wound away from w > iso) and face vectors [F, 3]."""
    P = np.asarray(pos, np.float64).T
    tris, vecs = [], []
    for ci in range(len(cells)):
        cw = np.asarray(w, np.float64)[cidx[ci]]
        cp = P[cidx[ci]]
        above = [bool(x > iso) for x in cw]
        if all(above) or not any(above):
            continue
        for loop in cube_loops(above):
            q = []
            for e in loop:
                u, v = CUBE_EDGES[e]
                t = (iso - cw[u]) / (cw[v] - cw[u])
                q.append(cp[u] + t * (cp[v] - cp[u]))
            for i in range(1, len(q) - 1):
                tris.append(np.stack([q[0], q[i], q[i + 1]]))
                vecs.append(np.cross(q[i] - q[0], q[i + 1] - q[0]))
    if not tris:
        return np.zeros((0, 3, 3)), np.zeros((0, 3))
    return np.array(tris), np.array(vecs)


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


def extract(cells, cidx, pos, w, iso, surface="cubes"):
    """The w_bar level set by Marching Cubes (surface='cubes', the paper's) or by marching
    tetrahedra (surface='tets')."""
    if surface == "cubes":
        return marching_cubes(cells, cidx, pos, w, iso)
    if surface == "tets":
        return marching_tets(cells, cidx, pos, w, iso)
    raise ValueError(f"unknown surface {surface!r}")


def level_set(P, N, area, delta, lam=0.0, eps=0.0, depth=8, dilate=1, beta=0.0, leaf=32, iso="points",
              surface="cubes"):
    """(triangles [F,3,3], face vectors [F,3], w_bar, corner positions [3,m], corner w [m])."""
    cells, lo, side = grid_cells(P, depth, dilate)
    _, pos, cidx = corners(cells, lo, side, depth)
    w = _field(P, N, area, delta, pos, lam, eps, beta, leaf)
    if iso == "points":
        iso = float(np.mean(_field(P, N, area, delta, P, lam, eps, beta, leaf)))
    else:
        iso = float(np.mean(w))
    tris, vecs = extract(cells, cidx, pos, w, iso, surface)
    return tris, vecs, iso, pos, w


def update(P, N, area, delta, lam=0.0, eps=0.0, depth=8, dilate=1, k=10, beta=0.0, leaf=32, iso="points",
           surface="cubes"):
    """One iteration of the paper's update: (N_new [3,n], iso, number of faces, faces per
    point [n])."""
    tris, vecs, iso, _, _ = level_set(P, N, area, delta, lam, eps, depth, dilate, beta, leaf, iso, surface)
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
