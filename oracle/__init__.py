"""CPU FP64 oracle for the Diffusing Winding Gradients hot path (arXiv 2405.13839).

TEST INFRASTRUCTURE ONLY: the slow, plain definition that the GPU library is checked
against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it. It shares no code with ``paper_2405_13839_amd`` and never
calls it; the GPU library never imports this package.

The arithmetic lives in ``dwg_oracle.c`` (plain C, double precision, Neumaier sums,
OpenMP over independent queries), ``tree_oracle.c`` (the octree evaluation of Sec. 5.2)
and ``mlp.py`` (NumPy float64). This module is the
ctypes binding: it promotes the caller's FP32 arrays exactly to float64 and returns
float64 results.

Parity pins (closed forms, finite differences, invariants, published test vectors,
library special cases) are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwg_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "tree_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc (-O2 -fopenmp, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        lib.orc_gwn.argtypes = [dp, dp, dp, dp, i64, dp, i64, ctypes.c_double, ctypes.c_double, dp, dp, ip]
        lib.orc_update.argtypes = [dp, dp, i64, dp, dp]
        lib.orc_stats.argtypes = [dp, dp, i64, ctypes.c_double, dp]
        lib.orc_top_count.argtypes = [i64, ctypes.c_double]
        lib.orc_top_count.restype = i64
        lib.orc_dwg_run.argtypes = [dp, dp, dp, i64, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_knn_self.argtypes = [dp, i64, ctypes.c_int, ip, dp]
        lib.orc_knn.argtypes = [dp, i64, dp, i64, ip, ctypes.c_int, ip, dp]
        lib.orc_delta.argtypes = [dp, i64, ctypes.c_int, dp]
        lib.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_splitmix64.restype = ctypes.c_uint64
        lib.orc_random_normals.argtypes = [ctypes.c_uint64, i64, dp]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.orc_octree.argtypes = [dp, i64, ctypes.c_int, lp, lp, i64]
        lib.orc_octree.restype = i64
        lib.orc_tree_gwn.argtypes = [dp, dp, dp, dp, i64, dp, i64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, dp, dp, ip, lp]
        _lib = lib
    return _lib


def _d(a, shape=None):
    """Contiguous float64 copy (exact promotion of FP32 inputs)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a, ct=ctypes.c_double):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the oracle's later OpenMP loops (results do not depend on it)."""
    _load().orc_set_num_threads(int(t))


def gwn(P, N, area, delta, Q, lam=0.0, eps=0.0, grad=True):
    """w[m], grad w [3,m] (or None) and flags[m] of the (screened, clamped) GWN at Q.

    P, N: [3,n] sources and normals; area: [n]; delta: [n] or None; Q: [3,m].
    """
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    N = _d(N, (3, n))
    area = _d(area, (n,))
    delta = None if delta is None else _d(delta, (n,))
    Q = _d(Q)
    m = Q.shape[1]
    w = np.zeros(m)
    g = np.zeros((3, m)) if grad else None
    fl = np.zeros(m, dtype=np.int32)
    rc = lib.orc_gwn(_p(P), _p(N), _p(area), _p(delta), n, _p(Q), m, float(lam), float(eps), _p(w), _p(g),
                     _p(fl, ctypes.c_int32))
    if rc != 0:
        raise ValueError("orc_gwn rejected its arguments")
    return w, g, fl


def update(g, N_old):
    """Eq. 7 point-wise: (N_new [3,n], chord [n])."""
    lib = _load()
    g = _d(g)
    n = g.shape[1]
    N_old = _d(N_old, (3, n))
    N_new = np.zeros((3, n))
    ch = np.zeros(n)
    lib.orc_update(_p(g), _p(N_old), n, _p(N_new), _p(ch))
    return N_new, ch


def top_count(n: int, top_frac: float = 0.01) -> int:
    return int(_load().orc_top_count(n, top_frac))


def stats(w, chord, top_frac=0.01):
    """(wmean, top_mean_deg, mean_chord)."""
    lib = _load()
    w = _d(w)
    chord = _d(chord, w.shape)
    out = np.zeros(3)
    rc = lib.orc_stats(_p(w), _p(chord), w.shape[0], float(top_frac), _p(out))
    if rc != 0:
        raise ValueError("orc_stats rejected its arguments")
    return float(out[0]), float(out[1]), float(out[2])


def dwg_run(P, area, delta, N0, lam=0.0, eps=0.0, max_iters=30, fixed_iters=True, eps_deg=0.1,
            top_frac=0.01):
    """Algorithm 1 (point-wise, Jacobi). Returns (N_final [3,n], stats [T,3])."""
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    area = _d(area, (n,))
    delta = None if delta is None else _d(delta, (n,))
    N = _d(N0, (3, n)).copy()
    st = np.zeros((max_iters, 3))
    done = lib.orc_dwg_run(_p(P), _p(area), _p(delta), n, _p(N), float(lam), float(eps), int(max_iters),
                           int(bool(fixed_iters)), float(eps_deg), float(top_frac), _p(st))
    if done < 1:
        raise RuntimeError("orc_dwg_run failed (%d)" % done)
    return N, st[:done]


def knn_self(P, k):
    """k nearest other points of every point: (idx int32 [n,k], dist float64 [n,k])."""
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    idx = np.zeros((n, k), dtype=np.int32)
    dist = np.zeros((n, k))
    if lib.orc_knn_self(_p(P), n, int(k), _p(idx, ctypes.c_int32), _p(dist)) != 0:
        raise ValueError("orc_knn_self rejected its arguments")
    return idx, dist


def knn(R, Q, k, skip=None):
    """k nearest points of R for each query of Q, skipping R[skip[i]] for query i."""
    lib = _load()
    R = _d(R)
    Q = _d(Q)
    m = Q.shape[1]
    sk = None if skip is None else np.ascontiguousarray(np.asarray(skip, dtype=np.int32))
    idx = np.zeros((m, k), dtype=np.int32)
    dist = np.zeros((m, k))
    if lib.orc_knn(_p(R), R.shape[1], _p(Q), m, _p(sk, ctypes.c_int32), int(k), _p(idx, ctypes.c_int32),
                   _p(dist)) != 0:
        raise ValueError("orc_knn rejected its arguments")
    return idx, dist


def delta(P, k=10):
    """delta_i = mean distance to the k nearest other points [n]."""
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    out = np.zeros(n)
    if lib.orc_delta(_p(P), n, int(k), _p(out)) != 0:
        raise ValueError("orc_delta rejected its arguments")
    return out


def splitmix64(seed: int, t: int) -> int:
    return int(_load().orc_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(t)))


def random_normals(seed: int, n: int):
    lib = _load()
    out = np.zeros((3, n))
    lib.orc_random_normals(ctypes.c_uint64(seed), n, _p(out))
    return out


def anchor_delta(P, k=10, n_anchor=4096, scale=1.0):
    """scale x mean distance from every point to its k nearest anchors (every stride-th
    point, stride = max(1, n // n_anchor); an anchor skips itself)."""
    P = _d(P)
    n = P.shape[1]
    stride = max(1, n // n_anchor)
    A = np.ascontiguousarray(P[:, ::stride])
    skip = np.where(np.arange(n) % stride == 0, np.arange(n) // stride, -1).astype(np.int32)
    _, dist = knn(A, P, k, skip=skip)
    return scale * dist.mean(axis=1)


def pca_normals(P, k=16):
    """PCA initial normals (Sec. 5.1, "Normal Initialization"): the eigenvector (numpy eigh)
    of the smallest eigenvalue of the covariance of p_i and its k nearest other points about
    their mean. The paper leaves the sign open; this one points away from the origin
    (n . p_i > 0), and where n . p_i == 0 makes the largest-magnitude component positive."""
    P = _d(P)
    n = P.shape[1]
    idx, _ = knn_self(P, k)
    nb = np.concatenate([np.arange(n)[:, None], idx], axis=1)  # [n, k+1]
    X = P[:, nb].transpose(1, 2, 0)  # [n, k+1, 3]
    X = X - X.mean(axis=1, keepdims=True)
    C = np.einsum("nki,nkj->nij", X, X)
    w, V = np.linalg.eigh(C)
    v = V[:, :, 0]
    s = np.sum(v * P.T, axis=1)
    lead = v[np.arange(n), np.argmax(np.abs(v), axis=1)]
    s = np.where(s == 0.0, lead, s)
    return (v * np.where(s < 0, -1.0, 1.0)[:, None]).T


def gauss_normals(P):
    """Gauss-map initial normals (Sec. 5.1, "Normal Initialization"): p_i / |p_i|, the
    projection onto the unit sphere about the origin; (0, 0, 1) at the origin."""
    P = _d(P)
    r = np.linalg.norm(P, axis=0)
    out = np.where(r > 0, P / np.where(r > 0, r, 1.0), np.array([[0.0], [0.0], [1.0]]))
    return out


TREE_DEPTH = 21


def octree(P, leaf=32):
    """Octree of Sec. 5.2 as built by tree_oracle.c: (perm int64 [n], info int64 [nodes, 4] =
    (start, end, level, skip) in depth-first pre-order)."""
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    perm = np.zeros(n, dtype=np.int64)
    cap = max(64, 4 * n)
    while True:
        info = np.zeros((cap, 4), dtype=np.int64)
        cnt = lib.orc_octree(_p(P), n, int(leaf), _p(perm, ctypes.c_int64), _p(info, ctypes.c_int64), cap)
        if cnt < 0:
            raise ValueError("orc_octree rejected its arguments")
        if cnt <= cap:
            return perm, info[:cnt].copy()
        cap = int(cnt)


def tree_gwn(P, N, area, delta, Q, lam=0.0, eps=0.0, beta=2.3, leaf=32, grad=True, work=False):
    """Octree-approximated w [m], grad w [3,m] (or None), flags [m] (and, when work=True, per
    query [m, 4] = visited nodes, far nodes taken as one dipole, source pairs summed at
    leaves, sources inside the far nodes): Sec. 5.2 traversal with opening radius
    max(beta r, r + dmax)."""
    lib = _load()
    P = _d(P)
    n = P.shape[1]
    N = _d(N, (3, n))
    area = _d(area, (n,))
    delta = None if delta is None else _d(delta, (n,))
    Q = _d(Q)
    m = Q.shape[1]
    w = np.zeros(m)
    g = np.zeros((3, m)) if grad else None
    fl = np.zeros(m, dtype=np.int32)
    wk = np.zeros((m, 4), dtype=np.int64)
    rc = lib.orc_tree_gwn(_p(P), _p(N), _p(area), _p(delta), n, _p(Q), m, float(lam), float(eps), float(beta),
                          int(leaf), _p(w), _p(g), _p(fl, ctypes.c_int32), _p(wk, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_tree_gwn rejected its arguments")
    return (w, g, fl, wk) if work else (w, g, fl)


def voronoi_area(P, m=15):
    """Area weights of Sec. 5.1: per point, the m nearest other points, the tangent plane
    through p_i normal to the smallest-eigenvalue eigenvector (numpy eigh) of their
    covariance with p_i about the mean, and the area of p_i's cell in the 2D Voronoi diagram
    of the projections, bounded by the square [-R, R]^2 (R = largest projected distance) on
    the axes u = n x e_k / |n x e_k| (e_k the coordinate axis with the smallest |n_k|) and
    n x u, computed as a half-plane intersection by qhull
    (scipy.spatial.HalfspaceIntersection)."""
    from scipy.spatial import ConvexHull, HalfspaceIntersection
    P = _d(P)
    n = P.shape[1]
    idx, _ = knn_self(P, m)
    out = np.zeros(n)
    for i in range(n):
        nb = P[:, idx[i]]
        X = np.concatenate([P[:, i:i + 1], nb], axis=1)
        C = np.cov(X, bias=True) * X.shape[1]
        _, V = np.linalg.eigh(C)
        nv = V[:, 0]
        k = int(np.argmin(np.abs(nv)))  # the axis least aligned with the normal (first on ties)
        u = np.cross(nv, np.eye(3)[k])
        u /= np.linalg.norm(u)
        B = np.stack([u, np.cross(nv, u)], axis=1)  # the square's axes; a flipped nv flips only u
        q = B.T @ (nb - P[:, i:i + 1])  # [2, m]
        R = np.linalg.norm(q, axis=0).max()
        if not R > 0:
            continue
        c = 0.5 * np.sum(q * q, axis=0)
        keep = c > 0
        hs = [[q[0, j], q[1, j], -c[j]] for j in np.nonzero(keep)[0]]
        hs += [[1.0, 0.0, -R], [-1.0, 0.0, -R], [0.0, 1.0, -R], [0.0, -1.0, -R]]
        h = HalfspaceIntersection(np.array(hs), np.zeros(2))
        out[i] = ConvexHull(h.intersections).volume
    return out


def delta_knn_window(P, k=10, vmin=0.0015, vmax=0.015):
    """Kernel radius of Sec. 5.2: mean of the k-NN distances inside [vmin, vmax]; when none
    is inside, the mean of all k clamped to the window."""
    _, dist = knn_self(P, k)
    inside = (dist >= vmin) & (dist <= vmax)
    cnt = inside.sum(axis=1)
    win = np.where(cnt > 0, (dist * inside).sum(axis=1) / np.maximum(cnt, 1), 0.0)
    allm = np.clip(dist.mean(axis=1), vmin, vmax)
    return np.where(cnt > 0, win, allm)
