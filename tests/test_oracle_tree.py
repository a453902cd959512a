"""Pins of the octree oracle (Sec. 5.2 "Octree Traversal") against facts that do not come
from its own code: the exact all-pairs sum (an opening radius that opens every node), an
octree built by explicit geometric subdivision, the far-field error falling with the
opening factor and staying within the first-order remainder bound of its far dipoles, and
the area-weighted dipole of a far cluster."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13839_amd import synth


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    P = (rng.uniform(-1, 1, (3, n)) * np.array([[1.0], [0.6], [0.3]])).astype(np.float32)
    N = rng.normal(size=(3, n))
    N = (N / np.linalg.norm(N, axis=0)).astype(np.float32)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32) * np.float32(4.0 / n)
    d = rng.uniform(0.0, 0.05, n).astype(np.float32)
    return P, N, a, d


@pytest.mark.parametrize("lam", [0.0, 10.0])
@pytest.mark.parametrize("leaf", [1, 16])
def test_tree_opening_everything_is_exact(lam, leaf):
    """beta -> infinity opens every node: the traversal then sums every point exactly once
    with the modified kernel, which is the all-pairs definition."""
    P, N, a, d = _cloud(3000, 1)
    Q = np.concatenate([P[:, :200], np.random.default_rng(2).uniform(-1.2, 1.2, (3, 50))], axis=1)
    w, g, _ = oracle.gwn(P, N, a, d, Q, lam=lam)
    wt, gt, _ = oracle.tree_gwn(P, N, a, d, Q, lam=lam, beta=1e30, leaf=leaf)
    assert np.abs(wt - w).max() <= 1e-12 * max(1.0, np.abs(w).max())
    assert np.abs(gt - g).max() <= 1e-12 * max(1.0, np.abs(g).max())


def _geometric_octree(P, leaf, depth=21):
    """Nodes as (level, sorted point indices) by explicit recursive subdivision of the cube
    (a cell with a single non-empty child is represented by that child)."""
    P = np.asarray(P, np.float64)
    lo = P.min(axis=1)
    ext = (P.max(axis=1) - lo).max()
    out = []

    def children(idx, level):
        h = ext / 2 ** (level + 1)
        kids = {}
        for i in idx:
            c = tuple(int(min(max(math.floor((P[d, i] - lo[d]) / h), 0), 2 ** (level + 1) - 1)) for d in range(3))
            kids.setdefault(c, []).append(i)
        return [kids[c] for c in sorted(kids, key=lambda c: [((c[0] >> b) & 1, (c[1] >> b) & 1, (c[2] >> b) & 1)
                                                              for b in range(level, -1, -1)])]

    def rec(idx, level):
        if len(idx) <= leaf or level == depth:
            out.append((level, tuple(sorted(idx))))
            return
        kids = children(idx, level)
        if len(kids) == 1:  # same point set as its only child: one node, at the deeper cell
            rec(kids[0], level + 1)
            return
        out.append((level, tuple(sorted(idx))))
        for k in kids:
            rec(k, level + 1)

    rec(list(range(P.shape[1])), 0)
    return out


@pytest.mark.parametrize("n,leaf", [(1, 1), (7, 1), (300, 4), (2000, 16), (-400, 4)])
def test_octree_matches_geometric_subdivision(n, leaf):
    if n > 0:
        P = _cloud(n, 3 + n)[0]
    else:  # two tight clusters far apart: long single-child chains, and duplicate points
        n = -n
        rng = np.random.default_rng(9)
        P = np.concatenate([rng.normal(0, 1e-4, (3, n // 2)), 1 + rng.normal(0, 1e-5, (3, n // 2))], axis=1)
        P[:, 5] = P[:, 6]
        P = P.astype(np.float32)
    perm, info = oracle.octree(P, leaf)
    ref = _geometric_octree(P, leaf)
    assert len(info) == len(ref)
    for (s, e, lev, skip), (rl, ri) in zip(info, ref):
        assert lev == rl and tuple(sorted(perm[s:e])) == ri
    # pre-order: skip is the index just past the subtree; children tile the parent's range
    assert sorted(perm.tolist()) == list(range(n))
    assert len(info) <= 2 * n
    for k, (s, e, lev, skip) in enumerate(info):
        assert skip > k and (skip == len(info) or info[skip][0] >= e)
        assert skip == k + 1 or info[k + 1][1] < e  # an internal node has >= 2 children
        c, pos = k + 1, s
        while c < skip:
            assert info[c][2] > lev and info[c][0] == pos
            pos = info[c][1]
            c = info[c][3]
        assert skip == k + 1 or pos == e


def test_tree_error_falls_with_beta():
    """Exact outward normals on a sphere: w = 1 inside, 0 outside. The node-dipole (order-0)
    far field has an error that shrinks as the opening factor grows."""
    s = synth.fibonacci_sphere(20000)
    Q = np.array([[0, 0, 0], [0.3, 0.2, -0.1], [1.5, 0, 0], [0, 2, 0]], dtype=np.float64).T
    truth = np.array([1.0, 1.0, 0.0, 0.0])
    err = []
    for beta in [2.3, 4.0, 8.0]:
        w, _, _ = oracle.tree_gwn(s.P, s.N_true, s.area, None, Q, beta=beta)
        err.append(np.abs(w - truth).max())
    assert err[0] <= 0.03 and err[1] < err[0] and err[2] < err[1], err


def test_far_cluster_is_area_weighted_dipole():
    """A far node stands for one dipole: moment sum a_j n_j at the area-weighted centre."""
    P = np.array([[0.0, 0.01, 0.0], [0.0, 0.0, 0.02], [0.0, 0.0, 0.0]])
    N = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    a = np.array([1.0, 2.0, 5.0])
    q = np.array([[0.3], [0.1], [2.0]])
    w, _, _ = oracle.tree_gwn(P, N, a, None, q, beta=2.3, leaf=1)
    cm = (P * a).sum(axis=1) / a.sum()
    d = cm - q[:, 0]
    ref = a.sum() * d[2] / (4 * math.pi * np.linalg.norm(d) ** 3)
    assert abs(w[0] - ref) <= 1e-14 * abs(ref)
    d0 = P.mean(axis=1) - q[:, 0]  # unweighted centre: visibly different
    assert abs(a.sum() * d0[2] / (4 * math.pi * np.linalg.norm(d0) ** 3) - ref) > 1e-6 * abs(ref)


def test_far_test_keeps_the_clamp():
    """Two points 10 apart with radius 1 and a query 0.5 from one of them: the near point
    is opened and clamped (its distance is inside its radius), the other counts as a far
    single-point node, which is exact -- so the octree value equals the all-pairs value."""
    P = np.array([[0.0, 10.0], [0.0, 0.0], [0.0, 0.0]])
    N = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    a = np.array([1.0, 1.0])
    d = np.array([1.0, 1.0])
    q = np.array([[0.3], [0.4], [0.0]])
    for lam in [0.0, 10.0]:
        w, g, _ = oracle.gwn(P, N, a, d, q, lam=lam)
        wt, gt, _ = oracle.tree_gwn(P, N, a, d, q, lam=lam, beta=2.3, leaf=1)
        np.testing.assert_allclose(wt, w, rtol=1e-14)
        np.testing.assert_allclose(gt, g, rtol=1e-14, atol=1e-300)


def test_traversal_work_partitions_the_sources():
    """Per query, the far nodes and the leaf pairs of the traversal cover every source exactly
    once (a far node stands for its sources), for any opening factor; a query far from the
    cloud takes the root as one dipole; with beta -> infinity only nodes of zero radius (one
    point, or coincident points) can still be far, so far nodes hold one point each here."""
    c = synth.torus_ellipsoids(6000, seed=9)
    d = oracle.anchor_delta(c.P)
    Q = np.concatenate([c.P[:, ::37], np.array([[50.0], [0.0], [0.0]], np.float32)], axis=1)
    _, _, _, wk = oracle.tree_gwn(c.P, c.N_true, c.area, d, Q, lam=10.0, beta=2.3, leaf=16, grad=False,
                                  work=True)
    np.testing.assert_array_equal(wk[:, 2] + wk[:, 3], c.n)
    assert wk[:-1, 1].min() > 0 and wk[:-1, 2].min() > 0
    assert tuple(wk[-1, 1:]) == (1, 0, c.n)
    _, _, _, wk = oracle.tree_gwn(c.P, c.N_true, c.area, d, Q[:, :20], beta=1e9, leaf=16, grad=False, work=True)
    np.testing.assert_array_equal(wk[:, 2] + wk[:, 3], c.n)
    np.testing.assert_array_equal(wk[:, 1], wk[:, 3])


def _far_remainder_bounds(P, N, a, Q, beta, leaf):
    """Per query, bounds on |w_tree - w| and |grad_tree - grad w| (plain kernel, no clamp
    radius) from the node list, and the size of the far terms themselves: a far node
    replaces its sources' dipoles m_j at p_j by their sum M at the area-weighted centre c.
    Along the segment from c to p_j the source stays in the node's ball (radius
    r = max |p_j - c|), at distance >= d - r from q (d = |c - q| > beta r). For
    K(x) = m.x / (4 pi |x|^3), |grad_x K| <= 4|m| / (4 pi |x|^3) and the Hessian's norm is
    <= 24|m| / (4 pi |x|^4), so the node's error in w is at most S / (pi (d - r)^3) and in
    grad w at most 6 S / (pi (d - r)^4), S = sum |m_j| |p_j - c|. The far terms' size is
    sum |M.(c - q)| / (4 pi d^3). The traversal (open a node unless |q - c| > crit =
    max(beta r, r)) is redone here from the oracle's node list."""
    P = np.asarray(P, np.float64)
    N = np.asarray(N, np.float64)
    a = np.asarray(a, np.float64)
    perm, info = oracle.octree(P, leaf)
    nn = len(info)
    C = np.zeros((nn, 3))
    M = np.zeros((nn, 3))
    R = np.zeros(nn)
    S = np.zeros(nn)
    for k, (s, e, _, _) in enumerate(info):
        idx = perm[s:e]
        ak = a[idx]
        c = (P[:, idx] * ak).sum(axis=1) / ak.sum()
        dist = np.linalg.norm(P[:, idx] - c[:, None], axis=0)
        m = N[:, idx] * ak
        C[k], M[k], R[k], S[k] = c, m.sum(axis=1), dist.max(), (np.linalg.norm(m, axis=0) * dist).sum()
    crit = np.maximum(beta * R, R)
    bw = np.zeros(Q.shape[1])
    bg = np.zeros(Q.shape[1])
    far = np.zeros(Q.shape[1])
    nfar = np.zeros(Q.shape[1], np.int64)
    for i in range(Q.shape[1]):
        q = np.asarray(Q[:, i], np.float64)
        stack = [0]
        while stack:
            k = stack.pop()
            x = C[k] - q
            d = np.linalg.norm(x)
            if d > crit[k]:
                nfar[i] += 1
                bw[i] += S[k] / (math.pi * (d - R[k]) ** 3)
                bg[i] += 6.0 * S[k] / (math.pi * (d - R[k]) ** 4)
                far[i] += abs(M[k] @ x) / (4 * math.pi * d ** 3)
            elif info[k][3] != k + 1:  # not a leaf: its children follow it in pre-order
                c = k + 1
                while c < info[k][3]:
                    stack.append(c)
                    c = info[c][3]
    return bw, bg, far, nfar


def _remainder_case(shape, beta):
    if shape == "sphere":
        c = synth.fibonacci_sphere(4000)
        P, N, a = c.P, c.N_true, c.area
    else:
        P, N, a, _ = _cloud(4000, 21)
    rng = np.random.default_rng(5)
    Q = np.concatenate([np.asarray(P[:, ::40], np.float64), rng.uniform(-1.5, 1.5, (3, 60))], axis=1)
    w, g, _ = oracle.gwn(P, N, a, None, Q)
    wt, gt, fl = oracle.tree_gwn(P, N, a, None, Q, beta=beta, leaf=8)
    bw, bg, far, nfar = _far_remainder_bounds(P, N, a, Q, beta, 8)
    ok = fl == 0
    return w, g, wt, gt, ok, bw, bg, far, nfar


@pytest.mark.parametrize("beta", [2.3, 16.0])
@pytest.mark.parametrize("shape", ["sphere", "random_normals"])
def test_tree_error_within_the_far_remainder_bound(shape, beta):
    """The octree value differs from the exact all-pairs sum by no more than the first-order
    remainder of its far dipoles (bound derived in _far_remainder_bounds), for w and grad w at
    every query the oracle does not flag (observed: within 1-5% of the bound)."""
    w, g, wt, gt, ok, bw, bg, far, nfar = _remainder_case(shape, beta)
    assert ok.mean() > 0.95 and (nfar[ok] > 0).all()
    ew = np.abs(wt - w)[ok]
    eg = np.linalg.norm(gt - g, axis=0)[ok]
    assert (ew <= bw[ok] * (1 + 1e-9) + 1e-13).all(), (ew / bw[ok]).max()
    assert (eg <= bg[ok] * (1 + 1e-9) + 1e-12).all(), (eg / bg[ok]).max()


def test_far_remainder_bound_is_below_the_far_field():
    """The bound above is a pin, not a formality: with exact outward normals and beta = 16
    it is several times smaller than the far terms themselves, so far dipoles with a wrong
    sign, a wrong scale or left out would exceed it."""
    w, g, wt, gt, ok, bw, bg, far, nfar = _remainder_case("sphere", 16.0)
    assert np.median(bw[ok]) < 0.25 * np.median(far[ok])
