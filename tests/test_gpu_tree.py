"""Octree mode (Sec. 5.2 "Octree Traversal") through the C ABI against the octree oracle:
the tree itself bit-exact (dwg_octree: Morton order and pre-order nodes), w and grad w to the
GWN tolerance at sizes that span many nodes and leaves, one full iteration, and sampled
queries at 1M points. Every input comes from the seeded generators or the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_13839_amd import synth
from tests.helpers import TOL_G, TOL_W, cuda, e_g, e_w, host, unit_rows

pytestmark = pytest.mark.gpu


def _dwg():
    from paper_2405_13839_amd import dwg
    return dwg


def _clusters(n, seed):
    rng = np.random.default_rng(seed)
    P = np.concatenate([rng.normal(0, 1e-4, (3, n // 2)), 1 + rng.normal(0, 1e-5, (3, n - n // 2))], axis=1)
    P[:, 5] = P[:, 6]
    P[:, 7] = P[:, 6]
    return P.astype(np.float32)


CLOUDS = {
    "single": lambda: np.array([[0.5], [0.25], [1.0]], np.float32),
    "uniform_17": lambda: np.random.default_rng(1).uniform(-1, 1, (3, 17)).astype(np.float32),
    "uniform_5000": lambda: np.random.default_rng(2).uniform(-1, 1, (3, 5000)).astype(np.float32),
    "clusters_dups_4000": lambda: _clusters(4000, 3),
    "all_equal_100": lambda: np.zeros((3, 100), np.float32),
    "torus_ellipsoids_100K": lambda: synth.torus_ellipsoids(100_000, seed=501).P,
}


@pytest.mark.parametrize("leaf", [1, 4, 16])
@pytest.mark.parametrize("cloud", list(CLOUDS))
def test_octree_matches_oracle(cloud, leaf):
    dwg = _dwg()
    P = CLOUDS[cloud]()
    perm, nodes = dwg.octree(cuda(P), leaf)
    operm, oinfo = oracle.octree(P, leaf)
    np.testing.assert_array_equal(host(perm).astype(np.int64), operm)
    np.testing.assert_array_equal(host(nodes).astype(np.int64), oinfo)


CASES = [
    # generator, lambda, use delta, compensated, beta, leaf, queries (None = the sources)
    ("sphere_3000", 0.0, False, True, 2.3, 16, None),
    ("sphere_3000", 10.0, True, False, 2.3, 4, None),
    ("torus_ellipsoids_20000", 10.0, True, True, 2.3, 16, None),
    ("torus_ellipsoids_20000", 0.0, True, True, 4.0, 16, None),
    ("torus_ellipsoids_20000", 10.0, True, True, 2.3, 1, 3001),
    ("superquadrics_plates_30000", 0.0, True, True, 2.3, 32, None),
]


def _gen(name):
    kind, n = name.rsplit("_", 1)
    n = int(n)
    if kind == "sphere":
        return synth.sphere(n, 0.005, 100)
    return getattr(synth, kind)(n, seed=777)


@pytest.mark.parametrize("gen,lam,use_delta,comp,beta,leaf,nq", CASES)
def test_tree_gwn_matches_oracle(gen, lam, use_delta, comp, beta, leaf, nq):
    dwg = _dwg()
    c = _gen(gen)
    rng = np.random.default_rng(11)
    N = unit_rows(rng, c.n)
    d = oracle.anchor_delta(c.P).astype(np.float32) if use_delta else None
    Q = c.P if nq is None else rng.uniform(c.P.min(axis=1, keepdims=True), c.P.max(axis=1, keepdims=True),
                                           (3, nq)).astype(np.float32)
    prm = dwg.Params(lam=lam, compensated=comp, beta=beta, leaf=leaf)
    Pc = cuda(c.P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), None if d is None else cuda(d), Pc if nq is None else cuda(Q), prm)
    w_ref, g_ref, flag = oracle.tree_gwn(c.P, N, c.area, d, Q, lam=lam, beta=beta, leaf=leaf)
    ok = flag == 0
    assert ok.mean() > 0.99
    ew, eg = e_w(host(w)[ok], w_ref[ok]), e_g(host(g)[:, ok], g_ref[:, ok])
    print(f"[tree] {gen} lam={lam} beta={beta} leaf={leaf}: e_w={ew:.2e} e_g={eg:.2e} flagged={int((~ok).sum())}")
    assert ew <= TOL_W and eg <= TOL_G


@pytest.mark.parametrize("m", [2, 5, 40])
def test_tree_sparse_wavefront_leaves_match_oracle(m):
    """A leaf opened by at most half of a wavefront's lanes is spread over the idle lanes:
    k groups of lanes (k a power of two, k x lanes <= 64) each take every k-th source for one
    query, and the partial sums return to the querying lanes through LDS. m queries at
    scattered points put a single lane on most leaves (the lanes past m repeat the last
    query), so the spread loop runs with up to 32 groups; w and grad w match the oracle, and
    with m = 2 the wavefront needs fewer leaf iterations than the live queries have pairs."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(20_000, seed=509)
    rng = np.random.default_rng(13)
    N = unit_rows(rng, c.n)
    d = oracle.anchor_delta(c.P).astype(np.float32)
    Q = np.ascontiguousarray(c.P[:, np.sort(rng.choice(c.n, m, replace=False))])
    prm = dwg.Params(lam=10.0, beta=2.3, leaf=32)
    w, g = dwg.gwn(cuda(c.P), cuda(N), cuda(c.area), cuda(d), cuda(Q), prm)
    w_ref, g_ref, flag = oracle.tree_gwn(c.P, N, c.area, d, Q, lam=10.0, beta=2.3, leaf=32)
    ok = flag == 0
    assert e_w(host(w)[ok], w_ref[ok]) <= TOL_W and e_g(host(g)[:, ok], g_ref[:, ok]) <= TOL_G
    if m == 2:
        wk = dwg.octree_work(cuda(c.P), cuda(c.area), cuda(d), cuda(Q), prm)
        assert wk.leaf_steps < wk.pairs


def test_tree_huge_beta_is_the_all_pairs_sum():
    """beta = 1e30 opens every node: the octree kernel then sums every source one by one."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(8000, seed=778)
    rng = np.random.default_rng(12)
    N = unit_rows(rng, c.n)
    d = oracle.anchor_delta(c.P).astype(np.float32)
    Pc = cuda(c.P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), cuda(d), Pc, dwg.Params(lam=10.0, beta=1e30))
    w_ref, g_ref, flag = oracle.gwn(c.P, N, c.area, d, c.P, lam=10.0)
    assert e_w(host(w), w_ref) <= TOL_W and e_g(host(g), g_ref, skip=flag) <= TOL_G


def test_tree_iteration_matches_oracle():
    """One dwg_iterate step in octree mode: n_new = -grad / |grad| of the oracle's octree
    gradient on the same inputs, and the same mean w."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(20_000, seed=779)
    N0 = oracle.random_normals(5, c.n).astype(np.float32)
    d = oracle.anchor_delta(c.P).astype(np.float32)
    Nt = cuda(N0)
    st, stats = dwg.iterate(cuda(c.P), cuda(c.area), cuda(d), Nt, dwg.Params(lam=10.0, beta=2.3), max_iters=1,
                            fixed_iters=True)
    w_ref, g_ref, flag = oracle.tree_gwn(c.P, N0, c.area, d, c.P, lam=10.0, beta=2.3)
    N1, _ = oracle.update(g_ref, N0)
    from tests.helpers import angle_deg
    ang = angle_deg(host(Nt), N1)
    ok = flag == 0
    assert np.percentile(ang[ok], 99.9) <= 1e-2 and np.mean(ang[ok] <= 1e-3) > 0.99
    assert abs(stats[0, 0] - w_ref.mean()) <= 1e-5 * max(1.0, abs(w_ref.mean()))


def test_tree_full_size_sampled_1M():
    """1M points (torus + 2 ellipsoids, screened): all queries on the GPU in octree mode,
    300 sampled queries recomputed by the octree oracle over all sources; the octree error
    against the exact sum is printed."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(1_000_000, seed=102)
    rng = np.random.default_rng(17)
    N = unit_rows(rng, c.n)
    from tests.test_gpu_configs import anchor_radius
    d = anchor_radius(c.P)
    Pc = cuda(c.P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), cuda(d), Pc, dwg.Params(lam=10.0, beta=2.3))
    sel = np.sort(rng.choice(c.n, 300, replace=False))
    Q = np.ascontiguousarray(c.P[:, sel])
    w_ref, g_ref, flag = oracle.tree_gwn(c.P, N, c.area, d, Q, lam=10.0, beta=2.3)
    ok = flag == 0
    wg, gg = host(w)[sel], host(g)[:, sel]
    ew, eg = e_w(wg[ok], w_ref[ok]), e_g(gg[:, ok], g_ref[:, ok])
    w_ex, g_ex, _ = oracle.gwn(c.P, N, c.area, d, Q[:, :50], lam=10.0)
    print(f"[tree] 1M: e_w={ew:.2e} e_g={eg:.2e} flagged={int((~ok).sum())}; octree vs exact on 50 queries: "
          f"e_w={e_w(wg[:50], w_ex):.2e} e_g={e_g(gg[:, :50], g_ex):.2e}")
    assert ew <= TOL_W and eg <= TOL_G


def test_tree_trajectory_matches_oracle():
    """Ten Jacobi iterations in octree mode from random normals on the C1 sphere (2,000
    points, plain kernel) against the oracle iterating its own octree evaluation: the
    normals stay together (a decision on a flagged query can move one normal slightly)."""
    from tests.helpers import angle_deg
    dwg = _dwg()
    s = synth.sphere(2000, 0.005, 100)
    N0 = oracle.random_normals(200, s.n)
    d = oracle.delta(s.P, 10) * 2.0
    Nt = cuda(N0.astype(np.float32))
    st, stats = dwg.iterate(cuda(s.P), cuda(s.area), cuda(d.astype(np.float32)), Nt, dwg.Params(beta=2.3, leaf=8),
                            max_iters=10, fixed_iters=True)
    N = N0.astype(np.float32).astype(np.float64)
    for t in range(10):
        w, g, _ = oracle.tree_gwn(s.P, N, s.area, d.astype(np.float32), s.P, beta=2.3, leaf=8)
        N, _ = oracle.update(g, N)
        N = N.astype(np.float32).astype(np.float64)  # the GPU keeps FP32 normals between iterations
        assert abs(stats[t, 0].item() - w.mean()) <= 1e-5
    ang = angle_deg(host(Nt), N)
    assert np.median(ang) <= 1e-3 and np.mean(ang <= 0.05) >= 0.995, np.percentile(ang, [50, 99, 100])


def test_tree_mode_is_deterministic():
    """Two octree-mode evaluations and two 3-iteration solves on the same inputs agree bit for
    bit (node radii come from order-free atomic maxima; every sum has a fixed order)."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(60_000, seed=780)
    rng = np.random.default_rng(13)
    N = cuda(unit_rows(rng, c.n))
    P, a = cuda(c.P), cuda(c.area)
    d = cuda(oracle.anchor_delta(c.P).astype(np.float32))
    prm = dwg.Params(lam=10.0, beta=2.3)
    w1, g1 = dwg.gwn(P, N, a, d, P, prm)
    w2, g2 = dwg.gwn(P, N, a, d, P, prm)
    assert torch.equal(w1, w2) and torch.equal(g1, g2)
    N1, N2 = N.clone(), N.clone()
    dwg.iterate(P, a, d, N1, prm, max_iters=3, fixed_iters=True)
    dwg.iterate(P, a, d, N2, prm, max_iters=3, fixed_iters=True)
    assert torch.equal(N1, N2)


@pytest.mark.parametrize("n,leaf,qkind", [(20_000, 32, "points"), (20_000, 8, "points"), (50_000, 32, "box")])
def test_traversal_work_matches_oracle(n, leaf, qkind):
    """dwg_octree_work: the far dipoles and leaf pairs the GPU traversal takes, totalled over
    the queries, equal the oracle's counts of the same decisions (the opening test is FP64 on
    both sides; queries the oracle flags as within 1e-7 of an opening radius may decide
    differently and are allowed one node's worth of difference each)."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(n, seed=507)
    d = oracle.anchor_delta(c.P).astype(np.float32)
    rng = np.random.default_rng(8)
    Q = c.P if qkind == "points" else rng.uniform(-1.6, 1.6, (3, 3000)).astype(np.float32)
    prm = dwg.Params(lam=10.0, beta=2.3, leaf=leaf)
    wk_gpu = dwg.octree_work(cuda(c.P), cuda(c.area), cuda(d), cuda(Q) if qkind != "points" else cuda(c.P), prm)
    far, pairs = wk_gpu.far, wk_gpu.pairs
    _, _, fl, wk = oracle.tree_gwn(c.P, c.N_true, c.area, d, Q, lam=10.0, beta=2.3, leaf=leaf, grad=False,
                                   work=True)
    print(f"[tree work] n={n} leaf={leaf} {qkind}: far {far} pairs {pairs} (oracle {wk[:, 1].sum()} "
          f"{wk[:, 2].sum()}), flagged {int(fl.sum())}")
    nfl = int(fl.sum())
    assert abs(far - int(wk[:, 1].sum())) <= 8 * nfl
    assert abs(pairs - int(wk[:, 2].sum())) <= 8 * leaf * nfl
    if nfl == 0:
        assert far == int(wk[:, 1].sum()) and pairs == int(wk[:, 2].sum())
    # a wavefront step serves at most 64 and at least one of its queries
    assert wk_gpu.far_steps <= far <= 64 * wk_gpu.far_steps
    assert wk_gpu.leaf_steps <= pairs <= 64 * wk_gpu.leaf_steps


@pytest.mark.parametrize("m", [1, 64, 200])
def test_traversal_wave_counts_of_one_repeated_query(m):
    """m copies of one query: every lane of a wavefront takes the same decisions, so each
    far step adds one dipole per query and each leaf iteration one pair per query; with m = 1
    (63 lanes past m) the wavefront counts equal the per-query counts."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(20_000, seed=508)
    d = oracle.anchor_delta(c.P).astype(np.float32)
    Q = np.repeat(np.array([[0.9], [0.05], [0.1]], np.float32), m, axis=1)
    prm = dwg.Params(lam=10.0, beta=2.3, leaf=32)
    wk = dwg.octree_work(cuda(c.P), cuda(c.area), cuda(d), cuda(Q), prm)
    _, _, fl, wo = oracle.tree_gwn(c.P, c.N_true, c.area, d, Q[:, :1], lam=10.0, beta=2.3, leaf=32, grad=False,
                                   work=True)
    waves = -(-m // 64)
    assert fl.sum() == 0
    assert wk.far == m * int(wo[0, 1]) and wk.pairs == m * int(wo[0, 2])
    assert wk.far_steps == waves * int(wo[0, 1]) and wk.leaf_steps == waves * int(wo[0, 2])
