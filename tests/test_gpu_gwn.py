"""GPU parity of the all-pairs GWN / gradient kernels against the FP64 oracle.

Inputs are seeded synthetic clouds (FP32); both sides get the same arrays. Bar: e_w and
e_g (see helpers) <= 1e-4, queries flagged by the oracle as branch-ambiguous at the clamp
radius excluded from e_g.
"""
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


def _cloud(n, seed):
    c = synth.torus_ellipsoids(max(n, 64), seed=seed) if n >= 64 else synth.sphere(n, 0.01, seed=seed)
    rng = np.random.default_rng(seed)
    P = c.P[:, :n].copy()
    N = unit_rows(rng, n)
    a = c.area[:n].copy()
    d = (rng.uniform(0.5, 1.5, n) * 0.04).astype(np.float32)
    return P, N, a, d


CASES = [
    # n, m (None = queries are the sources), lam, use_delta, compensated, split
    (1, 7, 0.0, False, True, 0),
    (2, None, 0.0, True, True, 0),
    (63, None, 10.0, True, True, 0),
    (255, 300, 0.0, True, False, 0),
    (256, None, 10.0, False, True, 0),
    (257, 1000, 100.0, True, True, 3),
    (1000, None, 0.0, True, True, 0),
    (1000, None, 10.0, True, True, 1),
    (4097, 1500, 0.0, False, True, 0),
    (4097, None, 10.0, True, False, 5),
    # one query: the block's query box is a point, so every far tile takes the separated loop
    (5000, 1, 10.0, True, True, 0),
    (5000, 1, 0.0, True, True, 0),
]


@pytest.mark.parametrize("n,m,lam,use_delta,comp,split", CASES)
def test_gwn_grad_matches_oracle(n, m, lam, use_delta, comp, split):
    dwg = _dwg()
    P, N, a, d = _cloud(n, 1000 + n)
    if m is None:
        Q = P
    else:
        rng = np.random.default_rng(n + 7)
        lo, hi = P.min(1, keepdims=True) - 0.2, P.max(1, keepdims=True) + 0.2
        Q = rng.uniform(lo, hi, (3, m)).astype(np.float32)
        Q[:, : min(m, n)] = P[:, : min(m, n)]  # some queries coincide with sources
    D = d if use_delta else None
    prm = dwg.Params(lam=lam, compensated=comp, split=split)
    w, g, wm = dwg.gwn(cuda(P), cuda(N), cuda(a), None if D is None else cuda(D), cuda(Q), prm, grad=True,
                       want_wmean=True)
    torch.cuda.synchronize()
    w_ref, g_ref, flag = oracle.gwn(P, N, a, D, Q, lam=lam)
    assert e_w(host(w), w_ref) <= TOL_W
    assert e_g(host(g), g_ref, skip=flag) <= TOL_G
    assert abs(host(wm)[0] - np.mean(host(w).astype(np.float64))) <= 1e-12 * max(1.0, abs(host(wm)[0]))
    # w-only entry point agrees with the gradient entry point's w
    w2 = dwg.gwn(cuda(P), cuda(N), cuda(a), None if D is None else cuda(D), cuda(Q), prm, grad=False)
    assert e_w(host(w2), w_ref) <= TOL_W


def test_eps_floor_and_zero_delta_are_the_same_kernel():
    dwg = _dwg()
    P, N, a, d = _cloud(700, 3)
    Pc, Nc, ac = cuda(P), cuda(N), cuda(a)
    w1, g1 = dwg.gwn(Pc, Nc, ac, cuda(np.full(700, 0.03, np.float32)), Pc)
    w2, g2 = dwg.gwn(Pc, Nc, ac, None, Pc, dwg.Params(eps=0.03))
    assert torch.equal(w1, w2) and torch.equal(g1, g2)
    w3, g3 = dwg.gwn(Pc, Nc, ac, cuda(np.zeros(700, np.float32)), Pc)
    w4, g4 = dwg.gwn(Pc, Nc, ac, None, Pc)
    assert torch.equal(w3, w4) and torch.equal(g3, g4)


@pytest.mark.parametrize("lam", [0.0, 10.0])
def test_duplicate_sources(lam):
    """Exact duplicates among the sources (a point repeated three times, with different normals
    and areas): every copy at distance 0 from a query contributes nothing, the others count in
    full; the queries are the sources themselves, so each duplicate group meets both cases."""
    dwg = _dwg()
    P, N, a, d = _cloud(1500, 21)
    rng = np.random.default_rng(22)
    dup = rng.choice(1500, 60, replace=False)
    P = np.concatenate([P, P[:, dup], P[:, dup]], axis=1)
    N = np.concatenate([N, unit_rows(rng, 120)], axis=1)
    a = np.concatenate([a, a[dup], 2 * a[dup]]).astype(np.float32)
    d = np.concatenate([d, d[dup], d[dup]]).astype(np.float32)
    w, g = dwg.gwn(cuda(P), cuda(N), cuda(a), cuda(d), cuda(P), dwg.Params(lam=lam))
    w_ref, g_ref, flag = oracle.gwn(P, N, a, d, P, lam=lam)
    assert e_w(host(w), w_ref) <= TOL_W
    assert e_g(host(g), g_ref, skip=flag) <= TOL_G


@pytest.mark.parametrize("lam,beta", [(10.0, 0.0), (0.0, 0.0), (10.0, 2.3)])
def test_offset_cloud_clamp_boundary(lam, beta):
    """A cloud far from the origin (unit cube at 4096) with delta = 0.1 for every source: ~80
    pairs lie within 1e-3 delta of their clamp radius. Scaling absolute positions by kappa in
    FP32 would move r by up to ~4e-4 here and flip the clamp branch of some of them (an FP32
    emulation counts 58 at lambda = 10); the kernels take kappa (p - q) from differences, so
    only pairs within the oracle's 1e-6 delta flag band may differ."""
    dwg = _dwg()
    n = 2000
    rng = np.random.default_rng(31)
    P = (rng.random((3, n)) + 4096.0).astype(np.float32)
    N = unit_rows(rng, n)
    a = np.full(n, 1.0 / n, np.float32)
    d = np.full(n, 0.1, np.float32)
    Pc = cuda(P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(a), cuda(d), Pc, dwg.Params(lam=lam, beta=beta))
    if beta > 0:
        w_ref, g_ref, flag = oracle.tree_gwn(P, N, a, d, P, lam=lam, beta=beta)
    else:
        w_ref, g_ref, flag = oracle.gwn(P, N, a, d, P, lam=lam)
    ok = flag == 0
    assert ok.mean() > 0.99
    ew, eg = e_w(host(w)[ok], w_ref[ok]), e_g(host(g)[:, ok], g_ref[:, ok])
    print(f"[offset] lam={lam} beta={beta}: e_w={ew:.2e} e_g={eg:.2e} flagged={int((~ok).sum())}")
    assert ew <= TOL_W and eg <= TOL_G


@pytest.mark.parametrize("lam,offset", [(10.0, 0.0), (0.0, 0.0), (10.0, 4096.0)])
def test_tile_classes_in_one_launch(lam, offset):
    """One block of 512 queries in a cube of half-width 0.05 and 512 sources in the cube,
    4,096 on a shell of radius 0.12 and 16,384 on a shell of radius 0.6 around it (radius
    0.005 each): the all-pairs kernel sorts the sources into tiles of 256 and takes, per
    tile, the general loop (tiles overlapping the query box), the far difference loop (box
    gap above the tile's radius but below the largest distance of a query from the block's
    middle query, 0.09-0.17 here) or the separated loop (|p|^2 and m . p staged per source).
    A host replay of the tiling in Morton order counts about 28, 15 and 39 tiles of the
    three kinds, so all of them meet in one launch; it is compared with the oracle. At
    offset 4096 the scene sits far from the origin, where the staged |p|^2 and m . p stay
    block-relative."""
    dwg = _dwg()
    rng = np.random.default_rng(71)
    m = 512

    def shell(k, rad):
        v = rng.standard_normal((3, k))
        return rad * v / np.linalg.norm(v, axis=0)

    Q = rng.uniform(-0.05, 0.05, (3, m))
    P = np.concatenate([Q[:, :256], rng.uniform(-0.05, 0.05, (3, 256)), shell(4096, 0.12), shell(16384, 0.6)], axis=1)
    Q = (Q + offset).astype(np.float32)
    P = (P + offset).astype(np.float32)
    n = P.shape[1]
    N = unit_rows(rng, n)
    a = np.full(n, 1.0 / n, np.float32)
    d = np.full(n, 0.005, np.float32)
    prm = dwg.Params(lam=lam)
    w, g = dwg.gwn(cuda(P), cuda(N), cuda(a), cuda(d), cuda(Q), prm)
    w_ref, g_ref, flag = oracle.gwn(P, N, a, d, Q, lam=lam)
    ew, eg = e_w(host(w), w_ref), e_g(host(g), g_ref, skip=flag)
    # the w-only kernels have their own separated loops
    w2 = dwg.gwn(cuda(P), cuda(N), cuda(a), cuda(d), cuda(Q), prm, grad=False)
    ew2 = e_w(host(w2), w_ref)
    print(f"[tile classes] lam={lam} offset={offset}: e_w={ew:.2e} e_g={eg:.2e} w-only e_w={ew2:.2e} "
          f"flagged={int(flag.sum())}")
    assert ew <= TOL_W and eg <= TOL_G and ew2 <= TOL_W


def test_sphere_closed_form_on_gpu():
    """Screened GWN of a sphere with exact normals (closed form) evaluated by the kernel."""
    dwg = _dwg()
    c = synth.fibonacci_sphere(20000)
    Q = np.array([[0.3, 0.2, -0.1], [0, 0, 0.6], [1.5, 0, 0], [1.2, 0.9, 0.3]], np.float32).T
    lam = 10.0
    s = np.sqrt(lam)
    rho = np.linalg.norm(Q.astype(np.float64), axis=0)
    C = (1 + s) * np.exp(-s)
    w_in = C * np.sinh(s * rho) / (s * rho)
    w_out = -np.exp(-s * rho) * (s * np.cosh(s) - np.sinh(s)) / (s * rho)
    w, g = dwg.gwn(cuda(c.P), cuda(c.N_true), cuda(c.area), None, cuda(Q), dwg.Params(lam=lam))
    np.testing.assert_allclose(host(w), np.where(rho < 1, w_in, w_out), rtol=1e-4, atol=1e-5)
    w0 = dwg.gwn(cuda(c.P), cuda(c.N_true), cuda(c.area), None, cuda(Q), dwg.Params(), grad=False)
    np.testing.assert_allclose(host(w0), np.where(rho < 1, 1.0, 0.0), atol=2e-5)


@pytest.mark.parametrize("n,lam", [(100_000, 10.0), (100_000, 0.0)])
def test_gwn_grad_large_sampled(n, lam):
    """Full-size launch (100K sources and queries, the split the library picks); the oracle
    recomputes 1000 sampled queries one by one."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(n, seed=101)
    rng = np.random.default_rng(5)
    N = unit_rows(rng, n)
    d = (rng.uniform(0.5, 1.5, n) * 0.01).astype(np.float32)
    Pc = cuda(c.P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), cuda(d), Pc, dwg.Params(lam=lam))
    sel = rng.choice(n, 1000, replace=False)
    w_ref, g_ref, flag = oracle.gwn(c.P, N, c.area, d, c.P[:, sel], lam=lam)
    assert e_w(host(w)[sel], w_ref) <= TOL_W
    assert e_g(host(g)[:, sel], g_ref, skip=flag) <= TOL_G


def test_deterministic_bitwise():
    dwg = _dwg()
    P, N, a, d = _cloud(3000, 9)
    args = (cuda(P), cuda(N), cuda(a), cuda(d), cuda(P), dwg.Params(lam=10.0))
    w1, g1 = dwg.gwn(*args)
    w2, g2 = dwg.gwn(*args)
    assert torch.equal(w1, w2) and torch.equal(g1, g2)


def test_nan_input_propagates():
    dwg = _dwg()
    P, N, a, d = _cloud(500, 4)
    a[17] = np.nan
    w, g = dwg.gwn(cuda(P), cuda(N), cuda(a), cuda(d), cuda(P))
    assert torch.isnan(w).all()


def test_gwn_grad_full_size_sampled():
    """The bench configuration: 1M points (torus + 2 ellipsoids), screened lambda = 10, the
    anchor radius (mean distance to 10 of 4096 anchors, computed by the oracle), the split and
    spatial order the library picks; 200 sampled queries are recomputed by the oracle one by
    one."""
    dwg = _dwg()
    c = synth.torus_ellipsoids(1_000_000, seed=102)
    rng = np.random.default_rng(11)
    N = unit_rows(rng, c.n)
    Pc = cuda(c.P)
    d = oracle.anchor_delta(c.P, 10, 4096, 1.0).astype(np.float32)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), cuda(d), Pc, dwg.Params(lam=10.0))
    sel = rng.choice(c.n, 200, replace=False)
    w_ref, g_ref, flag = oracle.gwn(c.P, N, c.area, d, c.P[:, sel], lam=10.0)
    assert e_w(host(w)[sel], w_ref) <= TOL_W
    assert e_g(host(g)[:, sel], g_ref, skip=flag) <= TOL_G
