"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-type the oracle's kernel: they check it against closed-form integrals
(Gauss / solid-angle result and the Yukawa double layer on a sphere), central finite
differences, symmetries, a published RNG test vector and library routines.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13839_amd import synth


def _sphere_q():
    # interior and exterior query points at least 0.3 from the unit sphere
    return np.array([[0, 0, 0], [0.3, 0.2, -0.1], [0, 0, 0.6], [-0.4, 0.3, 0.2],
                     [1.5, 0, 0], [0, 2, 0], [1.2, 0.9, 0.3], [-1.0, -1.0, 1.0]], dtype=np.float64).T


@pytest.fixture(scope="module")
def fib():
    return synth.fibonacci_sphere(20000)


def test_plain_sphere_is_indicator(fib):
    """Eq. 1-2: with exact outward normals w = 1 inside, 0 outside, grad w = 0 off the surface."""
    Q = _sphere_q()
    w, g, fl = oracle.gwn(fib.P, fib.N_true, fib.area, None, Q)
    rho = np.linalg.norm(Q, axis=0)
    np.testing.assert_allclose(w, np.where(rho < 1, 1.0, 0.0), atol=1e-5)
    assert np.max(np.linalg.norm(g, axis=0)) < 1e-3
    assert not fl.any()


def test_plain_sphere_surface_half(fib):
    """At a sample point (self pair excluded) the double-layer integrand on a sphere is
    1 / (8 pi R r); the discrete sum is 1/2 minus the missing self-cell, which for a disc of
    area a is sqrt(a / pi) / (4 R)."""
    w, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, None, fib.P[:, :64])
    pred = 0.5 - math.sqrt(fib.area[0] / math.pi) / 4.0
    assert np.all(w < 0.5)
    np.testing.assert_allclose(w, pred, atol=1e-3)


@pytest.mark.parametrize("dl", [0.05, 0.1, 0.2])
def test_plain_sphere_surface_with_clamp(fib, dl):
    """The clamped branch (Sec. 5.2, rho = max(r, delta_j)) on a sphere of radius R = 1 with
    exact normals and a uniform radius delta: on the sphere the area inside chord r is
    exactly pi r^2, so the clamp changes the surface value by
    (1 / 4R) int_0^delta (r^3 / delta^3 - 1) dr = -3 delta / (16 R), and the self pair no
    longer matters (the clamped integrand vanishes at r = 0): w = 1/2 - 3 delta / 16. A
    dropped clamp misses by >= 0.009 here."""
    D = np.full(fib.n, dl, np.float32)
    Q = fib.P[:, :: fib.n // 64]
    w, _, fl = oracle.gwn(fib.P, fib.N_true, fib.area, D, Q)
    pred = 0.5 - 3.0 * float(np.float32(dl)) / 16.0
    np.testing.assert_allclose(w, pred, atol=3e-4)
    assert not fl.any()


def test_clamp_uses_the_source_radius(fib):
    """Two interleaved populations with radii d1 (even indices) and d2 (odd), each carrying
    half of the sphere's area: every sample point sees both, so w = 1/2 - 3 (d1 + d2) / 32.
    Taking the query's own radius instead would give 1/2 - 3 d_i / 16 (0.4906 or 0.4625
    against 0.4766)."""
    d1, d2 = 0.05, 0.2
    D = np.where(np.arange(fib.n) % 2 == 0, d1, d2).astype(np.float32)
    Q = fib.P[:, :: fib.n // 64]
    w, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, D, Q)
    np.testing.assert_allclose(w, 0.5 - 3.0 * (d1 + d2) / 32.0, atol=1e-3)


@pytest.mark.parametrize("lam,dl", [(1.0, 0.1), (10.0, 0.05), (10.0, 0.2), (100.0, 0.2)])
def test_screened_sphere_surface_with_clamp(fib, lam, dl):
    """Screened kernel and clamp together (Eq. 5 with rho = max(r, delta)): phi uses the true
    r and only r^3 is clamped, so on the sphere the surface value is the Yukawa double layer's
    e^-x [(2 + x) sinh x - x cosh x] / (2x) (x = s R) plus
    (1 / 4R) int_0^delta e^-sr (1 + sr) (r^3 / delta^3 - 1) dr (quadrature). Reading
    phi(rho) instead moves it by 1.6e-3 at lambda = 100, delta = 0.2."""
    from scipy.integrate import quad
    s = math.sqrt(lam)
    x = s
    dd = float(np.float32(dl))
    ws = math.exp(-x) * ((2 + x) * math.sinh(x) - x * math.cosh(x)) / (2 * x)
    corr = quad(lambda r: math.exp(-s * r) * (1 + s * r) * (r ** 3 / dd ** 3 - 1), 0, dd, epsabs=1e-14)[0] / 4
    D = np.full(fib.n, dl, np.float32)
    Q = fib.P[:, :: fib.n // 64]
    w, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, D, Q, lam=lam)
    np.testing.assert_allclose(w, ws + corr, atol=3e-4 if dl < 0.1 else 1.5e-4)


@pytest.mark.parametrize("lam", [0.0, 10.0])
def test_radius_below_every_pair_distance_changes_nothing(lam):
    """rho = max(r, delta_j): a radius below every pair's distance leaves every term, and so
    w and grad w, bit for bit as without a radius."""
    rng = np.random.default_rng(12)
    P, N, a, _ = _rand_cloud(rng, 60)
    Q = np.concatenate([P[:, :20], rng.uniform(-1, 1, (3, 20))], axis=1)
    r = np.linalg.norm(P[:, None, :] - Q[:, :, None], axis=0)
    dmin = r[r > 0].min()
    D = np.full(P.shape[1], 0.5 * dmin)
    w0, g0, _ = oracle.gwn(P, N, a, None, Q, lam=lam)
    w1, g1, _ = oracle.gwn(P, N, a, D, Q, lam=lam)
    np.testing.assert_array_equal(w0, w1)
    np.testing.assert_array_equal(g0, g1)


@pytest.mark.parametrize("lam", [1.0, 10.0, 100.0])
def test_screened_sphere_closed_form(fib, lam):
    """Eq. 5 on a sphere of radius R = 1 (Yukawa double layer, x = s R, s = sqrt(lambda)):
    inside w = (1+x) e^-x sinh(s rho)/(s rho), outside w = -e^(-s rho)(x cosh x - sinh x)/(s rho);
    radial gradients C (s rho cosh(s rho) - sinh(s rho))/(s rho^2) with C = (1+x) e^-x and
    (x cosh x - sinh x) e^(-s rho)(1 + s rho)/(s rho^2). The jump across the sphere is 1."""
    Q = _sphere_q()[:, 1:]  # skip the centre (radial direction undefined)
    w, g, _ = oracle.gwn(fib.P, fib.N_true, fib.area, None, Q, lam=lam)
    s = math.sqrt(lam)
    x = s
    rho = np.linalg.norm(Q, axis=0)
    C = (1 + x) * math.exp(-x)
    w_in = C * np.sinh(s * rho) / (s * rho)
    w_out = -np.exp(-s * rho) * (x * math.cosh(x) - math.sinh(x)) / (s * rho)
    np.testing.assert_allclose(w, np.where(rho < 1, w_in, w_out), rtol=1e-5, atol=1e-6)
    g_in = C * (s * rho * np.cosh(s * rho) - np.sinh(s * rho)) / (s * rho**2)
    g_out = (x * math.cosh(x) - math.sinh(x)) * np.exp(-s * rho) * (1 + s * rho) / (s * rho**2)
    radial = np.sum(g * Q, axis=0) / rho
    np.testing.assert_allclose(radial, np.where(rho < 1, g_in, g_out), rtol=1e-4, atol=1e-6)
    tang = np.linalg.norm(g - radial * Q / rho, axis=0)
    assert tang.max() < 1e-4
    # centre value
    w0, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, None, np.zeros((3, 1)), lam=lam)
    assert abs(w0[0] - C) < 1e-5 * max(1.0, C)


def test_screened_jump_is_one(fib):
    """The jump condition k = 1 (Sec. 4.2): w(R - t) - w(R + t) -> 1 as t -> 0."""
    lam = 10.0
    dirs = np.array([[0.3, -0.5, 0.81], [-0.7, 0.1, 0.2]]).T
    dirs = dirs / np.linalg.norm(dirs, axis=0)
    t = 0.25
    w_i, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, None, dirs * (1 - t), lam=lam)
    w_o, _, _ = oracle.gwn(fib.P, fib.N_true, fib.area, None, dirs * (1 + t), lam=lam)
    s = math.sqrt(lam)
    # closed-form jump of the two one-sided values at distance t, which tends to 1
    C = (1 + s) * math.exp(-s)
    pred = C * math.sinh(s * (1 - t)) / (s * (1 - t)) + math.exp(-s * (1 + t)) * (s * math.cosh(s) - math.sinh(s)) / (s * (1 + t))
    np.testing.assert_allclose(w_i - w_o, pred, rtol=1e-5)
    assert abs(C * math.sinh(s) / s + math.exp(-s) * (s * math.cosh(s) - math.sinh(s)) / s - 1.0) < 1e-12


def _rand_cloud(rng, n=40):
    P = rng.uniform(-1, 1, (3, n))
    N = rng.standard_normal((3, n))
    N /= np.linalg.norm(N, axis=0)
    a = rng.uniform(0.01, 0.1, n)
    d = rng.uniform(0.05, 0.4, n)
    return P, N, a, d


@pytest.mark.parametrize("lam", [0.0, 10.0])
@pytest.mark.parametrize("use_delta", [False, True])
def test_gradient_matches_finite_differences(lam, use_delta):
    """grad w is the derivative of w with respect to the query (normals fixed, Sec. 4.1),
    including the clamped branch and the s^2 term of the screened kernel."""
    rng = np.random.default_rng(7)
    P, N, a, d = _rand_cloud(rng)
    D = d if use_delta else None
    Q = rng.uniform(-1, 1, (3, 60))
    h = 1e-5
    w, g, fl = oracle.gwn(P, N, a, D, Q, lam=lam)
    # keep queries away from the clamp boundary |r - delta_j| (finite differences straddle it)
    r = np.linalg.norm(P[:, None, :] - Q[:, :, None], axis=0)  # [m, n]
    ok = np.ones(Q.shape[1], bool)
    if use_delta:
        ok = np.min(np.abs(r - d[None, :]), axis=1) > 1e-3
        assert np.any(np.min(r - d[None, :], axis=1) < 0), "no query exercises the clamped branch"
    fd = np.zeros_like(g)
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = h
        wp, _, _ = oracle.gwn(P, N, a, D, Q + e, lam=lam, grad=False)
        wm, _, _ = oracle.gwn(P, N, a, D, Q - e, lam=lam, grad=False)
        fd[k] = (wp - wm) / (2 * h)
    err = np.linalg.norm(g - fd, axis=0)[ok] / np.maximum(np.linalg.norm(g, axis=0)[ok], 1.0)
    assert err.max() < 1e-5, err.max()


def test_invariants():
    """Linearity in a, odd in n, translation invariance, rotation equivariance and the
    scaling law p -> alpha p, a -> alpha^2 a, delta -> alpha delta, lambda -> lambda/alpha^2:
    w unchanged, grad w -> grad w / alpha."""
    rng = np.random.default_rng(3)
    P, N, a, d = _rand_cloud(rng, 50)
    Q = rng.uniform(-1.2, 1.2, (3, 30))
    lam = 7.0
    w, g, _ = oracle.gwn(P, N, a, d, Q, lam=lam)
    w2, g2, _ = oracle.gwn(P, N, 2.5 * a, d, Q, lam=lam)
    np.testing.assert_allclose(w2, 2.5 * w, rtol=1e-12, atol=1e-14)
    w3, g3, _ = oracle.gwn(P, -N, a, d, Q, lam=lam)
    np.testing.assert_allclose(w3, -w, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g3, -g, rtol=1e-12, atol=1e-12)
    t = np.array([[0.3], [-1.1], [0.7]])
    w4, g4, _ = oracle.gwn(P + t, N, a, d, Q + t, lam=lam)
    np.testing.assert_allclose(w4, w, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(g4, g, rtol=1e-8, atol=1e-9)
    Rm = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    w5, g5, _ = oracle.gwn(Rm @ P, Rm @ N, a, d, Rm @ Q, lam=lam)
    np.testing.assert_allclose(w5, w, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(g5, Rm @ g, rtol=1e-8, atol=1e-9)
    al = 1.7
    w6, g6, _ = oracle.gwn(al * P, N, al * al * a, al * d, al * Q, lam=lam / al**2)
    np.testing.assert_allclose(w6, w, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(g6, g / al, rtol=1e-8, atol=1e-9)


def test_coincident_source_contributes_nothing():
    """A query sitting exactly on a source gets nothing from it (self pair at an input point)."""
    rng = np.random.default_rng(5)
    P, N, a, d = _rand_cloud(rng, 30)
    for lam, D in [(0.0, None), (10.0, d)]:
        w, g, _ = oracle.gwn(P, N, a, D, P[:, :5], lam=lam)
        for i in range(5):
            keep = np.arange(30) != i
            wi, gi, _ = oracle.gwn(P[:, keep], N[:, keep], a[keep], None if D is None else D[keep],
                                   P[:, i:i + 1], lam=lam)
            assert abs(wi[0] - w[i]) <= 1e-12 * max(1, abs(w[i]))
            np.testing.assert_allclose(gi[:, 0], g[:, i], rtol=1e-12, atol=1e-12)


def test_delta_zero_and_eps_floor():
    """delta = 0 is the unmodified kernel; eps acts as a global floor on the radius."""
    rng = np.random.default_rng(11)
    P, N, a, d = _rand_cloud(rng, 30)
    Q = rng.uniform(-1, 1, (3, 20))
    w0, g0, _ = oracle.gwn(P, N, a, None, Q)
    w1, g1, _ = oracle.gwn(P, N, a, np.zeros(30), Q)
    np.testing.assert_array_equal(w0, w1)
    np.testing.assert_array_equal(g0, g1)
    w2, g2, _ = oracle.gwn(P, N, a, np.full(30, 0.2), Q)
    w3, g3, _ = oracle.gwn(P, N, a, None, Q, eps=0.2)
    np.testing.assert_array_equal(w2, w3)
    np.testing.assert_array_equal(g2, g3)


def test_update_and_stats():
    """Eq. 7: unit normals anti-parallel to the gradient; zero gradient keeps the old normal.
    The top-1% statistic equals the mean of the largest ceil(0.01 n) angles (numpy sort)."""
    rng = np.random.default_rng(2)
    n = 1000
    g = rng.standard_normal((3, n))
    g[:, 7] = 0.0
    N0 = rng.standard_normal((3, n))
    N0 /= np.linalg.norm(N0, axis=0)
    N1, ch = oracle.update(g, N0)
    np.testing.assert_allclose(np.linalg.norm(N1, axis=0), 1.0, rtol=1e-14)
    keep = np.arange(n) != 7
    cosang = np.sum(N1 * g, axis=0)[keep] / np.linalg.norm(g, axis=0)[keep]
    np.testing.assert_allclose(cosang, -1.0, rtol=1e-14)
    np.testing.assert_array_equal(N1[:, 7], N0[:, 7])
    np.testing.assert_allclose(ch, np.linalg.norm(N1 - N0, axis=0), rtol=1e-14)
    w = rng.standard_normal(n)
    wm, top, mc = oracle.stats(w, ch, 0.01)
    ang = np.degrees(np.arccos(np.clip(np.sum(N1 * N0, axis=0), -1, 1)))
    k = math.ceil(0.01 * n)
    assert oracle.top_count(n, 0.01) == k == 10
    np.testing.assert_allclose(top, np.sort(ang)[::-1][:k].mean(), rtol=1e-9)
    np.testing.assert_allclose(wm, w.mean(), rtol=1e-13)
    np.testing.assert_allclose(mc, ch.mean(), rtol=1e-13)
    assert oracle.top_count(1, 0.01) == 1 and oracle.top_count(150, 0.01) == 2


def test_splitmix64_published_vector():
    """SplitMix64 reference outputs for seed 1234567 (Vigna's splitmix64.c test vector)."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [oracle.splitmix64(1234567, t) for t in range(5)] == want


def test_random_normals_uniform_on_sphere():
    n = 200_000
    N = oracle.random_normals(42, n)
    np.testing.assert_allclose(np.linalg.norm(N, axis=0), 1.0, rtol=1e-13)
    tol = 5.0 / math.sqrt(n)
    assert np.all(np.abs(N.mean(axis=1)) < tol)
    np.testing.assert_allclose((N**2).mean(axis=1), 1 / 3, atol=tol)
    assert np.abs(np.mean(N[0] * N[1])) < tol
    assert not np.array_equal(N, oracle.random_normals(43, n))
    np.testing.assert_array_equal(N[:, :100], oracle.random_normals(42, 100))


def test_knn_against_kdtree():
    from scipy.spatial import cKDTree
    c = synth.torus_ellipsoids(3000, seed=5)
    P = c.P.astype(np.float64)
    idx, dist = oracle.knn_self(P, 10)
    dd, ii = cKDTree(P.T).query(P.T, k=11)
    np.testing.assert_allclose(dist, dd[:, 1:], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(idx, ii[:, 1:])
    delta = oracle.delta(P, 10)
    np.testing.assert_allclose(delta, dd[:, 1:].mean(axis=1), rtol=1e-12)
    R = P[:, ::7]
    idx2, dist2 = oracle.knn(R, P, 16)
    d3, i3 = cKDTree(R.T).query(P.T, k=16)
    np.testing.assert_allclose(dist2, d3, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(idx2, i3)


@pytest.mark.slow
def test_sphere_method_level():
    """Sec. 4.1 and Eq. 4: exact outward normals are (nearly) a fixed point of the update, and
    from random normals the iteration orients the sphere consistently (either global sign)."""
    c = synth.sphere(1500, 0.005, seed=100)
    P = c.P.astype(np.float64)
    # kernel radius: the anchor rule (mean distance to the 10 nearest anchors, every
    # stride-th point) with 256 anchors, the resolution parameter for one convex solid; this
    # gives delta = 0.25 R. The iteration orients the sphere from random normals once
    # delta >~ R / 8 (512 anchors, delta = 0.16: yes; 1024 anchors, delta = 0.11: 77%).
    delta = oracle.anchor_delta(c.P, k=10, n_anchor=256)
    N1, st = oracle.dwg_run(P, c.area, delta, c.N_true, max_iters=1)
    cos = np.sum(N1 * c.N_true, axis=0)
    assert np.all(cos > 0)
    assert np.degrees(np.arccos(np.clip(cos, -1, 1))).mean() < 10.0
    N0 = oracle.random_normals(200, c.n)
    NT, st = oracle.dwg_run(P, c.area, delta, N0, max_iters=40)
    cos = np.sum(NT * c.N_true, axis=0)
    agree = max(np.mean(cos > 0), np.mean(cos < 0))
    assert agree >= 0.999, agree


def test_anchor_delta_against_kdtree():
    """Radius from the k nearest anchors (every stride-th point, an anchor skips itself)."""
    from scipy.spatial import cKDTree
    c = synth.torus_ellipsoids(5000, seed=6)
    P = c.P.astype(np.float64)
    d = oracle.anchor_delta(P, k=10, n_anchor=300, scale=1.5)
    stride = 5000 // 300
    A = P[:, ::stride]
    dd, ii = cKDTree(A.T).query(P.T, k=11)
    is_anchor = np.arange(5000) % stride == 0
    ref = np.where(is_anchor, dd[:, 1:].mean(axis=1), dd[:, :10].mean(axis=1)) * 1.5
    np.testing.assert_allclose(d, ref, rtol=1e-12)


def test_pca_normals_plane_closed_form():
    """Sec. 5.1 PCA init: points on the plane z = 0.5 + 0.3 x - 0.2 y (off the origin, so a
    covariance taken about the origin instead of the mean fails) have the plane normal
    (-0.3, 0.2, 1)/|.| as the smallest-eigenvalue eigenvector, turned away from the origin."""
    rng = np.random.default_rng(3)
    x, y = rng.uniform(-1, 1, (2, 500))
    P = np.stack([x, y, 0.5 + 0.3 * x - 0.2 * y])
    N = oracle.pca_normals(P, 16)
    ref = np.array([-0.3, 0.2, 1.0]) / math.sqrt(1.13)
    np.testing.assert_allclose(N, np.repeat(ref[:, None], 500, axis=1), atol=1e-9)
    # the mirrored plane z = -0.5 - 0.3 x + 0.2 y lies below the origin: its normal turns down
    N2 = oracle.pca_normals(P * np.array([[1.0], [1.0], [-1.0]]), 16)
    ref2 = np.array([-0.3, 0.2, -1.0]) / math.sqrt(1.13)
    np.testing.assert_allclose(N2, np.repeat(ref2[:, None], 500, axis=1), atol=1e-9)


def test_pca_normals_sphere_is_outward_radial(fib):
    """On a dense sphere about the origin the smallest-variance direction of a 16-NN patch is
    the radius, to O(h) of the patch size (the largest eigenvector would be tangent), and the
    sign rule turns every one outward."""
    N = oracle.pca_normals(fib.P, 16)
    c = np.sum(N * fib.N_true, axis=0)
    assert c.min() > 0.999


def test_gauss_normals_sphere_exact():
    """Sec. 5.1 Gauss map: on a sphere about the origin p / |p| is the outward normal; the
    origin itself maps to (0, 0, 1)."""
    s = synth.fibonacci_sphere(1000)
    P = s.P * 2.5
    np.testing.assert_allclose(oracle.gauss_normals(P), s.N_true, atol=1e-6)
    np.testing.assert_array_equal(oracle.gauss_normals(np.zeros((3, 1))), [[0.0], [0.0], [1.0]])


def test_arithmetic_against_50_digit_brute_force():
    """The oracle's FP64 arithmetic (Neumaier sums, exp/sqrt) against the same sum in 50-digit
    mpmath on 48 sources, plain and screened, with some pairs clamped: <= 1e-13 relative."""
    import mpmath
    mpmath.mp.dps = 50
    rng = np.random.default_rng(8)
    n = 48
    P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    N = rng.normal(size=(3, n))
    N = (N / np.linalg.norm(N, axis=0)).astype(np.float32)
    a = rng.uniform(0.01, 0.1, n).astype(np.float32)
    d = rng.uniform(0.0, 0.4, n).astype(np.float32)
    Q = np.concatenate([P[:, :3], rng.uniform(-1.2, 1.2, (3, 5)).astype(np.float32)], axis=1)
    for lam in [0.0, 10.0]:
        w, g, _ = oracle.gwn(P, N, a, d, Q, lam=lam)
        s = mpmath.sqrt(lam)
        for i in range(Q.shape[1]):
            q = [mpmath.mpf(float(x)) for x in Q[:, i]]
            W, G = mpmath.mpf(0), [mpmath.mpf(0)] * 3
            for j in range(n):
                dv = [mpmath.mpf(float(P[k, j])) - q[k] for k in range(3)]
                r2 = sum(x * x for x in dv)
                if r2 == 0:
                    continue
                r = mpmath.sqrt(r2)
                fl = mpmath.mpf(float(d[j]))
                rho = r if r > fl else fl
                nv = [mpmath.mpf(float(x)) for x in N[:, j]]
                c = sum(dv[k] * nv[k] for k in range(3))
                E = mpmath.exp(-s * r)
                kk = mpmath.mpf(float(a[j])) / (4 * mpmath.pi)
                W += kk * E * (1 + s * r) * c / rho ** 3
                coef = (3 * (1 + s * r) / r2 if rho == r else 0) + s * s
                G = [G[k] + kk * E / rho ** 3 * (coef * c * dv[k] - (1 + s * r) * nv[k]) for k in range(3)]
            assert abs(w[i] - float(W)) <= 1e-13 * max(1.0, abs(float(W)))
            gn = math.sqrt(sum(float(x) ** 2 for x in G))
            for k in range(3):
                assert abs(g[k, i] - float(G[k])) <= 1e-13 * max(1.0, gn)
