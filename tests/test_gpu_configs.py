"""Parity of the all-pairs kernel on every workload configuration at its full size: the
sphere (2K, plain), torus + 2 ellipsoids (100K and 1M, screened), superquadrics + thin
plates (5M, plain and screened) and 20 ellipsoids / tori (15M, screened). All sources take
part; a seeded sample of queries is evaluated on the GPU and recomputed one by one by the
FP64 oracle; the 1M, 5M and 15M configurations are also run as full launches (every point a
query) and compared on a seeded 10K-point subset. Inputs (points, random unit normals,
anchor radius by scipy's cKDTree) come from the seeded generators, never from the GPU path.
Prints e_w / e_g per configuration."""
import numpy as np
import pytest

import oracle
from paper_2405_13839_amd import synth
from tests.helpers import TOL_G, TOL_W, cuda, e_g, e_w, host, unit_rows

pytestmark = pytest.mark.gpu

CONFIGS = [
    # name, generator, lambda, sampled queries
    ("C1 sphere 2K", lambda: synth.sphere(2000, 0.005, 100), 0.0, 2000),
    ("C2 torus+ellipsoids 100K", lambda: synth.torus_ellipsoids(100_000, seed=101), 10.0, 400),
    ("C3 torus+ellipsoids 1M", lambda: synth.torus_ellipsoids(1_000_000, seed=102), 10.0, 300),
    ("C4 superquadrics+plates 5M", lambda: synth.superquadrics_plates(5_000_000, seed=103), 0.0, 200),
    ("C4 superquadrics+plates 5M screened", lambda: synth.superquadrics_plates(5_000_000, seed=103), 10.0, 200),
    ("C5 ellipsoids+tori 15M", lambda: synth.ellipsoids_tori(15_000_000, seed=104), 10.0, 150),
]


def anchor_radius(P, k=10, n_anchor=4096):
    from scipy.spatial import cKDTree
    n = P.shape[1]
    stride = max(1, n // n_anchor)
    X = np.asarray(P, np.float64).T
    d, _ = cKDTree(X[::stride]).query(X, k=k + 1, workers=16)
    is_anchor = np.arange(n) % stride == 0
    return np.where(is_anchor, d[:, 1:].mean(axis=1), d[:, :k].mean(axis=1)).astype(np.float32)


@pytest.mark.parametrize("name,gen,lam,nq", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_config_full_size_sampled(name, gen, lam, nq):
    from paper_2405_13839_amd import dwg
    c = gen()
    rng = np.random.default_rng(17)
    N = unit_rows(rng, c.n)
    d = anchor_radius(c.P)
    sel = np.sort(rng.choice(c.n, min(nq, c.n), replace=False))
    Q = np.ascontiguousarray(c.P[:, sel])
    w, g = dwg.gwn(cuda(c.P), cuda(N), cuda(c.area), cuda(d), cuda(Q), dwg.Params(lam=lam))
    w_ref, g_ref, flag = oracle.gwn(c.P, N, c.area, d, Q, lam=lam)
    ew, eg = e_w(host(w), w_ref), e_g(host(g), g_ref, skip=flag)
    print(f"[accuracy] {name}: n={c.n} lambda={lam} queries={len(sel)} e_w={ew:.2e} e_g={eg:.2e} "
          f"flagged={int(flag.sum())}")
    assert ew <= TOL_W and eg <= TOL_G


FULL_LAUNCH = [
    # name, generator, lambda
    ("C3 torus+ellipsoids 1M screened", lambda: synth.torus_ellipsoids(1_000_000, seed=102), 10.0),
    ("C4 superquadrics+plates 5M", lambda: synth.superquadrics_plates(5_000_000, seed=103), 0.0),
    ("C4 superquadrics+plates 5M screened", lambda: synth.superquadrics_plates(5_000_000, seed=103), 10.0),
    ("C5 ellipsoids+tori 15M screened", lambda: synth.ellipsoids_tori(15_000_000, seed=104), 10.0),
]


@pytest.mark.parametrize("name,gen,lam", FULL_LAUNCH, ids=[c[0] for c in FULL_LAUNCH])
def test_full_launch_10k_subset(name, gen, lam, capsys):
    """A configuration evaluated as the iteration does: every point is a query of one launch
    (all query blocks, the library's default split), and w and grad w of a seeded 10K-point
    subset are compared with the FP64 oracle. In the 5M scene, scaling absolute positions by
    kappa in FP32 would flip the clamp branch of a few near pairs (e_g ~ 6e-2 at one query in
    10K); the kernels take kappa (p - q) from differences. The 15M launch takes about two
    minutes on the GPU and the oracle's subset about as long on 16 cores, so each stage
    reports when it is done."""
    from paper_2405_13839_amd import dwg

    def done(msg):
        with capsys.disabled():
            print(f"\n[full launch] {name}: {msg}", flush=True)

    c = gen()
    rng = np.random.default_rng(17)
    N = unit_rows(rng, c.n)
    d = anchor_radius(c.P)
    sel = np.sort(rng.choice(c.n, 10_000, replace=False))
    done(f"inputs ready (n={c.n})")
    Pc = cuda(c.P)
    w, g = dwg.gwn(Pc, cuda(N), cuda(c.area), cuda(d), Pc, dwg.Params(lam=lam))
    wg, gg = host(w)[sel], host(g)[:, sel]
    del w, g, Pc
    done("GPU launch done")
    parts = []
    for k, part in enumerate(np.array_split(sel, 4)):
        parts.append(oracle.gwn(c.P, N, c.area, d, np.ascontiguousarray(c.P[:, part]), lam=lam))
        done(f"oracle part {k + 1}/4 done")
    w_ref = np.concatenate([p[0] for p in parts])
    g_ref = np.concatenate([p[1] for p in parts], axis=1)
    flag = np.concatenate([p[2] for p in parts])
    ew, eg = e_w(wg, w_ref), e_g(gg, g_ref, skip=flag)
    print(f"[accuracy] {name} full launch: 10K-point subset e_w={ew:.2e} e_g={eg:.2e} "
          f"flagged={int(flag.sum())}")
    assert ew <= TOL_W and eg <= TOL_G
