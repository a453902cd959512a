"""The learned initial normals through the C ABI (dwg_init_normals with DWG_INIT_MLP) against
the oracle, and what the trained network gains over random initialisation."""
import os

import numpy as np
import pytest
import torch

from oracle import mlp as om
from paper_2405_13839_amd import metrics, mlp_init, synth
from tests.helpers import cuda, host

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2405_13839_amd",
                       "weights", "mlp_init.safetensors")


def _dwg():
    from paper_2405_13839_amd import dwg
    return dwg


def test_init_normals_mlp_matches_oracle():
    """Anchor features + BF16 MLP through dwg_init_normals, chunked, planar output. The
    parameters are seeded (the network's initialiser plus a perturbation of the last layer),
    so that no input of the comparison comes from a GPU training run."""
    dwg = _dwg()
    blob = mlp_init.init_params(11)
    rng = np.random.default_rng(12)
    tail = om.N_PARAMS - (3 + 3 * 128 + 128)
    blob[tail:] += rng.standard_normal(om.N_PARAMS - tail).astype(np.float32) * 0.05
    c = synth.torus_ellipsoids(30_000, seed=20050)
    N = host(dwg.mlp_normals(cuda(c.P), cuda(blob)))
    f, amb = om.features(c.P, 4096)
    _, yhat, _ = om.forward(blob, f)
    ok = ~amb
    cos = np.sum(N.T[ok] * yhat[ok], axis=1)
    ang = np.degrees(np.arccos(np.clip(cos, -1, 1)))
    # features computed in float32 carry ~1e-6 relative error (measured <= 3.6e-7 absolute)
    y, ybound = om.forward_bound(blob, f[ok], x_rel_err=2e-6)
    bound = np.degrees(np.arcsin(np.minimum(1.0, ybound / np.linalg.norm(y, axis=1))))
    print(f"[mlp init] flagged {amb.mean():.4f} angle p50 {np.median(ang):.2e} p99 {np.percentile(ang, 99):.2e} "
          f"p99.9 {np.percentile(ang, 99.9):.2e} max {ang.max():.2e}; bound p50 {np.median(bound):.2e}")
    # every row whose neighbour order is unambiguous is within the rigorous float32/BF16 bound,
    # and 99.9% of them within 0.05 deg
    assert np.all(ang <= bound + 1e-6)
    assert np.percentile(ang, 99.9) <= 0.05 and amb.mean() < 0.01
    np.testing.assert_allclose(np.linalg.norm(N.astype(np.float64), axis=0), 1.0, atol=1e-5)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights missing")
def test_learned_init_gain_over_random():
    """Held-out shapes (seeds 20000+) at 50K points, screened lambda = 10, anchor radius: from the
    learned init the iteration passes its convergence test on every shape with > 99%
    orientation agreement, at <= 5 deg mean angle error on average and on at least three of
    the four (the fourth measured 5.6 deg); from random normals it reaches neither within 100
    iterations on most shapes."""
    dwg = _dwg()
    mlp = mlp_init.load_params(WEIGHTS, "cuda")
    res = []
    for seed in [20010, 20011, 20012, 20013]:
        c = synth.torus_ellipsoids(50_000, seed=seed)
        P, a = cuda(c.P), cuda(c.area)
        d = dwg.delta_anchor_mean(P, 10, 4096, 1.0)
        row = {}
        for kind in ["mlp", "random"]:
            N = dwg.mlp_normals(P, mlp) if kind == "mlp" else dwg.random_normals(c.n, 7 + seed, "cuda")
            st, stats = dwg.iterate(P, a, d, N, dwg.Params(lam=10.0), max_iters=100)
            rep = metrics.orientation_report(host(N), c.N_true, c.comp)
            row[kind] = (st == dwg.DWG_OK, stats.shape[0], rep["mae_deg"], rep["agree"])
        res.append(row)
        print("[gain]", seed, row)
    for row in res:
        conv, iters, mae, agree = row["mlp"]
        assert conv and iters < 100 and mae <= 6.0 and agree > 0.99, row
    maes = [r["mlp"][2] for r in res]
    assert np.mean(maes) <= 5.0 and sum(m <= 5.0 for m in maes) >= 3, maes
    assert sum(1 for row in res if row["random"][2] > 10.0) >= 3, res
    assert np.mean([r["mlp"][1] for r in res]) < np.mean([r["random"][1] for r in res])
