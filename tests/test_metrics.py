"""The divergence-theorem sign rule that orients the MLP's training targets and aligns the
orientation metrics (no ground truth needed): sum_i a_i <n_i, p_i - c> = 3 x volume > 0 for
outward normals on a closed surface."""
import math

import numpy as np

from paper_2405_13839_amd import metrics, synth


def test_divergence_identity_on_a_sphere():
    s = synth.fibonacci_sphere(20000, R=0.8)
    c = s.P.mean(axis=1, keepdims=True)
    v = np.sum(s.area * np.sum(s.N_true * (s.P - c), axis=0))
    assert abs(v - 3 * (4.0 / 3.0) * math.pi * 0.8 ** 3) < 1e-3 * v


def test_divergence_sign_per_component():
    c = synth.ellipsoids_tori(30000, seed=5)
    N = c.N_true.astype(np.float64).copy()
    comps = sorted(k for k in np.unique(c.comp) if k >= 0)
    flip = comps[0]
    N[:, c.comp == flip] *= -1
    sg = metrics.divergence_sign(c.P, N, c.area, c.comp)
    assert sg[flip] == -1.0 and all(sg[k] == 1.0 for k in comps if k != flip)


def test_orientation_report_aligns_components():
    c = synth.ellipsoids_tori(20000, seed=6)
    N = c.N_true.astype(np.float64).copy()
    comps = sorted(k for k in np.unique(c.comp) if k >= 0)
    N[:, c.comp == comps[0]] *= -1  # one component flipped: still fully consistent per component
    rep = metrics.orientation_report(N, c.N_true, c.comp)
    assert len(comps) > 2
    assert rep["agree"] == 1.0 and rep["mae_deg"] < 0.01  # FP32 unit vectors: ~1e-3 deg
    assert rep["agree_global"] < 1.0
