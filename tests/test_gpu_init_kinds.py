"""The paper's PCA and Gauss-map initial normals (Sec. 5.1, "Normal Initialization") through
dwg_init_normals against the oracle on the same seeded points."""
import numpy as np
import pytest

import oracle
from paper_2405_13839_amd import synth
from tests.helpers import cuda, host

pytestmark = pytest.mark.gpu


def _dwg():
    from paper_2405_13839_amd import dwg
    return dwg


@pytest.mark.parametrize("n", [1, 7, 1000, 65_537])
def test_gauss_normals_match_oracle(n):
    dwg = _dwg()
    rng = np.random.default_rng(n)
    P = rng.normal(size=(3, n)).astype(np.float32)
    P[:, 0] = 0.0  # the origin maps to (0, 0, 1)
    N = host(dwg.gauss_normals(cuda(P)))
    ref = oracle.gauss_normals(P)
    np.testing.assert_allclose(N, ref, atol=2e-7, rtol=0)


@pytest.mark.parametrize("case", ["torus_ellipsoids_20K", "sphere_17", "sphere_4097"])
def test_pca_normals_match_oracle(case):
    """Same line as the oracle's eigenvector (|cos| ~ 1) on all but near-tied neighbour sets
    or near-degenerate eigenvalues; where n . p is clear of zero, the same sign; unit length
    everywhere."""
    dwg = _dwg()
    if case == "torus_ellipsoids_20K":
        P = synth.torus_ellipsoids(20_000, seed=303).P
    else:
        P = synth.sphere(int(case.split("_")[1]), 0.002, 5).P
    N = host(dwg.pca_normals(cuda(P))).astype(np.float64)
    ref = oracle.pca_normals(P, 16)
    c = np.sum(N * ref, axis=0)
    assert np.mean(np.abs(c) > 1 - 1e-6) >= 0.999, np.sort(np.abs(c))[:10]
    P64 = np.asarray(P, np.float64)
    clear = (np.abs(np.sum(ref * P64, axis=0)) > 1e-3 * np.linalg.norm(P64, axis=0)) & (np.abs(c) > 1 - 1e-6)
    assert clear.mean() > 0.9
    assert np.all(c[clear] > 0)
    np.testing.assert_allclose(np.linalg.norm(N, axis=0), 1.0, atol=1e-6)


def test_pca_rejects_too_few_points():
    """16 points have no 16 nearest other points: DWG_E_INVALID, raised as DwgError."""
    dwg = _dwg()
    P = cuda(np.random.default_rng(0).normal(size=(3, 16)).astype(np.float32))
    with pytest.raises(dwg.DwgError):
        dwg.pca_normals(P)
