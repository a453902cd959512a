"""Shared test helpers: error metrics of the GPU path against the oracle, and fixtures."""
import numpy as np
import torch

TOL_W = 1e-4  # e_w bound
TOL_G = 1e-4  # e_g bound


def e_w(w_gpu, w_ref):
    """max_i |dw_i| / max(|w_ref_i|, 1): w is a dimensionless O(1) quantity."""
    w_gpu = np.asarray(w_gpu, np.float64)
    return float(np.max(np.abs(w_gpu - w_ref) / np.maximum(np.abs(w_ref), 1.0)))


def e_g(g_gpu, g_ref, skip=None):
    """max_i |dg_i| / max(|g_ref_i|, 1e-3 median |g_ref|), skipping flagged queries."""
    g_gpu = np.asarray(g_gpu, np.float64)
    nr = np.linalg.norm(g_ref, axis=0)
    floor = 1e-3 * np.median(nr)
    err = np.linalg.norm(g_gpu - g_ref, axis=0) / np.maximum(nr, max(floor, 1e-30))
    if skip is not None:
        err = err[~skip.astype(bool)]
    return float(err.max()) if err.size else 0.0


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def unit_rows(rng, n):
    v = rng.standard_normal((3, n))
    return (v / np.linalg.norm(v, axis=0)).astype(np.float32)


def angle_deg(a, b):
    """Angle between column vectors in degrees, atan2(|a x b|, a.b) in float64 (robust for
    tiny angles; FP32-stored unit vectors have norms 1 +- 1e-7, which arccos would amplify)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    cr = np.linalg.norm(np.cross(a.T, b.T), axis=1)
    return np.degrees(np.arctan2(cr, np.sum(a * b, axis=0)))


def knn_radius(P, k=10, scale=1.0):
    """scale x mean distance to the k nearest other points, by scipy's cKDTree in float64
    (an input for both sides that does not come from the GPU path)."""
    from scipy.spatial import cKDTree
    X = np.asarray(P, np.float64).T
    d, _ = cKDTree(X).query(X, k=k + 1)
    return (scale * d[:, 1:].mean(axis=1)).astype(np.float32)
