"""Orientation-quality metrics (host side, float64). Not part of the hot path.

Both global orientations are fixed points of the iteration, and disconnected solids may
settle with independent signs, so the metrics align signs per connected component by
majority vote before measuring angles. Outliers (comp < 0) are excluded.
"""
from __future__ import annotations

import numpy as np


def _unit(N):
    N = np.asarray(N, np.float64)
    return N / np.maximum(np.linalg.norm(N, axis=0), 1e-300)


def component_signs(N, N_true, comp):
    """+1/-1 per component: the sign that makes the majority of its points agree with truth."""
    cos = np.sum(_unit(N) * np.asarray(N_true, np.float64), axis=0)
    signs = {}
    for k in np.unique(comp[comp >= 0]):
        m = comp == k
        signs[int(k)] = 1.0 if np.mean(cos[m] > 0) >= 0.5 else -1.0
    return signs


def orientation_report(N, N_true, comp):
    """dict: agree (per-component sign-aligned fraction of inliers with cos > 0), agree_global
    (one sign for all inliers), mae_deg (mean angle error, per-component aligned), p95_deg."""
    N = _unit(N)
    T = np.asarray(N_true, np.float64)
    comp = np.asarray(comp)
    inl = comp >= 0
    cos = np.sum(N * T, axis=0)
    sg = component_signs(N, T, comp)
    s = np.ones(N.shape[1])
    for k, v in sg.items():
        s[comp == k] = v
    ca = (cos * s)[inl]
    ang = np.degrees(np.arccos(np.clip(ca, -1, 1)))
    g = cos[inl]
    return dict(agree=float(np.mean(ca > 0)), agree_global=float(max(np.mean(g > 0), np.mean(g < 0))),
                mae_deg=float(ang.mean()), p95_deg=float(np.percentile(ang, 95)),
                components=len(sg))


def divergence_sign(P, N, area, comp):
    """Sign per component from the divergence theorem: sum_i a_i <n_i, p_i - c> equals
    3 x volume > 0 for outward normals (c = the component's centroid). Needs no truth."""
    P = np.asarray(P, np.float64)
    N = _unit(N)
    a = np.asarray(area, np.float64)
    out = {}
    for k in np.unique(comp[comp >= 0]):
        m = comp == k
        c = P[:, m].mean(axis=1, keepdims=True)
        v = np.sum(a[m] * np.sum(N[:, m] * (P[:, m] - c), axis=0))
        out[int(k)] = 1.0 if v >= 0 else -1.0
    return out
