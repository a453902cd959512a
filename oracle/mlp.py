"""FP64 NumPy oracle of the learned initial normals (an extension of the paper's random /
PCA / Gauss-map initialisation, Sec. 5.1 "Normal Initialization").

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py). Written from the definitions:

* features: for point i, its 16 nearest anchors (anchors = every stride-th point,
  stride = max(1, n // n_anchor), the anchor i itself excluded when i is one), ordered by
  (distance, index); feature = (anchor - p_i) / s_i with s_i the mean of the 16 distances.
* MLP 48 -> 128 -> 128 -> 3 with ReLU, output normalised. The GPU rounds every GEMM
  operand to BF16 (round to nearest even) and accumulates in FP32; this oracle rounds the
  same operands (X, W1, W2, W3, h1, h2 in the forward; the upstream gradients and
  activations of every backward GEMM) and computes everything else in float64.
  `bf16=False` gives the plain float64 network.
* loss = mean over kept rows of (1 - <y/|y|, t>); gradients by the chain rule written out
  layer by layer; Adam (Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

from . import knn as _knn

IN, HID, OUT, K = 48, 128, 3, 16
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)),
          ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64. Values are first
    rounded to float32, as the GPU holds them."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


U32 = 2.0 ** -24  # unit roundoff of float32


def _bf16_tie_gap(v):
    """Distance of each value to the nearest bfloat16 rounding boundary (the midpoint of two
    consecutive bfloat16 numbers, exactly representable in float32)."""
    v = np.asarray(v, np.float64)
    u = np.ascontiguousarray(v.astype(np.float32)).view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    hi_prev = ((u & np.uint32(0xFFFF0000)) - np.uint32(0x10000)) | np.uint32(0x8000)
    m1 = lo.view(np.float32).astype(np.float64)
    m0 = hi_prev.view(np.float32).astype(np.float64)
    return np.minimum(np.abs(v - m1), np.abs(v - m0))


def _bf16_ulp(v):
    """Spacing of the bfloat16 numbers around each value (2^(e - 7) for |v| in [2^e, 2^(e+1)))."""
    v = np.abs(np.asarray(v, np.float64))
    e = np.floor(np.log2(np.maximum(v, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def forward_bound(blob, X, x_rel_err=0.0):
    """A bound, per row, on |y_gpu - y| between this oracle's forward pass and any float32
    evaluation of the same network on BF16-rounded operands (bound [B]), with y [B, 3].

    Interval propagation, layer by layer: a float32 dot product of K terms is off by at most
    K u sum|terms| (u = 2^-24); an activation whose uncertainty reaches a bfloat16 rounding
    boundary may round to the neighbouring bfloat16 value (one more ulp); ReLU and the
    rounding to nearest are 1-Lipschitz otherwise. With x_rel_err > 0 the inputs carry that
    relative error (features computed in float32) and may round either way too."""
    p = unpack(blob)
    X = np.asarray(X, np.float64)
    W1, W2, W3 = bf16(p["W1"]), bf16(p["W2"]), bf16(p["W3"])
    X0 = bf16(X)
    dX = np.zeros_like(X0)
    if x_rel_err > 0:
        ex = x_rel_err * np.abs(X)
        dX = ex + np.where(_bf16_tie_gap(X) <= ex, _bf16_ulp(X), 0.0)

    def layer(h, dh, W, b, K):
        z = h @ W.T + b
        dz = np.abs(dh) @ np.abs(W).T + 2 * K * U32 * (np.abs(h) @ np.abs(W).T + np.abs(b))
        return z, dz

    def act(z, dz):
        a = np.maximum(z, 0.0)
        hr = bf16(a)
        # the float32 side's activation lies within dz of a; its rounding within one ulp
        flip = _bf16_tie_gap(a) <= dz
        return hr, dz + np.where(flip, _bf16_ulp(a), 0.0)

    z1, dz1 = layer(X0, dX, W1, p["b1"], IN)
    h1, dh1 = act(z1, dz1)
    z2, dz2 = layer(h1, dh1, W2, p["b2"], HID)
    h2, dh2 = act(z2, dz2)
    y, dy = layer(h2, dh2, W3, p["b3"], HID)
    return y, np.linalg.norm(dy, axis=1)


def unpack(blob):
    """Parameter blob (W1, b1, W2, b2, W3, b3 row-major) -> dict of float64 arrays."""
    blob = np.asarray(blob, np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = blob[o:o + k].reshape(shp)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def forward(blob, X, bf16_ops=True):
    """Returns (y [B,3], yhat [B,3], cache)."""
    p = unpack(blob)
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, np.float64))
    X0 = r(X)
    z1 = X0 @ r(p["W1"]).T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = r(h1)
    z2 = h1r @ r(p["W2"]).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    h2r = r(h2)
    y = h2r @ r(p["W3"]).T + p["b3"]
    yn = np.linalg.norm(y, axis=1, keepdims=True)
    yhat = y / np.maximum(yn, 1e-30)
    return y, yhat, dict(X0=X0, z1=z1, h1r=h1r, z2=z2, h2r=h2r, y=y, yn=yn, yhat=yhat, p=p, r=r)


def loss_and_grad(blob, X, T, mask=None, bf16_ops=True):
    """(loss, grad blob). loss = mean over kept rows of 1 - <yhat, t>."""
    y, yhat, c = forward(blob, X, bf16_ops)
    T = np.asarray(T, np.float64)
    keep = np.ones(len(y), bool) if mask is None else np.asarray(mask).astype(bool)
    nk = max(int(keep.sum()), 1)
    cos = np.sum(yhat * T, axis=1)
    loss = float(np.sum((1.0 - cos)[keep]) / nk)
    r, p = c["r"], c["p"]
    # d loss / d y for one row: -(t - <yhat,t> yhat) / |y| / nk
    dy = -(T - cos[:, None] * yhat) / np.maximum(c["yn"], 1e-30) / nk
    dy[~keep] = 0.0
    g = {}
    g["W3"] = dy.T @ c["h2r"]
    g["b3"] = dy.sum(0)
    dh2 = dy @ r(p["W3"])
    dz2 = dh2 * (c["z2"] > 0)
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ c["h1r"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2r @ r(p["W2"])
    dz1 = dh1 * (c["z1"] > 0)
    dz1r = r(dz1)
    g["W1"] = dz1r.T @ c["X0"]
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam(blob, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (float64): returns (blob, m, v)."""
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * grad
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * grad * grad
    mh = m / (1 - b1**step)
    vh = v / (1 - b2**step)
    return np.asarray(blob, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(P, n_anchor=4096):
    """[n, 48] float64 features and the ambiguity flags (True where two of the 17 nearest
    anchor distances are within 1e-5 relative, so FP32 may order them differently)."""
    P = np.asarray(P, np.float64)
    n = P.shape[1]
    stride = max(1, n // n_anchor)
    A = P[:, ::stride]
    skip = np.where(np.arange(n) % stride == 0, np.arange(n) // stride, -1).astype(np.int32)
    idx, dist = _knn(A, P, K + 1, skip=skip)
    s = dist[:, :K].mean(axis=1)
    rel = A[:, idx[:, :K]] - P[:, :, None]  # [3, n, K]
    f = (rel / s[None, :, None]).transpose(1, 2, 0).reshape(n, K * 3)
    gaps = np.diff(dist, axis=1) / np.maximum(dist[:, 1:], 1e-30)
    amb = np.any(gaps < 1e-5, axis=1)
    return f, amb
