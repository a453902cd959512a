"""Pins of the MLP / feature oracle: torch autograd and torch.optim.Adam (independent
implementations), finite differences, published bfloat16 rounding, feature invariants."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as om
from paper_2405_13839_amd import synth


def _params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in om.SHAPES:
        fan_in = shp[1] if len(shp) == 2 else 16
        p[name] = rng.standard_normal(shp) * math.sqrt(2.0 / fan_in) * (1 if len(shp) == 2 else 0.1)
    return om.pack(p)


def _batch(seed=1, B=200):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, om.IN))
    T = rng.standard_normal((B, 3))
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    mask = rng.uniform(size=B) < 0.8
    return X, T, mask


def _torch_loss(blob, X, T, mask):
    P = om.unpack(blob)
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    x = torch.tensor(X)
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    y = h2 @ t["W3"].T + t["b3"]
    yh = y / y.norm(dim=1, keepdim=True)
    m = torch.tensor(mask)
    loss = (1 - (yh * torch.tensor(T)).sum(1))[m].sum() / m.sum()
    loss.backward()
    return float(loss.detach()), np.concatenate([t[name].grad.numpy().ravel() for name, _ in om.SHAPES])


def test_backward_matches_torch_autograd():
    blob = _params()
    X, T, mask = _batch()
    loss, g = om.loss_and_grad(blob, X, T, mask, bf16_ops=False)
    tl, tg = _torch_loss(blob, X, T, mask)
    assert abs(loss - tl) < 1e-12
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-12)
    assert om.N_PARAMS == 23171


def test_backward_matches_finite_differences():
    blob = _params(3)
    X, T, mask = _batch(4, 64)
    _, g = om.loss_and_grad(blob, X, T, mask, bf16_ops=False)
    rng = np.random.default_rng(5)
    h = 1e-6
    for i in rng.choice(om.N_PARAMS, 40, replace=False):
        e = np.zeros_like(blob)
        e[i] = h
        lp, _ = om.loss_and_grad(blob + e, X, T, mask, bf16_ops=False)
        lm, _ = om.loss_and_grad(blob - e, X, T, mask, bf16_ops=False)
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_adam_matches_torch():
    blob = _params(7)
    X, T, mask = _batch(8)
    m = np.zeros_like(blob)
    v = np.zeros_like(blob)
    tp = torch.tensor(blob, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    b = blob.copy()
    for step in range(1, 4):
        _, g = om.loss_and_grad(b, X, T, mask, bf16_ops=False)
        b, m, v = om.adam(b, m, v, g, step, 1e-3)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(b, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-9, -2.5, 3.0e-3, 65504.0, 1e30], dtype=np.float64)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16(x), ref)
    assert om.bf16(np.array([1 + 2**-8]))[0] == 1.0  # tie to even
    rng = np.random.default_rng(0)
    y = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    ref = torch.tensor(y, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16(y), ref)


def test_feature_invariants():
    c = synth.torus_ellipsoids(6000, seed=12)
    P = c.P.astype(np.float64)
    f, amb = om.features(P, n_anchor=512)
    assert f.shape == (6000, 48)
    norms = np.linalg.norm(f.reshape(-1, 16, 3), axis=2)
    np.testing.assert_allclose(norms.mean(axis=1), 1.0, rtol=1e-12)  # s_i is the mean distance
    assert np.all(np.diff(norms, axis=1) >= -1e-12)  # ascending distance
    ok = ~amb
    f2, _ = om.features(P + np.array([[0.3], [-2.0], [1.1]]), n_anchor=512)
    np.testing.assert_allclose(f2[ok], f[ok], atol=1e-9)
    f3, _ = om.features(2.7 * P, n_anchor=512)
    np.testing.assert_allclose(f3[ok], f[ok], atol=1e-9)
    R = np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))[0]
    f4, _ = om.features(R @ P, n_anchor=512)
    rot = (f.reshape(-1, 16, 3) @ R.T).reshape(-1, 48)
    np.testing.assert_allclose(f4[ok], rot[ok], atol=1e-9)
    # an anchor never sees itself
    stride = 6000 // 512
    assert np.all(norms[::stride, 0] > 0)


def test_forward_bound_covers_a_float32_evaluation():
    """om.forward_bound bounds |y_fp32 - y| for any float32 evaluation on BF16 operands: a
    float32 NumPy forward pass (its own summation order, its own BF16 flips of activations
    near a rounding boundary) stays inside the bound on every row, including rows with such
    flips, and the bound is not vacuous (median relative bound well below 1)."""
    from oracle import mlp as om
    from paper_2405_13839_amd import mlp_init
    blob = mlp_init.init_params(3)
    rng = np.random.default_rng(4)
    blob[om.N_PARAMS - 3 - 3 * 128 - 128:] += rng.standard_normal(3 + 3 * 128 + 128).astype(np.float32) * 0.05
    X = rng.standard_normal((4000, 48)).astype(np.float32)
    p = om.unpack(blob)

    def r32(a):
        return om.bf16(a).astype(np.float32)

    h1 = r32(np.maximum(r32(X) @ r32(p["W1"]).T + p["b1"].astype(np.float32), 0))
    h2 = r32(np.maximum(h1 @ r32(p["W2"]).T + p["b2"].astype(np.float32), 0))
    y32 = (h2 @ r32(p["W3"]).T + p["b3"].astype(np.float32)).astype(np.float64)
    y, bound = om.forward_bound(blob, X)
    err = np.linalg.norm(y32 - y, axis=1)
    assert np.all(err <= bound)
    assert np.median(bound / np.linalg.norm(y, axis=1)) < 0.05
    # some rows do differ by a flip (the bound is exercised, not only the accumulation term)
    y_noflip, _, _ = om.forward(blob, X)
    assert np.any(err > 1e-4 * np.linalg.norm(y_noflip, axis=1))
