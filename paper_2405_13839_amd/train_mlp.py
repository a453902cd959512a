"""Trains the learned initial-normal MLP with the library's own GPU kernels.

    python -m paper_2405_13839_amd.train_mlp --shapes 2000 --n 50000 --epochs 3 \
        --out paper_2405_13839_amd/weights/mlp_init.safetensors

Data: seeded shapes of the torus + 2 ellipsoids family (seeds 10000 + k, 5% outliers,
noise 0.25% of the diagonal). Targets: the plain method's converged normals -- dwg_iterate
(screened, lambda = 10, radius = mean distance to the 10 nearest of 4096 anchors) run to its
convergence test from
the analytic normals, i.e. the fixed point of the same iteration in the consistently
oriented basin -- with each component's sign fixed by the divergence theorem; outliers are
masked out of the loss. Features: dwg_features (16 nearest of 4096 anchors). Optimiser:
dwg_mlp_train_step (BF16 MFMA forward / backward, FP32 Adam), cosine learning-rate decay.

`--eval K` then compares learned and random initialisation on K held-out shapes
(seeds 20000 + k): iterations to the convergence test and mean angle error.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _gen(args):
    from paper_2405_13839_amd import synth
    seed, n = args
    c = synth.torus_ellipsoids(n, seed=seed)
    return c.P, c.area, c.N_true, c.comp, c.inlier


def _shapes(seeds, n, workers):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        yield from ex.map(_gen, [(s, n) for s in seeds], chunksize=4)


def converged_targets(dwg, metrics, P, area, N_true, comp, lam, ws, dev, seed):
    """Fixed point of the iteration reached from the analytic normals (outliers start random)."""
    import torch
    n = P.shape[1]
    Pt = torch.from_numpy(P).to(dev)
    at = torch.from_numpy(area).to(dev)
    d = dwg.delta_anchor_mean(Pt, 10, 4096, 1.0, ws=ws)
    N0 = dwg.random_normals(n, seed, dev)
    inl = torch.from_numpy(comp >= 0).to(dev)
    N0[:, inl] = torch.from_numpy(N_true).to(dev)[:, inl]
    st, stats = dwg.iterate(Pt, at, d, N0, dwg.Params(lam=lam), max_iters=40, ws=ws)
    Nc = N0.cpu().numpy()
    sg = metrics.divergence_sign(P, Nc, area, comp)
    for k, s in sg.items():
        Nc[:, comp == k] *= s
    return Pt, Nc, int(stats.shape[0])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", type=int, default=2000)
    ap.add_argument("--n", type=int, default=50_000)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lam", type=float, default=10.0)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--eval", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights", "mlp_init.safetensors"))
    ap.add_argument("--log", default="train_mlp.json")
    args = ap.parse_args(argv)
    import torch

    from paper_2405_13839_amd import dwg, metrics, mlp_init

    dev = torch.device("cuda", 0)
    n = args.n
    ws = dwg.workspace(n, n, dev, dwg.Params(lam=args.lam))
    X = torch.empty((args.shapes * n, 48), dtype=torch.float32, device=dev)
    T = torch.empty((args.shapes * n, 3), dtype=torch.float32, device=dev)
    M = torch.empty(args.shapes * n, dtype=torch.uint8, device=dev)
    t0 = time.time()
    iters = []
    for k, (P, area, N_true, comp, inl) in enumerate(_shapes(range(10000, 10000 + args.shapes), n, args.workers)):
        Pt, Nc, it = converged_targets(dwg, metrics, P, area, N_true, comp, args.lam, ws, dev, 300000 + k)
        iters.append(it)
        X[k * n:(k + 1) * n] = dwg.features(Pt, 4096, ws=ws)
        T[k * n:(k + 1) * n] = torch.from_numpy(np.ascontiguousarray(Nc.T)).to(dev)
        M[k * n:(k + 1) * n] = torch.from_numpy(inl.astype(np.uint8)).to(dev)
        if k % 200 == 0:
            print(f"[data] shape {k}/{args.shapes}  {time.time() - t0:.0f}s  target iters {it}", flush=True)
    t_data = time.time() - t0
    print(f"[data] done in {t_data:.0f}s, mean target iterations {np.mean(iters):.1f}", flush=True)

    blob = torch.from_numpy(mlp_init.init_params(0)).to(dev)
    m1 = torch.zeros_like(blob)
    m2 = torch.zeros_like(blob)
    rows = X.shape[0]
    steps_per_epoch = rows // args.batch
    total = steps_per_epoch * args.epochs
    g = torch.Generator(device=dev)
    g.manual_seed(1234)
    step = 0
    t1 = time.time()
    hist = []
    for ep in range(args.epochs):
        perm = torch.randperm(rows, device=dev, generator=g)
        run = 0.0
        for b in range(steps_per_epoch):
            idx = perm[b * args.batch:(b + 1) * args.batch]
            step += 1
            lr = args.lr * 0.5 * (1 + math.cos(math.pi * step / total))
            loss, _ = dwg.mlp_train_step(blob, m1, m2, step, max(lr, 1e-6), X[idx].contiguous(), T[idx].contiguous(),
                                         M[idx].contiguous())
            if b % 500 == 0:
                lv = float(loss.item())
                hist.append((step, lv))
                print(f"[train] epoch {ep} step {b}/{steps_per_epoch} loss {lv:.4f} lr {lr:.2e} "
                      f"{time.time() - t1:.0f}s", flush=True)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    mlp_init.save_params(args.out, blob.cpu().numpy(), meta=dict(shapes=args.shapes, n=n, epochs=args.epochs,
                                                                 batch=args.batch, lr=args.lr, lam=args.lam))
    del X, T, M
    torch.cuda.empty_cache()

    ev = []
    for k, (P, area, N_true, comp, inl) in enumerate(_shapes(range(20000, 20000 + args.eval), n, args.workers)):
        Pt = torch.from_numpy(P).to(dev)
        at = torch.from_numpy(area).to(dev)
        d = dwg.delta_anchor_mean(Pt, 10, 4096, 1.0, ws=ws)
        row = {}
        for kind in ["mlp", "random"]:
            N0 = dwg.mlp_normals(Pt, blob, ws=ws) if kind == "mlp" else dwg.random_normals(n, 400000 + k, dev)
            r0 = metrics.orientation_report(N0.cpu().numpy(), N_true, comp)
            st, stats = dwg.iterate(Pt, at, d, N0, dwg.Params(lam=args.lam), max_iters=100, ws=ws)
            r1 = metrics.orientation_report(N0.cpu().numpy(), N_true, comp)
            row[kind] = dict(init_mae=r0["mae_deg"], iters=int(stats.shape[0]), converged=st == dwg.DWG_OK,
                             mae=r1["mae_deg"], agree=r1["agree"])
        ev.append(row)
        print(f"[eval] {k}: {json.dumps(row)}", flush=True)
    summ = {}
    for kind in ["mlp", "random"]:
        summ[kind] = {key: float(np.mean([r[kind][key] for r in ev])) for key in ["init_mae", "iters", "mae", "agree"]}
        summ[kind]["frac_mae_le_5deg"] = float(np.mean([r[kind]["mae"] <= 5.0 for r in ev]))
    out = dict(t_data=t_data, t_train=t_train, target_iters=float(np.mean(iters)), loss=hist, eval=summ, per_shape=ev)
    os.makedirs(os.path.dirname(os.path.abspath(args.log)), exist_ok=True)
    json.dump(out, open(args.log, "w"), indent=1)
    print("[done]", json.dumps(summ), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
