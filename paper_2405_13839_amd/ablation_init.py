"""Convergence from the four initialisations (random, PCA, Gauss map, learned) across the
screening coefficient, in the spirit of the paper's initialisation ablation (Sec. 5.1,
"Normal Initialization"): per shape, lambda and init, the iterations to the convergence
test, whether it passed, the mean angle error and the orientation agreement.

    python -m paper_2405_13839_amd.ablation_init --n 50000 --out ablation_init.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

SHAPES = {
    # name: (generator, seed, kwargs)
    "torus+2ellipsoids": ("torus_ellipsoids", 20010, {}),
    "torus+2ellipsoids/b": ("torus_ellipsoids", 20011, {}),
    "torus+2ellipsoids noisy 0.75%": ("torus_ellipsoids", 20012, dict(noise_frac=0.0075)),
    "superquadrics+plates": ("superquadrics_plates", 20020, {}),
    "ellipsoids+tori": ("ellipsoids_tori", 20030, {}),
    "sphere": ("sphere", 20040, dict(noise=0.0025)),
}
INITS = ["random", "pca", "gauss", "mlp"]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=50_000)
    ap.add_argument("--lams", default="0,4,10,50,100")
    ap.add_argument("--shapes", default=",".join(SHAPES))
    ap.add_argument("--inits", default=",".join(INITS))
    ap.add_argument("--max-iters", type=int, default=100)
    ap.add_argument("--out", default="ablation_init.json")
    args = ap.parse_args(argv)
    import torch

    from paper_2405_13839_amd import dwg, metrics, mlp_init, synth

    dev = torch.device("cuda", 0)
    mlp = mlp_init.load_params(os.path.join(os.path.dirname(__file__), "weights", "mlp_init.safetensors"), dev)
    rows = []
    for name in args.shapes.split(","):
        gen, seed, kw = SHAPES[name]
        c = getattr(synth, gen)(args.n, seed=seed, **kw)
        P, a = torch.from_numpy(c.P).to(dev), torch.from_numpy(c.area).to(dev)
        ws = dwg.workspace(c.n, c.n, dev, dwg.Params(lam=10.0))
        d = dwg.delta_anchor_mean(P, 10, 4096, 1.0, ws=ws)
        for kind in args.inits.split(","):
            if kind == "random":
                N0 = dwg.random_normals(c.n, seed + 7, dev)
            elif kind == "pca":
                N0 = dwg.pca_normals(P, ws=ws)
            elif kind == "gauss":
                N0 = dwg.gauss_normals(P)
            else:
                N0 = dwg.mlp_normals(P, mlp, ws=ws)
            r0 = metrics.orientation_report(N0.cpu().numpy(), c.N_true, c.comp)
            for lam in [float(x) for x in args.lams.split(",")]:
                N = N0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, stats = dwg.iterate(P, a, d, N, dwg.Params(lam=lam), max_iters=args.max_iters, ws=ws)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                r1 = metrics.orientation_report(N.cpu().numpy(), c.N_true, c.comp)
                row = dict(shape=name, n=c.n, init=kind, lam=lam, iters=int(stats.shape[0]),
                           converged=bool(st == dwg.DWG_OK), init_mae=round(r0["mae_deg"], 2),
                           mae=round(r1["mae_deg"], 2), agree=round(r1["agree"], 5), seconds=round(dt, 3))
                rows.append(row)
                print("[ablation]", json.dumps(row), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    json.dump(rows, open(args.out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
