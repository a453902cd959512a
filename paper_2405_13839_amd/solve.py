"""One orientation solve on a named synthetic workload, printed as one JSON line.

    python -m paper_2405_13839_amd.solve --config C5 --mode octree --anchors 16384
    python -m paper_2405_13839_amd.solve --config C3 --mode allpairs --init random --max-iters 50

Configs (synth.CONFIGS): C1 sphere 2K, C2 torus + 2 ellipsoids 100K, C3 the same at 1M, C4 8
superquadrics + 4 thin plates 5M, C5 10 ellipsoids + 10 tori 15M (`--n` overrides the size).
Kernel radius (`--radius`): `anchor` = mean distance to the 10 nearest of `--anchors` anchor
points (the scene's resolution parameter, like the paper's octree depth); `window` = the
paper's rule (Sec. 5.2): the mean of the 10-NN distances inside [0.0015, 0.015] x the longest
side of the bounding box (the paper's window in units of its models' size). Modes: `allpairs`
(exact sum), `octree` (Sec. 5.2 traversal, beta 2.3), `warm` (octree solves with the opening
factors `--warm-betas`, each from the last one's normals, until their convergence tests pass,
then the all-pairs solve from those normals until the all-pairs test passes: the exact
method's fixed point, reached mostly with octree iterations), `mc` (the paper's level-set update on a grid of `--depth`, Marching Cubes
unless `--surface tets`, octree evaluation). Timing covers the radius, the initial normals and
the iterations, with the points already on the GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="C3", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--seed", type=int, default=-1)
    ap.add_argument("--mode", default="octree", choices=["allpairs", "octree", "warm", "mc"])
    ap.add_argument("--warm-betas", default="2.3,8,32", help="opening factors of the octree stages of --mode warm")
    ap.add_argument("--init", default="mlp", choices=["mlp", "random", "pca", "gauss"])
    ap.add_argument("--anchors", type=int, default=4096)
    ap.add_argument("--lam", type=float, default=10.0)
    ap.add_argument("--max-iters", type=int, default=100)
    ap.add_argument("--depth", type=int, default=8)
    ap.add_argument("--radius", default="anchor", choices=["anchor", "window"])
    ap.add_argument("--surface", default="cubes", choices=["cubes", "tets"])
    ap.add_argument("--mc-k", type=int, default=10)
    args = ap.parse_args(argv)
    import torch

    from paper_2405_13839_amd import dwg, metrics, mlp_init, synth

    gen = {"C1": (synth.sphere, 2000, 100), "C2": (synth.torus_ellipsoids, 100_000, 101),
           "C3": (synth.torus_ellipsoids, 1_000_000, 102), "C4": (synth.superquadrics_plates, 5_000_000, 103),
           "C5": (synth.ellipsoids_tori, 15_000_000, 104)}[args.config]
    n = args.n or gen[1]
    seed = args.seed if args.seed >= 0 else gen[2]
    c = gen[0](n, seed=seed) if args.config != "C1" else synth.sphere(n, 0.005, seed)
    dev = torch.device("cuda", 0)
    P, area = torch.from_numpy(c.P).to(dev), torch.from_numpy(c.area).to(dev)
    warm_betas = [float(b) for b in args.warm_betas.split(",")]
    prm = dwg.Params(lam=args.lam, beta={"allpairs": 0.0, "warm": warm_betas[0]}.get(args.mode, 2.3))
    # one workspace for every stage of `warm`
    ws = dwg.workspace(c.n, c.n, dev, prm, dwg.Params(lam=args.lam), *(dwg.Params(lam=args.lam, beta=b) for b in warm_betas))
    mws = dwg.mc_workspace(P, prm, args.depth, 1, args.mc_k, surface=args.surface) if args.mode == "mc" else None
    side = float((P.max(dim=1).values - P.min(dim=1).values).max())
    mlp = None
    if args.init == "mlp":
        mlp = mlp_init.load_params(os.path.join(os.path.dirname(__file__), "weights", "mlp_init.safetensors"), dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.radius == "anchor":
        delta = dwg.delta_anchor_mean(P, 10, args.anchors, 1.0, ws=ws)
    else:
        delta = dwg.delta_knn_window(P, 10, 0.0015 * side, 0.015 * side, ws=ws)
    if args.init == "mlp":
        N = dwg.mlp_normals(P, mlp, ws=ws)
    elif args.init == "pca":
        N = dwg.pca_normals(P, ws=ws)
    elif args.init == "gauss":
        N = dwg.gauss_normals(P)
    else:
        N = dwg.random_normals(c.n, 7, dev)
    if args.mode == "mc":
        st, stats = dwg.iterate_mc(P, area, delta, N, prm, depth=args.depth, k=args.mc_k, max_iters=args.max_iters,
                                   ws=mws, surface=args.surface)
    else:
        st, stats = dwg.iterate(P, area, delta, N, prm, max_iters=args.max_iters, ws=ws)
    warm_iters = None
    if args.mode == "warm":
        warm_iters = [int(stats.shape[0])]
        for b in warm_betas[1:]:
            st, stats = dwg.iterate(P, area, delta, N, dwg.Params(lam=args.lam, beta=b), max_iters=args.max_iters, ws=ws)
            warm_iters.append(int(stats.shape[0]))
        st, stats = dwg.iterate(P, area, delta, N, dwg.Params(lam=args.lam), max_iters=args.max_iters, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rep = metrics.orientation_report(N.cpu().numpy(), c.N_true, c.comp)
    print(json.dumps({"config": args.config, "n": c.n, "mode": args.mode, "init": args.init, "anchors": args.anchors,
                      "radius": args.radius, "surface": args.surface if args.mode == "mc" else None,
                      "depth": args.depth if args.mode == "mc" else None, "lambda": args.lam, "converged": st == dwg.DWG_OK,
                      "octree_iterations": warm_iters, "iterations": int(stats.shape[0]),
                      "seconds": dt, "eval_ms_median": float(stats[:, 3].median()),
                      "median_delta": float(delta.median()), "mae_deg": rep["mae_deg"], "agree": rep["agree"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
