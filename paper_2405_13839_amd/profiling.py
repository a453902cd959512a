"""Small fixed workloads to run under rocprofv3 (kernel trace and PMC counters).

    python -m paper_2405_13839_amd.profiling gwn  --n 1000000 --lam 10 --reps 2
    python -m paper_2405_13839_amd.profiling tree --n 1000000 --lam 10 --reps 5
    python -m paper_2405_13839_amd.profiling treework --n 1000000 --lam 10
    python -m paper_2405_13839_amd.profiling mc   --n 1000000 --lam 10 --reps 5
    python -m paper_2405_13839_amd.profiling copy --mib 1024 --reps 3
    python -m paper_2405_13839_amd.profiling mlp  --n 1000000 --reps 3
    python -m paper_2405_13839_amd.profiling area --n 1000000 --reps 3

`gwn` launches the all-pairs kernel through dwg_gwn_grad on the C3 workload shape (anchor
radius: mean distance to 10 of 4096 anchors, random normals); `iterate` runs dwg_iterate
with fixed iterations on it; `tree` the same in octree mode (beta 2.3); `treework` prints
the octree traversal's work on it (dwg_octree_work: far dipoles, leaf pairs, wavefront
steps and the lane occupancy they imply); `mc` runs
dwg_iterate_mc (the level-set update, depth 8, octree evaluation) on it; `mlp` computes
the learned initial normals (anchor kNN, features, MLP inference) with the shipped weights;
`area` the tangent-plane Voronoi area weights (15 neighbours) and the windowed 10-NN radius;
`copy`
runs a plain device-to-device copy of a known size, used to calibrate the FETCH_SIZE /
WRITE_SIZE counters (bytes the counters report per byte actually moved).
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["gwn", "copy", "iterate", "tree", "treework", "mc", "mlp", "area"])
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--lam", type=float, default=10.0)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--mib", type=int, default=1024)
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    dev = torch.device("cuda", 0)
    if args.what == "copy":
        x = torch.ones(args.mib * 262144, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(args.reps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copied {args.mib} MiB x {args.reps}")
        return 0
    from paper_2405_13839_amd import dwg, synth

    c = synth.torus_ellipsoids(args.n, seed=102)
    P = torch.from_numpy(c.P).to(dev)
    a = torch.from_numpy(c.area).to(dev)
    prm = dwg.Params(lam=args.lam, beta=2.3 if args.what in ("tree", "treework", "mc") else 0.0)
    ws = dwg.workspace(c.n, c.n, dev, prm)
    d = dwg.delta_anchor_mean(P, 10, 4096, 1.0, ws=ws)  # the benchmark's kernel radius
    N = dwg.random_normals(c.n, 202, dev)
    if args.what == "mlp":
        import os

        from paper_2405_13839_amd import mlp_init

        mlp = mlp_init.load_params(os.path.join(os.path.dirname(__file__), "weights", "mlp_init.safetensors"), dev)
        for _ in range(args.reps):
            dwg.mlp_normals(P, mlp, ws=ws)
        torch.cuda.synchronize()
    elif args.what == "area":
        for _ in range(args.reps):
            dwg.voronoi_area(P, 15, ws=ws)
            dwg.delta_knn_window(P, 10, ws=ws)
        torch.cuda.synchronize()
    elif args.what == "gwn":
        for _ in range(args.reps):
            dwg.gwn(P, N, a, d, P, prm, ws=ws)
        torch.cuda.synchronize()
    elif args.what == "treework":
        wk = dwg.octree_work(P, a, d, P, prm, ws=ws)
        print(f"far dipoles {wk.far} ({wk.far / c.n:.1f} per query), leaf pairs {wk.pairs} "
              f"({wk.pairs / c.n:.1f} per query); wavefront far steps {wk.far_steps}, leaf iterations "
              f"{wk.leaf_steps}; lane occupancy: far steps {wk.far_lanes:.3f}, leaf loops {wk.leaf_lanes:.3f}")
    elif args.what == "mc":
        del ws
        st, stats = dwg.iterate_mc(P, a, d, N, prm, depth=8, dilate=1, k=10, max_iters=args.reps, fixed_iters=True)
        print("evaluation ms per iteration:", np.round(stats[:, 3].numpy(), 3).tolist())
    else:  # iterate / tree
        st, stats = dwg.iterate(P, a, d, N, prm, max_iters=args.reps, fixed_iters=True, ws=ws)
        print("kernel ms per iteration:", np.round(stats[:, 3].numpy(), 3).tolist())
    print(f"{args.what}: n={c.n} lam={args.lam} reps={args.reps} done")
    return 0


if __name__ == "__main__":
    sys.exit(main())
