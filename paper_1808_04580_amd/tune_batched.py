"""Tune the NFFT parameters of the batched workload and write the cache.

The workload: 64 independent Gaussian-mixture clouds in d = 3 (3..8
components, std U[0.01, 0.05]), n log-uniform in [1e3, 2e5], sigma per graph
U[0.03, 0.15] (seed 0).  Each graph is tuned with nfl_autotune to relative
error 1e-5 on 256 sampled rows; results are merged into the text cache keyed
by (d, size class, sigma band, target), which later runs verify per graph.

    python -m paper_1808_04580_amd.tune_batched [--out PATH] [--graphs 64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.txt")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--graphs", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--target", type=float, default=1e-5)
    ap.add_argument("--rows", type=int, default=256)
    ap.add_argument("--fresh", action="store_true", help="start from an empty cache")
    args = ap.parse_args()

    import torch

    import paper_1808_04580_amd as nfl
    import synth

    torch.cuda.set_device(0)
    if args.fresh and os.path.exists(args.out):
        os.remove(args.out)
    t0 = time.time()
    for g, (v, sigma) in enumerate(synth.batched_clouds(args.graphs, seed=args.seed)):
        P = nfl.Plan(3)
        P.set_points(torch.as_tensor(v, device="cuda"))
        r = P.autotune(sigma, target=args.target, rows=args.rows, seed=g + 1, cache=args.out)
        r.update(graph=g, n=len(v), sigma=round(sigma, 6))
        print(json.dumps(r), flush=True)
        P.close()
    print("tuned %d graphs in %.1fs -> %s" % (args.graphs, time.time() - t0, args.out), flush=True)


if __name__ == "__main__":
    main()
