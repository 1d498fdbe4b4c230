"""Train the CG warm-start network on the GPU.

The training pairs are the method's own solves: for resampled point clouds
of the semi-supervised workload (two crescents + Swiss roll, n nodes,
sigma = 0.04, N = 64, m = 6), one-vs-rest right-hand sides f with 2% labels,
and the solution u* of (I + tau L_s) u = f from CG to 1e-6.  Each solve is
followed by one Adam step on `nsample` randomly drawn nodes.  Forward,
backward and the optimiser are the library's BF16 matrix-core kernels.

    python -m paper_1808_04580_amd.train_warmstart --seeds 100 --draws 7 \\
        --out paper_1808_04580_amd/warmstart_moons_roll.bin

Training clouds use seeds 1..S; evaluation uses seeds from 100001 on.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_moons_roll.bin")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--seeds", type=int, default=100)
    ap.add_argument("--draws", type=int, default=7, help="label draws per class and cloud")
    ap.add_argument("--nsample", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tau", type=float, default=10.0)
    ap.add_argument("--sigma", type=float, default=0.04)
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--m", type=int, default=6)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1808_04580_amd as nfl
    import synth

    torch.cuda.set_device(0)
    net = nfl.WarmStart(n_classes=3, seed=0)
    total = args.seeds * args.draws * 3
    step = 0
    t0 = time.time()
    for s in range(1, args.seeds + 1):
        v, lab = synth.moons_and_roll(args.n, seed=s)
        P = nfl.plan(torch.as_tensor(v, device="cuda"), args.sigma, N=args.N, m=args.m)
        losses, iters = [], []
        for dr in range(args.draws):
            for c in range(3):
                f = synth.ssl_rhs(lab, c, frac=0.02, seed=1000 * s + 10 * dr + c)
                fd = torch.as_tensor(f, device="cuda")
                r = P.cg_solve(fd, tau=args.tau, tol=1e-6, maxit=500)
                iters.append(r["iters"])
                # cosine decay of the learning rate over all solves
                lr = args.lr * 0.5 * (1 + np.cos(np.pi * step / total))
                losses.append(net.train_step(P, fd, r["u"], c, args.nsample, step, lr))
                step += 1
        P.close()
        if s == 1 or s % 5 == 0 or s == args.seeds:
            print("seed %d/%d  solves %d  mean CG iters %.1f  loss %.4g  %.0fs" % (
                s, args.seeds, step, float(np.mean(iters)), float(np.mean(losses)),
                time.time() - t0), flush=True)
    net.save(args.out)
    print("saved", args.out, flush=True)


if __name__ == "__main__":
    main()
