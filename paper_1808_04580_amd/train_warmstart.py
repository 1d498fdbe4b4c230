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

Loss "mse": mean squared error of u against u*.  Loss "energy": the energy
norm e^T (I + tau L_s) e of the warm-start error e = u - u*, the quantity CG
from u0 = u actually feels; its gradient with respect to the output at node i
is 2 ((I + tau L_s) e)_i, which the mean-squared-error training step receives
through the pseudo-target u_i - ((I + tau L_s) e)_i (one extra L_s product
per step).
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
    ap.add_argument("--loss", choices=["mse", "energy"], default="mse")
    ap.add_argument("--init", default=None, help="start from these weights")
    ap.add_argument("--first-seed", type=int, default=1)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1808_04580_amd as nfl
    import synth

    torch.cuda.set_device(0)
    net = nfl.WarmStart(n_classes=3, seed=0)
    if args.init:
        net.load(args.init)
    total = args.seeds * args.draws * 3
    step = 0
    t0 = time.time()
    for s in range(args.first_seed, args.first_seed + args.seeds):
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
                target = r["u"]
                if args.loss == "energy":
                    u = net.predict(P, fd, c)
                    e = (u - r["u"]).float()
                    Me = e.double() + args.tau * P.apply_Ls(e).double()
                    target = u - Me
                losses.append(net.train_step(P, fd, target, c, args.nsample, step, lr))
                step += 1
        P.close()
        k = s - args.first_seed + 1
        if k == 1 or k % 5 == 0 or k == args.seeds:
            print("seed %d/%d  solves %d  mean CG iters %.1f  loss %.4g  %.0fs" % (
                k, args.seeds, step, float(np.mean(iters)), float(np.mean(losses)),
                time.time() - t0), flush=True)
    net.save(args.out)
    print("saved", args.out, flush=True)


if __name__ == "__main__":
    main()
