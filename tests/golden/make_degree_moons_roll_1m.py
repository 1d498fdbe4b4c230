"""Writes the exact FP64 degree vector of the n = 1e6 moons-and-roll cloud
(seed 1, sigma = 0.04) that the L_s parity test at full size and the
benchmark's accuracy block compare against.

Calls only the oracle's direct sums (Section 2: d_j = sum_{i != j} W_ji with
the Gaussian weight of eq. W_gaussian), O(n^2) = 1e12 pair terms: about
4-10 minutes on 8-16 host threads.  Writes
    degree_moons_roll_n1000000_seed1_sigma0.04.npy   (float64, n)
    degree_moons_roll_n1000000_seed1_sigma0.04.json  (n, seed, sigma, SHA-1 of
                                                      the float32 coordinates)
next to this script.  Run:  python tests/golden/make_degree_moons_roll_1m.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import graph, lib  # noqa: E402

N, SEED, SIGMA = 1_000_000, 1, 0.04
STEM = os.path.join(HERE, "degree_moons_roll_n%d_seed%d_sigma%g" % (N, SEED, SIGMA))


def main():
    v, _ = synth.moons_and_roll(N, seed=SEED)
    v = np.ascontiguousarray(v, dtype=np.float32)
    sha = hashlib.sha1(v.tobytes()).hexdigest()
    t0 = time.time()
    d = graph.degree(v, SIGMA)
    dt = time.time() - t0
    np.save(STEM + ".npy", d)
    with open(STEM + ".json", "w") as f:
        json.dump({"n": N, "seed": SEED, "sigma": SIGMA, "coords_sha1": sha,
                   "generator": "synth.moons_and_roll", "oracle": "oracle.graph.degree",
                   "threads": int(lib().oracle_num_threads()), "seconds": round(dt, 1)},
                  f, indent=1)
        f.write("\n")
    print("wrote %s.npy (%d degrees, min %.6g max %.6g) in %.0f s"
          % (STEM, d.size, d.min(), d.max(), dt))


if __name__ == "__main__":
    main()
