"""GPU parity at the full sizes of the large workloads, in the launch
configuration the benchmark times.

At n = 1e6 and 1e7 the oracle cannot form the operator, so the checks are
(a) rows of W x and of the degree vector, each computed by the oracle's
direct FP64 sum one row at a time, and (b) properties that hold at any size:
L_s D^{1/2} 1 = 0, symmetry, the spectrum in [0, 2], eigen-residuals and
orthonormality of the returned vectors.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from oracle import graph

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "degree_moons_roll_n1000000_seed1_sigma0.04")


def golden_degree(v):
    """The exact FP64 degrees of the n = 1e6 cloud, written by
    tests/golden/make_degree_moons_roll_1m.py from the oracle's direct sums;
    refused if the generator's coordinates changed since."""
    meta = json.load(open(GOLDEN + ".json"))
    sha = hashlib.sha1(np.ascontiguousarray(v, dtype=np.float32).tobytes()).hexdigest()
    assert meta["coords_sha1"] == sha, "the cloud changed since the degrees were written"
    return np.load(GOLDEN + ".npy")


def _sampled_rows(P, v, sigma, x, rows):
    import torch
    yW = P.apply_W(torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)[rows]
    dg = P.degree().cpu().numpy().astype(np.float64)[rows]
    refW = graph.w_rows(v, sigma, x.astype(np.float64), rows)
    refd = graph.degree(v, sigma, rows)
    return (np.abs(dg - refd).max() / np.abs(refd).max(),
            np.abs(yW - refW).max() / np.abs(refW).max())


def test_moons_and_roll_1M_full_size(nfl):
    """n = 1e6 (two crescents + Swiss roll), sigma = 0.04, N = 64, m = 6,
    eps_B = 0: sampled rows of d and W x within 1e-5 of the direct oracle;
    the normalised operator's null vector and symmetry at full size."""
    import torch
    n, sigma = 1_000_000, 0.04
    v, _ = synth.moons_and_roll(n, seed=1)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=64, m=6, eps_B=0.0)
    x = synth.normal_vectors(n, seed=12345)
    rows = np.sort(np.random.default_rng(3).choice(n, size=256, replace=False))
    rd, rw = _sampled_rows(P, v, sigma, x, rows)
    assert rd <= 1e-5 and rw <= 1e-5, (rd, rw)
    # L_s D^{1/2} 1 = 0 for the approximate operator (its own degrees)
    d = P.degree().double()
    s = torch.sqrt(d).float()
    r = P.apply_Ls(s).double()
    assert (r.abs().max() / s.double().abs().max()).item() <= 1e-5
    # x^T L_s y = y^T L_s x
    y = torch.as_tensor(synth.normal_vectors(n, seed=777), device="cuda")
    xt = torch.as_tensor(x, device="cuda")
    a = torch.dot(xt.double(), P.apply_Ls(y).double()).item()
    b = torch.dot(y.double(), P.apply_Ls(xt).double()).item()
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b)) / 2 + 1e-3, (a, b)
    P.close()


def test_moons_and_roll_1M_Ls_rows_against_the_direct_oracle(nfl):
    """eq. nomlap at the benchmark's launch configuration (n = 1e6, sigma =
    0.04, N = 64, m = 6, eps_B = 0, tile 4, items of <= 512 nodes): L_s x of
    one product against (L_s x)_j = x_j - d_j^{-1/2} sum_{i != j} W_ji
    d_i^{-1/2} x_i on 4096 seeded rows, with the exact degree vector of all
    1e6 nodes (direct FP64 sums, cached); rel_inf <= 1e-5.  And the
    approximate degrees d_E against all 1e6 exact ones."""
    import torch
    n, sigma = 1_000_000, 0.04
    v, _ = synth.moons_and_roll(n, seed=1)
    dref = golden_degree(v)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=64, m=6, eps_B=0.0)
    dg = P.degree().double().cpu().numpy()
    rd = np.abs(dg - dref).max() / np.abs(dref).max()
    assert rd <= 1e-5, rd
    x = synth.normal_vectors(n, seed=12345)
    y = P.apply_Ls(torch.as_tensor(x, device="cuda")).double().cpu().numpy()
    rows = np.sort(np.random.default_rng(7).choice(n, size=4096, replace=False))
    ref = graph.Ls_rows(v, sigma, x.astype(np.float64), rows, dref)
    rel = np.abs(y[rows] - ref).max() / np.abs(ref).max()
    print("n = 1e6: rel_inf(d) %.3g over all nodes, rel_inf(L_s x) %.3g on 4096 rows" % (rd, rel))
    assert rel <= 1e-5, rel
    P.close()


def test_gmm_10M_block_lanczos(nfl):
    """n = 1e7 Gaussian mixture (10 components, std U[0.005, 0.03]),
    sigma = 0.02, N = 128 (grid 256^3), m = 6; block Lanczos (block 4) for the
    20 smallest eigenpairs of L_s with FP64 reorthogonalisation."""
    import torch
    n, sigma = 10_000_000, 0.02
    v = synth.gmm(n, d=3, k=10, seed=0)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=128, m=6, eps_B=0.0)
    x = synth.normal_vectors(n, seed=4)
    rows = np.sort(np.random.default_rng(9).choice(n, size=48, replace=False))
    rd, rw = _sampled_rows(P, v, sigma, x, rows)
    assert rd <= 1e-5 and rw <= 1e-5, (rd, rw)

    r = P.lanczos_smallest(20, tol=1e-6, maxit=400, block=4)
    assert r["converged"], (r["iters"], r["max_resid"])
    lam = r["evals"]
    assert np.all(np.diff(lam) >= -1e-12) and lam[0] >= -1e-6 and lam[-1] <= 2.0
    assert abs(lam[0]) <= 1e-6
    V = r["evecs"]                                     # (n, 20) FP64, caller order
    G = (V.T @ V).cpu().numpy()
    assert np.abs(G - np.eye(20)).max() <= 1e-8
    for i in range(20):
        vi = V[:, i].contiguous()
        Lv = P.apply_Ls(vi.float()).double()
        res = torch.linalg.vector_norm(Lv - lam[i] * vi).item()
        assert res <= 1e-5, (i, lam[i], res)
    P.close()
