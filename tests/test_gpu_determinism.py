"""Run-to-run reproducibility of the products (the remark after
tab:fastsum_param: Alg. nfft_fastsum is a deterministic linear map, which the
error analysis of Section 3.1 writes as W~ + E).

With the default deterministic spread (int64 fixed-point accumulation of the
work items' padded tiles, NFL_OPT_DETERMINISTIC = 1) every product, the
degrees, and the Krylov solvers built on them (fixed-order reductions) give
bitwise identical results when run twice on the same input.  With FP32
atomic accumulation (option 0) the results differ from them only by
rounding.  Both paths agree with the FP64 direct oracle on sampled rows.
"""
import numpy as np
import pytest

import synth
from oracle import graph

pytestmark = pytest.mark.gpu


def tt(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("d,n,sigma,N,m", [(3, 300_000, 0.04, 64, 6), (3, 20_000, 0.08, 64, 4),
                                           (2, 20_000, 0.08, 64, 4), (1, 5_000, 0.08, 64, 4)])
def test_products_are_bitwise_reproducible(nfl, d, n, sigma, N, m):
    import torch
    if n > 100_000:
        v, _ = synth.moons_and_roll(n, seed=2)
    else:
        v = synth.gmm(n, d=d, k=4, seed=40 + d)
    x = tt(synth.normal_vectors(n, seed=9))
    outs = []
    for rep in range(2):
        P = nfl.plan(tt(v), sigma, N=N, m=m, eps_B=0.0)   # degrees recomputed per plan
        deg = P.degree()
        y1 = P.apply_Ls(x)
        y2 = P.apply_Ls(x)          # the same plan again (grid left clean by the first)
        w = P.apply_W(x)
        outs.append((deg, y1, y2, w))
        P.close()
    (d0, a0, b0, w0), (d1, a1, b1, w1) = outs
    assert torch.equal(d0, d1)
    assert torch.equal(a0, b0) and torch.equal(a0, a1) and torch.equal(b0, b1)
    assert torch.equal(w0, w1)
    # and against the oracle on sampled rows (both paths must stay accurate)
    rows = np.sort(np.random.default_rng(1).choice(n, size=min(n, 256), replace=False))
    ref = graph.w_rows(v, sigma, synth.normal_vectors(n, seed=9).astype(np.float64), rows)
    got = w0.cpu().numpy().astype(np.float64)[rows]
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def test_float_atomic_mode_differs_only_by_rounding(nfl):
    import torch
    n = 200_000
    v, _ = synth.moons_and_roll(n, seed=3)
    x = tt(synth.normal_vectors(n, seed=4))
    Pd = nfl.plan(tt(v), 0.04, N=64, m=6, eps_B=0.0)
    Pf = nfl.plan(tt(v), 0.04, N=64, m=6, eps_B=0.0, deterministic=0)
    yd, yf = Pd.apply_W(x), Pf.apply_W(x)
    rel = (yd - yf).abs().max().item() / yd.abs().max().item()
    print("deterministic vs float-atomic W x: rel diff %.3e" % rel)
    assert rel <= 2e-6
    # switching the option on an existing plan keeps the product valid
    Pf.set_option(nfl.OPT_DETERMINISTIC, 1)
    assert torch.equal(Pf.apply_W(x), yd)
    Pd.close()
    Pf.close()


def test_solvers_are_bitwise_reproducible(nfl):
    import torch
    n = 100_000
    v, lab = synth.moons_and_roll(n, seed=5)
    f = tt(synth.ssl_rhs(lab, 1, frac=0.02, seed=6))
    res = []
    for rep in range(2):
        P = nfl.plan(tt(v), 0.04, N=64, m=6, eps_B=0.0)
        cg = P.cg_solve(f, tau=10.0, tol=1e-6, maxit=200)
        lz = P.lanczos_smallest(6, tol=1e-6, maxit=200, block=4, vectors=False)
        res.append((cg, lz))
        P.close()
    (c0, l0), (c1, l1) = res
    assert c0["iters"] == c1["iters"] and torch.equal(c0["u"], c1["u"])
    assert c0["relres"] == c1["relres"]
    assert np.array_equal(np.asarray(l0["evals"]), np.asarray(l1["evals"]))
