"""The all-FP64 NFFT path (NFL_OPT_PRECISION 64).

Tab. fastsum_param: with the window cut-off m = 8 the NFFT is accurate to
about IEEE double precision.  So at m = 8 the FP64 path must reproduce the
exact trigonometric operator that Alg. nfft_fastsum approximates (Oracle B:
direct nonequispaced DFTs in FP64, the same coefficients b_l) to ~1e-12,
in d = 1, 2, 3; the FP32 path stops at ~1e-7.  Against the direct FP64 sums
(Oracle A) what remains is the kernel-approximation error of the chosen N,
and the eigenvalues from the FP64 operator match LAPACK far below the FP32
path's 1e-6 gate.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum, graph

pytestmark = pytest.mark.gpu


def tt(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("d,n,sigma,N", [(1, 900, 0.03, 64), (2, 2000, 0.05, 32),
                                         (3, 1500, 0.06, 16)])
def test_m8_matches_exact_trig_operator_to_double_precision(nfl, d, n, sigma, N):
    m = 8
    v = synth.gmm(n, d=d, k=3, seed=31)
    P = nfl.plan(tt(v), sigma, N=N, m=m, eps_B=0.0, precision=64)
    TG = fastsum.TrigGraph(v, sigma, N, 0.0, m)
    dg = P.degree64().cpu().numpy()
    rd = np.abs(dg - TG.d).max() / np.abs(TG.d).max()
    x = synth.normal_vectors(n, seed=3).astype(np.float64)
    y = P.apply_A64(tt(x)).cpu().numpy()
    ref = x - TG.apply_Ls(x)                      # A x = x - L_s x
    ra = np.abs(y - ref).max() / np.abs(ref).max()
    # the FP32 path on the same operator, for scale
    P32 = nfl.plan(tt(v), sigma, N=N, m=m, eps_B=0.0)
    y32 = P32.apply_A64(tt(x)).cpu().numpy()
    r32 = np.abs(y32 - ref).max() / np.abs(ref).max()
    print("d=%d m=8: FP64 path rel_inf(d) %.2e, rel_inf(A x) %.2e; FP32 path rel_inf(A x) %.2e"
          % (d, rd, ra, r32))
    assert rd <= 1e-12 and ra <= 1e-12, (rd, ra)
    assert r32 > 1e-10          # the FP32 path cannot get there
    P.close()
    P32.close()


def test_m6_fp64_path_against_direct_sums_and_fp32_path(nfl):
    """n = 2e5 moons-and-roll, sigma = 0.04, N = 64, m = 6: the FP64 path's
    error against the direct FP64 sums is the kernel approximation's alone
    (below the FP32 path's), and the two paths agree to FP32 rounding."""
    n, sigma = 200_000, 0.04
    v, _ = synth.moons_and_roll(n, seed=8)
    P64 = nfl.plan(tt(v), sigma, N=64, m=6, eps_B=0.0, precision=64)
    P32 = nfl.plan(tt(v), sigma, N=64, m=6, eps_B=0.0)
    x = synth.normal_vectors(n, seed=2).astype(np.float64)
    rows = np.sort(np.random.default_rng(4).choice(n, size=512, replace=False))
    d64 = P64.degree64().cpu().numpy()
    d32 = P32.degree64().cpu().numpy()
    dref = graph.degree(v, sigma, rows)
    # W x = D^{1/2} A D^{1/2} x from the FP64 A-product
    s64 = np.sqrt(d64)
    w64 = s64 * P64.apply_A64(tt(s64 * x)).cpu().numpy()
    s32 = np.sqrt(d32)
    w32 = s32 * P32.apply_A64(tt(s32 * x)).cpu().numpy()
    wref = graph.w_rows(v, sigma, x, rows)
    e64 = np.abs(w64[rows] - wref).max() / np.abs(wref).max()
    e32 = np.abs(w32[rows] - wref).max() / np.abs(wref).max()
    ed64 = np.abs(d64[rows] - dref).max() / dref.max()
    ed32 = np.abs(d32[rows] - dref).max() / dref.max()
    agree = np.abs(w64 - w32).max() / np.abs(w64).max()
    print("n=2e5 m=6: rel_inf W x FP64 %.2e FP32 %.2e; degrees FP64 %.2e FP32 %.2e; paths %.2e"
          % (e64, e32, ed64, ed32, agree))
    assert e64 <= 1e-9 and ed64 <= 1e-9
    assert e64 < e32 and ed64 < ed32
    assert agree <= 2e-6
    P64.close()
    P32.close()


def test_fp64_lanczos_and_cg_against_lapack(nfl):
    """n = 5000 two blobs, sigma = 0.05, eps_B = 1/16, N = 64, m = 8: the 10
    smallest eigenvalues of L_s from the FP64 path within 1e-12 of LAPACK on
    the dense FP64 matrix (the FP32 path: ~1e-7); CG for (I + 10 L_s) u = f
    within 1e-10 of LAPACK's solve."""
    v = synth.blobs2d(5000, seed=0)
    P = nfl.plan(tt(v), 0.05, N=64, m=8, eps_B=1.0 / 16, precision=64)
    r = P.lanczos_smallest(10, tol=1e-10, maxit=300, vectors=False)
    lam_ref, _ = graph.smallest_eigs_dense(v, 0.05, 10)
    err = np.abs(np.asarray(r["evals"]) - lam_ref)
    print("FP64 path: max |lambda - lambda*| = %.2e" % err.max())
    assert r["converged"] and err.max() <= 1e-12, err
    f = np.zeros(5000)
    f[::50], f[1::50] = 1.0, -1.0
    c = P.cg_solve(tt(f), tau=10.0, tol=1e-11, maxit=500)
    u_ref = np.linalg.solve(np.eye(5000) + 10.0 * graph.dense_Ls(v, 0.05), f)
    eu = np.abs(c["u"].cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
    print("FP64 path CG: iters %d, true relres %.2e, rel_inf(u - u*) %.2e"
          % (c["iters"], c["relres"], eu))
    assert c["converged"] and c["relres"] <= 2e-11 and eu <= 1e-10
    P.close()


def test_fp64_option_errors(nfl):
    v = synth.gmm(1000, d=3, seed=1)
    P = nfl.Plan(3)
    with pytest.raises(nfl.NFLError):
        P.set_option(nfl.OPT_PRECISION, 16)
    P.close()
    with pytest.raises(nfl.NFLError) as e:
        nfl.plan(tt(v), 0.05, N=32, m=4, eps_B=0.0, precision=64, kind="laplacian_rbf")
    assert e.value.code == nfl.NFL_ERR_UNSUPPORTED
