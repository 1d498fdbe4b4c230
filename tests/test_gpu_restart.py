"""GPU tests of thick-restart (block) Lanczos (NFL_OPT_RESTARTS).

The restarted solver runs on the same FP32 NFFT operator as the plain one,
so the two must agree to the solver tolerance; both are compared with LAPACK
on the dense L_s of the oracle (Section 2) within the fast-summation error.
"""
import numpy as np
import pytest

import synth
from oracle import graph

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("block,basis", [(1, 40), (2, 40), (4, 48)])
def test_thick_restart_matches_plain_lanczos_and_lapack(nfl, block, basis):
    import torch
    n, sigma, k = 3000, 0.03, 12
    v = synth.gmm(n, d=3, k=6, seed=3)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=64, m=6)
    plain = P.lanczos_smallest(k, tol=1e-8, maxit=300, block=block)
    rs = P.lanczos_smallest(k, tol=1e-8, maxit=basis, block=block, restarts=60)
    assert plain["converged"] and rs["converged"], (plain["iters"], rs["iters"])
    # each Ritz value lies within its residual (<= tol) of an eigenvalue of the
    # operator, so two converged runs differ by at most 2 tol (plus the FP32
    # operator's slight asymmetry)
    np.testing.assert_allclose(rs["evals"], plain["evals"], atol=3e-8)
    V = rs["evecs"]
    G = (V.T @ V).cpu().numpy()
    assert np.abs(G - np.eye(k)).max() <= 1e-8
    for i in range(k):
        vi = V[:, i].contiguous()
        r = P.apply_Ls(vi.float()).double() - rs["evals"][i] * vi
        assert torch.linalg.vector_norm(r).item() <= 1e-5, i
    # a basis too small for k + 2 blocks is refused
    with pytest.raises(nfl.NFLError):
        P.lanczos_smallest(k, tol=1e-8, maxit=k + block, block=block, restarts=5)
    P.close()
    ref = np.linalg.eigvalsh(graph.dense_Ls(v, sigma))[:k]
    np.testing.assert_allclose(rs["evals"], ref, atol=1e-6)
