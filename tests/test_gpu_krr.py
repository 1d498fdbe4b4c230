"""GPU parity of kernel ridge regression (Section 6.3): CG on
(K + beta I) alpha = f with FP32 NFFT products.

The oracle's reference system is the dense matrix M of the exact
trigonometric operator with the same kernel, parameter and regularisation
(M approximates K, diagonal included; what separates M from the library's
operator is the window, FFT and FP32 error).  Gates: the library's alpha
solves the oracle's system to a relative residual of 10 tol plus FP32
rounding of the products, 1e-7 || |M| |alpha| || / ||f|| (unit roundoff
times the absolute sums the products add up: large for the inverse
multiquadric, whose K(0) = 1/c), and its distance to alpha_M = (M + beta I)^{-1} f is within
||f - (M + beta I) alpha|| / lambda_min(M + beta I) (exact linear algebra, no
tolerance guessed).  The kernel-approximation error between M and the exact
Gram matrix is reported by the oracle's pins, not gated here.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum, krr

pytestmark = pytest.mark.gpu

CASES = [
    # cloud, kind, param, beta, N, m, eps_B
    ("blobs2d", "gaussian", 0.05, 0.1, 64, 6, 0.0),
    ("gmm3d", "inverse_multiquadric", 0.1, 1.0, 32, 6, 1 / 8),
    ("gmm3d", "gaussian", 0.05, 0.5, 32, 6, 0.0),
]


def _cloud(name):
    return synth.blobs2d(3000, seed=3) if name == "blobs2d" else synth.gmm(2000, d=3, k=4, seed=5)


@pytest.mark.parametrize("cloud,kind,c,beta,N,m,eps_B", CASES)
def test_krr_matches_oracle_system(nfl, cloud, kind, c, beta, N, m, eps_B):
    import torch
    v = _cloud(cloud)
    n = v.shape[0]
    f = np.sign(v[:, 0] + 1e-9).astype(np.float64)      # two-class labels
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=N, m=m, eps_B=eps_B, kind=kind)
    r = P.krr_solve(f, beta, tol=1e-6, maxit=5000)
    a = r["alpha"].cpu().numpy()
    # warm start from the solution: far fewer iterations
    r2 = P.krr_solve(f, beta, tol=1e-6, maxit=5000, alpha0=r["alpha"])
    # prediction at the training points: K alpha = W alpha + K(0) alpha
    K0 = 1.0 if kind == "gaussian" else 1.0 / c
    Wa = P.apply_W(torch.as_tensor(a.astype(np.float32), device="cuda")).cpu().numpy()
    P.close()
    T = fastsum.TrigGraph(v, c, N, eps_B, m, kind)
    M = T.scale * fastsum.trig_matrix(T.vt, T.bhat, N) + beta * np.eye(n)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    lam_min = ev[0]
    assert lam_min > 0
    gate = 10 * 1e-6 + 1e-7 * np.linalg.norm(np.abs(M) @ np.abs(a)) / np.linalg.norm(f)
    assert r["converged"] and r["relres"] <= gate, (r["iters"], r["relres"], gate)
    assert r2["iters"] <= max(2, r["iters"] // 4), (r["iters"], r2["iters"])
    res = f - M @ a
    assert np.linalg.norm(res) <= gate * np.linalg.norm(f)
    aM = np.linalg.solve(M, f)
    assert np.linalg.norm(a - aM) <= 1.01 * np.linalg.norm(res) / lam_min + 1e-12
    # K alpha = f - beta alpha, to the product's FP32 accuracy
    pred = Wa.astype(np.float64) + K0 * a
    assert np.abs(pred - (f - beta * a)).max() <= 1e-4 * np.abs(f).max()
    # the exact Gram system is solved to the kernel-approximation level
    aE = krr.solve(v, c, beta, f, kind)
    assert np.linalg.norm(a - aE) <= 0.05 * np.linalg.norm(aE)


def test_krr_argument_errors(nfl):
    import torch
    v = synth.blobs2d(500, seed=1)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.05, N=32, m=4)
    f = np.ones(500)
    with pytest.raises(nfl.NFLError):
        P.krr_solve(f, -1.0)
    with pytest.raises(nfl.NFLError):
        P.krr_solve(f, 1.0, tol=0.0)
    P.close()
