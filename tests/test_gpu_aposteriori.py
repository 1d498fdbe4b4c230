"""A-posteriori error of the HIP operator (Section 3.1) at n = 1000.

The fast summation is linear, so the library's product is W~_E = W + K(0) I + E
(the remark after the parameter table of Section 3).  Its columns are the
products with the n unit vectors, which gives, exactly up to the FP32 output
rounding:
* ||E||_inf = || sum_i |W~_E e_i - W e_i - K(0) e_i| ||_inf
  (eq. epsilon_norm_aposteriori) and eps = ||E||_inf / ||W||_inf,
* ||A - A_E||_inf = || sum_i |A e_i - A_E e_i| ||_inf, A_E the library's
  normalised operator (degrees d_E from the same operator, Alg.
  nfft_normalized_matvec step 4),
and these are checked against
* the Lemma on normalisation: ||A - A_E||_inf <= eps (1 + eta)/(eta (eta - eps)),
* Oracle B: the HIP E minus the exact trigonometric operator's error matrix is
  the NFFT's own (window + FP32) error, small next to E at N = 32,
* the library's estimates (nfl_error_estimate): eta from d_E within the
  Lemma's |d_E - d| <= ||E||_inf, the sampled ||K_ERR||_inf equal to the
  oracle's on the same sample points, and eps <= n ||K_ERR||_inf / ||W||_inf
  (eq. epsilon_KERR_estimate).
The configurations (N = 32) put eps near 6e-5, so that the kernel error
dominates the FP32 noise of the unit-vector products by orders of magnitude.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum, graph

pytestmark = pytest.mark.gpu

CASES = [
    ("blobs2d", lambda: synth.blobs2d(1000, seed=2), 0.05),
    ("gmm3d", lambda: synth.gmm(1000, d=3, k=3, std_lo=0.03, std_hi=0.06, seed=3), 0.05),
]


@pytest.mark.parametrize("name,gen,sigma", CASES, ids=[c[0] for c in CASES])
def test_aposteriori_error_of_the_gpu_operator(nfl, name, gen, sigma):
    import torch
    v = gen()
    n, d = v.shape
    N, m, eps_B = 32, 6, 0.0
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=N, m=m, eps_B=eps_B)
    I = torch.eye(n, dtype=torch.float32, device="cuda")
    WE = P.apply_W(I).double().cpu().numpy().T      # column i = W_E e_i
    AE = P.apply_A(I).double().cpu().numpy().T
    W = graph.dense_W(v, sigma)
    deg = W.sum(axis=1)
    Winf = deg.max()
    eta = deg.min() / Winf
    E = WE - W
    eps = np.abs(E).sum(axis=1).max() / Winf
    A = W / np.sqrt(np.outer(deg, deg))
    a_err = np.abs(A - AE).sum(axis=1).max()
    assert 0.0 < eps < eta, (eps, eta)
    bound = fastsum.lemma_bound(eps, eta)
    assert a_err <= bound, (a_err, bound)

    # Oracle B: the kernel-approximation error of the exact trigonometric
    # operator with the library's own scaled width
    info = P.info()
    st = info["sigma_tilde"]
    c, rho, vt = fastsum.scaling(v, eps_B)
    b = fastsum.coefficients(st, N, d, eps_B, m)
    EB = fastsum.trig_matrix(vt, b, N) - W - np.eye(n)
    epsB = np.abs(EB).sum(axis=1).max() / Winf
    nfft_part = np.abs(E - EB).sum(axis=1).max() / Winf
    assert nfft_part <= 0.05 * epsB, (nfft_part, epsB)
    assert abs(eps - epsB) <= nfft_part * (1 + 1e-9)

    # the library's estimates
    est = P.error_estimate(samples=20000, seed=1)
    lo, hi = (eta - eps) / (1 + eps), (eta + eps) / (1 - eps)
    assert lo * (1 - 1e-5) <= est["eta"] <= hi * (1 + 1e-5), (est["eta"], lo, hi)
    assert eps <= est["eps_est"], (eps, est["eps_est"])
    rng = np.random.default_rng(8)
    g = rng.normal(size=(4000, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = (0.5 - eps_B) * rng.uniform(0.0, 1.0, size=4000) ** (1.0 / d)
    y = g * r[:, None]
    kerr_oracle = float(np.abs(fastsum.gaussian(r, st) - fastsum.K_RF(y, b, N).real).max())
    kerr_lib = P.error_estimate(points=y)["kerr_inf"]
    assert abs(kerr_lib - kerr_oracle) <= 1e-12 + 1e-9 * kerr_oracle, (kerr_lib, kerr_oracle)
    P.close()
