"""GPU parity of the multiquadric and inverse multiquadric kernels (eq.
W_general, Alg. nfft_normalized_matvec).

The library's products are compared with the oracle's exact trigonometric
operator built from the same kernel, parameter and regularisation (what is
left is the window, FFT and FP32 error of the NFFT: gate 1e-5 relative, as for
the Gaussian), and with the direct dense sums in the original coordinates
within the kernel-approximation bound ||x||_1 ||K_ERR||_inf times the
homogeneity factor.  Lanczos on L_s is compared with LAPACK on the dense L_s,
within the Lemma of Section 3.1 (eigenvalues move by at most ||A - A_E||).
"""
import numpy as np
import pytest

import synth
from oracle import fastsum, graph

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


CASES = [
    # kind, c, N, m, eps_B
    ("multiquadric", 0.2, 32, 6, 1 / 8),
    ("inverse_multiquadric", 0.2, 32, 6, 1 / 8),
    ("inverse_multiquadric", 0.08, 64, 5, 1 / 8),
    ("multiquadric", 0.1, 64, 4, 1 / 16),
]


@pytest.mark.parametrize("kind,c,N,m,eps_B", CASES)
def test_other_kernels_match_trig_operator(nfl, kind, c, N, m, eps_B):
    import torch
    n = 1500
    v = synth.gmm(n, d=3, k=4, seed=21)
    x = synth.normal_vectors(n, seed=5)
    T = fastsum.TrigGraph(v, c, N, eps_B, m, kind)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=N, m=m, eps_B=eps_B, kind=kind)
    xd = torch.as_tensor(x, device="cuda")
    d = P.degree().cpu().numpy().astype(np.float64)
    Wx = P.apply_W(xd).cpu().numpy().astype(np.float64)
    Lx = P.apply_Ls(xd).cpu().numpy().astype(np.float64)
    info = P.info()
    P.close()
    x64 = x.astype(np.float64)
    assert _rel(d, T.d) <= 1e-5
    assert _rel(Wx, T.apply_W(x64)) <= 1e-5
    assert _rel(Lx, T.apply_Ls(x64)) <= 1e-5
    assert abs(info["dmin"] - T.d.min()) <= 1e-5 * T.d.max()
    # against the direct sums in the original coordinates
    W = graph.dense_W(v, c, kind)
    kerr = fastsum.kerr_sampled(T.bhat, N, T.sigma_t, eps_B, 3, samples=20000, kind=kind)
    bound = 2.0 * T.scale * kerr * np.abs(x64).sum() + 1e-5 * np.abs(W @ x64).max()
    assert np.abs(Wx - W @ x64).max() <= bound
    assert np.abs(d - W.sum(axis=1)).max() <= 2.0 * T.scale * kerr * n + 1e-5 * T.d.max()


@pytest.mark.parametrize("kind,c", [("inverse_multiquadric", 0.1), ("inverse_multiquadric", 0.05)])
def test_other_kernels_lanczos(nfl, kind, c):
    """The 6 smallest eigenvalues of L_s for a non-Gaussian W, against LAPACK
    on the dense matrix: |lambda - lambda*| <= Lemma bound + solver tolerance.
    (The multiquadric L_s of these clouds has a cluster of eigenvalues equal
    to 1e-5, which single-vector Lanczos is not meant to resolve.)"""
    import torch
    n, N, m, eps_B = 1200, 64, 6, 1 / 8
    v = synth.gmm(n, d=3, k=4, seed=23)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=N, m=m, eps_B=eps_B, kind=kind)
    r = P.lanczos_smallest(6, tol=1e-7, maxit=300)
    P.close()
    assert r["converged"]
    W = graph.dense_W(v, c, kind)
    ref = np.linalg.eigvalsh(graph.dense_Ls(v, c, kind))[:6]
    _, rho, _ = fastsum.scaling(v, eps_B)
    ct = fastsum.scaled_param(kind, c, rho)
    b = fastsum.coefficients(ct, N, 3, eps_B, m, kind)
    kerr = fastsum.kerr_sampled(b, N, ct, eps_B, 3, samples=20000, kind=kind)
    Wn = W.sum(axis=1).max()
    eps = 2.0 * fastsum.output_scale(kind, rho) * kerr * n / Wn
    eta = W.sum(axis=1).min() / Wn
    tol = fastsum.lemma_bound(eps, eta) + 1e-5
    assert tol < 1e-2
    np.testing.assert_allclose(r["evals"], ref, atol=tol)


LAPLACE_CASES = [
    # d, n, sigma, N, m, eps_B
    (3, 1500, 0.05, 64, 6, 1 / 8),
    (2, 2000, 0.04, 64, 5, 1 / 8),
]


def test_laplacian_near_field_items_longer_than_a_workgroup(nfl):
    """Near field of the Laplacian RBF kernel on a clustered 2-D cloud whose
    tiles hold up to ~2,800 nodes: work items of more than 256 targets run in
    full batches plus a partial last batch (shared among thread groups).
    Degrees, W x and L_s x against the oracle's exact trigonometric operator
    plus its dense near-field sum (1e-5)."""
    import torch
    n, d, s, N, m, eps_B = 12000, 2, 0.04, 64, 5, 1 / 8
    v = synth.gmm(n, d=d, k=4, seed=42)
    x = synth.normal_vectors(n, seed=7)
    T = fastsum.TrigGraph(v, s, N, eps_B, m, "laplacian_rbf", eps_I=m / N)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), s, N=N, m=m, eps_B=eps_B,
                 kind="laplacian_rbf")
    xd = torch.as_tensor(x, device="cuda")
    dg = P.degree().cpu().numpy().astype(np.float64)
    Wx = P.apply_W(xd).cpu().numpy().astype(np.float64)
    Lx = P.apply_Ls(xd).cpu().numpy().astype(np.float64)
    P.close()
    x64 = x.astype(np.float64)
    assert _rel(dg, T.d) <= 1e-5
    assert _rel(Wx, T.apply_W(x64)) <= 1e-5
    assert _rel(Lx, T.apply_Ls(x64)) <= 1e-5


@pytest.mark.parametrize("d,n,s,N,m,eps_B", LAPLACE_CASES)
def test_laplacian_rbf_with_near_field(nfl, d, n, s, N, m, eps_B):
    """Laplacian RBF kernel (eq. W_laplacian_rbf): the regularised kernel's
    products plus the near-field sum on r <= eps_I = p/N.  Against the oracle's
    exact trigonometric operator of the same regularised kernel plus its dense
    near-field sum (1e-5: window, FFT and FP32 error), and against the direct
    sums within ||x||_1 max|K_R - K_RF|."""
    import torch
    v = synth.gmm(n, d=d, k=4, seed=40 + d)
    x = synth.normal_vectors(n, seed=6)
    eps_I = m / N
    T = fastsum.TrigGraph(v, s, N, eps_B, m, "laplacian_rbf", eps_I=eps_I)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), s, N=N, m=m, eps_B=eps_B,
                 kind="laplacian_rbf")
    xd = torch.as_tensor(x, device="cuda")
    dg = P.degree().cpu().numpy().astype(np.float64)
    Wx = P.apply_W(xd).cpu().numpy().astype(np.float64)
    Lx = P.apply_Ls(xd).cpu().numpy().astype(np.float64)
    r = P.lanczos_smallest(4, tol=1e-7, maxit=200)
    with pytest.raises(nfl.NFLError):               # no near field between two node sets
        P.evaluate(xd, nfl.target_plan(torch.as_tensor(v[:10], device="cuda"), P))
    P.close()
    x64 = x.astype(np.float64)
    assert _rel(dg, T.d) <= 1e-5
    assert _rel(Wx, T.apply_W(x64)) <= 1e-5
    assert _rel(Lx, T.apply_Ls(x64)) <= 1e-5
    W = graph.dense_W(v, s, "laplacian_rbf")
    rng = np.random.default_rng(0)
    g = rng.normal(size=(20000, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    rr = (0.5 - eps_B) * rng.uniform(0.0, 1.0, size=20000) ** (1.0 / d)
    kerr = np.abs(T.reg(rr) - fastsum.K_RF(g * rr[:, None], T.bhat, N).real).max()
    assert np.abs(Wx - W @ x64).max() <= 2.0 * kerr * np.abs(x64).sum() + 1e-5 * np.abs(W @ x64).max()
    assert r["converged"]
    if d < 3:      # the Lemma bound is too loose at this N to say anything in 2-D
        return
    ref = np.linalg.eigvalsh(graph.dense_Ls(v, s, "laplacian_rbf"))[:4]
    Wn = W.sum(axis=1).max()
    tol = fastsum.lemma_bound(2.0 * kerr * n / Wn, W.sum(axis=1).min() / Wn) + 1e-5
    np.testing.assert_allclose(r["evals"], ref, atol=tol)
