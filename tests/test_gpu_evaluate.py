"""GPU parity of the fast summation at target nodes distinct from the
sources (nfl_set_points_frame + nfl_evaluate) and of the kernel ridge
regression prediction F(t) = sum_i alpha_i K(t - v_i) (Section 6.3).

The library's sums are compared with the oracle's exact trigonometric
operator with targets (same kernel, parameter and regularisation; gate 1e-5
relative: the window, FFT and FP32 error) and with the direct cross sums
within ||x||_1 ||K_ERR||_inf times the homogeneity factor.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum, krr

pytestmark = pytest.mark.gpu


def _targets(v, n_t, seed, shrink=0.95):
    """n_t points uniform in the ball of the sources around their centre."""
    V = v.astype(np.float64)
    c = 0.5 * (V.min(axis=0) + V.max(axis=0))
    R = np.sqrt(((V - c) ** 2).sum(axis=1)).max()
    u = synth.uniform_ball(n_t, d=v.shape[1], seed=seed).astype(np.float64)
    u /= np.sqrt((u * u).sum(axis=1)).max()
    return (c + shrink * R * u).astype(np.float32)


CASES = [
    # d, kind, param, N, m, eps_B, n_src, n_tgt
    (3, "gaussian", 0.05, 32, 6, 0.0, 2000, 777),
    (3, "inverse_multiquadric", 0.1, 32, 6, 1 / 8, 1500, 513),
    (2, "gaussian", 0.05, 64, 5, 1 / 16, 3000, 1001),
    (1, "gaussian", 0.03, 128, 4, 0.0, 900, 333),
]


@pytest.mark.parametrize("d,kind,c,N,m,eps_B,n,nt", CASES)
def test_evaluate_matches_oracle(nfl, d, kind, c, N, m, eps_B, n, nt):
    import torch
    v = synth.gmm(n, d=d, k=4, seed=30 + d)
    t = _targets(v, nt, seed=7)
    x = synth.normal_vectors(n, seed=8)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=N, m=m, eps_B=eps_B, kind=kind)
    T = nfl.target_plan(torch.as_tensor(t, device="cuda"), P)
    y = P.evaluate(torch.as_tensor(x, device="cuda"), T).cpu().numpy().astype(np.float64)
    yself = P.evaluate(torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    Wx = P.apply_W(torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    T.close()
    P.close()
    x64 = x.astype(np.float64)
    K0 = 1.0 if kind == "gaussian" else 1.0 / c
    # at the sources themselves: W x + K(0) x
    assert np.abs(yself - (Wx + K0 * x64)).max() <= 1e-5 * np.abs(yself).max()
    # against the exact trigonometric operator with targets
    c0, rho, vs = fastsum.scaling(v, eps_B)
    vt = (t.astype(np.float64) - c0) * rho
    ct = fastsum.scaled_param(kind, c, rho)
    b = fastsum.coefficients(ct, N, d, eps_B, m, kind)
    ref = fastsum.output_scale(kind, rho) * fastsum.trig_operator(vs, x64, b, N, targets=vt)
    assert np.abs(y - ref).max() <= 1e-5 * np.abs(ref).max()
    # against the direct cross sums in the original coordinates
    direct = krr.predict(v, x64, t, c, kind)
    kerr = fastsum.kerr_sampled(b, N, ct, eps_B, d, samples=20000, kind=kind)
    bound = 2.0 * fastsum.output_scale(kind, rho) * kerr * np.abs(x64).sum()
    assert np.abs(y - direct).max() <= bound + 1e-5 * np.abs(direct).max()


def test_krr_prediction_at_new_points(nfl):
    """Train on 2-D two-class data (Gaussian kernel), predict at new points:
    the library's prediction with its own alpha matches the direct sum with
    that alpha, and the predicted classes agree with the oracle's dense solve."""
    import torch
    v = synth.blobs2d(3000, seed=3)
    f = np.sign(v[:, 0] + 1e-9).astype(np.float64)
    c, beta = 0.05, 0.1
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=64, m=6)
    r = P.krr_solve(f, beta, tol=1e-8, maxit=5000)
    assert r["converged"]
    t = _targets(v, 1200, seed=9, shrink=0.9)
    T = nfl.target_plan(torch.as_tensor(t, device="cuda"), P)
    F = P.krr_predict(r["alpha"], T).cpu().numpy().astype(np.float64)
    T.close()
    P.close()
    a = r["alpha"].cpu().numpy()
    ref = krr.predict(v, a.astype(np.float32).astype(np.float64), t, c)
    assert np.abs(F - ref).max() <= 1e-5 * np.abs(a).sum()
    Fo = krr.predict(v, krr.solve(v, c, beta, f), t, c)
    sure = np.abs(Fo) > 1e-2
    assert np.mean(np.sign(F[sure]) == np.sign(Fo[sure])) >= 0.999


def test_target_plan_errors(nfl):
    import torch
    v = synth.gmm(800, d=3, k=3, seed=5)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.05, N=32, m=4)
    far = _targets(v, 50, seed=2, shrink=1.5)          # outside the sources' ball
    with pytest.raises(nfl.NFLError):
        nfl.target_plan(torch.as_tensor(far, device="cuda"), P)
    T = nfl.target_plan(torch.as_tensor(_targets(v, 50, seed=2), device="cuda"), P)
    with pytest.raises(nfl.NFLError):                    # a target plan has no degrees
        T.apply_Ls(torch.zeros(50, device="cuda"))
    with pytest.raises(nfl.NFLError):
        T.lanczos_smallest(2, maxit=10)
    # a target plan with other kernel parameters is refused
    T.set_kernel(0.06, 32, 4, 0.0)
    with pytest.raises(nfl.NFLError):
        P.evaluate(torch.zeros(800, device="cuda"), T)
    T.close()
    P.close()


def test_products_around_full_transform_passes(nfl):
    """A plan's own products run the d = 3 FFT passes on the z-lines its
    nodes' windows touch only, keeping the rest of the spectrum zero; an
    evaluation at other targets and a convolution of a caller's grid run the
    full passes.  On a clustered cloud whose support leaves most lines out,
    with targets spread over the whole ball: the targets' sums match the
    exact trigonometric operator (1e-5), and L_s x before, between and after
    the full passes is bitwise the same (deterministic spread)."""
    import torch
    d, c, N, m, eps_B, n = 3, 0.05, 32, 6, 0.0, 3000
    v = synth.gmm(n, d=d, k=4, seed=61)
    t = _targets(v, 700, seed=9)
    x = synth.normal_vectors(n, seed=10)
    xd = torch.as_tensor(x, device="cuda")
    P = nfl.plan(torch.as_tensor(v, device="cuda"), c, N=N, m=m, eps_B=eps_B)
    y1 = P.apply_Ls(xd).cpu().numpy()
    T = nfl.target_plan(torch.as_tensor(t, device="cuda"), P)
    yt = P.evaluate(xd, T).cpu().numpy().astype(np.float64)
    y2 = P.apply_Ls(xd).cpu().numpy()
    g = P.convolve(P.spread(xd))
    y3 = P.apply_Ls(xd).cpu().numpy()
    f = P.interp(g).cpu().numpy().astype(np.float64)
    T.close()
    P.close()
    np.testing.assert_array_equal(y1, y2)
    np.testing.assert_array_equal(y1, y3)
    x64 = x.astype(np.float64)
    c0, rho, vs = fastsum.scaling(v, eps_B)
    vt = (t.astype(np.float64) - c0) * rho
    b = fastsum.coefficients(c * rho, N, d, eps_B, m, "gaussian")
    ref = fastsum.trig_operator(vs, x64, b, N, targets=vt)
    assert np.abs(yt - ref).max() <= 1e-5 * np.abs(ref).max()
    # the step-by-step product at the sources: the trigonometric sum itself
    refs = fastsum.trig_operator(vs, x64, b, N)
    assert np.abs(f - refs).max() <= 1e-5 * np.abs(refs).max()
