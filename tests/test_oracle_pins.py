"""Pins of the oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each check is a closed form,
brute force on a tiny input, an identity of Section 2, a special case that
reduces to a numpy/LAPACK routine, or the Lemma of Section 3.1.
"""
import math

import numpy as np
import pytest

from oracle import fastsum, graph, krr, krylov, nystrom
import synth


# ---- Oracle A: the graph of Section 2 ----------------------------------------

def test_closed_form_three_points():
    """Three points at distances sigma, 2 sigma, sqrt(5) sigma: W = e^-1, e^-4, e^-5
    (eq. W_gaussian), zero diagonal; degrees are row sums (Section 2)."""
    s = 0.05
    v = np.array([[0.0, 0.0], [s, 0.0], [0.0, 2 * s]])
    e1, e4, e5 = math.exp(-1), math.exp(-4), math.exp(-5)
    Wref = np.array([[0, e1, e4], [e1, 0, e5], [e4, e5, 0]])
    x = np.array([1.0, -2.0, 0.5])
    np.testing.assert_allclose(graph.apply_W(v, s, x), Wref @ x, rtol=1e-14)
    np.testing.assert_allclose(graph.degree(v, s), Wref.sum(axis=1), rtol=1e-14)
    np.testing.assert_allclose(graph.dense_W(v, s), Wref, rtol=1e-14)


def test_duplicates_and_diagonal():
    """Only the diagonal is zero: duplicate points j != i have weight exp(0) = 1."""
    v = np.array([[0.1, 0.2, 0.0], [0.1, 0.2, 0.0], [0.5, 0.5, 0.5]])
    W = graph.dense_W(v, 0.01)
    assert W[0, 1] == 1.0 and W[0, 0] == 0.0 and W[1, 1] == 0.0
    np.testing.assert_allclose(graph.degree(v, 0.01)[:2], [1.0, 1.0], atol=1e-300)


def test_direct_sums_match_dense_matrix():
    """The C loops and the explicitly formed matrix are two independent paths."""
    v = synth.gmm(57, d=3, k=3, seed=4)
    x = synth.normal_vectors(57, nvec=3, seed=1).astype(np.float64)
    W = graph.dense_W(v, 0.07)
    np.testing.assert_allclose(graph.apply_W(v, 0.07, x), x @ W.T, rtol=1e-13, atol=1e-13)
    rows = np.array([0, 13, 56])
    np.testing.assert_allclose(graph.w_rows(v, 0.07, x, rows), (x @ W.T)[:, rows], rtol=1e-13, atol=1e-13)


def test_laplacian_identities():
    """u^T L u = 1/2 sum W_ji (u_j - u_i)^2, L 1 = 0 (Section 2), L_s D^{1/2} 1 = 0,
    symmetry of L_s (eq. nomlap), spec(L_s) in [0, 2] with smallest eigenvalue 0."""
    v = synth.gmm(40, d=2, k=2, seed=2)
    s = 0.06
    rng = np.random.default_rng(0)
    u, y = rng.standard_normal(40), rng.standard_normal(40)
    quad = 0.0
    for j in range(40):                       # brute force double loop
        for i in range(40):
            if i != j:
                dist2 = float(((v[j].astype(np.float64) - v[i]) ** 2).sum())
                quad += math.exp(-dist2 / s**2) * (u[j] - u[i]) ** 2
    assert abs(u @ graph.apply_L(v, s, u) - 0.5 * quad) <= 1e-12 * abs(quad)
    np.testing.assert_allclose(graph.apply_L(v, s, np.ones(40)), 0.0, atol=1e-12)
    d = graph.degree(v, s)
    np.testing.assert_allclose(graph.apply_Ls(v, s, np.sqrt(d)), 0.0, atol=1e-12)
    assert abs(y @ graph.apply_Ls(v, s, u) - u @ graph.apply_Ls(v, s, y)) < 1e-12
    lam = np.linalg.eigvalsh(graph.dense_Ls(v, s))
    assert lam[0] > -1e-12 and lam[-1] < 2 + 1e-12 and abs(lam[0]) < 1e-12


# ---- the regularised kernel and its coefficients (Section 3) ----------------

def test_gaussian_derivatives_against_finite_differences():
    """Radial derivatives of the Gaussian against central differences of the
    next-lower derivative (step 1e-5, truncation error ~ (h/sigma)^2)."""
    s, r0, p = 0.07, 0.06, 6
    D = fastsum.gaussian_radial_derivs(r0, s, p)
    h = 1e-5
    assert abs(D[0] - math.exp(-(r0 / s) ** 2)) < 1e-16
    for k in range(1, p):
        lo = fastsum.gaussian_radial_derivs(r0 - h, s, k)[k - 1]
        hi = fastsum.gaussian_radial_derivs(r0 + h, s, k)[k - 1]
        fd = (hi - lo) / (2 * h)
        assert abs(D[k] - fd) <= 1e-6 * max(abs(D[k]), abs(D[k - 1]) / s), k


@pytest.mark.parametrize("p", [2, 4, 6])
def test_two_point_taylor_conditions(p):
    """T_B matches K and p-1 derivatives at 1/2 - eps_B; value K(1/2) and zero
    derivatives at 1/2 (so the constant continuation is C^{p-1})."""
    s, eps = 0.25, 1.0 / 8
    K = fastsum.RegKernel(s, eps, p)
    poly = np.polynomial.Polynomial(K.coef)
    h = 0.5 - K.r0
    A = fastsum.gaussian_radial_derivs(K.r0, s, p)
    for k in range(p):
        dk = poly.deriv(k) if k else poly
        # rounding scale of the k-th derivative at t = 1
        scale = sum(abs(c) * q**k for q, c in enumerate(K.coef)) / h**k
        assert abs(dk(0.0) / h**k - A[k]) <= 1e-12 * scale + 1e-14
        want = math.exp(-(0.5 / s) ** 2) if k == 0 else 0.0
        assert abs(dk(1.0) / h**k - want) <= 1e-12 * scale + 1e-14
    # K_R continuous across both junctions
    r = np.array([K.r0 - 1e-12, K.r0 + 1e-12, 0.5 - 1e-12, 0.5 + 1e-12])
    vals = K(r)
    assert abs(vals[0] - vals[1]) < 1e-9 and abs(vals[2] - vals[3]) < 1e-9


@pytest.mark.parametrize("d,N,eps", [(1, 16, 0.0), (2, 16, 1.0 / 8), (3, 8, 1.0 / 4)])
def test_coefficients_interpolate_samples(d, N, eps):
    """With the N^{-d} normalisation, K_RF(j/N) = K_R(j/N) on all nodes of I_N^d
    (the defining property of the trapezoidal coefficients, eq. b_l::K_RF)."""
    s = 0.2
    b = fastsum.coefficients(s, N, d, eps, 3)
    j = fastsum.index_set(N)
    nodes = np.stack(np.meshgrid(*([j / N] * d), indexing="ij"), axis=-1).reshape(-1, d)
    K = fastsum.RegKernel(s, eps, 3)
    got = fastsum.K_RF(nodes, b, N)
    np.testing.assert_allclose(got.real, K(np.linalg.norm(nodes, axis=1)), atol=1e-13)
    assert np.abs(got.imag).max() < 1e-13


def test_coefficients_closed_form_small_sigma():
    """For a narrow Gaussian the regularisation is inert and the trapezoidal
    coefficients are, by Poisson summation, sum_r c(l + rN) with the
    continuous transform c(xi) = (sqrt(pi) sigma)^d exp(-pi^2 sigma^2 |xi|^2)
    (the analytic coefficients Section 3 mentions for small sigma)."""
    s, N, d = 0.05, 32, 2
    b = fastsum.coefficients(s, N, d, 0.0, 4)
    l = fastsum.index_set(N)
    L1, L2 = np.meshgrid(l, l, indexing="ij")
    ref = np.zeros_like(b)
    for r1 in range(-3, 4):
        for r2 in range(-3, 4):
            xi2 = (L1 + r1 * N) ** 2 + (L2 + r2 * N) ** 2
            ref += (math.sqrt(math.pi) * s) ** d * np.exp(-(math.pi * s) ** 2 * xi2)
    np.testing.assert_allclose(b, ref, atol=1e-15)


@pytest.mark.parametrize("kind", ["multiquadric", "inverse_multiquadric"])
def test_power_kernel_derivatives(kind):
    """Radial derivatives of (r^2 + c^2)^alpha: the first two against the
    textbook closed forms, all against central differences of the next-lower
    one (step 1e-5, truncation ~ (h/c)^2)."""
    c, r0, p = 0.3, 0.37, 7
    D = fastsum.radial_derivs(kind, r0, c, p)
    u = r0 * r0 + c * c
    if kind == "multiquadric":
        closed = [math.sqrt(u), r0 / math.sqrt(u), c * c / u ** 1.5]
    else:
        closed = [u ** -0.5, -r0 * u ** -1.5, (2 * r0 * r0 - c * c) * u ** -2.5]
    for k in range(3):
        assert abs(D[k] - closed[k]) <= 1e-14 * max(1.0, abs(closed[k])), k
    h = 1e-5
    for k in range(1, p):
        lo = fastsum.radial_derivs(kind, r0 - h, c, k)[k - 1]
        hi = fastsum.radial_derivs(kind, r0 + h, c, k)[k - 1]
        fd = (hi - lo) / (2 * h)
        assert abs(D[k] - fd) <= 1e-6 * max(abs(D[k]), abs(D[k - 1]) / c), k


@pytest.mark.parametrize("kind,p", [("multiquadric", 4), ("inverse_multiquadric", 6)])
def test_two_point_taylor_conditions_other_kernels(kind, p):
    """The regularisation of the other kernels meets the same Hermite
    conditions: K and p-1 derivatives at 1/2 - eps_B, K(1/2) and flat at 1/2."""
    c, eps = 0.15, 1.0 / 8
    K = fastsum.RegKernel(c, eps, p, kind)
    poly = np.polynomial.Polynomial(K.coef)
    h = 0.5 - K.r0
    A = fastsum.radial_derivs(kind, K.r0, c, p)
    want_half = float(fastsum.radial_kernel(kind, c)(0.5))
    for k in range(p):
        dk = poly.deriv(k) if k else poly
        scale = sum(abs(cf) * q**k for q, cf in enumerate(K.coef)) / h**k
        assert abs(dk(0.0) / h**k - A[k]) <= 1e-12 * scale + 1e-14
        assert abs(dk(1.0) / h**k - (want_half if k == 0 else 0.0)) <= 1e-12 * scale + 1e-14


@pytest.mark.parametrize("kind", ["multiquadric", "inverse_multiquadric"])
def test_coefficients_interpolate_samples_other_kernels(kind):
    """K_RF(j/N) = K_R(j/N) on I_N^d for the other kernels too."""
    d, N, eps, c = 2, 16, 1.0 / 8, 0.1
    b = fastsum.coefficients(c, N, d, eps, 4, kind)
    j = fastsum.index_set(N)
    nodes = np.stack(np.meshgrid(*([j / N] * d), indexing="ij"), axis=-1).reshape(-1, d)
    K = fastsum.RegKernel(c, eps, 4, kind)
    got = fastsum.K_RF(nodes, b, N)
    np.testing.assert_allclose(got.real, K(np.linalg.norm(nodes, axis=1)), atol=1e-12)


@pytest.mark.parametrize("kind,c", [("multiquadric", 0.2), ("inverse_multiquadric", 0.2)])
def test_other_kernels_scaled_operator_matches_direct_sums(kind, c):
    """In the scaled coordinates the parameter is rho c and the sums carry the
    homogeneity factor (rho for the multiquadric, 1/rho for the inverse
    multiquadric), which the operator divides out: W x and the degrees then
    match the direct sums in the original coordinates within
    ||x||_1 ||K_ERR||_inf times that factor.  (The other reading, c / rho with
    the reverse factors, misses by orders of magnitude.)"""
    v = synth.gmm(300, d=3, k=3, seed=11)
    N, eps, p = 64, 1.0 / 8, 6
    T = fastsum.TrigGraph(v, c, N, eps, p, kind)
    W = graph.dense_W(v, c, kind)
    x = np.random.default_rng(2).standard_normal(300)
    kerr = fastsum.kerr_sampled(T.bhat, N, T.sigma_t, eps, 3, samples=20000, kind=kind)
    bound = 2.0 * T.scale * kerr * np.abs(x).sum()
    err = np.abs(T.apply_W(x) - W @ x).max()
    assert err <= bound
    assert np.abs(T.d - W.sum(axis=1)).max() <= 2.0 * T.scale * kerr * 300
    # and the bound is meaningful: well below the size of W x
    assert bound < 1e-2 * np.abs(W @ x).max()
    # the inverted reading of the parameter scaling is far off
    c2, rho, vt = fastsum.scaling(v, eps)
    b_wrong = fastsum.coefficients(c / rho, N, 3, eps, p, kind)
    wrong = (1.0 / fastsum.output_scale(kind, rho)) * fastsum.trig_operator(vt, x, b_wrong, N)
    assert np.abs(wrong - T.K0 * x - W @ x).max() > 100 * bound


def test_laplacian_rbf_derivatives_and_inner_regularisation():
    """exp(-r/s): derivatives against central differences; T_I is even and
    meets the Hermite conditions at +-eps_I (so K_R is C^{p-1} across the
    junction), and the near-field correction K - K_R vanishes beyond eps_I."""
    s, p, eps_I = 0.05, 6, 0.09
    D = fastsum.radial_derivs("laplacian_rbf", 0.07, s, p)
    h = 1e-6
    K = fastsum.radial_kernel("laplacian_rbf", s)
    assert abs(D[1] - (K(0.07 + h) - K(0.07 - h)) / (2 * h)) <= 1e-7 * abs(D[1])
    R = fastsum.RegKernel(s, 1.0 / 8, p, "laplacian_rbf", eps_I)
    r = np.linspace(0.0, eps_I, 7)
    np.testing.assert_allclose(R.T_I(r), R.T_I(-r), rtol=1e-12, atol=1e-14)
    poly = np.polynomial.Polynomial(R.coef_I)
    h2 = 2 * eps_I
    A = fastsum.radial_derivs("laplacian_rbf", eps_I, s, p)
    for k in range(p):
        dk = poly.deriv(k) if k else poly
        scale = sum(abs(c) * q ** k for q, c in enumerate(R.coef_I)) / h2 ** k
        assert abs(dk(1.0) / h2 ** k - A[k]) <= 1e-11 * scale + 1e-13, k
    assert np.all(R.near(np.array([eps_I * 1.01, 0.2, 0.4])) == 0.0)
    assert R.near(np.array([0.0]))[0] == pytest.approx(1.0 - R.T_I(0.0))


def test_laplacian_rbf_near_field_restores_the_direct_sums():
    """Trigonometric operator of the regularised kernel plus the near-field sum
    equals the direct sums of eq. W_laplacian_rbf within
    ||x||_1 max |K_R - K_RF| (the near field restores K exactly on r <= eps_I);
    without the near field the kink of K at 0 leaves errors ~1e-2."""
    v = synth.gmm(800, d=3, k=4, seed=3)
    s, N, m, eps_B = 0.05, 64, 6, 1.0 / 8
    T = fastsum.TrigGraph(v, s, N, eps_B, m, "laplacian_rbf", eps_I=m / N)
    x = np.random.default_rng(5).standard_normal(800)
    W = graph.dense_W(v, s, "laplacian_rbf")
    rng = np.random.default_rng(0)
    g = rng.normal(size=(20000, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    rr = (0.5 - eps_B) * rng.uniform(0.0, 1.0, size=20000) ** (1.0 / 3)
    kerr = np.abs(T.reg(rr) - fastsum.K_RF(g * rr[:, None], T.bhat, N).real).max()
    err = np.abs(T.apply_W(x) - W @ x).max()
    assert err <= 2.0 * kerr * np.abs(x).sum()
    assert err <= 1e-4 * np.abs(W @ x).max()
    T0 = fastsum.TrigGraph(v, s, N, eps_B, m, "laplacian_rbf")
    assert np.abs(T0.apply_W(x) - W @ x).max() > 1e-3 * np.abs(W @ x).max()


# ---- Oracle B: the exact trigonometric operator -----------------------------

def test_trig_operator_on_grid_nodes_is_the_direct_sum():
    """On nodes lying on the lattice j/N inside the ball of radius 1/4 - eps_B/2,
    every difference v_j - v_i is a lattice node with norm <= 1/2 - eps_B, where
    K_RF interpolates K_R = K exactly; so the trigonometric operator equals the
    direct sum sum_i x_i K(v_j - v_i) = (W x)_j + x_j."""
    N, d, s = 32, 2, 0.09
    j = fastsum.index_set(N)
    g = np.stack(np.meshgrid(j / N, j / N, indexing="ij"), axis=-1).reshape(-1, 2)
    g = g[np.linalg.norm(g, axis=1) <= 0.25 - 1.0 / 16]
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.shape[0])
    b = fastsum.coefficients(s, N, d, 1.0 / 8, 4)
    f = fastsum.trig_operator(g, x, b, N)
    np.testing.assert_allclose(f, graph.apply_W(g, s, x) + x, atol=1e-12)


def test_trig_operator_with_targets_on_grid_nodes_is_the_direct_cross_sum():
    """Sources and distinct targets on the lattice j/N inside the ball of radius
    1/4 - eps_B/2: every difference is a lattice node where K_RF = K_R = K, so
    the operator with targets is sum_i x_i K(t_j - v_i) exactly; with targets
    equal to the sources it is the operator without targets."""
    N, d, s = 32, 2, 0.09
    j = fastsum.index_set(N)
    g = np.stack(np.meshgrid(j / N, j / N, indexing="ij"), axis=-1).reshape(-1, 2)
    g = g[np.linalg.norm(g, axis=1) <= 0.25 - 1.0 / 16]
    rng = np.random.default_rng(4)
    src, tgt = g[::2], g[1::3]
    x = rng.standard_normal(src.shape[0])
    b = fastsum.coefficients(s, N, d, 1.0 / 8, 4)
    f = fastsum.trig_operator(src, x, b, N, targets=tgt)
    D = np.exp(-((tgt[:, None, :] - src[None, :, :]) ** 2).sum(axis=2) / s ** 2)
    np.testing.assert_allclose(f, D @ x, atol=1e-12)
    np.testing.assert_allclose(fastsum.trig_operator(src, x, b, N, targets=src),
                               fastsum.trig_operator(src, x, b, N), atol=1e-13)


def test_trig_operator_matches_matrix_and_kerr_bound():
    """Two code paths for the same operator agree; and |f - f_RF| <=
    ||x||_1 ||K_ERR||_inf (eq. KERR_estimate) against the direct sum."""
    v = synth.gmm(300, d=3, k=3, seed=7)
    s, N, eps = 0.05, 16, 0.0
    c, rho, vt = fastsum.scaling(v, eps)
    b = fastsum.coefficients(s * rho, N, 3, eps, 4)
    x = np.random.default_rng(1).standard_normal(300)
    f = fastsum.trig_operator(vt, x, b, N)
    M = fastsum.trig_matrix(vt, b, N)
    np.testing.assert_allclose(f, M @ x, atol=1e-11)
    kerr = fastsum.kerr_sampled(b, N, s * rho, eps, 3, samples=40000)
    err = np.abs(f - (graph.apply_W(v, s, x) + x)).max()
    # the sampled maximum under-estimates the true sup slightly: allow 2x
    assert err <= 2.0 * np.abs(x).sum() * kerr
    assert err > 0.0


def test_scaling_puts_nodes_in_ball_and_preserves_weights():
    v = synth.gmm(200, d=3, seed=1)
    eps = 6.0 / 64
    c, rho, vt = fastsum.scaling(v, eps)
    assert abs(np.linalg.norm(vt, axis=1).max() - (0.25 - eps / 2)) < 1e-15
    W1 = graph.dense_W(v, 0.04)
    W2 = graph.dense_W(vt, 0.04 * rho)
    np.testing.assert_allclose(W1, W2, rtol=1e-12, atol=1e-300)


def test_lemma_bound_holds():
    """Lemma normalization_propagation with the exact eps, eta and ||A - A_E||_inf
    computed from the full matrices (eq. epsilon_norm_aposteriori)."""
    v = synth.blobs2d(240, seed=5)
    s, N, eps_B = 0.05, 32, 0.0
    c, rho, vt = fastsum.scaling(v, eps_B)
    b = fastsum.coefficients(s * rho, N, 2, eps_B, 4)
    Wt_E = fastsum.trig_matrix(vt, b, N)          # W~_E = W + I + E
    W = graph.dense_W(v, s)
    E = Wt_E - W - np.eye(W.shape[0])
    Wn = np.abs(W).sum(axis=1).max()
    eps = np.abs(E).sum(axis=1).max() / Wn
    d = W.sum(axis=1)
    eta = d.min() / Wn
    assert 0 < eps < eta
    W_E = W + E
    dE = W_E.sum(axis=1)
    A = W / np.sqrt(np.outer(d, d))
    A_E = W_E / np.sqrt(np.outer(dE, dE))
    err = np.abs(A - A_E).sum(axis=1).max()
    assert err <= fastsum.lemma_bound(eps, eta)
    # and the bound is not vacuous here
    assert fastsum.lemma_bound(eps, eta) < 1.0


def test_lemma_bound_hand_values_and_proof_chain():
    """The Lemma's bound eps (1 + eta) / (eta (eta - eps)) at hand-computed
    points (eps = 0.01, eta = 0.1: 0.011 / 0.009 = 11/9; eps = 0.2, eta = 0.5:
    0.3 / 0.15 = 2), infinite where eps >= eta, and equal to the unsimplified
    sum of the three terms in the proof of the Lemma (Section 3.1):
    ((eta-eps)^{-1/2} - eta^{-1/2}) (eta^{-1/2} + (1+eps)(eta-eps)^{-1/2})
    + (eta-eps)^{-1/2} eps eta^{-1/2}."""
    assert abs(fastsum.lemma_bound(0.01, 0.1) - 11.0 / 9.0) < 1e-15
    assert abs(fastsum.lemma_bound(0.2, 0.5) - 2.0) < 1e-15
    assert fastsum.lemma_bound(0.3, 0.3) == np.inf and fastsum.lemma_bound(0.4, 0.3) == np.inf
    rng = np.random.default_rng(11)
    for _ in range(50):
        eta = rng.uniform(1e-3, 1.0)
        eps = eta * rng.uniform(0.0, 0.99)
        a, b = (eta - eps) ** -0.5, eta ** -0.5
        chain = (a - b) * (b + (1.0 + eps) * a) + a * eps * b
        assert abs(fastsum.lemma_bound(eps, eta) - chain) <= 1e-12 * chain + 1e-300


def test_K_RF_single_coefficient_and_kerr_of_a_constant():
    """eq. K_RF with one nonzero coefficient b at l* is b exp(2 pi i l*.y)
    (closed form); kerr_sampled of the constant K_RF = 3 against the Gaussian
    of width 0.05 is 3 - min K over the samples, i.e. 3 up to e^{-80}
    (samples reach radius ~1/2, where K ~ e^{-100})."""
    rng = np.random.default_rng(12)
    N = 8
    for d in (1, 2, 3):
        y = rng.uniform(-0.5, 0.5, size=(40, d))
        b = np.zeros((N,) * d)
        lstar = rng.integers(-N // 2, N // 2, size=d)
        b[tuple(lstar + N // 2)] = 1.75
        want = 1.75 * np.exp(2j * np.pi * (y @ lstar))
        np.testing.assert_allclose(fastsum.K_RF(y, b, N), want, rtol=0, atol=1e-13)
        c = np.zeros((N,) * d)
        c[(N // 2,) * d] = 3.0
        k = fastsum.kerr_sampled(c, N, 0.05, 0.0, d, samples=5000, seed=1)
        assert abs(k - 3.0) < 1e-12, (d, k)


# ---- Krylov solvers (Section 4) -----------------------------------------------

def test_lanczos_matches_lapack_and_top_eigenpair():
    """Largest eigenvalue of A is 1 with eigenvector D^{1/2} 1 (Section 2);
    the k largest Ritz values match LAPACK's eigh."""
    v = synth.blobs2d(400, seed=2)
    s = 0.05
    A = graph.dense_A(v, s)
    theta, V, res, steps = krylov.lanczos_largest(lambda q: A @ q, 400, 6, tol=1e-11)
    ref = np.linalg.eigvalsh(A)[::-1][:6]
    np.testing.assert_allclose(theta, ref, atol=1e-10)
    assert abs(theta[0] - 1.0) < 1e-12
    d = graph.degree(v, s)
    u = np.sqrt(d) / np.linalg.norm(np.sqrt(d))
    assert abs(abs(V[:, 0] @ u) - 1.0) < 1e-9
    for i in range(6):
        assert np.linalg.norm(A @ V[:, i] - theta[i] * V[:, i]) < 1e-9


def test_cg_matches_dense_solve():
    """CG on (I + tau L_s) u = f (eq. ssl::system) against LAPACK's solve."""
    v, lab = synth.moons_and_roll(600, seed=3)
    s, tau = 0.04, 10.0
    M = np.eye(600) + tau * graph.dense_Ls(v, s)
    f = synth.ssl_rhs(lab, 0, frac=0.05, seed=1)
    u, it, rel = krylov.cg(lambda p: M @ p, f, tol=1e-10, maxit=500)
    np.testing.assert_allclose(u, np.linalg.solve(M, f), atol=1e-8)
    assert rel <= 1e-10 and it < 200


# ---- Nystrom-Gaussian-NFFT (Alg. nystrom_hybrid) --------------------------------

def _lowrank(n, lam, seed):
    """A = U diag(lam) U^T with a random orthonormal U (n x len(lam))."""
    U, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, len(lam))))
    return (U * np.asarray(lam)[None, :]) @ U.T, U


def test_nystrom_exact_for_low_rank_psd():
    """For A positive semidefinite of rank r <= M <= L, range(A G) = range(A),
    so the rank-M Nystrom matrix is A itself: the k largest eigenpairs come out
    exactly, and M shrinks to r (the other eigenvalues of Q^T A Q are zero)."""
    lam = np.array([1.0, 0.8, 0.55, 0.4, 0.25, 0.1])
    A, U = _lowrank(60, lam, seed=5)
    G = np.random.default_rng(6).standard_normal((60, 12))
    th, V, m_used = nystrom.nystrom_gaussian(lambda X: A @ X, G, k=4, M=8)
    assert m_used == 6
    np.testing.assert_allclose(th, lam[:4], atol=1e-12)
    np.testing.assert_allclose(np.abs(np.sum(V * U[:, :4], axis=0)), 1.0, atol=1e-10)


def test_nystrom_keeps_only_the_positive_part():
    """With negative eigenvalues in the range (A indefinite, as the graph's A
    is), step 5 drops them: the result is the positive part of A."""
    A_pos, U = _lowrank(50, [0.9, 0.7, 0.5], seed=7)
    w = np.random.default_rng(8).standard_normal(50)
    w -= U @ (U.T @ w)
    w /= np.linalg.norm(w)
    A = A_pos - 0.8 * np.outer(w, w)
    G = np.random.default_rng(9).standard_normal((50, 8))
    th, V, m_used = nystrom.nystrom_gaussian(lambda X: A @ X, G, k=3, M=8)
    assert m_used == 3
    np.testing.assert_allclose(th, [0.9, 0.7, 0.5], atol=1e-12)
    assert np.abs(V.T @ w).max() < 1e-10


def test_nystrom_full_sample_is_the_truncated_eigendecomposition():
    """L = n: Q is square orthogonal, Q^T A Q is similar to A, and the rank-M
    matrix is A's truncation to its M largest (positive) eigenvalues; on a
    graph A of Section 2 these match LAPACK's eigh."""
    v, _, sc = synth.spirals(60, seed=1)
    A = graph.dense_A(v, 3.5 * sc)
    G = np.random.default_rng(2).standard_normal((60, 60))
    th, V, m_used = nystrom.nystrom_gaussian(lambda X: A @ X, G, k=8, M=8)
    ev, EV = np.linalg.eigh(A)
    np.testing.assert_allclose(th, ev[::-1][:8], atol=1e-11)
    assert abs(th[0] - 1.0) < 1e-12          # top eigenvalue of A is 1 (Section 2)
    for i in range(8):
        assert np.linalg.norm(A @ V[:, i] - th[i] * V[:, i]) < 1e-9


def test_nystrom_steps_6_7_match_the_dense_nystrom_matrix():
    """Steps 6-7 (QR of B1 U_M, eigendecomposition of Rh Sigma^{-1} Rh^T) are
    the eigendecomposition of (A Q)(Q^T A Q)_M^{-1}(A Q)^T; formed densely
    with Q from an SVD instead, LAPACK's eigh gives the same pairs."""
    v, _, sc = synth.spirals(400, seed=3)
    A = graph.dense_A(v, 3.5 * sc)
    G = np.random.default_rng(4).standard_normal((400, 20))
    th, V, m_used = nystrom.nystrom_gaussian(lambda X: A @ X, G, k=10, M=10)
    assert m_used == 10
    N = nystrom.nystrom_matrix(lambda X: A @ X, G, 10)
    ev = np.linalg.eigvalsh(N)[::-1][:10]
    np.testing.assert_allclose(th, ev, atol=1e-11)
    np.testing.assert_allclose((V * th[None, :]) @ V.T, N, atol=1e-11)
    np.testing.assert_allclose(V.T @ V, np.eye(10), atol=1e-12)


def test_nystrom_depends_on_the_range_of_G_only():
    """Q = orth(A G) is unchanged (up to rotation) by G -> G S, S invertible,
    and every later step is invariant under that rotation."""
    v, _, sc = synth.spirals(300, seed=5)
    A = graph.dense_A(v, 3.5 * sc)
    rng = np.random.default_rng(6)
    G = rng.standard_normal((300, 16))
    S = rng.standard_normal((16, 16)) + 4.0 * np.eye(16)
    t1, V1, _ = nystrom.nystrom_gaussian(lambda X: A @ X, G, k=6, M=10)
    t2, V2, _ = nystrom.nystrom_gaussian(lambda X: A @ X, G @ S, k=6, M=10)
    np.testing.assert_allclose(t1, t2, atol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(V1 * V2, axis=0)), 1.0, atol=1e-8)


def test_nystrom_rejects_bad_sizes():
    A = np.eye(10)
    with pytest.raises(ValueError):
        nystrom.nystrom_gaussian(lambda X: A @ X, np.ones((10, 4)), k=5, M=4)
    with pytest.raises(ValueError):
        nystrom.nystrom_gaussian(lambda X: -(A @ X), np.eye(10)[:, :4], k=1, M=2)


# ---- kernel ridge regression (Section 6.3) -----------------------------------

@pytest.mark.parametrize("kind,param", [("gaussian", 0.3), ("inverse_multiquadric", 0.2)])
def test_krr_closed_forms(kind, param):
    """One point: alpha = f / (K(0) + beta).  Two points at distance r:
    [[K0 + b, k], [k, K0 + b]]^{-1} f by the 2 x 2 inverse.  Large beta:
    alpha -> f / beta."""
    K0 = 1.0 if kind == "gaussian" else 1.0 / param
    one = np.array([[0.1, 0.2]])
    a1 = krr.solve(one, param, 0.5, [3.0], kind)
    assert abs(a1[0] - 3.0 / (K0 + 0.5)) < 1e-15
    two = np.array([[0.0, 0.0], [0.3, 0.4]])
    r2 = 0.25
    k = math.exp(-r2 / param ** 2) if kind == "gaussian" else 1.0 / math.sqrt(r2 + param ** 2)
    b, f = 0.7, np.array([1.0, -2.0])
    det = (K0 + b) ** 2 - k * k
    ref = np.array([(K0 + b) * f[0] - k * f[1], -k * f[0] + (K0 + b) * f[1]]) / det
    np.testing.assert_allclose(krr.solve(two, param, b, f, kind), ref, rtol=1e-14)
    v = synth.blobs2d(50, seed=1)
    f = np.random.default_rng(0).standard_normal(50)
    big = 1e9
    np.testing.assert_allclose(krr.solve(v, param, big, f, kind) * big, f, rtol=1e-6)


def test_krr_matches_cg_and_predicts_training_values():
    """The dense solve agrees with CG on the same SPD system, and the
    prediction at the training points is K alpha = f - beta alpha."""
    v = synth.blobs2d(300, seed=4)
    f = np.sign(v[:, 0]).astype(np.float64)
    s, b = 0.05, 0.1
    K = krr.gram(v, s)
    a = krr.solve(v, s, b, f)
    u, it, rel = krylov.cg(lambda p: K @ p + b * p, f, tol=1e-12, maxit=2000)
    np.testing.assert_allclose(a, u, atol=1e-8 * np.abs(a).max())
    np.testing.assert_allclose(krr.predict(v, a, v, s), f - b * a, atol=1e-9)


# ---- the warm-start network reference -----------------------------------------

def test_mlp_gradient_matches_finite_differences():
    """Analytic backward of the FP64 network against central differences."""
    from oracle import mlp
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, size=mlp.NP)
    X = rng.normal(size=(37, 16))
    t = rng.normal(size=37)
    L, g = mlp.loss_and_grad(p, X, t, emulate=False)
    idx = np.concatenate([rng.choice(1024, 8), 1024 + rng.choice(64, 4), 1088 + rng.choice(4096, 8),
                          5184 + rng.choice(64, 4), 5248 + rng.choice(4096, 8),
                          9344 + rng.choice(64, 4), 9408 + rng.choice(64, 4), [9472]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NP)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t, emulate=False)[0]
              - mlp.loss_and_grad(p - e, X, t, emulate=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_rounding_is_nearest_even():
    from oracle import mlp
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-3.0) == -3.0
