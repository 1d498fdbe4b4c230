"""GPU parity of the NFFT steps and operators against the oracle.

Every test calls the HIP library through its C-ABI (the ctypes binding) and
compares with the FP64 oracle on the same seeded float32 inputs, or with
independent FP64 helpers written here (gridding with the Kaiser-Bessel
window, numpy FFTs).  Tolerances follow from FP32 arithmetic: a product
with the FP32 grid carries ~1e-7 relative error per term; the gates below
allow 1e-5 relative (the target of the FP32 path).
"""
import math

import numpy as np
import pytest

import synth
from oracle import fastsum, graph

pytestmark = pytest.mark.gpu

B = 1.5 * math.pi


def tt(a, dev="cuda"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def host(t):
    return t.detach().cpu().numpy()


def kb_psi(t, m):
    t = np.asarray(t, dtype=np.float64)
    s = np.sqrt(np.maximum(m * m - t * t, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.where(s > 0, np.sinh(B * s) / np.where(s > 0, s, 1.0), B) / (B * math.exp(B * m))
    return np.where((t > -m) & (t <= m), v, 0.0)


def grid_coords(v, rho, eps_B, nos):
    c, _, _ = fastsum.scaling(v, eps_B)
    V = np.asarray(v, dtype=np.float64)
    V = V[:, None] if V.ndim == 1 else V
    return nos * (rho * (V - c) + 0.5)


def cpu_spread(u, x, m, nos):
    """g[k] = sum_i x_i prod_t psi(k_t - u_it) over the 2m cells per axis with
    t in (-m, m], periodic; FP64."""
    n, d = u.shape
    fl = np.floor(u).astype(np.int64)
    offs = np.arange(-m + 1, m + 1)
    g = np.zeros((nos,) * d)
    idx = [(fl[:, t, None] + offs[None, :]) for t in range(d)]
    w = [kb_psi(idx[t] - u[:, t, None], m) for t in range(d)]
    if d == 1:
        np.add.at(g, idx[0] % nos, x[:, None] * w[0])
    elif d == 2:
        val = x[:, None, None] * w[0][:, :, None] * w[1][:, None, :]
        I0 = np.broadcast_to(idx[0][:, :, None], val.shape) % nos
        I1 = np.broadcast_to(idx[1][:, None, :], val.shape) % nos
        np.add.at(g, (I0, I1), val)
    else:
        val = (x[:, None, None, None] * w[0][:, :, None, None] * w[1][:, None, :, None]
               * w[2][:, None, None, :])
        I0 = np.broadcast_to(idx[0][:, :, None, None], val.shape) % nos
        I1 = np.broadcast_to(idx[1][:, None, :, None], val.shape) % nos
        I2 = np.broadcast_to(idx[2][:, None, None, :], val.shape) % nos
        np.add.at(g, (I0, I1, I2), val)
    return g.reshape(-1)


def make(nfl, v, sigma, N, m, eps_B=0.0, tile=None, chunk=None, kernel=0):
    import torch
    v = np.asarray(v, dtype=np.float32)
    d = 1 if v.ndim == 1 else v.shape[1]
    P = nfl.Plan(d)
    P.set_option(nfl.OPT_KERNEL, kernel)
    if tile:
        P.set_option(nfl.OPT_TILE, tile)
    if chunk:
        P.set_option(nfl.OPT_CHUNK, chunk)
    P.set_points(torch.as_tensor(v.reshape(len(v), d), device="cuda"))
    P.set_kernel(sigma, N, m, eps_B)
    return P


CASES = [
    # (d, n, N, m, tile, chunk, kernel) -- several tiles, ragged n, several items
    # per tile; kernel 0 = matrix cores (tile-stationary where tile + 2m - 1 <= 16,
    # else per-cell runs), 1 = vector ALU, 2 = matrix cores with per-cell runs
    # (d = 3 only)
    (3, 2777, 32, 4, 8, 256, 0),
    (3, 2222, 32, 3, 8, 100, 0),
    (3, 3333, 32, 6, 4, 200, 2),
    (3, 4099, 32, 5, 4, 96, 2),
    (3, 3001, 16, 4, 4, 64, 2),
    (3, 3001, 16, 4, 4, 64, 0),
    (3, 3001, 16, 4, 4, 64, 1),
    (3, 2500, 32, 6, 8, 128, 0),
    (3, 2500, 32, 6, 8, 128, 1),
    (3, 4099, 32, 5, 4, 96, 0),
    (3, 3333, 32, 6, 4, 200, 0),
    (3, 2001, 32, 7, 16, 700, 0),
    (3, 1777, 16, 2, 4, 64, 0),
    (3, 1500, 32, 8, 8, 300, 0),
    (2, 2999, 32, 5, None, None, 0),
    (1, 777, 64, 3, None, None, 0),
    # d <= 2 spread sums padded tiles of tile + 2m - 1 <= 19 cells per item
    (2, 3001, 32, 8, 4, 64, 0),
    (2, 5000, 16, 2, 16, 300, 0),
    (2, 2000, 64, 4, 32, 128, 0),      # tile 32 is clamped so that the padded tile fits
    (1, 1500, 128, 6, 8, 64, 0),
]


@pytest.mark.parametrize("d,n,N,m,tile,chunk,kernel", CASES)
def test_spread_matches_cpu_gridding(nfl, d, n, N, m, tile, chunk, kernel):
    v = synth.gmm(n, d=d, k=4, seed=11 + d)
    P = make(nfl, v, 0.08, N, m, 0.0, tile, chunk, kernel)
    x = synth.normal_vectors(n, seed=5)
    g = host(P.spread(tt(x)))
    u = grid_coords(v, P.info()["rho"], 0.0, 2 * N)
    ref = cpu_spread(u, x.astype(np.float64), m, 2 * N)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


@pytest.mark.parametrize("n_sparse,n_dense,N,m,tile", [
    (2500, 0, 64, 4, 4), (2000, 6000, 64, 6, 4), (1500, 9000, 32, 4, 8), (3000, 3000, 64, 2, 8)])
def test_tile_forms_on_mixed_clouds(nfl, n_sparse, n_dense, N, m, tile):
    """A sparse uniform ball (most tiles hold a node or two) plus one dense
    cluster: the tile forms' workgroups then take several tiles one after the
    other (each reusing the LDS of the one before) and the dense tiles are
    split over several workgroups.  Spread element-wise against the FP64
    gridding, interpolation on sampled nodes against its transpose."""
    rng = np.random.default_rng(42)
    dense = rng.normal(size=(n_dense, 3)) * 0.004 + np.array([0.05, 0.02, -0.03])
    v = np.concatenate([synth.uniform_ball(n_sparse, d=3, seed=41), dense]).astype(np.float32)
    n = len(v)
    P = make(nfl, v, 0.08, N, m, 0.0, tile)
    x = synth.normal_vectors(n, seed=5)
    g = host(P.spread(tt(x)))
    u = grid_coords(v, P.info()["rho"], 0.0, 2 * N)
    ref = cpu_spread(u, x.astype(np.float64), m, 2 * N)
    assert np.abs(g - ref).max() <= 2e-6 * np.abs(ref).max()
    rng = np.random.default_rng(3)
    G = rng.standard_normal((2 * N) ** 3).astype(np.float32)
    f = host(P.interp(tt(G)))
    rows = np.arange(0, n, 37)
    ref_f = np.array([cpu_spread(u[i:i + 1], np.ones(1), m, 2 * N) @ G for i in rows])
    np.testing.assert_allclose(f[rows], ref_f, rtol=0, atol=3e-6 * np.abs(ref_f).max())


@pytest.mark.parametrize("d,N", [(1, 64), (1, 256), (2, 32), (2, 128), (3, 16), (3, 32), (3, 64)])
def test_convolve_matches_numpy_fft(nfl, d, N):
    v = synth.gmm(500, d=d, k=3, seed=2)
    P = make(nfl, v, 0.1, N, 3 if N <= 16 else 4)
    nos = 2 * N
    rng = np.random.default_rng(7)
    G = rng.standard_normal((nos,) * d).astype(np.float32)
    out = host(P.convolve(tt(G.reshape(-1)))).reshape((nos,) * d)
    filt = P.filter().reshape([N + 1] * (d - 1) + [N // 2 + 1])
    H = np.zeros([nos] * (d - 1) + [nos // 2 + 1])
    ext = np.arange(-N // 2, N // 2 + 1) % nos
    sl = np.ix_(*([ext] * (d - 1) + [np.arange(N // 2 + 1)]))
    H[sl] = filt
    ref = np.fft.irfftn(np.fft.rfftn(G.astype(np.float64)) * H, s=(nos,) * d, axes=tuple(range(d))) * nos ** d
    err = np.abs(out - ref).max() / np.abs(ref).max()
    assert err < 2e-6, err


@pytest.mark.parametrize("d,n,N,m,tile,chunk,kernel", CASES)
def test_interp_is_transpose_of_spread(nfl, d, n, N, m, tile, chunk, kernel):
    v = synth.gmm(n, d=d, k=4, seed=21)
    P = make(nfl, v, 0.08, N, m, 0.0, tile, chunk, kernel)
    x = synth.normal_vectors(n, seed=8)
    rng = np.random.default_rng(1)
    g = rng.standard_normal((2 * N) ** d).astype(np.float32)
    lhs = float(np.dot(host(P.spread(tt(x))).astype(np.float64), g))
    f = host(P.interp(tt(g)))
    rhs = float(np.dot(x.astype(np.float64), f))
    u = grid_coords(v, P.info()["rho"], 0.0, 2 * N)
    # interp against the FP64 gridding transpose
    ref_f = np.array([cpu_spread(u[i:i + 1], np.ones(1), m, 2 * N) @ g for i in range(0, n, 97)])
    np.testing.assert_allclose(f[::97], ref_f, rtol=0, atol=3e-6 * np.abs(ref_f).max())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + 1e-30)


@pytest.mark.parametrize("d,n,sigma,N,m,eps_B", [
    (2, 2000, 0.05, 32, 6, 1.0 / 16),
    (3, 1500, 0.06, 16, 6, 0.0),
    (3, 1200, 0.15, 16, 5, 1.0 / 8),
    (1, 900, 0.03, 64, 4, 0.0),
])
def test_operators_match_exact_trig_operator(nfl, d, n, sigma, N, m, eps_B):
    """GPU (NFFT, FP32) vs the exact trigonometric operator (direct NDFT, FP64):
    isolates window + FFT + FP32 error from the kernel approximation."""
    v = synth.gmm(n, d=d, k=3, seed=31)
    P = make(nfl, v, sigma, N, m, eps_B)
    TG = fastsum.TrigGraph(v, sigma, N, eps_B, m)
    x = synth.normal_vectors(n, seed=3).astype(np.float64)
    d_gpu = host(P.degree()).astype(np.float64)
    assert np.abs(d_gpu - TG.d).max() <= 1e-5 * np.abs(TG.d).max()
    yW = host(P.apply_W(tt(x.astype(np.float32)))).astype(np.float64)
    refW = TG.apply_W(x)
    assert np.abs(yW - refW).max() <= 1e-5 * np.abs(refW).max()
    yL = host(P.apply_Ls(tt(x.astype(np.float32)))).astype(np.float64)
    refL = TG.apply_Ls(x)
    assert np.abs(yL - refL).max() <= 1e-5 * np.abs(refL).max()


@pytest.mark.parametrize("m,tile,kernel", [
    (6, 4, 0),    # tile-stationary spread and interpolation (the default form)
    (4, 8, 0),    # tile-stationary, 8-cell tiles
    (6, 8, 0),    # padded tile 19 > 16: per-cell runs on the matrix cores
    (6, 4, 2),    # per-cell runs forced
    (6, 4, 1),    # vector ALU
])
def test_operators_across_tile_sizes_and_kernel_forms(nfl, m, tile, kernel):
    """Products of a plan's own nodes take the FFT passes on the z-lines its
    nodes' windows touch; the support is built from the tile size and m, and
    every kernel form must write and read inside it.  Degrees, W x and L_s x
    against the exact trigonometric operator (1e-5) for each form, on a
    clustered cloud whose support leaves lines out."""
    n, sigma, N = 2500, 0.06, 16
    v = synth.gmm(n, d=3, k=3, seed=37)
    P = make(nfl, v, sigma, N, m, 0.0, tile, None, kernel)
    TG = fastsum.TrigGraph(v, sigma, N, 0.0, m)
    x = synth.normal_vectors(n, seed=5).astype(np.float64)
    d_gpu = host(P.degree()).astype(np.float64)
    assert np.abs(d_gpu - TG.d).max() <= 1e-5 * np.abs(TG.d).max()
    yW = host(P.apply_W(tt(x.astype(np.float32)))).astype(np.float64)
    refW = TG.apply_W(x)
    assert np.abs(yW - refW).max() <= 1e-5 * np.abs(refW).max()
    yL = host(P.apply_Ls(tt(x.astype(np.float32)))).astype(np.float64)
    refL = TG.apply_Ls(x)
    assert np.abs(yL - refL).max() <= 1e-5 * np.abs(refL).max()


def test_blobs2d_full_config_vs_direct_oracle(nfl):
    """The small workload: n = 5000 two blobs in 2-D, sigma = 0.05, eps_B = 1/16,
    m = 4.  At N = 32 the kernel approximation alone leaves ~1e-5 relative
    error in L_s x; at N = 64 the FP32 path meets 1e-5 against the direct sum."""
    v = synth.blobs2d(5000, seed=0)
    x = synth.normal_vectors(5000, seed=1).astype(np.float64)
    dref = graph.degree(v, 0.05)
    refL = graph.apply_Ls(v, 0.05, x, dref)
    refW = graph.apply_W(v, 0.05, x)
    for N, gate in [(64, 1e-5), (32, 5e-5)]:
        P = make(nfl, v, 0.05, N, 4, 1.0 / 16)
        dg = host(P.degree()).astype(np.float64)
        yL = host(P.apply_Ls(tt(x.astype(np.float32)))).astype(np.float64)
        yW = host(P.apply_W(tt(x.astype(np.float32)))).astype(np.float64)
        relL = np.abs(yL - refL).max() / np.abs(refL).max()
        relD = np.abs(dg - dref).max() / np.abs(dref).max()
        epsW = np.abs(yW - refW).max() / (dref.max() * np.abs(x).max())
        assert relL <= gate and relD <= gate and epsW <= gate, (N, relL, relD, epsW)


def test_invariants_of_the_approximate_operator(nfl):
    """L_{s,E} D_E^{1/2} 1 = 0 and x^T L_{s,E} y = y^T L_{s,E} x hold for the
    approximate operator itself (same deterministic degree pass, interp =
    spread^T, real even filter)."""
    v = synth.gmm(20000, d=3, k=6, seed=9)
    P = make(nfl, v, 0.05, 32, 5)
    dE = host(P.degree()).astype(np.float64)
    s = np.sqrt(dE).astype(np.float32)
    y = host(P.apply_Ls(tt(s))).astype(np.float64)
    assert np.abs(y).max() <= 2e-5 * np.abs(s).max()
    a = synth.normal_vectors(20000, seed=1)
    b = synth.normal_vectors(20000, seed=2)
    La = host(P.apply_Ls(tt(a))).astype(np.float64)
    Lb = host(P.apply_Ls(tt(b))).astype(np.float64)
    lhs, rhs = b.astype(np.float64) @ La, a.astype(np.float64) @ Lb
    assert abs(lhs - rhs) <= 1e-5 * (np.abs(a).sum() * np.abs(Lb).max())
    # multiple vectors in one call equal single calls
    Y = host(P.apply_Ls(tt(np.stack([a, b]))))
    assert np.abs(Y[0] - La).max() <= 1e-6 * np.abs(La).max()
    assert np.abs(Y[1] - Lb).max() <= 1e-6 * np.abs(Lb).max()


@pytest.mark.parametrize("block", [1, 3, 4, 6])
def test_lanczos_matches_dense_eigh(nfl, block):
    """10 smallest eigenpairs of L_s on the n = 5000 blob workload (N = 64),
    single-vector and block Lanczos (block 6: two passes of four and two
    vectors over the basis): eigenvalues within 1e-6 of LAPACK on the
    dense FP64 matrix; residuals of the returned vectors against the dense
    matrix small."""
    v = synth.blobs2d(5000, seed=0)
    P = make(nfl, v, 0.05, 64, 4, 1.0 / 16)
    r = P.lanczos_smallest(10, tol=1e-8, maxit=300, block=block)
    lam_ref, U = graph.smallest_eigs_dense(v, 0.05, 10)
    assert r["converged"]
    assert np.abs(r["evals"] - lam_ref).max() <= 1e-6, (r["evals"], lam_ref)
    assert abs(r["evals"][0]) <= 1e-6
    V = host(r["evecs"])
    Ls = graph.dense_Ls(v, 0.05)
    for i in range(10):
        res = np.linalg.norm(Ls @ V[:, i] - r["evals"][i] * V[:, i])
        assert res <= 1e-4, (i, res)


@pytest.mark.parametrize("block", [1, 4])
def test_image_subsample_lanczos_matches_dense_eigh(nfl, block):
    """Image-segmentation graph (316 x 316 RGB, 6 regions, noise 0.02) on a
    seeded 5000-pixel subsample, sigma = 0.1, N = 64, m = 5: the 10 smallest
    eigenvalues of L_s within 1e-6 of LAPACK on the dense FP64 matrix."""
    img = synth.image_rgb(316, seed=0)
    idx = np.sort(np.random.default_rng(5).choice(img.shape[0], size=5000, replace=False))
    v = np.ascontiguousarray(img[idx])
    P = make(nfl, v, 0.1, 64, 5)
    r = P.lanczos_smallest(10, tol=1e-8, maxit=300, block=block, vectors=False)
    lam_ref, _ = graph.smallest_eigs_dense(v, 0.1, 10)
    assert r["converged"], r
    assert np.abs(r["evals"] - lam_ref).max() <= 1e-6, (r["evals"], lam_ref)


def test_cg_matches_dense_solve(nfl):
    """(I + tau L_s) u = f by CG on the GPU vs LAPACK's solve with the exact
    FP64 matrix; tau = 10, 2% labels, n = 4000 moons-and-roll."""
    v, lab = synth.moons_and_roll(4000, seed=4)
    P = make(nfl, v, 0.04, 64, 6)
    f = synth.ssl_rhs(lab, 2, frac=0.02, seed=3)
    r = P.cg_solve(tt(f), tau=10.0, tol=1e-8, maxit=500)
    M = np.eye(4000) + 10.0 * graph.dense_Ls(v, 0.04)
    u_ref = np.linalg.solve(M, f)
    u = host(r["u"])
    assert r["relres"] <= 1e-6, r
    assert np.abs(u - u_ref).max() <= 1e-5 * np.abs(u_ref).max()
    # warm start from the solution converges immediately; user warm start honoured
    r2 = P.cg_solve(tt(f), tau=10.0, tol=1e-6, maxit=500, u0=r["u"])
    assert r2["iters"] <= 1
    # without the closing true-residual product: the same iterations and
    # bitwise the same solution (the solve is deterministic), no residual
    r3 = P.cg_solve(tt(f), tau=10.0, tol=1e-8, maxit=500, true_residual=False)
    assert r3["relres"] is None and r3["converged"] and r3["iters"] == r["iters"]
    np.testing.assert_array_equal(host(r3["u"]), u)


def test_error_paths(nfl):
    import torch
    v = synth.gmm(1000, d=3, seed=1)
    P = nfl.Plan(3)
    x = torch.zeros(1000, device="cuda")
    rc = nfl.lib().nfl_apply_Ls(P._h, x.data_ptr(), x.data_ptr(), 1, 1000)
    assert rc == nfl.NFL_ERR_ORDER
    with pytest.raises(nfl.NFLError) as e:
        P.set_kernel(0.05, 32, 4)
    assert e.value.code == nfl.NFL_ERR_ORDER
    P.set_points(tt(v))
    for args, code in [((0.05, 31, 4), nfl.NFL_ERR_ARG), ((0.05, 48, 4), nfl.NFL_ERR_UNSUPPORTED),
                       ((0.0, 32, 4), nfl.NFL_ERR_ARG), ((0.05, 32, 0), nfl.NFL_ERR_ARG),
                       ((0.05, 32, 4, 0.5), nfl.NFL_ERR_ARG), ((0.05, 32, 9), nfl.NFL_ERR_UNSUPPORTED)]:
        with pytest.raises(nfl.NFLError) as e:
            P.set_kernel(*args)
        assert e.value.code == code, args
    # eps >= eta: a very narrow Gaussian on a coarse grid gives negative degrees
    with pytest.raises(nfl.NFLError) as e:
        P.set_kernel(0.001, 8, 2)
    assert e.value.code == nfl.NFL_ERR_DEGREE
    with pytest.raises(nfl.NFLError) as e:
        P.apply_Ls(x)
    assert e.value.code == nfl.NFL_ERR_ORDER
    P.set_kernel(0.05, 32, 4)
    r = P.cg_solve(tt(np.ones(1000)), tau=10.0, tol=1e-12, maxit=1)
    assert not r["converged"] and r["iters"] == 1
    P.close()
