"""GPU edge cases of the fast summation, against the oracle's direct FP64
sums (Section 2): the fewest points, duplicated points, all points
identical (zero radius), degenerate geometry (a line and a plane in 3-D),
everything in one grid tile (many work items per tile), and the largest grid
this build supports (N = 256 in 3-D, 512^3 points), on sampled rows.
Gate: relative max-norm error 1e-5 of W x and d, as for the other products.
"""
import numpy as np
import pytest

import synth
from oracle import graph

pytestmark = pytest.mark.gpu


def _check(nfl, v, sigma, N, m, eps_B=0.0, rows=None, tol=1e-5, **opts):
    import torch
    v = np.ascontiguousarray(v.astype(np.float32))
    n = v.shape[0]
    x = synth.normal_vectors(n, seed=n % 1000 + 1)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), sigma, N=N, m=m, eps_B=eps_B, **opts)
    Wx = P.apply_W(torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    d = P.degree().cpu().numpy().astype(np.float64)
    Ls = P.apply_Ls(torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
    P.close()
    sel = np.arange(n) if rows is None else rows
    refW = graph.w_rows(v, sigma, x.astype(np.float64), sel)
    refd = graph.degree(v, sigma, sel)
    assert np.abs(Wx[sel] - refW).max() <= tol * max(np.abs(refW).max(), 1e-30)
    assert np.abs(d[sel] - refd).max() <= tol * refd.max()
    assert np.all(np.isfinite(Ls))
    return Wx, d


def test_two_points(nfl):
    """The pair sits at the largest scaled distance (1/2 - eps_B): eps_B = 1/8
    and N = 128 resolve the kernel there; sigma keeps the weight well above
    FP32 rounding of W~ x - x."""
    v = np.array([[0.01, -0.02, 0.03], [0.05, 0.01, -0.02]])
    _check(nfl, v, 0.05, 128, 4, eps_B=1.0 / 8)


def test_duplicated_points(nfl):
    base = synth.gmm(600, d=3, k=3, seed=4)
    v = np.concatenate([base, base[:400], base[:50]], axis=0)
    _check(nfl, v, 0.05, 64, 5)


def test_all_points_identical(nfl):
    """Zero radius: every weight is K(0) = 1, W x = sum(x) - x, d = n - 1."""
    v = np.tile(np.array([[0.1, -0.2, 0.05]], dtype=np.float32), (500, 1))
    Wx, d = _check(nfl, v, 0.1, 32, 4)
    np.testing.assert_allclose(d, 499.0, rtol=1e-5)


@pytest.mark.parametrize("shape", ["line", "plane"])
def test_degenerate_geometry(nfl, shape):
    rng = np.random.default_rng(12)
    t = rng.uniform(-0.2, 0.2, size=(3000, 2))
    if shape == "line":
        v = np.stack([t[:, 0], 0.5 * t[:, 0], -0.3 * t[:, 0]], axis=1)
    else:
        v = np.stack([t[:, 0], t[:, 1], 0.0 * t[:, 0]], axis=1)
    _check(nfl, v, 0.04, 64, 5)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_everything_in_one_tile(nfl, d):
    """A tight cluster of 5,000 points plus two small far clusters (so the big
    one sits in one tile; isolated far points would have degrees near 0,
    outside the Lemma's eps < eta): many work items per tile, their flushes to
    the same cells."""
    rng = np.random.default_rng(20 + d)
    core = rng.normal(0.0, 1e-3, size=(5000, d))
    far = np.concatenate([rng.normal(0.0, 1e-3, size=(100, d)) + 0.2,
                          rng.normal(0.0, 1e-3, size=(100, d)) - 0.2])
    v = np.concatenate([core, far], axis=0)
    _check(nfl, v, 0.05, 64, 4, chunk=64)


def test_largest_grid_3d(nfl):
    """N = 256 (oversampled grid 512^3), m = 4, n = 200,000 narrow clusters,
    sigma = 0.01: sampled rows of W x and d."""
    v = synth.gmm(200_000, d=3, k=20, std_lo=0.003, std_hi=0.01, seed=9)
    rows = np.sort(np.random.default_rng(1).choice(200_000, size=128, replace=False))
    _check(nfl, v, 0.01, 256, 4, rows=rows)


def test_refused_inputs(nfl):
    import torch
    with pytest.raises(nfl.NFLError):        # one point: no graph
        nfl.plan(torch.zeros((1, 3), device="cuda"), 0.1, N=32, m=4)
    v = torch.as_tensor(synth.gmm(100, d=3, k=2, seed=1), device="cuda")
    with pytest.raises(nfl.NFLError):        # N not a power of 2
        nfl.plan(v, 0.1, N=48, m=4)
    with pytest.raises(nfl.NFLError):        # window wider than the grid allows
        nfl.plan(v, 0.1, N=8, m=6)
    bad = v.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(nfl.NFLError):
        nfl.plan(bad, 0.1, N=32, m=4)
