"""GPU parity of the batched launch: many graphs of different size, kernel
width and NFFT parameters, a block of vectors each, in one graph launch.

Each (graph, vector) result is compared with the exact trigonometric
operator of its own plan (the FP64 oracle of Alg. nfft_fastsum's output,
which isolates the FP32 window/FFT error; gate 1e-5 relative, looser for
windows narrower than m = 4, whose own error is larger), and with the
same plan's single-graph product (same kernels, same operator; only the
order of the floating-point atomic additions differs; gate 2e-6).  The
graph is replayed several times with eager work and synchronisations in
between, with both a change of buffers and a repeat of the same buffers.
"""
import numpy as np
import pytest

import synth
from oracle import fastsum

pytestmark = pytest.mark.gpu

# (n, sigma, N, m, tile, eps_B): window widths 4..14, z-merged and plain
# spreads, two tiles in one width group, ragged sizes
GRAPHS = [
    (1501, 0.10, 16, 4, 4, 0.0),
    (2203, 0.08, 32, 6, 4, 0.0),
    (777, 0.12, 16, 5, 8, 1.0 / 16),
    (1999, 0.09, 32, 7, 4, 0.0),
    (1200, 0.10, 16, 4, 8, 0.0),
    (300, 0.15, 16, 2, 4, 1.0 / 8),
    (1003, 0.11, 16, 3, 4, 0.0),
]
NVEC = 3

# Kaiser-Bessel window error bound at oversampling 2 (the NFFT literature's
# estimate 4 pi (sqrt(m) + m) (1/2)^(1/4) e^(-2 pi m / sqrt(2))), with a
# factor 4 of slack; below m = 4 the window, not FP32, limits the agreement.
def trig_gate(m):
    import math
    kb = 4 * math.pi * (math.sqrt(m) + m) * 0.5 ** 0.25 * math.exp(-2 * math.pi * m / math.sqrt(2))
    return max(1e-5, 4 * kb)


def _plans(nfl):
    import torch
    plans, clouds = [], []
    for g, (n, sigma, N, m, tile, eps_B) in enumerate(GRAPHS):
        v = synth.gmm(n, d=3, k=3 + g % 4, seed=100 + g)
        P = nfl.Plan(3)
        P.set_option(nfl.OPT_TILE, tile)
        P.set_points(torch.as_tensor(v, device="cuda"))
        P.set_kernel(sigma, N, m, eps_B)
        plans.append(P)
        clouds.append(v)
    return plans, clouds


def _blocks(seed):
    return [synth.normal_vectors(n, nvec=NVEC, seed=seed + g)
            for g, (n, *_r) in enumerate(GRAPHS)]


def test_batch_matches_oracle_and_single_plan(nfl):
    import torch
    plans, clouds = _plans(nfl)
    B = nfl.Batch(plans, NVEC)
    info = B.info()
    assert info["jobs"] == NVEC * len(GRAPHS)
    assert info["total_n"] == sum(g[0] for g in GRAPHS)
    assert np.array_equal(np.diff(B.offsets), [g[0] for g in GRAPHS])

    xa, xb = _blocks(10), _blocks(20)
    Xa, Xb = B.pack(xa), B.pack(xb)
    Ya, Yb = torch.empty_like(Xa), torch.empty_like(Xb)

    # expected: the oracle's exact operator per plan, and the single-plan product
    trig = [fastsum.TrigGraph(v, s, N, e, m) for v, (n, s, N, m, t, e) in zip(clouds, GRAPHS)]
    single = {}
    for key, xs in (("a", xa), ("b", xb)):
        single[key] = [P.apply_Ls(torch.as_tensor(x, device="cuda")).cpu().numpy()
                       for P, x in zip(plans, xs)]

    def check(Y, xs, key):
        torch.cuda.synchronize()
        for g, (blk, x) in enumerate(zip(B.unpack(Y), xs)):
            y = blk.cpu().numpy().astype(np.float64)
            for j in range(NVEC):
                ref = trig[g].apply_Ls(x[j].astype(np.float64))
                err = np.abs(y[j] - ref).max() / np.abs(ref).max()
                assert err <= trig_gate(GRAPHS[g][3]), (key, g, j, err)
                s = single[key][g][j].astype(np.float64)
                assert np.abs(y[j] - s).max() <= 2e-6 * np.abs(s).max(), (key, g, j)

    # replays: new buffers, other buffers, the same buffers again, with eager
    # work (single-plan products) and synchronisations between them
    B.apply_Ls(Xa, out=Ya)
    check(Ya, xa, "a")
    plans[0].apply_Ls(torch.as_tensor(xa[0], device="cuda"))
    Ya.zero_()
    B.apply_Ls(Xb, out=Yb)
    torch.cuda.synchronize()
    check(Yb, xb, "b")
    B.apply_Ls(Xa, out=Ya)
    check(Ya, xa, "a")
    Ya.zero_()
    B.apply_Ls(Xa, out=Ya)
    check(Ya, xa, "a")
    B.close()
    for P in plans:
        P.close()


def test_batch_single_graph_many_vectors(nfl):
    """One graph with a block of 8 vectors equals eight single products."""
    import torch
    v = synth.gmm(4097, d=3, k=5, seed=7)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.07, N=32, m=5, tile=4)
    B = nfl.Batch([P], 8)
    x = synth.normal_vectors(4097, nvec=8, seed=3)
    Y = B.apply_Ls(B.pack([x]))
    y = B.unpack(Y)[0].cpu().numpy()
    for j in range(8):
        s = P.apply_Ls(torch.as_tensor(x[j], device="cuda")).cpu().numpy()
        assert np.abs(y[j] - s).max() <= 2e-6 * np.abs(s).max(), j
    B.close()
    P.close()


def test_batch_errors(nfl):
    import torch
    v = synth.gmm(500, d=3, k=3, seed=1)
    P = nfl.plan(torch.as_tensor(v, device="cuda"), 0.1, N=16, m=3)
    with pytest.raises(nfl.NFLError) as e:
        nfl.Batch([P], 0)
    assert e.value.code == nfl.NFL_ERR_ARG
    P2 = nfl.plan(torch.as_tensor(synth.blobs2d(400, seed=0), device="cuda"), 0.05, N=16, m=3)
    with pytest.raises(nfl.NFLError) as e:
        nfl.Batch([P, P2], 2)
    assert e.value.code == nfl.NFL_ERR_UNSUPPORTED
    P3 = nfl.Plan(3)
    P3.set_points(torch.as_tensor(v, device="cuda"))
    with pytest.raises(nfl.NFLError) as e:
        nfl.Batch([P, P3], 2)
    assert e.value.code == nfl.NFL_ERR_ORDER
    B = nfl.Batch([P], 2)
    x = torch.zeros(2 * 500, device="cuda")
    B.apply_Ls(x)
    P.set_kernel(0.1, 16, 4, 0.0)          # plan changed after the batch was made
    with pytest.raises(nfl.NFLError) as e:
        B.apply_Ls(x)
    assert e.value.code == nfl.NFL_ERR_ORDER
    B.close()
    for Q in (P, P2, P3):
        Q.close()
