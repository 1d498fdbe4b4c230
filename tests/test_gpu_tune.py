"""GPU tests of the accuracy probe and the parameter search.

nfl_direct_rows (the library's exact sampled-row sums, FP64 on the GPU) is
compared with the oracle's direct sums; the configuration nfl_autotune
chooses is checked against the oracle on every row, and its cache is
exercised: a hit is verified on the new graph, a wrong entry is re-tuned.
"""
import numpy as np
import pytest

import synth
from oracle import graph

pytestmark = pytest.mark.gpu


def test_direct_rows_match_oracle(nfl):
    import torch
    v = synth.gmm(6001, d=3, k=5, seed=3)
    x = synth.normal_vectors(6001, seed=4)
    P = nfl.Plan(3)
    P.set_points(torch.as_tensor(v, device="cuda"))
    rows = np.sort(np.random.default_rng(0).choice(6001, size=300, replace=False))
    wx, dg = P.direct_rows(0.05, rows, torch.as_tensor(x, device="cuda"))
    refW = graph.w_rows(v, 0.05, x.astype(np.float64), rows)
    refd = graph.degree(v, 0.05, rows)
    np.testing.assert_allclose(dg, refd, rtol=1e-12, atol=0)
    np.testing.assert_allclose(wx, refW, rtol=0, atol=1e-12 * np.abs(refW).max())
    # degrees alone (no vector)
    _, dg2 = P.direct_rows(0.05, rows)
    np.testing.assert_array_equal(dg2, dg)
    with pytest.raises(nfl.NFLError) as e:
        P.direct_rows(0.05, [6001])
    assert e.value.code == nfl.NFL_ERR_ARG
    P.close()


def _check_config_against_oracle(P, v, sigma, target):
    """max(rel_inf(d), rel_inf(W x)) over all rows against the oracle."""
    import torch
    n = len(v)
    x = synth.normal_vectors(n, seed=77).astype(np.float64)
    refd = graph.degree(v, sigma)
    refW = graph.apply_W(v, sigma, x)
    dg = P.degree().cpu().numpy().astype(np.float64)
    yW = P.apply_W(torch.as_tensor(x.astype(np.float32), device="cuda")).cpu().numpy()
    rd = np.abs(dg - refd).max() / np.abs(refd).max()
    rw = np.abs(yW - refW).max() / np.abs(refW).max()
    return rd, rw


@pytest.mark.parametrize("sigma", [0.05, 0.12])
def test_autotune_meets_target_against_oracle(nfl, sigma, tmp_path):
    import torch
    v = synth.gmm(3000, d=3, k=4, seed=12)
    P = nfl.Plan(3)
    P.set_points(torch.as_tensor(v, device="cuda"))
    cache = str(tmp_path / "tune.txt")
    r = P.autotune(sigma, target=1e-5, rows=3000, seed=5, cache=cache)
    assert r["reached"] and not r["cached"], r
    assert r["err"] <= 1e-5
    assert 2 <= r["m"] <= 8 and r["N"] >= 8 and r["tile"] in (4, 8, 16)
    info = P.info()
    assert abs(info["eps_B"] - r["eps_B"]) < 1e-15
    # the degrees are x-independent: the same bound holds on every row; W x
    # for another random vector gets a factor 2 of room
    rd, rw = _check_config_against_oracle(P, v, sigma, 1e-5)
    assert rd <= 1e-5 and rw <= 2e-5, (r, rd, rw)
    # one window narrower misses 0.7 x target on the probe (or m is already 2)
    if r["m"] > 2:
        P.set_option(nfl.OPT_TILE, r["tile"])
        P.set_kernel(sigma, r["N"], r["m"] - 1, r["eps_B"])
        rd2, rw2 = _check_config_against_oracle(P, v, sigma, 1e-5)
        assert max(rd2, rw2) > 0.3e-5, (r, rd2, rw2)

    # cache hit on a second cloud of the same size class and sigma band
    v2 = synth.gmm(2900, d=3, k=4, seed=13)
    Q = nfl.Plan(3)
    Q.set_points(torch.as_tensor(v2, device="cuda"))
    r2 = Q.autotune(sigma, target=1e-5, rows=512, seed=6, cache=cache)
    assert r2["reached"] and r2["err"] <= 1e-5
    if r2["cached"]:
        assert (r2["N"], r2["m"], r2["tile"]) == (r["N"], r["m"], r["tile"])
    P.close()
    Q.close()


def test_autotune_rejects_a_wrong_cache_entry(nfl, tmp_path):
    import torch
    v = synth.gmm(3000, d=3, k=4, seed=21)
    sigma = 0.05
    P = nfl.Plan(3)
    P.set_points(torch.as_tensor(v, device="cuda"))
    cache = tmp_path / "tune.txt"
    r = P.autotune(sigma, target=1e-5, rows=1024, seed=5, cache=str(cache))
    assert r["reached"]
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[0].startswith("#")
    f = lines[1].split()
    # replace the entry by a far too coarse grid for this sigma
    f[4], f[5] = "8", "2"
    cache.write_text(lines[0] + "\n" + " ".join(f) + "\n")
    r2 = P.autotune(sigma, target=1e-5, rows=1024, seed=5, cache=str(cache))
    assert r2["reached"] and not r2["cached"]
    assert (r2["N"], r2["m"]) == (r["N"], r["m"])
    assert cache.read_text().splitlines()[1].split()[4] == str(r["N"])
    # the next call is served from the corrected cache
    r3 = P.autotune(sigma, target=1e-5, rows=1024, seed=5, cache=str(cache))
    assert r3["cached"] and (r3["N"], r3["m"], r3["tile"]) == (r["N"], r["m"], r["tile"])
    P.close()


def test_autotune_smaller_sigma_needs_finer_grid(nfl):
    import torch
    v = synth.gmm(2000, d=3, k=4, seed=31)
    P = nfl.Plan(3)
    P.set_points(torch.as_tensor(v, device="cuda"))
    wide = P.autotune(0.12, target=1e-5, rows=512)
    narrow = P.autotune(0.035, target=1e-5, rows=512)
    assert wide["reached"] and narrow["reached"]
    assert narrow["N"] >= wide["N"] and narrow["N"] >= 32
    P.close()
