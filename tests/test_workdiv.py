"""Host logic of the tile-stationary forms' work division (csrc/workdiv.h),
compiled with g++ on the CPU: every node in exactly one segment, segments
in sorted order inside their tile, one segment per tile and group, at most
G groups, and the groups' cost near the target (nodes + 256 per segment,
at least 768)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1808_04580_amd", "csrc")
SEG, MIN_GROUP, MIN_TAKE = 256.0, 768.0, 32

DRIVER = r"""
#include <cstdio>
#include "workdiv.h"
int main() {
  int G = 0; long nt = 0;
  if (scanf("%d %ld", &G, &nt) != 2) return 1;
  std::vector<uint32_t> hc((size_t)nt);
  long long n = 0;
  for (long t = 0; t < nt; ++t) { unsigned c; if (scanf("%u", &c) != 1) return 1; hc[t] = c; n += c; }
  std::vector<nfl::GroupSeg> gi; std::vector<int> goff;
  nfl::cost_groups(hc, n, G, gi, goff);
  printf("%zu %zu\n", goff.size(), gi.size());
  for (int o : goff) printf("%d\n", o);
  for (const auto &s : gi) printf("%d %d %d\n", s.tile, s.start, s.end);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("workdiv")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run([gxx, "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(driver, counts, G):
    inp = "%d %d\n%s\n" % (G, len(counts), " ".join(str(int(c)) for c in counts))
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split()
    ng, ns = int(out[0]), int(out[1])
    goff = np.array(out[2:2 + ng], dtype=np.int64)
    segs = np.array(out[2 + ng:2 + ng + 3 * ns], dtype=np.int64).reshape(ns, 3)
    return goff, segs


CASES = {
    # clustered: ~400 occupied tiles of log-normal size, 1e6 nodes in all
    "clustered": lambda rng: np.where(rng.random(4000) < 0.1,
                                      np.maximum(1, rng.lognormal(7.0, 1.5, 4000)), 0).astype(np.int64),
    # sparse: most tiles one to three nodes
    "sparse": lambda rng: rng.integers(0, 4, 20000),
    "one_tile": lambda rng: np.array([0, 0, 1_000_003, 0]),
    "tiny": lambda rng: np.array([0, 2, 0, 3]),
    "dense_and_sparse": lambda rng: np.concatenate([rng.integers(0, 3, 3000), [250_000], rng.integers(0, 3, 3000)]),
}


@pytest.mark.parametrize("G", [1, 7, 1024, 4096])
@pytest.mark.parametrize("case", sorted(CASES))
def test_groups_cover_every_node_once(driver, case, G):
    counts = CASES[case](np.random.default_rng(5))
    n = int(counts.sum())
    goff, segs = run(driver, counts, G)
    ng = len(goff) - 1
    assert 1 <= ng <= G
    assert goff[0] == 0 and goff[-1] == len(segs) and np.all(np.diff(goff) > 0)
    # segments tile the sorted order, each inside its own tile's range
    assert segs[0, 1] == 0 and segs[-1, 2] == n
    assert np.all(segs[1:, 1] == segs[:-1, 2]) and np.all(segs[:, 2] > segs[:, 1])
    tstart = np.concatenate([[0], np.cumsum(counts)])
    t = segs[:, 0]
    assert np.all(counts[t] > 0)
    assert np.all(segs[:, 1] >= tstart[t]) and np.all(segs[:, 2] <= tstart[t + 1])
    # a tile appears at most once in a group
    for g in range(ng):
        tg = t[goff[g]:goff[g + 1]]
        assert np.all(np.diff(tg) > 0)


@pytest.mark.parametrize("case", ["clustered", "sparse", "dense_and_sparse"])
def test_group_costs_near_target(driver, case):
    counts = CASES[case](np.random.default_rng(9))
    n, G = int(counts.sum()), 1024
    goff, segs = run(driver, counts, G)
    nocc = int((counts > 0).sum())
    target = max(MIN_GROUP, (n + SEG * (nocc + G)) / G)
    lens = segs[:, 2] - segs[:, 1]
    cost = np.array([lens[goff[g]:goff[g + 1]].sum() + SEG * (goff[g + 1] - goff[g])
                     for g in range(len(goff) - 1)])
    # every group but the last closes once it reaches the target; a segment
    # takes at most the room left (or the minimum take)
    assert np.all(cost[:-1] <= target + MIN_TAKE + 1)
    assert cost[-1] <= 2.0 * target
    # the groups used cover the work without much slack
    assert cost.sum() <= len(cost) * (target + MIN_TAKE + 1)
