// Host-side division of the tile-stationary forms' work into workgroups
// (plain C++, no device code: the plan set-up and a CPU test include it).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace nfl {

// the nodes start .. end - 1 (sorted order) of one tile inside a group
struct GroupSeg {
  int tile;
  int start;
  int end;
};

// The tile-stationary forms' work: the sorted nodes in at most G groups of
// near-equal cost, G the workgroups the GPU holds at once, so that all groups
// run in one round and end together (work items of a fixed size leave the
// CUs of the last round partly idle, and a second round of smaller groups
// measured slower).  A segment (the nodes of one tile inside a group,
// contiguous in the sort) costs its nodes plus kSegCost node-equivalents:
// the interpolation stages the tile's padded grid block and the spread
// flushes it whatever the number of nodes, each a chain of dependent memory
// accesses, so a group's time grows with its segments even where the CU has
// other work (at the benchmark workload a product took 261, 233, 215, 202,
// 196 and 200 us with 64, 96, 128, 192, 256 and 384).  A tile's nodes in one
// group form one segment, so they are staged and flushed once.  Small
// problems get fewer, larger groups: none costs less than a segment of 512
// nodes (many groups of ~100 nodes in a few dense tiles flush into the same
// cells at once: on the 316 x 316 RGB image, 1e5 nodes, 88 against 77 us).
// In: hc, the nodes of each tile in sorted tile order (empty tiles hold 0);
// n, their sum; G >= 1.  Out: the segments in sorted-node order, and group g
// = segments goff[g] .. goff[g + 1] - 1 (at most G groups, none empty).
inline void cost_groups(const std::vector<uint32_t> &hc, int64_t n, int G,
                        std::vector<GroupSeg> &gi, std::vector<int> &goff) {
  constexpr double kSegCost = 256.0, kMinGroupCost = 512.0 + kSegCost;
  constexpr int64_t kMinTake = 32;
  int64_t nocc = 0;
  for (uint32_t c : hc) nocc += c > 0;
  const double target =
      std::max(kMinGroupCost, ((double)n + kSegCost * (double)(nocc + G)) / G);
  gi.clear();
  goff.assign(1, 0);
  double gc = 0.0;
  int64_t start = 0;
  for (size_t t = 0; t < hc.size(); ++t) {
    int64_t pos = start, rem = hc[t];
    start += hc[t];
    while (rem > 0) {
      const bool last = (int)goff.size() == G;   // the last group takes the rest
      const double room = target - gc - kSegCost;
      if (!last && gc > 0.0 && room < (double)kMinTake) {
        goff.push_back((int)gi.size());
        gc = 0.0;
        continue;
      }
      const int64_t take =
          last ? rem : std::min<int64_t>(rem, std::max<int64_t>(kMinTake, (int64_t)std::ceil(room)));
      gi.push_back(GroupSeg{(int)t, (int)pos, (int)(pos + take)});
      gc += kSegCost + (double)take;
      pos += take;
      rem -= take;
      if (!last && gc >= target) {
        goff.push_back((int)gi.size());
        gc = 0.0;
      }
    }
  }
  if (goff.back() != (int)gi.size()) goff.push_back((int)gi.size());
}

}  // namespace nfl
