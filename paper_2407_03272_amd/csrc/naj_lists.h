// Per-wave item lists of the per-pass kernel, built on the host when a system is created (host code
// only: the library uploads the result, and a host test checks it).  Wave w of a launch of `grid`
// workgroups of `wpb` waves (w = workgroup * wpb + wave in workgroup) sweeps items[off[w] .. off[w+1]),
// an item being long row i (< n_long) or slice i - n_long.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

#include "naj_partition.h"

namespace naj {

// Balanced lists (sorted layout): items assigned longest first, each to the wave with the least work
// so far (ties to the lowest wave); every wave sweeps its items in increasing order.  cost[i] is item
// i's work.
inline void balanced_wave_lists(const std::vector<int64_t>& cost, int waves, std::vector<int32_t>& off,
                                std::vector<int32_t>& items) {
  const int64_t nitems = (int64_t)cost.size();
  std::vector<int32_t> order((size_t)nitems);
  for (int64_t i = 0; i < nitems; ++i) order[(size_t)i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[(size_t)x] > cost[(size_t)y]; });
  using Load = std::pair<int64_t, int32_t>;   // (work so far, wave)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int32_t w = 0; w < waves; ++w) heap.push({0, w});
  std::vector<int32_t> owner((size_t)nitems);
  for (const int32_t it : order) {
    Load l = heap.top();
    heap.pop();
    owner[(size_t)it] = l.second;
    l.first += cost[(size_t)it];
    heap.push(l);
  }
  off.assign((size_t)waves + 1, 0);
  items.assign((size_t)nitems, 0);
  for (int64_t i = 0; i < nitems; ++i) off[(size_t)owner[(size_t)i] + 1] += 1;
  for (int w = 0; w < waves; ++w) off[(size_t)w + 1] += off[(size_t)w];
  std::vector<int32_t> pos(off.begin(), off.end() - 1);
  for (int64_t i = 0; i < nitems; ++i) items[(size_t)pos[(size_t)owner[(size_t)i]]++] = (int32_t)i;
}

// Blocked lists (regular layout, no long rows): the slices of every L2 domain (the contiguous range the
// slice partition gives it; workgroup w runs on domain w mod ndom) are visited band by band, a band
// being `band` consecutive slices, in blocks of `blk` slices: block 0 of every band of the domain, then
// block 1, and so on.  The domain's waves take that order in turn.  Returns false (no lists) when a band
// is no longer than a block.
inline bool blocked_wave_lists(int64_t ns, int64_t n_long, int64_t band, int64_t blk, int ndom_req, int grid,
                               int wpb, std::vector<int32_t>& off, std::vector<int32_t>& items) {
  if (ns <= 0 || blk <= 0 || band <= blk || grid < 1 || wpb < 1) return false;
  const int waves = grid * wpb;
  const int ndom = effective_domains(grid, ndom_req);
  const int nwd = grid / ndom * wpb;   // waves of one domain
  std::vector<std::vector<int32_t>> lists((size_t)waves);
  for (int d = 0; d < ndom; ++d) {
    const int64_t lo = ns * d / ndom, hi = ns * (d + 1) / ndom;
    int64_t k = 0;   // position in the domain's blocked order
    for (int64_t c = 0; c * blk < band; ++c)
      for (int64_t z = lo / band; z * band < hi; ++z) {
        const int64_t a = std::max(lo, z * band + c * blk);
        const int64_t b = std::min(hi, std::min(z * band + (c + 1) * blk, (z + 1) * band));
        for (int64_t sl = a; sl < b; ++sl, ++k) {
          const int q = (int)(k % nwd);              // the domain's wave that takes it
          const int w = (q / wpb) * ndom + d;        // its workgroup
          lists[(size_t)w * wpb + q % wpb].push_back((int32_t)(n_long + sl));
        }
      }
  }
  off.assign((size_t)waves + 1, 0);
  items.clear();
  items.reserve((size_t)ns);
  for (int w = 0; w < waves; ++w) {
    items.insert(items.end(), lists[(size_t)w].begin(), lists[(size_t)w].end());
    off[(size_t)w + 1] = (int32_t)items.size();
  }
  return true;
}

}  // namespace naj
