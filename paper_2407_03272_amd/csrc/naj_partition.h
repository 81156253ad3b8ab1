// Assignment of 64-row slices to wavefronts (host- and device-callable).
//
// Workgroups are dispatched round-robin over `ndom` L2 domains (the XCDs of
// the chip), so workgroup w runs in domain w % ndom.  The slices are cut into
// ndom contiguous ranges; the waves of a domain sweep its range together with
// a common stride, so rows that neighbour each other are read close in time
// by the same L2.  When the grid cannot be split evenly over the domains
// (fewer workgroups than domains, or a remainder) a single domain is used.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define NAJ_HD __host__ __device__
#else
#define NAJ_HD
#endif

namespace naj {

struct SliceRange {
  int64_t first, end, step;
};

NAJ_HD inline int effective_domains(int grid, int ndom) {
  return (ndom > 1 && grid >= ndom && grid % ndom == 0) ? ndom : 1;
}

// Slices visited by wave `wave` (0 <= wave < waves_per_block) of workgroup `w` (0 <= w < grid):
// first, first + step, ... while < end.  step >= 1 always.  `bounds` (ndom_req + 1
// non-decreasing entries from 0 to nslices, or null for equal slice counts)
// gives each domain's range, e.g. balanced by stored entries.
NAJ_HD inline SliceRange slice_range(int64_t nslices, int ndom_req, int grid, int w, int wave, int waves_per_block,
                                     const int64_t* bounds = nullptr) {
  const int ndom = effective_domains(grid, ndom_req);
  const int dom = w % ndom;
  const int j = w / ndom;
  const int per_dom = grid / ndom;
  const bool use_b = bounds != nullptr && ndom == ndom_req && ndom > 1;
  SliceRange r;
  const int64_t lo = use_b ? bounds[dom] : nslices * dom / ndom;
  r.first = lo + (int64_t)j * waves_per_block + wave;
  r.end = use_b ? bounds[dom + 1] : nslices * (dom + 1) / ndom;
  r.step = (int64_t)per_dom * waves_per_block;
  return r;
}

// Domain boundaries splitting slices [0, nslices) into ndom contiguous ranges of
// nearly equal weight (weight prefix sums wpre[0..nslices]); bounds[ndom+1].
NAJ_HD inline void balanced_bounds(const int64_t* wpre, int64_t nslices, int ndom, int64_t* bounds) {
  const int64_t total = wpre[nslices];
  int64_t s = 0;
  bounds[0] = 0;
  for (int d = 1; d < ndom; ++d) {
    const int64_t target = total / ndom * d + (total % ndom) * d / ndom;
    while (s < nslices && wpre[s] < target) ++s;
    bounds[d] = s;
  }
  bounds[ndom] = nslices;
}

}  // namespace naj
