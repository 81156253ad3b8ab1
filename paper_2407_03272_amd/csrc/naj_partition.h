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
// first, first + step, ... while < end.  step >= 1 always.
NAJ_HD inline SliceRange slice_range(int64_t nslices, int ndom_req, int grid, int w, int wave, int waves_per_block) {
  const int ndom = effective_domains(grid, ndom_req);
  const int dom = w % ndom;
  const int j = w / ndom;
  const int per_dom = grid / ndom;
  SliceRange r;
  r.first = nslices * dom / ndom + (int64_t)j * waves_per_block + wave;
  r.end = nslices * (dom + 1) / ndom;
  r.step = (int64_t)per_dom * waves_per_block;
  return r;
}

}  // namespace naj
