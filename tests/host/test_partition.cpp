// Host check of the slice-to-wave assignment used by every solve kernel:
// for many (slices, domains, grid, block) shapes, every slice is visited by
// exactly one wave and every stride is positive (a zero stride would never end).
#include <cstdio>
#include <vector>

#include "naj_partition.h"

int main() {
  long checked = 0;
  const int waves_opts[] = {4, 8, 16};
  const int dom_opts[] = {1, 2, 8};
  const int grid_opts[] = {1, 2, 3, 7, 8, 9, 16, 24, 64, 1000, 1024, 2048};
  const long long slice_opts[] = {0, 1, 2, 5, 63, 64, 65, 100, 1000, 4097, 32768};
  for (int wpb : waves_opts)
    for (int nd : dom_opts)
      for (int G : grid_opts)
        for (long long ns : slice_opts) {
          // weights: decreasing widths as in a degree-sorted layout
          std::vector<int64_t> wpre(ns + 1, 0);
          for (long long s = 0; s < ns; ++s) wpre[s + 1] = wpre[s] + 1 + (ns - s) % 97;
          std::vector<int64_t> bounds(nd + 1);
          naj::balanced_bounds(wpre.data(), ns, nd, bounds.data());
          for (int d = 0; d < nd; ++d)
            if (bounds[d] > bounds[d + 1]) { std::printf("FAIL bounds not monotone\n"); return 1; }
          for (int use_bounds = 0; use_bounds < 2; ++use_bounds) {
          std::vector<int> hits(ns, 0);
          for (int w = 0; w < G; ++w)
            for (int v = 0; v < wpb; ++v) {
              naj::SliceRange r = naj::slice_range(ns, nd, G, w, v, wpb, use_bounds ? bounds.data() : nullptr);
              if (r.step < 1) { std::printf("FAIL zero step ns=%lld nd=%d G=%d w=%d\n", ns, nd, G, w); return 1; }
              if (r.end > ns) { std::printf("FAIL end beyond slices\n"); return 1; }
              for (long long s = r.first; s < r.end; s += r.step) {
                if (s < 0) { std::printf("FAIL negative slice\n"); return 1; }
                hits[s] += 1;
              }
            }
          for (long long s = 0; s < ns; ++s)
            if (hits[s] != 1) {
              std::printf("FAIL slice %lld visited %d times (ns=%lld nd=%d G=%d wpb=%d)\n", s, hits[s], ns, nd, G, wpb);
              return 1;
            }
          ++checked;
          }
        }
  std::printf("ok %ld shapes\n", checked);
  return 0;
}
