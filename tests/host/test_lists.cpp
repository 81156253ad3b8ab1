// Host check of the per-wave item lists of the per-pass kernel (naj_lists.h), for many shapes:
//  * balanced lists: every item in exactly one wave's list, each list increasing, and the most loaded
//    wave within one item of the least loaded one's work plus the largest item (the LPT bound);
//  * blocked lists: every slice in exactly one list, each wave's slices inside its domain's range
//    (workgroup w on domain w mod ndom), the domain's waves taking its blocked order in turn, and that
//    order visiting block c of every band before block c + 1.
#include <cstdio>
#include <vector>

#include "naj_lists.h"

static int fail(const char* what, long long a, long long b) {
  std::printf("FAIL %s (%lld, %lld)\n", what, a, b);
  return 1;
}

int main() {
  long checked = 0;
  // balanced lists
  const int wave_opts[] = {1, 3, 64, 3072};
  const long long item_opts[] = {1, 2, 7, 100, 5000};
  for (int waves : wave_opts)
    for (long long n : item_opts) {
      std::vector<int64_t> cost((size_t)n);
      for (long long i = 0; i < n; ++i) cost[(size_t)i] = 1 + (i * 7919) % 53 + (i < 5 ? 400 : 0);
      std::vector<int32_t> off, items;
      naj::balanced_wave_lists(cost, waves, off, items);
      if ((long long)off.size() != waves + 1 || off[0] != 0 || off[waves] != n) return fail("balanced offsets", waves, n);
      std::vector<int> hits((size_t)n, 0);
      int64_t maxc = 0, lo = INT64_MAX, hi = 0;
      for (long long i = 0; i < n; ++i) maxc = std::max(maxc, cost[(size_t)i]);
      for (int w = 0; w < waves; ++w) {
        int64_t load = 0;
        for (int i = off[w]; i < off[w + 1]; ++i) {
          if (items[i] < 0 || items[i] >= n) return fail("balanced item range", w, items[i]);
          if (i > off[w] && items[i] <= items[i - 1]) return fail("balanced list not increasing", w, i);
          hits[(size_t)items[i]] += 1;
          load += cost[(size_t)items[i]];
        }
        lo = std::min(lo, load);
        hi = std::max(hi, load);
      }
      for (long long i = 0; i < n; ++i)
        if (hits[(size_t)i] != 1) return fail("balanced item count", i, hits[(size_t)i]);
      if (n >= waves && hi > lo + maxc) return fail("balanced LPT bound", hi, lo + maxc);
      ++checked;
    }
  // blocked lists
  const int dom_opts[] = {1, 2, 8};
  const int grid_opts[] = {1, 7, 8, 16, 24, 768};
  const int wpb_opts[] = {4, 8};
  const long long ns_opts[] = {1, 63, 400, 1000, 4096, 8000, 13824};
  const long long band_opts[] = {25, 36, 256, 400, 576};
  const long long blk_opts[] = {8, 32};
  for (int nd : dom_opts)
    for (int G : grid_opts)
      for (int wpb : wpb_opts)
        for (long long ns : ns_opts)
          for (long long band : band_opts)
            for (long long blk : blk_opts) {
              std::vector<int32_t> off, items;
              const bool built = naj::blocked_wave_lists(ns, 0, band, blk, nd, G, wpb, off, items);
              if (band <= blk) {
                if (built) return fail("blocked lists built for a band within one block", band, blk);
                continue;
              }
              if (!built) return fail("blocked lists not built", band, blk);
              const int waves = G * wpb;
              if ((int)off.size() != waves + 1 || off[waves] != ns) return fail("blocked offsets", waves, ns);
              const int ndom = naj::effective_domains(G, nd);
              const int nwd = G / ndom * wpb;
              std::vector<int> hits((size_t)ns, 0);
              for (int w = 0; w < waves; ++w) {
                const int wg = w / wpb, d = wg % ndom;
                const long long lo = ns * d / ndom, hi = ns * (d + 1) / ndom;
                for (int i = off[w]; i < off[w + 1]; ++i) {
                  const long long s = items[i];
                  if (s < lo || s >= hi) return fail("blocked slice outside its domain", w, s);
                  hits[(size_t)s] += 1;
                }
              }
              for (long long s = 0; s < ns; ++s)
                if (hits[(size_t)s] != 1) return fail("blocked slice count", s, hits[(size_t)s]);
              // rebuild each domain's order from the lists (position k is wave k mod nwd's (k / nwd)-th
              // item) and check that block indices never decrease along it
              for (int d = 0; d < ndom; ++d) {
                const long long lo = ns * d / ndom, hi = ns * (d + 1) / ndom;
                long long prev_c = -1, prev_z = -1;
                for (long long k = 0; k < hi - lo; ++k) {
                  const int q = (int)(k % nwd);
                  const int w = (q / wpb) * ndom + d;
                  const int wave = w * wpb + q % wpb;
                  const int idx = off[wave] + (int)(k / nwd);
                  if (idx >= off[wave + 1]) return fail("blocked order shorter than the domain", d, k);
                  const long long s = items[idx];
                  const long long c = (s % band) / blk, z = s / band;
                  if (c < prev_c || (c == prev_c && z < prev_z)) return fail("blocked order", s, k);
                  prev_c = c;
                  prev_z = z;
                }
              }
              ++checked;
            }
  std::printf("ok %ld shapes\n", checked);
  return 0;
}
