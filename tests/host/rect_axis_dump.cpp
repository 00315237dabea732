// Prints the library's rectangular tilings of an axis (rect_axis and
// rect_span of csrc/engine.hpp) for every length L in [2, LMAX] and every
// half-cycle height h with L >= 2h, one line per (L, h, tiling):
//   L h par t start0 width0 start1 width1 ...
// The tests compare these spans with the oracle's model of the same tilings.
// Host code only: built with --cuda-host-only, no device is touched.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1602_07558_amd/csrc/engine.hpp"

int main(int argc, char** argv) {
  const int lmax = argc > 1 ? std::atoi(argv[1]) : 64;
  for (int L = 2; L <= lmax; ++L)
    for (int h = 1; 2 * h <= L; ++h) {
      const swept::RAxis a = swept::rect_axis(L, h);
      for (int par = 0; par < 2; ++par) {
        std::printf("%d %d %d %d", L, h, par, a.t);
        for (int i = 0; i < a.t; ++i) {
          int s = 0, w = 0;
          swept::rect_span(a, par, i, s, w);
          std::printf(" %d %d", s, w);
        }
        std::printf("\n");
      }
    }
  return 0;
}
