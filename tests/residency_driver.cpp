// Host driver for the pump admission rule (paper_2509_01425_amd/csrc/residency.h):
// reads cases "cap new_wgs n" followed by n lines "wgs done same_stream shares_channel"
// from stdin and prints the indices of the launches to wait for, one line per case.
#include <cstdio>
#include <vector>

#include "residency.h"

int main() {
  unsigned long long cap, nw, n;
  while (std::scanf("%llu %llu %llu", &cap, &nw, &n) == 3) {
    std::vector<hicr::LiveLaunch> live(n);
    for (auto &l : live) {
      unsigned long long w;
      int d, s, c;
      if (std::scanf("%llu %d %d %d", &w, &d, &s, &c) != 4) return 1;
      l.wgs = w;
      l.done = d != 0;
      l.same_stream = s != 0;
      l.shares_channel = c != 0;
    }
    const std::vector<size_t> w = hicr::residency_waits(live, nw, cap);
    std::printf("%zu", w.size());
    for (size_t i : w) std::printf(" %zu", i);
    std::printf("\n");
  }
  return 0;
}
