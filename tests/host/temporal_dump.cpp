// Prints the library's host-side dG(r) constants for r = 0..3 as JSON lines
// (one per r), for comparison with the oracle.
#include <cstdio>

#include "temporal.h"

static void arr(const char* name, const double* v, int n, bool last = false) {
  std::printf("\"%s\": [", name);
  for (int i = 0; i < n; ++i) std::printf("%s%.17g", i ? ", " : "", v[i]);
  std::printf("]%s", last ? "" : ", ");
}

int main() {
  for (int r = 0; r <= 3; ++r) {
    const bt::TemporalConstants c = bt::make_temporal(r);
    std::printf("{\"r\": %d, ", r);
    arr("s", c.s, 4); arr("w", c.w, 4); arr("T", c.T, 16); arr("g", c.g, 4);
    arr("Q", c.Q, 16); arr("Qi", c.Qi, 16); arr("alpha", c.alpha, 4); arr("beta", c.beta, 4, true);
    std::printf("}\n");
  }
  return 0;
}
