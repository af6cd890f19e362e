// Prints the library's host-side dG(r) constants for r = 0..3 as JSON lines
// (one per r), for comparison with the oracle, with the preconditioner's level
// order (Q's order and the two-pass order of the square-block factorisation).
#include <cstdio>

#include "temporal.h"

static void arr(const char* name, const double* v, int n, bool last = false) {
  std::printf("\"%s\": [", name);
  for (int i = 0; i < n; ++i) std::printf("%s%.17g", i ? ", " : "", v[i]);
  std::printf("]%s", last ? "" : ", ");
}
static void iarr(const char* name, const int* v, int n) {
  std::printf("\"%s\": [", name);
  for (int i = 0; i < n; ++i) std::printf("%s%d", i ? ", " : "", v[i]);
  std::printf("], ");
}
static void order(const char* name, const bt::LevelOrder& o) {
  std::printf("\"%s\": {", name);
  iarr("perm", o.perm, 4); iarr("first", o.first, o.npairs); iarr("second", o.second, o.npairs);
  arr("beta", o.beta, o.npairs, true);
  std::printf("}, ");
}

int main() {
  for (int r = 0; r <= 3; ++r) {
    const bt::TemporalConstants c = bt::make_temporal(r);
    std::printf("{\"r\": %d, ", r);
    order("order_q", bt::level_order(c, false));
    order("order_pass", bt::level_order(c, true));
    arr("s", c.s, 4); arr("w", c.w, 4); arr("T", c.T, 16); arr("g", c.g, 4);
    arr("Q", c.Q, 16); arr("Qi", c.Qi, 16); arr("alpha", c.alpha, 4); arr("beta", c.beta, 4, true);
    std::printf("}\n");
  }
  return 0;
}
