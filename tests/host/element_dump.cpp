// Prints the library's host-side element matrices (tau = 1) for a 2D and a 3D
// box cell as JSON lines, for comparison with the oracle.
#include <cstdio>
#include <vector>

#include "element.h"

static void arr(const char* name, const std::vector<double>& v, bool last = false) {
  std::printf("\"%s\": [", name);
  for (size_t i = 0; i < v.size(); ++i) std::printf("%s%.17g", i ? ", " : "", v[i]);
  std::printf("]%s", last ? "" : ", ");
}

int main() {
  const double h[3] = {0.3, 0.7, 1.1};
  for (int d = 2; d <= 3; ++d) {
    std::printf("{\"d\": %d, ", d);
    arr("A", bt::elast_element(d, h, 1.3, 0.7, 1.0));
    arr("E", bt::coupling_element(d, h), true);
    std::printf("}\n");
  }
  return 0;
}
