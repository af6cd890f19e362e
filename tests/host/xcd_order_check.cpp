// Host-only check of the XCD-aware tile order (common.h): for every list
// length, workgroup b -> tile xcd_tile(b, n) is a permutation of 0..n-1, and
// the workgroups of each XCD (b % 8) take one contiguous, increasing run.
#include <cstdio>
#include <vector>

#include "common.h"

int main() {
  for (long long n = 1; n <= 2000; ++n) {
    std::vector<int> seen(n, 0);
    std::vector<long long> last(bt::kXcds, -1), first(bt::kXcds, -1), count(bt::kXcds, 0);
    for (long long b = 0; b < n; ++b) {
      const long long t = bt::xcd_tile(b, n);
      if (t < 0 || t >= n || seen[t]++) {
        std::printf("n=%lld: tile %lld of workgroup %lld out of range or repeated\n", n, t, b);
        return 1;
      }
      const int x = (int)(b % bt::kXcds);
      if (last[x] >= 0 && t != last[x] + 1) {
        std::printf("n=%lld: XCD %d run not contiguous at workgroup %lld\n", n, x, b);
        return 1;
      }
      if (first[x] < 0) first[x] = t;
      last[x] = t;
      ++count[x];
    }
    // runs follow each other in XCD order
    long long next = 0;
    for (int x = 0; x < bt::kXcds; ++x) {
      if (count[x] == 0) continue;
      if (first[x] != next) {
        std::printf("n=%lld: XCD %d run starts at %lld, expected %lld\n", n, x, first[x], next);
        return 1;
      }
      next += count[x];
    }
  }
  std::printf("ok\n");
  return 0;
}
