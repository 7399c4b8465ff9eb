// Prints rocRAND's Philox4x32-10 output words for (seed, subsequence, offset) triples read
// from stdin.  rocRAND's engine is an implementation of the published generator that is
// independent of this project's; the oracle's Philox is checked against it.
// With offset = 4*c the engine's counter is (c mod 2^32, c >> 32, sub mod 2^32, sub >> 32)
// and its key is (seed mod 2^32, seed >> 32).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
