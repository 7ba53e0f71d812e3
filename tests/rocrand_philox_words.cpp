// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, as
// an independent check of the oracle's Philox.  rocRAND's engine takes
// (seed, subsequence, offset): key = seed, counter words 0-1 = offset / 4,
// counter words 2-3 = subsequence.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal)
// on stdin and prints the 4 output words in decimal.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const unsigned long long seed = k0 | (k1 << 32);
    const unsigned long long subsequence = c2 | (c3 << 32);
    const unsigned long long offset = (c0 | (c1 << 32)) * 4ull;
    rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
    const uint4 v = e.next4();
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
