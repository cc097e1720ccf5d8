// Black-box Philox4x32-10 from PyTorch's header-only engine, used to pin the
// oracle's generator.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin and
// prints the four output words.  torch maps key = seed, counter = (offset, subsequence).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::Philox4_32 e(k0 | (k1 << 32), c2 | (c3 << 32), c0 | (c1 << 32));
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
