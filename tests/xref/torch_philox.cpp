// Cross-check helper for the oracle's Philox4x32-10: runs ATen's header-only
// at::philox_engine (torch/include/ATen/core/PhiloxRNGEngine.h).
// stdin: lines "seed subsequence offset"; stdout: the 4 outputs of that block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cinttypes>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::philox_engine e(seed, sub, off);
    uint32_t a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
