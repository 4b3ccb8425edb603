// Cross-check helper for the oracle's Philox4x32-10: runs rocRAND's header
// implementation (rocrand/rocrand_philox4x32_10.h) on the host.
// stdin: lines "c0 c1 c2 c3 k0 k1"; stdout: the 4 outputs of that block.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  probe p;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 o = p.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
