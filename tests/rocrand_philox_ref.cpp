// Independent Philox4x32-10 reference for the oracle's pin: drives the
// ten-round block function of the rocRAND host/device engine (open-source
// header shipped with ROCm) on explicit (counter, key) pairs read from stdin,
// one "c0 c1 c2 c3 k0 k1" line per block, and prints the four output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Exposed : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  Exposed e;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
    uint2 k; k.x = k0; k.y = k1;
    uint4 r = e.block(c, k);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
