// Known-answer generator for the Philox4x32-10 pin: runs rocRAND's own
// implementation (an independent, published Philox4x32-10) on counters and
// keys read from stdin ("c0 c1 c2 c3 k0 k1" per line) and prints the four
// output words per line. Host code only; built with g++ by the CPU tests.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct philox_probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned a, b, c, d, e, f;
  philox_probe p;
  while (scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &e, &f) == 6) {
    uint4 o = p.block(uint4{a, b, c, d}, uint2{e, f});
    printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
