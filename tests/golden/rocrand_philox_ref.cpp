// Host-side reference for Philox4x32-10 taken from the open-source rocRAND
// engine, used only by the oracle's pin tests. Reads lines of six hex words
// (ctr0..3, key0..1) on stdin and prints the four output words of the block.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct philox_block : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  philox_block p;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 out = p.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", out.x, out.y, out.z, out.w);
  }
  return 0;
}
