// Genome model 2: Trap-4 on a 64-bit string (Deb and Goldberg's deceptive trap
// of order 4): 16 four-bit blocks, a block with u one bits scoring 4 if u = 4,
// else 3 - u. The sum is 48 - ones + 5 * (blocks with all four bits set).
// Included by models.hpp.
#pragma once

namespace ga {

struct Trap4Eval {
  __device__ static float evaluate(uint32_t p0, uint32_t p1) {
    const uint32_t ones = __popc(p0) + __popc(p1);
    const uint32_t full0 = p0 & (p0 >> 1) & (p0 >> 2) & (p0 >> 3) & 0x11111111u;
    const uint32_t full1 = p1 & (p1 >> 1) & (p1 >> 2) & (p1 >> 3) & 0x11111111u;
    return (float)(48u - ones + 5u * (__popc(full0) + __popc(full1)));
  }
};
using Trap4Model = StringModel<Trap4Eval>;

}  // namespace ga
