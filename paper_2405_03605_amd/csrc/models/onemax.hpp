// Genome model 1: OneMax on a 64-bit string; the fitness is the number of
// one bits. Included by models.hpp.
#pragma once

namespace ga {

struct OneMaxEval {
  __device__ static float evaluate(uint32_t p0, uint32_t p1) {
    return (float)(__popc(p0) + __popc(p1));
  }
};
using OneMaxModel = StringModel<OneMaxEval>;

}  // namespace ga
