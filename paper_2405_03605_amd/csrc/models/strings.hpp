// Shared parts of the genome models that carry a 64-bit string (words P0,
// P1; bit b is bit b % 32 of word b / 32) beside the fitness: founders draw
// the string, mutation flips one bit, and the fitness is re-evaluated after
// every flip. A string model supplies only its evaluate(p0, p1).
// Included by models.hpp.
#pragma once

namespace ga {

template <typename Eval>
struct StringModel {
  static constexpr bool kString = true;

  // founders: words 0 and 1 of the agent's sampling-stream block at
  // generation 2^64 - 1 (a counter no generation reaches), and their fitness
  __device__ static void initialize(Genome& g, const Block& draw) {
    g.P0 = draw.x;
    g.P1 = draw.y;
    g.f = Eval::evaluate(draw.x, draw.y);
  }

  __device__ static float evaluate(const Genome& g) { return Eval::evaluate(g.P0, g.P1); }

  // with the same probability p as the fitness-valued genome (word 2 of the
  // selection block below p32), flip bit (w3 mod 64): the bits the fitness
  // delta would use, disjoint from the differentia bit (w3's top bit)
  __device__ static void mutate(Genome& c, const Block& r, const MutateArgs& a) {
    if (r.z < a.p32) {
      const uint32_t bit = r.w & 63u;
      const uint32_t mask = 1u << (bit & 31u);
      c.P0 ^= bit < 32u ? mask : 0u;
      c.P1 ^= bit < 32u ? 0u : mask;
      c.f = Eval::evaluate(c.P0, c.P1);
    }
  }
};

}  // namespace ga
