// Genome model 0: the fitness-valued genome of the paper's own runs (Sec. 3):
// the genome is its fitness value and mutation changes it directly.
// Included by models.hpp.
#pragma once

namespace ga {

struct FitnessModel {
  static constexpr bool kString = false;

  // founders: fitness +0 (the all-zero fill of a new run); nothing is drawn
  __device__ static void initialize(Genome&, const Block&) {}

  __device__ static float evaluate(const Genome& g) { return g.f; }

  // r: the child's selection-stream block; mutate iff its word 2 < p32.
  // Law 0: f + delta, delta = (hi32((w3 & 0x7FFFFFFF) * 10) - 2) / 2, i.e.
  //   uniform on {-1, -1/2, 0, 1/2, 1}.
  // Law 1 (the paper's treatments, Sec. 3): beneficial (+|Z|) iff w2 < p_ben,
  //   deleterious (-|Z|) iff p_ben <= w2 < p_any; Z is the variance-matched
  //   sum of the eight 16-bit halves of the child's mutation-stream block
  //   (Irwin-Hall n = 8), one correctly rounded product.
  __device__ static void mutate(Genome& c, const Block& r, const MutateArgs& a) {
    if (a.law == 0) {
      if (r.z < a.p32) {
        // di * 0.5 is exact, so a fused multiply-add rounds like the plain add
        const int di = (int)__umulhi(r.w & 0x7FFFFFFFu, 10u) - 2;  // -2..2
        c.f = __fadd_rn(c.f, (float)di * 0.5f);
      }
    } else {
      const bool ben = r.z < a.p_ben;
      const bool del = !ben && r.z < a.p_any;
      if (ben || del) {
        const Block m = a.mut->block(a.island);
        const uint32_t sum = (m.x & 0xFFFFu) + (m.x >> 16) + (m.y & 0xFFFFu) + (m.y >> 16) +
                             (m.z & 0xFFFFu) + (m.z >> 16) + (m.w & 0xFFFFu) + (m.w >> 16);
        const float size = fabsf(__fmul_rn((float)((int)sum - 262140), 0x1.3988e2p-16f));
        c.f = ben ? __fadd_rn(c.f, size) : __fsub_rn(c.f, size);
      }
    }
  }
};

}  // namespace ga
