// Device building blocks of the generation step, shared by every kernel
// family (per-generation streaming, LDS-resident tiles, asynchronous, batched):
// the counter-based RNG, the surface policy, cross-lane permutes, the torus
// geometry, coherent word accesses, and `breed`, the per-child part of a
// generation (tournament, copy, mutation, stratum deposit; paper Sec. 2).
#pragma once

#include <type_traits>

#include "ga_internal.hpp"

namespace ga {

constexpr uint32_t kMulA = 0xD2511F53u;   // Philox4x32 round multipliers
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;  // key schedule increments
constexpr uint32_t kWeylB = 0xBB67AE85u;

constexpr uint32_t kStreamSelect = 0u;
constexpr uint32_t kStreamMigrate = 1u;
constexpr uint32_t kStreamSample = 2u;
constexpr uint32_t kStreamMutate = 3u;

struct Block {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one gfx950 three-input bitwise op (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), rounds FIRST..9 applied
// to counter state (c0..c3) with the round-0 key (k0, k1): each round takes both
// halves of two 32x32->64 products and mixes the high halves with the other
// two words and the round key (k + round * Weyl increment).
template <int FIRST>
__device__ __forceinline__ Block philox_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = FIRST; round < 10; ++round) {
    const uint64_t pa = (uint64_t)kMulA * c0;
    const uint64_t pb = (uint64_t)kMulB * c2;
    const uint32_t n0 = xor3(hi32(pb), c1, k0 + (uint32_t)round * kWeylA);
    const uint32_t n2 = xor3(hi32(pa), c3, k1 + (uint32_t)round * kWeylB);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ Block philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
  return philox_rounds<0>(c0, c1, c2, c3, k0, k1);
}

// Per-child stream blocks for one lane across a chunk. The counter is
// (slot, island, t_lo, t_hi*4 + stream): only the island word changes between a lane's
// iterations, so everything of rounds 0-2 that does not depend on it is
// computed once. The remaining per-block cost is 2 + 7*2 products and 3 + 7*2
// three-input ops.
struct SelectStream {
  uint32_t x0;      // round 0: c0' = x0 ^ island
  uint32_t inv_a;   // round 1: c2'' = hi(M0*c0') ^ inv_a
  uint32_t inv_b;   // round 2: c0''' = hi(M1*c2'') ^ inv_b
  uint32_t inv_c;   // round 2: c2''' = inv_c ^ lo(M0*c0')
  uint32_t inv_d;   // round 2: c3''' = inv_d
  uint32_t k0, k1;

  __device__ __forceinline__ void init(uint32_t slot, uint32_t t_lo, uint32_t t_hi4, uint32_t key0,
                                       uint32_t key1, uint32_t stream) {
    k0 = key0;
    k1 = key1;
    // round 0 on (slot, island, t_lo, t_hi4)
    const uint64_t pa0 = (uint64_t)kMulA * slot;
    const uint64_t pb0 = (uint64_t)kMulB * t_lo;
    x0 = hi32(pb0) ^ key0;                       // c0' = hi(pb0) ^ island ^ k0
    const uint32_t c1_1 = (uint32_t)pb0;
    const uint32_t c2_1 = hi32(pa0) ^ (t_hi4 | stream) ^ key1;
    const uint32_t c3_1 = (uint32_t)pa0;
    // round 1: pb1 from c2_1 is invariant; pa1 from c0' is not
    const uint64_t pb1 = (uint64_t)kMulB * c2_1;
    const uint32_t c0_2 = hi32(pb1) ^ c1_1 ^ (key0 + kWeylA);
    const uint32_t c1_2 = (uint32_t)pb1;
    inv_a = c3_1 ^ (key1 + kWeylB);              // c2_2 = hi(pa1) ^ inv_a, c3_2 = lo(pa1)
    // round 2: pa2 from c0_2 is invariant; pb2 from c2_2 is not
    const uint64_t pa2 = (uint64_t)kMulA * c0_2;
    inv_b = c1_2 ^ (key0 + 2u * kWeylA);         // c0_3 = hi(pb2) ^ inv_b
    inv_c = hi32(pa2) ^ (key1 + 2u * kWeylB);    // c2_3 = inv_c ^ c3_2
    inv_d = (uint32_t)pa2;                       // c3_3
  }

  __device__ __forceinline__ Block block(uint32_t island) const {
    const uint32_t c0_1 = x0 ^ island;
    const uint64_t pa1 = (uint64_t)kMulA * c0_1;
    const uint32_t c2_2 = hi32(pa1) ^ inv_a;
    const uint32_t c3_2 = (uint32_t)pa1;
    const uint64_t pb2 = (uint64_t)kMulB * c2_2;
    const uint32_t c0_3 = hi32(pb2) ^ inv_b;
    const uint32_t c1_3 = (uint32_t)pb2;
    const uint32_t c2_3 = inv_c ^ c3_2;
    return philox_rounds<3>(c0_3, c1_3, c2_3, inv_d, k0, k1);
  }
};

// One agent's genome in registers: fitness, deposit counter, surface words
// and, for a genome model with a string, its two words.
struct Genome {
  float f = 0.f;
  uint32_t T = 0, D0 = 0, D1 = 0;
  uint32_t P0 = 0, P1 = 0;
};

// What a model's mutate may use beyond the child's selection-stream block:
// the mutation probability (and the treatment law's thresholds) and, for
// draws of its own, the lane's mutation stream at the child's island.
struct MutateArgs {
  uint32_t p32, law, p_ben, p_any;
  const SelectStream* mut;
  uint32_t island;
};

}  // namespace ga

#include "models/models.hpp"

namespace ga {

// Site written by the deposit of stratum rank r on S = 2^s sites when r >= S
// and r is a multiple of 2^e, e = bitlen(r) - s ("doubling steady" surface):
// the j-th rank written in epoch e takes over the site of rank (2j+1) << (e-1),
// which left the retained set when epoch e began. Written ranks have the form
// odd << shift, so the walk only renormalises the odd part until the rank
// falls below S.
static __device__ __noinline__ uint32_t surface_site_walk(uint32_t r, uint32_t e, uint32_t s) {
  const uint32_t half = 1u << (s - 1u);
  uint32_t odd = (((r >> e) - half) << 1) | 1u;
  uint32_t shift = e - 1u;
  for (;;) {
    const uint32_t len = 32u - __clz(odd);
    if (len + shift <= s) return odd << shift;
    const uint32_t lead = odd << (s - len);  // rank >> its epoch, in [S/2, S)
    shift = len + shift - s - 1u;
    odd = ((lead - half) << 1) | 1u;
  }
}

__device__ __forceinline__ uint32_t permute(uint32_t value, uint32_t byte_addr) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)byte_addr, (int)value);
}
__device__ __forceinline__ float permute(float value, uint32_t byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((int)byte_addr, __float_as_int(value)));
}

// Island next to (x, y) in direction q on the W x H torus:
// 0 north (y-1), 1 east (x+1), 2 south (y+1), 3 west (x-1).
__device__ __forceinline__ void torus_xy(uint32_t x, uint32_t y, uint32_t q, uint32_t W,
                                         uint32_t H, uint32_t* nx, uint32_t* ny) {
  const uint32_t xe = (x + 1u == W) ? 0u : x + 1u;
  const uint32_t xw = (x == 0u ? W : x) - 1u;
  const uint32_t yn = (y == 0u ? H : y) - 1u;
  const uint32_t ys = (y + 1u == H) ? 0u : y + 1u;
  *nx = q == 1u ? xe : (q == 3u ? xw : x);
  *ny = q == 0u ? yn : (q == 2u ? ys : y);
}
__device__ __forceinline__ uint32_t torus_step(uint32_t x, uint32_t y, uint32_t q, uint32_t W,
                                               uint32_t H) {
  uint32_t nx, ny;
  torus_xy(x, y, q, W, H, &nx, &ny);
  return ny * W + nx;
}

template <typename P>
__device__ __forceinline__ P* at_byte(P* base, uint32_t byte_off) {
  return reinterpret_cast<P*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename P>
__device__ __forceinline__ const P* at_byte(const P* base, uint32_t byte_off) {
  return reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Word accesses to memory that other workgroups (on any XCD) read and write
// while this one runs: relaxed atomics at device scope. Each such access is
// coherent across the XCDs by itself (its scope bits send it past the per-XCD
// L2's non-coherent state), so ordering two of them only needs the first to
// have completed before the second issues: drain_memory() waits for every
// memory access this wavefront has in flight. A device-scope fence would do
// the same but also write back and invalidate the whole L2 of the XCD, which
// under thousands of wavefronts streaming the population costs far more than
// the exchange itself.
__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t value) {
  __hip_atomic_store(p, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Two words at once (8-byte aligned), for entries whose stability the
// exchange protocol already guarantees while they are read.
__device__ __forceinline__ uint2 load_agent2(const uint32_t* p) {
  const uint64_t x = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
}
__device__ __forceinline__ void store_agent2(uint32_t* p, uint32_t lo, uint32_t hi) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), ((uint64_t)hi << 32) | lo, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void drain_memory() {
  // also a compiler barrier: no memory access moves across it
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// The dispatcher hands workgroups to the eight XCDs in turn (group g to XCD
// g mod 8), each XCD with its own L2. Renumbering the groups so that every XCD
// takes one contiguous band of the grid keeps an island's four neighbours, and
// the outbox entries it reads from them, mostly on its own XCD.
// The renumbering of groups g < n (a permutation of [0, n)), for grids whose
// first n groups are the ones with work.
__device__ __forceinline__ uint32_t xcd_band(uint32_t g, uint32_t n) {
  const uint32_t x = g & 7u, q = n >> 3, r = n & 7u;
  return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + (g >> 3);
}
__device__ __forceinline__ uint32_t xcd_band_group() { return xcd_band(blockIdx.x, gridDim.x); }

// Per-lane constants of one generation's children: the lane's slot in its
// island, the permute address of slot 0 of that island, and the selection
// (and, under the treatment law, mutation) stream with everything hoisted
// that depends only on the slot and the generation.
struct BreedLane {
  uint32_t slot;
  uint32_t lane0_addr;
  uint32_t t_lo, t_hi4;
  SelectStream sel, mut;
  // the mutation thresholds, compared lane by lane: held in vector registers
  // so that the loops do not keep (or reload) them in scalar ones
  uint32_t p32, p_ben, p_any;
};

// A copy of a wavefront-uniform value in a vector register.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
  uint32_t r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

template <int LC>
__device__ __forceinline__ BreedLane breed_lane(const RunView& v, uint64_t t) {
  const uint32_t L = LC >= 0 ? (uint32_t)LC : v.log2n;
  const uint32_t lane = __lane_id();
  BreedLane b;
  b.slot = lane & ((1u << L) - 1u);
  b.lane0_addr = (lane & ~((1u << L) - 1u)) << 2;
  b.t_lo = (uint32_t)t;
  b.t_hi4 = (uint32_t)(t >> 32) << 2;
  b.sel.init(b.slot, b.t_lo, b.t_hi4, v.seed, v.run_id, kStreamSelect);
  if (v.law) b.mut.init(b.slot, b.t_lo, b.t_hi4, v.seed, v.run_id, kStreamMutate);
  b.p32 = in_vgpr(v.p32);
  b.p_ben = in_vgpr(v.p_ben);
  b.p_any = in_vgpr(v.p_any);
  return b;
}

// Steps 3-7 of generation t for the child in this lane's slot of `island`
// (paper Sec. 2): evaluation (the fitness word), a tournament of k entrants
// drawn with replacement from the lane's island (first strict maximum in draw
// order wins; neutral runs take entrant 0), the winner's genome copied by
// cross-lane permutes, the model's mutation, and one stratum deposit at rank
// T followed by T + 1. `g` is this lane's post-immigration genome; every lane
// of the wavefront must call this together (the permutes read all lanes).
// LC / SWC: log2 N and surface words fixed at compile time, or -1 to read
// them from the view.
template <int LC, int SWC, typename Model, bool WIDE>
__device__ __forceinline__ Genome breed(const RunView& v, const BreedLane& b, const Genome& g,
                                        uint32_t island) {
  const uint32_t L = LC >= 0 ? (uint32_t)LC : v.log2n;
  const uint32_t SW = SWC >= 0 ? (uint32_t)SWC : v.words;
  // surface: S = 2^s_log sites of 2^dlog-bit differentia under the steady
  // policy; one bit on 32 or 64 sites is fixed at compile time, WIDE reads
  // the width, the site count and the policy from the view
  const uint32_t dlog = WIDE ? v.dlog : 0u;
  const bool tilted = WIDE && v.policy == 1u;
  const bool hybrid = WIDE && v.policy == 2u;
  const uint32_t s_log = WIDE ? v.s_log : 4u + SW;

  // 3-5. evaluate (read fitness) and run the tournament over permuted entrants
  const Block r = b.sel.block(island);
  uint32_t best = b.lane0_addr + (((r.x & 0xFFu) >> (8u - L)) << 2);
  float fbest = permute(g.f, best);
  // entrants 1..k-1: bytes 1..7 of (w0, w1), little-endian. Entrant 1 is
  // taken apart (k = 2 is the common size), the rest in a uniform loop (no
  // per-entrant condition kept live across the caller's loop).
  const uint32_t k = v.selection ? v.k : 1u;
  if (k > 1u) {
    const uint32_t cand = b.lane0_addr + ((((r.x >> 8) & 0xFFu) >> (8u - L)) << 2);
    const float fc = permute(g.f, cand);
    if (fc > fbest) {
      best = cand;
      fbest = fc;
    }
    uint64_t rest = (((uint64_t)r.y << 32) | r.x) >> 16;
    for (uint32_t m = 2; m < k; ++m) {
      const uint32_t cand_m = b.lane0_addr + ((((uint32_t)rest & 0xFFu) >> (8u - L)) << 2);
      rest >>= 8;
      const float fm = permute(g.f, cand_m);
      if (fm > fbest) {
        best = cand_m;
        fbest = fm;
      }
    }
  }
  Genome c;
  c.T = permute(g.T, best);
  c.D0 = permute(g.D0, best);
  c.D1 = SW > 1 ? permute(g.D1, best) : 0u;
  if (Model::kString) {
    c.P0 = permute(g.P0, best);
    c.P1 = permute(g.P1, best);
  }
  c.f = fbest;

  // 6. mutation, by the genome model
  MutateArgs ma{b.p32, v.law, b.p_ben, b.p_any, &b.mut, island};
  Model::mutate(c, r, ma);

  // 7. stratum deposit at rank T, then T + 1. The hybrid policy sends even
  //    ranks 2q to a 32-site steady half (sites 0..31) and odd ranks 2q + 1
  //    to a 32-site tilted half (sites 32..63), each as its rank q.
  uint32_t q = c.T, q_log = s_log, site_base = 0u;
  bool on_tilted = tilted;
  if (hybrid) {
    q = c.T >> 1;
    q_log = 5u;
    on_tilted = (c.T & 1u) != 0u;
    site_base = on_tilted ? 32u : 0u;
  }
  uint32_t site = q;
  bool write = true;
  if (on_tilted) {
    // level k = trailing zeros of q (capped at 31; q = 0 counts as 31), slot
    // (q >> (k+1)) mod m ((q >> 31) mod m on level 31), m = sites / 32
    const uint32_t m_log = q_log - 5u;
    const uint32_t k = q ? min((uint32_t)__ffs(q) - 1u, 31u) : 31u;
    const uint32_t ring = (k < 31u ? q >> (k + 1u) : q >> 31) & ((1u << m_log) - 1u);
    site = (k << m_log) + ring;
  } else if (q >= (1u << q_log)) {
    const uint32_t e = (32u - __clz(q)) - q_log;
    write = (q & ((1u << e) - 1u)) == 0u;
    if (write) site = surface_site_walk(q, e, q_log);
  }
  site += site_base;
  if (write) {
    // the differentia: one bit, the top bit of the selection block's w3;
    // b = 2^dlog > 1 bits, the top b bits of word 0 of a block of their own
    // (mutation stream, counter word 0 = slot + 256), drawn only by the
    // lanes that write
    const uint32_t pos = site << dlog;
    uint32_t value = r.w >> 31;
    if (WIDE && dlog != 0u)
      value = philox10(b.slot + 256u, island, b.t_lo, b.t_hi4 | kStreamMutate, v.seed, v.run_id).x >>
              (32u - (1u << dlog));
    const uint32_t field = ((2u << ((1u << dlog) - 1u)) - 1u) << (pos & 31u);
    const uint32_t bits = value << (pos & 31u);
    if (SW == 1 || pos < 32u) {
      c.D0 = (c.D0 & ~field) | bits;
    } else {
      c.D1 = (c.D1 & ~field) | bits;
    }
  }
  c.T += 1u;
  return c;
}

// ---------------------------------------------------------------------------
// Host-side dispatch to a kernel's compile-time shape.
// ---------------------------------------------------------------------------
template <int V>
using IntC = std::integral_constant<int, V>;
template <bool V>
using BoolC = std::integral_constant<bool, V>;

template <typename M, bool WD, typename F>
hipError_t dispatch_shapes(uint32_t L, uint32_t SW, F& f) {
  switch (L * 2u + (SW - 1u)) {
    case 0: return f(IntC<0>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 1: return f(IntC<0>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 2: return f(IntC<1>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 3: return f(IntC<1>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 4: return f(IntC<2>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 5: return f(IntC<2>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 6: return f(IntC<3>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 7: return f(IntC<3>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 8: return f(IntC<4>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 9: return f(IntC<4>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 10: return f(IntC<5>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 11: return f(IntC<5>{}, IntC<2>{}, M{}, BoolC<WD>{});
    case 12: return f(IntC<6>{}, IntC<1>{}, M{}, BoolC<WD>{});
    case 13: return f(IntC<6>{}, IntC<2>{}, M{}, BoolC<WD>{});
    default: return hipErrorInvalidValue;
  }
}

// Calls f(IntC<log2 N>, IntC<surface words>, Model, BoolC<wide differentia
// or another policy>) for the run's shape; f returns a hipError_t. Every
// kernel family is instantiated for every model of GA_FOR_EACH_MODEL.
template <typename F>
hipError_t dispatch(const RunView& v, F&& f) {
  const bool wide = v.dlog != 0u || v.policy != 0u;
#define GA_MODEL_CASE(ID, M)                                                   \
  case ID:                                                                     \
    return wide ? dispatch_shapes<M, true>(v.log2n, v.words, f)                \
                : dispatch_shapes<M, false>(v.log2n, v.words, f);
  switch (v.model) {
    GA_FOR_EACH_MODEL(GA_MODEL_CASE)
    default: return hipErrorInvalidValue;
  }
#undef GA_MODEL_CASE
}

// The template arguments of a kernel from dispatch's tag arguments
#define GA_SHAPE_ARGS(LC, SWC, M, WD) \
  decltype(LC)::value, decltype(SWC)::value, decltype(M), decltype(WD)::value

}  // namespace ga
