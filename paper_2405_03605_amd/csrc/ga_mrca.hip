// All-pairs MRCA-interval estimation from hereditary-stratigraphy surfaces on
// gfx950: the primitive under post hoc phylogenetic reconstruction (paper
// Fig. 1: markers on genomes let relatedness be estimated after the run; Sec. 3
// reconstructs from 10k sampled end-state genomes).
//
// For two surfaces with deposit counters Ta, Tb on S sites, the ranks both
// retain are the multiples of 2^e, e = max(e(Ta), e(Tb)), below min(Ta, Tb)
// (e(n) = max(0, ceil(log2 n) - log2 S), "doubling steady" surface). Ranks
// older than the MRCA hold identical differentia, so the first common rank
// whose differentia differ bounds the MRCA's counter from above (U); kc
// matching common ranks in a row below U make an MRCA earlier than them a
// 2^-(b kc) event for b-bit differentia (L).
//
// Layout of the work: `normalize_kernel` turns each surface into its retained
// differentia in rank order (field j, b bits wide, = rank j * 2^e(T)), a
// 64-bit string (S * b <= 64); for one-bit differentia the pair kernel keeps
// every 2^(e - e(T))-th bit of each string (stride compaction), XORs them and
// takes the lowest set bit, O(1) per pair; wider fields are compared field by
// field up to the first mismatch (at most S <= 32 of them). Integer only.
#include "ga_internal.hpp"

namespace ga {
namespace {

struct Normalized {
  unsigned long long bits;  // retained differentia in rank order
  uint32_t T;
  uint32_t epoch;
};

__device__ __forceinline__ uint32_t epoch_of(uint32_t n, uint32_t s) {
  // max(0, ceil(log2 n) - s); ceil(log2 n) = bitlen(n - 1) for n >= 1
  const uint32_t c = n <= 1u ? 0u : 32u - __clz(n - 1u);
  return c > s ? c - s : 0u;
}

// Site of rank r (a retained rank, so never a discard): ranks below S keep
// site r; otherwise walk to the rank whose site the j-th rank of its epoch
// took over, as in the generation step's deposit.
__device__ uint32_t site_of_retained(uint32_t r, uint32_t s) {
  const uint32_t half = 1u << (s - 1u);
  if (r < (half << 1)) return r;
  const uint32_t e = (32u - __clz(r)) - s;
  uint32_t odd = (((r >> e) - half) << 1) | 1u;
  uint32_t shift = e - 1u;
  for (;;) {
    const uint32_t len = 32u - __clz(odd);
    if (len + shift <= s) return odd << shift;
    const uint32_t lead = odd << (s - len);
    shift = len + shift - s - 1u;
    odd = ((lead - half) << 1) | 1u;
  }
}

__global__ void normalize_kernel(const uint32_t* __restrict__ T, const uint32_t* __restrict__ D,
                                 uint32_t n, uint32_t s, uint32_t dlog, Normalized* out) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const uint32_t words = (1u << (s + dlog)) >> 5;  // S * b / 32
  const uint32_t b = 1u << dlog;
  const unsigned long long fmask = (1ull << b) - 1ull;
  const uint32_t t = T[a];
  const uint32_t e = epoch_of(t, s);
  const uint32_t count = t == 0u ? 0u : ((t - 1u) >> e) + 1u;  // ceil(t / 2^e) <= S
  const unsigned long long w = (unsigned long long)D[(size_t)a * words] |
                               (words > 1 ? (unsigned long long)D[(size_t)a * words + 1] << 32
                                          : 0ull);
  unsigned long long bits = 0ull;
  for (uint32_t j = 0; j < count; ++j) {
    const uint32_t site = site_of_retained(j << e, s);
    bits |= ((w >> (site << dlog)) & fmask) << (j << dlog);
  }
  out[a] = Normalized{bits, t, e};
}

// keep bits 0, 2^d, 2*2^d, ... of x, packed to the bottom
__device__ __forceinline__ unsigned long long compact_stride(unsigned long long x, uint32_t d) {
  for (uint32_t i = 0; i < d; ++i) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  }
  return x;
}

// Interval for the pair (a, b) of normalised surfaces.
__device__ __forceinline__ uint2 pair_interval(const Normalized& a, const Normalized& b,
                                               uint32_t dlog, uint32_t kc) {
  const uint32_t e = a.epoch > b.epoch ? a.epoch : b.epoch;
  const uint32_t tmin = a.T < b.T ? a.T : b.T;
  const uint32_t common = tmin == 0u ? 0u : ((tmin - 1u) >> e) + 1u;  // ranks j*2^e < tmin
  uint32_t j = common;  // first mismatching common rank index, or common
  if (dlog == 0u) {
    const unsigned long long diff =
        compact_stride(a.bits, e - a.epoch) ^ compact_stride(b.bits, e - b.epoch);
    const unsigned long long mask = common >= 64u ? ~0ull : ((1ull << common) - 1ull);
    const unsigned long long hit = diff & mask;
    if (hit) j = (uint32_t)__ffsll((long long)hit) - 1u;
  } else if (a.epoch == b.epoch) {
    // common rank i is field i of both strings: the first differing field
    // holds the lowest set bit of the XOR
    const uint32_t used = common << dlog;  // bits of the common fields
    const unsigned long long mask = used >= 64u ? ~0ull : ((1ull << used) - 1ull);
    const unsigned long long hit = (a.bits ^ b.bits) & mask;
    if (hit) j = ((uint32_t)__ffsll((long long)hit) - 1u) >> dlog;
  } else {
    // common rank i is field i << (e - epoch) of each string
    const unsigned long long fmask = (1ull << (1u << dlog)) - 1ull;
    const uint32_t da = e - a.epoch, db = e - b.epoch;
    for (uint32_t i = 0; i < common; ++i) {
      const unsigned long long fa = (a.bits >> ((i << da) << dlog)) & fmask;
      const unsigned long long fb = (b.bits >> ((i << db) << dlog)) & fmask;
      if (fa != fb) {
        j = i;
        break;
      }
    }
  }
  const uint32_t upper = j < common ? j << e : tmin;
  const uint32_t lower = j < kc ? 0u : ((j - kc) << e) + 1u;
  return make_uint2(lower, upper);
}

// One thread per pair (x, y) in each of eight passes over 2,048 consecutive y
// (256 per pass, lane-consecutive, so loads and the two output rows are
// coalesced); rows of the grid are x.
__global__ __launch_bounds__(256) void pairs_kernel(const Normalized* __restrict__ nz, uint32_t n,
                                                    uint32_t dlog, uint32_t kc,
                                                    uint32_t* __restrict__ L,
                                                    uint32_t* __restrict__ U) {
  const uint32_t x = blockIdx.y;
  const Normalized a = nz[x];
  const size_t row = (size_t)x * n;
#pragma unroll
  for (uint32_t pass = 0; pass < 8; ++pass) {
    const uint32_t y = blockIdx.x * 2048u + pass * 256u + threadIdx.x;
    if (y < n) {
      const uint2 r = pair_interval(a, nz[y], dlog, kc);
      U[row + y] = r.y;
      L[row + y] = r.x;
    }
  }
}

// Tilted surfaces (S = 32 m sites, level k = site / m, slot j = site % m):
// the rank a slot holds after T deposits is the most recent rank below T of
// its level whose index along the level is j mod m. A rank sits at one site
// whatever T is, so the ranks two surfaces share are the slots where both
// hold the same rank.
// The rank slot j of level k holds after T deposits, or kNone. Level k < 31
// holds the odd multiples 2^k (2i + 1), level 31 the multiples i 2^31 (rank 0
// among them); slot j keeps the newest one below T with i = j mod 2^m_log.
constexpr uint32_t kNone = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t tilted_slot_rank(uint32_t T, uint32_t k, uint32_t j,
                                                     uint32_t m_log) {
  if (T == 0u) return kNone;
  const uint32_t q = (T - 1u) >> k;
  if (k < 31u && q == 0u) return kNone;
  const uint32_t imax = k < 31u ? (q - 1u) >> 1 : q;
  if (imax < j) return kNone;
  const uint32_t i = imax - ((imax - j) & ((1u << m_log) - 1u));
  return k < 31u ? ((2u * i + 1u) << k) : (i << 31);
}

// One thread per pair: U = the oldest common rank whose differentia differ
// (or min(Ta, Tb)); L = the kc-th common rank below U, plus one (0 if fewer).
// The common ranks (a rank sits at one site whatever T is, so they are the
// sites where both surfaces hold the same rank) are found once and kept in
// registers, S known at compile time.
template <uint32_t S>
__global__ __launch_bounds__(256) void pairs_tilted_kernel(const uint32_t* __restrict__ T,
                                                           const uint32_t* __restrict__ D,
                                                           uint32_t n, uint32_t dlog,
                                                           uint32_t kc,
                                                           uint32_t* __restrict__ L,
                                                           uint32_t* __restrict__ U) {
  constexpr uint32_t m_log = S == 64u ? 1u : 0u;
  const uint32_t y = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t x = blockIdx.y;
  if (y >= n) return;
  const uint32_t words = (S << dlog) >> 5;
  const uint32_t ta = T[x], tb = T[y];
  const unsigned long long wa = (unsigned long long)D[(size_t)x * words] |
                                (words > 1 ? (unsigned long long)D[(size_t)x * words + 1] << 32
                                           : 0ull);
  const unsigned long long wb = (unsigned long long)D[(size_t)y * words] |
                                (words > 1 ? (unsigned long long)D[(size_t)y * words + 1] << 32
                                           : 0ull);
  const unsigned long long fmask = (1ull << (1u << dlog)) - 1ull;
  const unsigned long long diff = wa ^ wb;
  uint32_t upper = ta < tb ? ta : tb;
  uint32_t common[S];  // the rank both hold at each site, or kNone
#pragma unroll
  for (uint32_t site = 0; site < S; ++site) {
    const uint32_t k = site >> m_log, j = site & ((1u << m_log) - 1u);
    const uint32_t ra = tilted_slot_rank(ta, k, j, m_log);
    const uint32_t rb = tilted_slot_rank(tb, k, j, m_log);
    common[site] = ra == rb ? ra : kNone;
    if (ra == rb && ra != kNone && ((diff >> (site << dlog)) & fmask) != 0ull && ra < upper)
      upper = ra;
  }
  // kc-th largest common rank below upper (the common ranks are distinct)
  uint32_t bound = upper;
  bool found = true;
  for (uint32_t c = 0; c < kc && found; ++c) {
    found = false;
    uint32_t best = 0u;
#pragma unroll
    for (uint32_t site = 0; site < S; ++site) {
      const uint32_t r = common[site];
      const bool ok = r != kNone && r < bound && (!found || r > best);
      best = ok ? r : best;
      found = found || ok;
    }
    bound = best;
  }
  const size_t at = (size_t)x * n + y;
  U[at] = upper;
  L[at] = found ? bound + 1u : 0u;
}

// Hybrid surfaces (64 one-bit sites): even ranks 2q sit on a 32-site steady
// half (sites 0..31), odd ranks 2q + 1 on a 32-site tilted half (sites
// 32..63). The common ranks of the steady halves are 2 j 2^E for
// j < common, E the larger epoch; those of the tilted halves are the slots
// holding the same rank in both. U and L as for the other policies, over the
// union of the two sets.
__global__ __launch_bounds__(256) void pairs_hybrid_kernel(const uint32_t* __restrict__ T,
                                                           const uint32_t* __restrict__ D,
                                                           uint32_t n, uint32_t kc,
                                                           uint32_t* __restrict__ L,
                                                           uint32_t* __restrict__ U) {
  const uint32_t y = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t x = blockIdx.y;
  if (y >= n) return;
  const uint32_t ta = T[x], tb = T[y];
  const unsigned long long diff =
      ((unsigned long long)D[(size_t)x * 2] | (unsigned long long)D[(size_t)x * 2 + 1] << 32) ^
      ((unsigned long long)D[(size_t)y * 2] | (unsigned long long)D[(size_t)y * 2 + 1] << 32);
  // steady halves: (t + 1) / 2 even deposits each
  const uint32_t na = (ta >> 1) + (ta & 1u), nb = (tb >> 1) + (tb & 1u);
  const uint32_t ea = epoch_of(na, 5u), eb = epoch_of(nb, 5u);
  const uint32_t E = ea > eb ? ea : eb;
  const uint32_t nmin = na < nb ? na : nb;
  const uint32_t cs = nmin == 0u ? 0u : ((nmin - 1u) >> E) + 1u;  // common steady ranks
  uint32_t upper = ta < tb ? ta : tb;
  for (uint32_t j = 0; j < cs; ++j) {
    const uint32_t q = j << E;
    if ((diff >> site_of_retained(q, 5u)) & 1ull) {
      upper = min(upper, 2u * q);
      break;
    }
  }
  // tilted halves: t / 2 odd deposits each, one slot per level; the common
  // ones (as odd ranks 2r + 1) found once and kept in registers
  const uint32_t ma = ta >> 1, mb = tb >> 1;
  uint32_t common[32];
#pragma unroll
  for (uint32_t k = 0; k < 32; ++k) {
    const uint32_t ra = tilted_slot_rank(ma, k, 0u, 0u);
    const uint32_t rb = tilted_slot_rank(mb, k, 0u, 0u);
    common[k] = ra == rb && ra != kNone ? 2u * ra + 1u : kNone;
    if (common[k] != kNone && ((diff >> (32u + k)) & 1ull) && common[k] < upper) upper = common[k];
  }
  // kc-th largest common rank below upper
  uint32_t bound = upper;
  bool found = true;
  for (uint32_t c = 0; c < kc && found; ++c) {
    found = false;
    uint32_t best = 0u;
    if (cs > 0u && bound > 0u) {
      uint32_t jm = (bound - 1u) >> (E + 1u);  // largest j with 2 j 2^E < bound
      if (jm > cs - 1u) jm = cs - 1u;
      best = 2u * (jm << E);
      found = true;
    }
#pragma unroll
    for (uint32_t k = 0; k < 32; ++k) {
      const uint32_t r = common[k];
      const bool ok = r != kNone && r < bound && (!found || r > best);
      best = ok ? r : best;
      found = found || ok;
    }
    bound = best;
  }
  const size_t at = (size_t)x * n + y;
  U[at] = upper;
  L[at] = found ? bound + 1u : 0u;
}

}  // namespace

size_t mrca_workspace_bytes(size_t n) { return n * sizeof(Normalized); }

hipError_t launch_mrca_matrix(const uint32_t* T, const uint32_t* D, uint32_t n, uint32_t s_log,
                              uint32_t dlog, uint32_t policy, uint32_t kc, void* workspace,
                              uint32_t* L, uint32_t* U, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (policy == 1u) {
    const dim3 grid((n + 255) / 256, n);
    if (s_log == 6u)
      pairs_tilted_kernel<64><<<grid, dim3(256), 0, stream>>>(T, D, n, dlog, kc, L, U);
    else if (s_log == 5u)
      pairs_tilted_kernel<32><<<grid, dim3(256), 0, stream>>>(T, D, n, dlog, kc, L, U);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (policy == 2u) {
    pairs_hybrid_kernel<<<dim3((n + 255) / 256, n), dim3(256), 0, stream>>>(T, D, n, kc, L, U);
    return hipGetLastError();
  }
  Normalized* nz = static_cast<Normalized*>(workspace);
  normalize_kernel<<<dim3((n + 255) / 256), dim3(256), 0, stream>>>(T, D, n, s_log, dlog, nz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pairs_kernel<<<dim3((n + 2047) / 2048, n), dim3(256), 0, stream>>>(nz, n, dlog, kc, L, U);
  return hipGetLastError();
}

}  // namespace ga
