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
#include <mutex>

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

// Tiled pairs for the tilted and hybrid policies. U and L are symmetric in
// the two surfaces, so a workgroup takes a 64 x 64 block of pairs (rows
// x0.., columns y0..) only when y0 >= x0 and writes the block and its mirror
// image. Each lane keeps its column surface's per-site ranks in registers for
// the 16 rows its wavefront visits (the rank computation is paid once per
// lane, not once per pair); the rows' ranks are built once per workgroup in
// LDS and read back as wavefront-uniform broadcasts. The mirror image goes
// out through an LDS transpose so both writes are whole-row and coalesced.
constexpr uint32_t kPairTile = 64;
constexpr uint32_t kRowsPerWave = kPairTile / 4;

struct PairStage {
  uint32_t u[kPairTile][kPairTile + 1];  // [row in block][column in block]
  uint32_t l[kPairTile][kPairTile + 1];
};

// Row r (x = x0 + r) of the block: write (x, y) directly and keep it for the
// mirror image.
__device__ __forceinline__ void put_pair(PairStage& st, uint32_t r, uint32_t lane, uint32_t x,
                                         uint32_t y, uint32_t n, uint32_t u, uint32_t l,
                                         uint32_t* __restrict__ L, uint32_t* __restrict__ U) {
  if (x < n && y < n) {
    const size_t at = (size_t)x * n + y;
    U[at] = u;
    L[at] = l;
  }
  st.u[r][lane] = u;
  st.l[r][lane] = l;
}

// The mirror image of an off-diagonal block: (y, x) for every staged (x, y).
__device__ __forceinline__ void put_mirror(const PairStage& st, uint32_t x0, uint32_t y0,
                                           uint32_t n, uint32_t* __restrict__ L,
                                           uint32_t* __restrict__ U) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t x = x0 + lane;
  for (uint32_t c = wid * kRowsPerWave; c < (wid + 1u) * kRowsPerWave; ++c) {
    const uint32_t y = y0 + c;
    if (x < n && y < n) {
      const size_t at = (size_t)y * n + x;
      U[at] = st.u[lane][c];
      L[at] = st.l[lane][c];
    }
  }
}

// The kc passes for L over the common ranks cr[site] (kNone: the site is not
// common). Pass p takes the largest common rank below bound (U on the first
// pass, then the previous pass's rank) and keeps it plus one; a pass that
// finds none gives 0, and 0 stays. The last pass's value is L: the kc-th
// common rank below U, plus one, or 0 when there are fewer. In unsigned
// arithmetic that value is bound minus the smallest (bound - 1) - cr: a rank
// at or above the bound wraps to a difference above the bound, and kNone
// gives exactly bound (nothing found), which is also where the search starts.
// `STEADY` adds the hybrid's steady half, whose common ranks 2 j 2^E (j < cs)
// give the largest one below a bound in closed form.
template <uint32_t S, bool STEADY>
__device__ __forceinline__ uint32_t kth_common_below(const uint32_t (&cr)[S], uint32_t upper,
                                                     uint32_t kc, uint32_t cs, uint32_t E) {
  uint32_t bound = upper, best = 0u;
  for (uint32_t p = 0; p < kc; ++p) {
    uint32_t gap = bound;
    if (STEADY && cs > 0u && bound > 0u) {
      uint32_t jm = (bound - 1u) >> (E + 1u);  // largest j with 2 j 2^E < bound
      if (jm > cs - 1u) jm = cs - 1u;
      gap = bound - (2u * (jm << E) + 1u);
    }
    const uint32_t below = bound - 1u;
#pragma unroll
    for (uint32_t site = 0; site < S; ++site) {
      const uint32_t d = below - cr[site];
      gap = d < gap ? d : gap;
    }
    best = bound - gap;
    bound = best - (best != 0u);
  }
  return best;
}

// All ones where bit `pos` of the word is set, else zero (one bit-field
// extract, sign-extended; pos is a constant once the site loops unroll).
__device__ __forceinline__ uint32_t bit_mask_dyn(uint32_t word, uint32_t pos) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)word, pos, 1);
}

template <uint32_t S, uint32_t DLOG>
__global__ __launch_bounds__(256) void pairs_tilted_tile_kernel(const uint32_t* __restrict__ T,
                                                                const uint32_t* __restrict__ D,
                                                                uint32_t n, uint32_t kc,
                                                                uint32_t* __restrict__ L,
                                                                uint32_t* __restrict__ U) {
  const uint32_t x0 = blockIdx.y * kPairTile, y0 = blockIdx.x * kPairTile;
  if (y0 < x0) return;
  constexpr uint32_t m_log = S == 64u ? 1u : 0u;
  constexpr uint32_t s_log = S == 64u ? 6u : 5u;
  constexpr uint32_t words = (S << DLOG) >> 5;
  __shared__ uint32_t xr[kPairTile][S];
  __shared__ PairStage st;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint32_t e = threadIdx.x; e < kPairTile * S; e += blockDim.x) {
    const uint32_t r = e >> s_log, site = e & (S - 1u);
    const uint32_t x = x0 + r;
    xr[r][site] = tilted_slot_rank(x < n ? T[x] : 0u, site >> m_log, site & ((1u << m_log) - 1u),
                                   m_log);
  }
  const uint32_t y = y0 + lane;
  const uint32_t yc = y < n ? y : n - 1u;  // a valid surface for lanes past the end
  const uint32_t tb = T[yc];
  const unsigned long long wb = (unsigned long long)D[(size_t)yc * words] |
                                (words > 1 ? (unsigned long long)D[(size_t)yc * words + 1] << 32
                                           : 0ull);
  uint32_t rb[S];
#pragma unroll
  for (uint32_t site = 0; site < S; ++site)
    rb[site] = tilted_slot_rank(tb, site >> m_log, site & ((1u << m_log) - 1u), m_log);
  __syncthreads();
#pragma unroll 1
  for (uint32_t i = 0; i < kRowsPerWave; ++i) {
    const uint32_t r = wid * kRowsPerWave + i, x = x0 + r;
    const uint32_t xc = x < n ? x : n - 1u;
    const uint32_t ta = T[xc];
    const unsigned long long wa = (unsigned long long)D[(size_t)xc * words] |
                                  (words > 1 ? (unsigned long long)D[(size_t)xc * words + 1] << 32
                                             : 0ull);
    unsigned long long diff = wa ^ wb;
    if (DLOG == 1u) diff |= diff >> 1;  // bit 2 s: field s differs
    // all ones over the sites whose fields agree: the sign-extended bit of ~diff
    const uint32_t agree_lo = ~(uint32_t)diff, agree_hi = ~(uint32_t)(diff >> 32);
    uint32_t upper = ta < tb ? ta : tb;
    uint32_t cr[S];  // the rank both surfaces hold at the site, or kNone
#pragma unroll
    for (uint32_t site = 0; site < S; ++site) {
      const uint32_t ra = xr[r][site];
      cr[site] = ra == rb[site] ? ra : kNone;
      const uint32_t pos = site << DLOG;
      const uint32_t agree = pos < 32u ? bit_mask_dyn(agree_lo, pos) : bit_mask_dyn(agree_hi, pos - 32u);
      const uint32_t cand = cr[site] | agree;  // kNone unless common and differing
      upper = cand < upper ? cand : upper;
    }
    put_pair(st, r, lane, x, y, n, upper, kth_common_below<S, false>(cr, upper, kc, 0u, 0u), L,
             U);
  }
  if (x0 == y0) return;
  __syncthreads();
  put_mirror(st, x0, y0, n, L, U);
}

// Steady half of a hybrid surface (sites 0..31 of the low word, (t + 1) / 2
// deposits on the even ranks) in rank order: bit j is the differentia of its
// j-th retained deposit, rank j 2^e of the half, e its epoch.
__device__ __forceinline__ uint32_t steady_half_bits(uint32_t t, uint32_t w_lo, uint32_t* epoch) {
  const uint32_t nh = (t >> 1) + (t & 1u);
  const uint32_t e = epoch_of(nh, 5u);
  const uint32_t count = nh == 0u ? 0u : ((nh - 1u) >> e) + 1u;  // <= 32
  uint32_t bits = 0u;
  for (uint32_t j = 0; j < count; ++j) bits |= ((w_lo >> site_of_retained(j << e, 5u)) & 1u) << j;
  *epoch = e;
  return bits;
}

// Keep bits 0, 2^d, 2 * 2^d, ... of a 32-bit string, packed to the bottom.
__device__ __forceinline__ uint32_t compact_stride32(uint32_t x, uint32_t d) {
  for (uint32_t i = 0; i < d && i < 5u; ++i) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
  }
  return x;
}

// Hybrid surfaces, tiled as above: the tilted half's ranks (odd ranks) per
// lane in registers and per row in LDS; the steady halves in rank order (per
// lane and per row), so their first differing common rank 2 j 2^E is the
// lowest set bit of the XOR of the two strings thinned to the common ranks,
// and the largest of their common ranks below a bound is closed-form.
__global__ __launch_bounds__(256) void pairs_hybrid_tile_kernel(const uint32_t* __restrict__ T,
                                                                const uint32_t* __restrict__ D,
                                                                uint32_t n, uint32_t kc,
                                                                uint32_t* __restrict__ L,
                                                                uint32_t* __restrict__ U) {
  const uint32_t x0 = blockIdx.y * kPairTile, y0 = blockIdx.x * kPairTile;
  if (y0 < x0) return;
  __shared__ uint32_t xr[kPairTile][32];
  __shared__ uint32_t xs[kPairTile][2];  // steady half in rank order, its epoch
  __shared__ PairStage st;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint32_t e = threadIdx.x; e < kPairTile * 32u; e += blockDim.x) {
    const uint32_t r = e >> 5, k = e & 31u;
    const uint32_t x = x0 + r;
    const uint32_t ra = tilted_slot_rank((x < n ? T[x] : 0u) >> 1, k, 0u, 0u);
    xr[r][k] = ra == kNone ? kNone : 2u * ra + 1u;
  }
  if (threadIdx.x < kPairTile) {
    const uint32_t x = x0 + threadIdx.x;
    uint32_t e = 0u;
    xs[threadIdx.x][0] = x < n ? steady_half_bits(T[x], D[(size_t)x * 2], &e) : 0u;
    xs[threadIdx.x][1] = e;
  }
  const uint32_t y = y0 + lane;
  const uint32_t yc = y < n ? y : n - 1u;
  const uint32_t tb = T[yc];
  const unsigned long long wb =
      (unsigned long long)D[(size_t)yc * 2] | (unsigned long long)D[(size_t)yc * 2 + 1] << 32;
  uint32_t rb[32];
#pragma unroll
  for (uint32_t k = 0; k < 32; ++k) {
    const uint32_t r = tilted_slot_rank(tb >> 1, k, 0u, 0u);
    rb[k] = r == kNone ? kNone : 2u * r + 1u;
  }
  const uint32_t nb = (tb >> 1) + (tb & 1u);
  uint32_t eb = 0u;
  const uint32_t sb = steady_half_bits(tb, (uint32_t)wb, &eb);
  __syncthreads();
#pragma unroll 1
  for (uint32_t i = 0; i < kRowsPerWave; ++i) {
    const uint32_t r = wid * kRowsPerWave + i, x = x0 + r;
    const uint32_t xc = x < n ? x : n - 1u;
    const uint32_t ta = T[xc];
    const unsigned long long diff =
        ((unsigned long long)D[(size_t)xc * 2] | (unsigned long long)D[(size_t)xc * 2 + 1] << 32) ^
        wb;
    // steady halves: common ranks 2 j 2^E for j < cs
    const uint32_t na = (ta >> 1) + (ta & 1u);
    const uint32_t ea = xs[r][1];
    const uint32_t E = ea > eb ? ea : eb;
    const uint32_t nmin = na < nb ? na : nb;
    const uint32_t cs = nmin == 0u ? 0u : ((nmin - 1u) >> E) + 1u;  // <= 32
    uint32_t upper = ta < tb ? ta : tb;
    const uint32_t hit = (compact_stride32(xs[r][0], E - ea) ^ compact_stride32(sb, E - eb)) &
                         (cs >= 32u ? 0xFFFFFFFFu : (1u << cs) - 1u);
    if (hit) upper = min(upper, 2u * ((uint32_t)(__ffs(hit) - 1) << E));
    const uint32_t agree_hi = ~(uint32_t)(diff >> 32);  // tilted half: sites 32..63
    uint32_t cr[32];  // the odd rank both surfaces hold at the level, or kNone
#pragma unroll
    for (uint32_t k = 0; k < 32; ++k) {
      const uint32_t ra = xr[r][k];
      cr[k] = ra == rb[k] ? ra : kNone;
      const uint32_t cand = cr[k] | bit_mask_dyn(agree_hi, k);  // kNone unless differing
      upper = cand < upper ? cand : upper;
    }
    put_pair(st, r, lane, x, y, n, upper, kth_common_below<32, true>(cr, upper, kc, cs, E), L, U);
  }
  if (x0 == y0) return;
  __syncthreads();
  put_mirror(st, x0, y0, n, L, U);
}

}  // namespace

size_t mrca_workspace_bytes(size_t n) { return n * sizeof(Normalized); }

// Workspace of the allocation-free relatedness call: one normalised surface
// per sample for up to kScratchSurfaces samples, in a file-scope device array.
// Each GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` only names the symbol: its device address, per
// device, comes from hipGetSymbolAddress.
static __device__ __align__(256) Normalized scratch[kScratchSurfaces];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void* scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> hold(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_mrca_matrix(const uint32_t* T, const uint32_t* D, uint32_t n, uint32_t s_log,
                              uint32_t dlog, uint32_t policy, uint32_t kc, void* workspace,
                              uint32_t* L, uint32_t* U, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (policy == 1u || policy == 2u) {
    const uint32_t tiles = (n + kPairTile - 1u) / kPairTile;
    const dim3 grid(tiles, tiles);
    if (policy == 2u)
      pairs_hybrid_tile_kernel<<<grid, dim3(256), 0, stream>>>(T, D, n, kc, L, U);
    else if (s_log == 6u && dlog == 0u)
      pairs_tilted_tile_kernel<64, 0><<<grid, dim3(256), 0, stream>>>(T, D, n, kc, L, U);
    else if (s_log == 5u && dlog == 0u)
      pairs_tilted_tile_kernel<32, 0><<<grid, dim3(256), 0, stream>>>(T, D, n, kc, L, U);
    else if (s_log == 5u && dlog == 1u)
      pairs_tilted_tile_kernel<32, 1><<<grid, dim3(256), 0, stream>>>(T, D, n, kc, L, U);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  Normalized* nz = static_cast<Normalized*>(workspace);
  normalize_kernel<<<dim3((n + 255) / 256), dim3(256), 0, stream>>>(T, D, n, s_log, dlog, nz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pairs_kernel<<<dim3((n + 2047) / 2048, n), dim3(256), 0, stream>>>(nz, n, dlog, kc, L, U);
  return hipGetLastError();
}

hipError_t launch_mrca_matrix_noalloc(const uint32_t* T, const uint32_t* D, uint32_t n,
                                      uint32_t s_log, uint32_t dlog, uint32_t policy, uint32_t kc,
                                      uint32_t* L, uint32_t* U, hipStream_t stream) {
  if (n > kScratchSurfaces) return hipErrorInvalidValue;
  void* ws = nullptr;
  if (n != 0 && policy == 0u) {
    // the normalise pass writes every one of the n entries it reads back,
    // so nothing left from an earlier call needs clearing
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return e;
  }
  return launch_mrca_matrix(T, D, n, s_log, dlog, policy, kc, ws, L, U, stream);
}

}  // namespace ga
