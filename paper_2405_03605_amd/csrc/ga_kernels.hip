// HIP kernels for the island-model GA generation step on gfx950 (CDNA4).
//
// Mapping: one wavefront owns a chunk of `ipw` consecutive islands. Lanes map
// to agent slots; with N agents per island a wavefront covers 64/N islands per
// iteration, so the tournament gathers and the parent copy are cross-lane
// permutes (ds_bpermute) inside the wavefront and never touch LDS storage or
// HBM twice. Before its iterations a wavefront draws the migration block of
// each of its islands in one pass (lane l -> island first + l), reads the four
// neighbour outbox headers of each, and keeps the result in two registers that
// later iterations fetch by permute; the migration stream thus costs one
// Philox block per island, not per agent.
//
// Generation t (paper Sec. 2): absorb arrivals emitted during t-1 (outbox
// parity (t-1)&1), emit into parity t&1, then tournament, copy, mutation and
// one stratum deposit for every child. Islands are updated in place: a
// wavefront reads all of an island's agents before it writes any child, and no
// other wavefront reads them.
#include "ga_internal.hpp"

namespace ga {
namespace {

constexpr uint32_t kMulA = 0xD2511F53u;   // Philox4x32 round multipliers
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;  // key schedule increments
constexpr uint32_t kWeylB = 0xBB67AE85u;

constexpr uint32_t kStreamSelect = 0u;
constexpr uint32_t kStreamMigrate = 1u;
constexpr uint32_t kStreamSample = 2u;

struct Block {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each takes
// both halves of two 32x32->64 products and mixes the high halves with the
// other two counter words and the round key.
__device__ __forceinline__ Block philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = (uint64_t)kMulA * c0;  // one v_mad_u64_u32 each
    const uint64_t pb = (uint64_t)kMulB * c2;
    const uint32_t a_hi = (uint32_t)(pa >> 32), a_lo = (uint32_t)pa;
    const uint32_t b_hi = (uint32_t)(pb >> 32), b_lo = (uint32_t)pb;
    c0 = b_hi ^ c1 ^ k0;
    c2 = a_hi ^ c3 ^ k1;
    c1 = b_lo;
    c3 = a_lo;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return {c0, c1, c2, c3};
}

// Site written by the deposit of stratum rank r on S = 2^s sites, or kDiscard
// ("doubling steady" surface): ranks below S keep site r; a rank r >= S is
// written only when its low e bits are clear, e = bitlen(r) - s, and the j-th
// rank written in epoch e takes over the site of rank (2j+1) << (e-1), which
// left the retained set when epoch e began. Written ranks are odd multiples
// odd << shift, so the walk only renormalises the odd part.
__device__ __forceinline__ uint32_t surface_site(uint32_t r, uint32_t s) {
  const uint32_t half = 1u << (s - 1u);
  if (r < (half << 1)) return r;
  const uint32_t e = (32u - __clz(r)) - s;
  if (r & ((1u << e) - 1u)) return kDiscard;
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

__device__ __forceinline__ uint32_t permute(uint32_t value, uint32_t src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src_lane << 2), (int)value);
}
__device__ __forceinline__ float permute(float value, uint32_t src_lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((int)(src_lane << 2), __float_as_int(value)));
}

// Island next to (x, y) in direction q on the W x H torus:
// 0 north (y-1), 1 east (x+1), 2 south (y+1), 3 west (x-1).
__device__ __forceinline__ uint32_t torus_step(uint32_t x, uint32_t y, uint32_t q, uint32_t W,
                                               uint32_t H) {
  const uint32_t xe = (x + 1u == W) ? 0u : x + 1u;
  const uint32_t xw = (x == 0u ? W : x) - 1u;
  const uint32_t yn = (y == 0u ? H : y) - 1u;
  const uint32_t ys = (y + 1u == H) ? 0u : y + 1u;
  const uint32_t nx = q == 1u ? xe : (q == 3u ? xw : x);
  const uint32_t ny = q == 0u ? yn : (q == 2u ? ys : y);
  return ny * W + nx;
}

// One generation for islands [base, base + v.ipw) of a run, by one wavefront.
// LC / SWC: log2 N and surface words fixed at compile time, or -1 to read them
// from the view.
template <int LC, int SWC>
__device__ __forceinline__ void chunk_generation(const RunView& v, uint32_t base, uint64_t t) {
  const uint32_t L = LC >= 0 ? (uint32_t)LC : v.log2n;
  const uint32_t SW = SWC >= 0 ? (uint32_t)SWC : v.words;
  const uint32_t s_log = 4u + SW;  // log2 S: 5 for 32 sites, 6 for 64
  const uint32_t lane = __lane_id();
  const uint32_t N = 1u << L;
  const uint32_t per_iter = 64u >> L;  // islands per wavefront iteration
  const uint32_t t_lo = (uint32_t)t;
  const uint32_t t_hi4 = (uint32_t)(t >> 32) << 2;
  const uint32_t rp = ((uint32_t)t & 1u) ^ 1u;  // parity absorbed from
  const uint32_t wp = (uint32_t)t & 1u;         // parity emitted into
  const uint32_t W = v.width, H = v.height;
  // parity-selected outbox planes (selects, not indexing, so views held in
  // registers never spill to scratch)
  const uint32_t* __restrict__ in_meta = rp ? v.ob_meta[1] : v.ob_meta[0];
  const float* __restrict__ in_f = rp ? v.ob_f[1] : v.ob_f[0];
  const uint32_t* __restrict__ in_T = rp ? v.ob_T[1] : v.ob_T[0];
  const uint32_t* __restrict__ in_D = rp ? v.ob_D[1] : v.ob_D[0];
  uint32_t* __restrict__ out_meta = wp ? v.ob_meta[1] : v.ob_meta[0];
  float* __restrict__ out_f = wp ? v.ob_f[1] : v.ob_f[0];
  uint32_t* __restrict__ out_T = wp ? v.ob_T[1] : v.ob_T[0];
  uint32_t* __restrict__ out_D = wp ? v.ob_D[1] : v.ob_D[0];

  // ---- per-island pass: lane l handles island base + l ---------------------
  uint32_t own = base + lane;
  if (lane >= v.ipw || own >= v.islands) own = base;
  const uint32_t ox = own % W, oy = own / W;
  const Block mig = philox10(0u, own, t_lo, t_hi4 | kStreamMigrate, v.seed, v.run_id);
  const uint32_t emig_slot = L ? (mig.x >> (32u - L)) : 0u;
  const uint32_t emig_dir = mig.y >> 30;
  uint32_t arrive = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t j = torus_step(ox, oy, q, W, H);
    if (in_meta[j] == (kMetaValid | (q ^ 2u))) arrive |= 1u << q;
  }
  const uint32_t info = emig_slot | (emig_dir << 8) | (arrive << 12);
  const uint32_t slots4 = mig.z;          // byte q: replacement slot draw for direction q
  const uint32_t xy = ox | (oy << 16);

  const uint32_t slot = lane & (N - 1u);
  const uint32_t lane0 = lane & ~(N - 1u);  // first lane of this lane's island
  const uint32_t A = v.agents;
  float* __restrict__ pf = v.pop_f;
  uint32_t* __restrict__ pT = v.pop_T;
  uint32_t* __restrict__ pD = v.pop_D;

  for (uint32_t it = 0; it * per_iter < v.ipw; ++it) {
    const uint32_t local = it * per_iter + (lane >> L);
    const uint32_t island = base + local;
    const bool active = island < v.islands;
    const uint32_t a = island * N + slot;

    float f = 0.f;
    uint32_t T = 0, D0 = 0, D1 = 0;
    if (active) {
      f = pf[a];
      T = pT[a];
      D0 = pD[a];
      if (SW > 1) D1 = pD[A + a];
    }
    const uint32_t my_info = permute(info, local);
    const uint32_t my_slots = permute(slots4, local);
    const uint32_t my_xy = permute(xy, local);

    // 1. absorb: the last arriving direction whose drawn slot is mine wins
    int from = -1;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t want = ((my_slots >> (8u * q)) & 0xFFu) >> (8u - L);
      if (((my_info >> (12u + q)) & 1u) && want == slot) from = (int)q;
    }
    if (active && from >= 0) {
      const uint32_t j = torus_step(my_xy & 0xFFFFu, my_xy >> 16, (uint32_t)from, W, H);
      f = in_f[j];
      T = in_T[j];
      D0 = in_D[j];
      if (SW > 1) D1 = in_D[v.islands + j];
    }

    // 2. emit a copy of the drawn member (post-absorb) toward the drawn neighbour
    if (active && slot == (my_info & 0xFFu)) {
      if (v.migration) {
        out_meta[island] = kMetaValid | ((my_info >> 8) & 3u);
        out_f[island] = f;
        out_T[island] = T;
        out_D[island] = D0;
        if (SW > 1) out_D[v.islands + island] = D1;
      } else {
        out_meta[island] = 0u;
      }
    }

    // 3-5. evaluate (read fitness) and run the tournament over permuted entrants
    const Block r = philox10(slot, island, t_lo, t_hi4 | kStreamSelect, v.seed, v.run_id);
    uint32_t best = (r.x & 0xFFu) >> (8u - L);
    float fbest = permute(f, lane0 + best);
    if (v.selection) {
#pragma unroll
      for (uint32_t m = 1; m < 8; ++m) {
        if (m < v.k) {
          const uint32_t byte = ((m < 4 ? r.x : r.y) >> (8u * (m & 3u))) & 0xFFu;
          const uint32_t cand = byte >> (8u - L);
          const float fc = permute(f, lane0 + cand);
          if (fc > fbest) {
            best = cand;
            fbest = fc;
          }
        }
      }
    }
    uint32_t cT = permute(T, lane0 + best);
    uint32_t cD0 = permute(D0, lane0 + best);
    uint32_t cD1 = SW > 1 ? permute(D1, lane0 + best) : 0u;
    float cf = fbest;

    // 6. mutation: delta index (w & 0x7FFFFFFF) * 5 >> 31 maps to {-1,-1/2,0,1/2,1}
    if (r.z < v.p32) {
      const uint32_t di = (uint32_t)(((uint64_t)(r.w & 0x7FFFFFFFu) * 5u) >> 31);
      cf = __fadd_rn(cf, 0.5f * (float)((int)di - 2));
    }

    // 7. stratum deposit at rank T, then T + 1
    const uint32_t site = surface_site(cT, s_log);
    if (site != kDiscard) {
      const uint32_t bit = r.w >> 31;
      const uint32_t sh = site & 31u;
      if (SW == 1 || site < 32u) {
        cD0 = (cD0 & ~(1u << sh)) | (bit << sh);
      } else {
        cD1 = (cD1 & ~(1u << sh)) | (bit << sh);
      }
    }
    cT += 1u;

    if (active) {
      pf[a] = cf;
      pT[a] = cT;
      pD[a] = cD0;
      if (SW > 1) pD[A + a] = cD1;
    }
  }
}

template <int LC, int SWC>
__global__ __launch_bounds__(1024) void generation_kernel(RunView v, uint32_t gen_offset) {
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) +
                        (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t base = wave * v.ipw;
  if (base >= v.islands) return;
  chunk_generation<LC, SWC>(v, base, *v.gen + gen_offset);
}

// Whole run in one workgroup: the generation loop stays on the GPU, with a
// workgroup barrier between generations (the outbox hand-over).
template <int LC, int SWC>
__global__ __launch_bounds__(1024) void resident_kernel(RunView v, uint64_t n_gens) {
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t base = wave * v.ipw;
  const uint64_t t0 = *v.gen;
  for (uint64_t g = 0; g < n_gens; ++g) {
    if (base < v.islands) chunk_generation<LC, SWC>(v, base, t0 + g);
    __syncthreads();
  }
  if (threadIdx.x == 0) *v.gen = t0 + n_gens;
}

__global__ void advance_kernel(unsigned long long* gen, uint64_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *gen = *gen + n;
}

__global__ void fill_kernel(uint32_t* p, uint32_t value, size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = value;
}

// One agent per island from the sampling stream at the current generation.
__global__ void sample_kernel(RunView v, uint32_t* ids) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.islands) return;
  const uint64_t t = *v.gen;
  const Block b = philox10(0u, i, (uint32_t)t, ((uint32_t)(t >> 32) << 2) | kStreamSample, v.seed,
                           v.run_id);
  const uint32_t slot = v.log2n ? (b.x >> (32u - v.log2n)) : 0u;
  ids[i] = (i << v.log2n) + slot;
}

__global__ void gather_kernel(RunView v, const uint32_t* ids, uint32_t n, uint32_t* T_out,
                              uint32_t* D_out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t a = ids[j];
  T_out[j] = v.pop_T[a];
  for (uint32_t w = 0; w < v.words; ++w) D_out[(size_t)w * n + j] = v.pop_D[(size_t)w * v.agents + a];
}

// Batched form: wavefront i works on tiles[i]; members whose budget for this
// block is spent sit the generation out.
__global__ __launch_bounds__(1024) void batch_generation_kernel(const RunView* __restrict__ views,
                                                                const Tile* __restrict__ tiles,
                                                                uint32_t n_tiles,
                                                                uint32_t gen_offset) {
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) +
                        (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave >= n_tiles) return;
  const Tile tile = tiles[wave];
  const RunView v = views[tile.run];
  if (*v.left <= gen_offset) return;
  chunk_generation<-1, -1>(v, tile.first, *v.gen + gen_offset);
}

__global__ void batch_advance_kernel(const RunView* views, uint32_t n_runs, uint64_t block) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_runs) return;
  const RunView v = views[i];
  const unsigned long long left = *v.left;
  const unsigned long long done = left < block ? left : block;
  *v.gen = *v.gen + done;
  *v.left = left - done;
}

}  // namespace

#define GA_DISPATCH(KERNEL, L, SW, ...)                                        \
  do {                                                                         \
    switch ((L) * 2 + ((SW) - 1)) {                                            \
      case 0: KERNEL<0, 1> __VA_ARGS__; break;                                 \
      case 1: KERNEL<0, 2> __VA_ARGS__; break;                                 \
      case 2: KERNEL<1, 1> __VA_ARGS__; break;                                 \
      case 3: KERNEL<1, 2> __VA_ARGS__; break;                                 \
      case 4: KERNEL<2, 1> __VA_ARGS__; break;                                 \
      case 5: KERNEL<2, 2> __VA_ARGS__; break;                                 \
      case 6: KERNEL<3, 1> __VA_ARGS__; break;                                 \
      case 7: KERNEL<3, 2> __VA_ARGS__; break;                                 \
      case 8: KERNEL<4, 1> __VA_ARGS__; break;                                 \
      case 9: KERNEL<4, 2> __VA_ARGS__; break;                                 \
      case 10: KERNEL<5, 1> __VA_ARGS__; break;                                \
      case 11: KERNEL<5, 2> __VA_ARGS__; break;                                \
      case 12: KERNEL<6, 1> __VA_ARGS__; break;                                \
      case 13: KERNEL<6, 2> __VA_ARGS__; break;                                \
      default: return hipErrorInvalidValue;                                    \
    }                                                                          \
  } while (0)

hipError_t launch_generation(const RunView& v, uint32_t gen_offset, uint32_t waves,
                             uint32_t waves_per_group, hipStream_t stream) {
  if (waves == 0) return hipSuccess;
  const uint32_t groups = (waves + waves_per_group - 1) / waves_per_group;
  const dim3 grid(groups), block(64 * waves_per_group);
  GA_DISPATCH(generation_kernel, v.log2n, v.words,
              <<<grid, block, 0, stream>>>(v, gen_offset));
  return hipGetLastError();
}

hipError_t launch_resident(const RunView& v, uint64_t n_gens, uint32_t waves, hipStream_t stream) {
  if (waves == 0 || waves > (uint32_t)kMaxWavesPerGroup) return hipErrorInvalidValue;
  const dim3 grid(1), block(64 * waves);
  GA_DISPATCH(resident_kernel, v.log2n, v.words, <<<grid, block, 0, stream>>>(v, n_gens));
  return hipGetLastError();
}

hipError_t launch_advance(unsigned long long* gen, uint64_t n, hipStream_t stream) {
  advance_kernel<<<1, 64, 0, stream>>>(gen, n);
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t* p, uint32_t value, size_t words, hipStream_t stream) {
  if (words == 0) return hipSuccess;
  size_t groups = (words + 255) / 256;
  if (groups > 65536) groups = 65536;
  fill_kernel<<<dim3((uint32_t)groups), dim3(256), 0, stream>>>(p, value, words);
  return hipGetLastError();
}

hipError_t launch_sample(const RunView& v, uint32_t* ids, hipStream_t stream) {
  const uint32_t groups = (v.islands + 255) / 256;
  sample_kernel<<<dim3(groups), dim3(256), 0, stream>>>(v, ids);
  return hipGetLastError();
}

hipError_t launch_gather(const RunView& v, const uint32_t* ids, uint32_t n, uint32_t* T_out,
                         uint32_t* D_out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  gather_kernel<<<dim3((n + 255) / 256), dim3(256), 0, stream>>>(v, ids, n, T_out, D_out);
  return hipGetLastError();
}

hipError_t launch_batch_generation(const RunView* views, const Tile* tiles, uint32_t n_tiles,
                                   uint32_t gen_offset, uint32_t waves_per_group,
                                   hipStream_t stream) {
  if (n_tiles == 0) return hipSuccess;
  const uint32_t groups = (n_tiles + waves_per_group - 1) / waves_per_group;
  batch_generation_kernel<<<dim3(groups), dim3(64 * waves_per_group), 0, stream>>>(
      views, tiles, n_tiles, gen_offset);
  return hipGetLastError();
}

hipError_t launch_batch_advance(const RunView* views, uint32_t n_runs, uint64_t block,
                                hipStream_t stream) {
  if (n_runs == 0) return hipSuccess;
  batch_advance_kernel<<<dim3((n_runs + 255) / 256), dim3(256), 0, stream>>>(views, n_runs, block);
  return hipGetLastError();
}

}  // namespace ga
