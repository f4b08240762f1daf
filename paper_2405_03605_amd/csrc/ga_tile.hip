// LDS-resident persistent form of the synchronous generation step.
//
// The torus is cut into tiles of tile_w x tile_h islands (ragged at the right
// and bottom edges); one workgroup owns one tile for the whole launch and keeps
// its population in LDS across generations, the way each processing element
// of the paper's wafer-scale design keeps its island in local memory (Sec. 2
// Methods). HBM then carries the population once at the start and once at the
// end of a launch, and in between only the emissions of the islands on a
// tile's edge (one outbox entry each per generation).
//
// Generation t in one workgroup, with the same results as the per-generation
// streaming kernel (and the oracle):
//   island pass   one thread per island: the migration draw; the four
//                 neighbours' emissions of generation t-1 (the LDS outbox for
//                 a neighbour in the tile, the LDS halo staging for one
//                 outside it); arrivals written into their drawn slots of the
//                 LDS population (later directions overwrite earlier ones);
//                 the drawn emigrant (post-immigration) copied to the LDS
//                 outbox of parity t&1 and, for an island with a neighbour
//                 outside the tile, to the HBM outbox;
//   iterations    lanes are agent slots, 64/N islands per wavefront
//                 iteration, tournament / copy / mutation / deposit (`breed`)
//                 in registers, children written back in place; iterations
//                 are handed out one at a time from an LDS counter, so the
//                 wavefronts finish together whatever the SIMDs favour;
//   publish       after its first iteration each wavefront drains its HBM
//                 stores and arrives on an LDS counter; the last one sets the
//                 tile's progress word to t+1: its emissions of t are readable
//                 and it has finished reading its neighbours' emissions of t-1;
//   halo          wavefront 0, once the tile is halfway through its
//                 iterations, polls the four neighbouring tiles' progress
//                 words and, once they read t+1,
//                 loads their edge emissions of t (the halo of generation t+1)
//                 into registers, staged in LDS after its last iteration (a
//                 bounded wait there if they are late).
// The emissions of t are fixed by the island pass, before the iterations, so
// the HBM round trips of the exchange (the drain of a tile's edge stores, the
// neighbours' loads of them) overlap the iterations instead of following
// them. A neighbour has finished reading the HBM outbox entries of parity
// (t+1)&1 (its island pass of t) when its progress word reads t+1, before
// this tile overwrites them in generation t+1.
//
// Every tile's workgroup must be resident at once (the host sizes the tiling
// by the occupancy query); each wait is bounded, and a wait that gave up is
// counted, which the host reports as an error when the state is read.
#include "ga_device.hpp"

namespace ga {
namespace {

extern __shared__ uint32_t tile_lds[];

// LDS words of a tile: the population as TA agent records and two scratch
// records (the same for strings; the scratch one takes arrivals that are not
// taken, so the island pass writes without a branch), the island-id and packed (x, y) tables of TA / N islands, the outbox for
// both parities (TI entries of ob_stride words each), the halo staging (one
// entry per edge island and outward direction, at most 2 (tile_w + tile_h)),
// the neighbour island each such pair reads, an arrival counter and two iteration
// counters (one per generation parity).
__host__ __device__ inline uint32_t tile_agents_padded(uint32_t ti_full, uint32_t log2n) {
  return ((ti_full << log2n) + 63u) & ~63u;
}
// words per agent: a 16-byte record (fitness, T, surface word 0, surface
// word 1 or 0) and, for a genome model with a string, an 8-byte one
__host__ __device__ inline uint32_t tile_agent_words(bool strings) {
  return 4u + (strings ? 2u : 0u);
}
// the island-id and (x, y) tables, each padded to a multiple of 4 words so
// what follows stays 16-byte aligned
__host__ __device__ inline uint32_t tile_table_words(uint32_t ta, uint32_t log2n) {
  return ((ta >> log2n) + 3u) & ~3u;
}

// Edge pairs of a tile of w x h islands on a W x H torus: (island, direction)
// whose neighbour lies in another tile. Indices: the north row's islands
// (0..w-1) and the south row's (w..2w-1) when the tile does not span the
// torus's height (h < H), then the west column's (..+h-1) and the east
// column's when it does not span the width.
struct EdgePairs {
  uint32_t w, h, n_ns, count;
  __device__ EdgePairs(uint32_t w_, uint32_t h_, uint32_t W, uint32_t H) : w(w_), h(h_) {
    n_ns = h < H ? 2u * w : 0u;
    count = n_ns + (w < W ? 2u * h : 0u);
  }
  // index of the pair (lx, ly, q); q's neighbour must lie outside the tile
  __device__ uint32_t index(uint32_t lx, uint32_t ly, uint32_t q) const {
    return q == 0u ? lx : q == 2u ? w + lx : q == 3u ? n_ns + ly : n_ns + h + ly;
  }
  // the pair's local island and direction
  __device__ void of(uint32_t p, uint32_t* lx, uint32_t* ly, uint32_t* q) const {
    if (p < n_ns) {
      const bool south = p >= w;
      *lx = south ? p - w : p;
      *ly = south ? h - 1u : 0u;
      *q = south ? 2u : 0u;
    } else {
      const uint32_t r = p - n_ns;
      const bool east = r >= h;
      *ly = east ? r - h : r;
      *lx = east ? w - 1u : 0u;
      *q = east ? 1u : 3u;
    }
  }
};

template <int LC, int SWC, typename Model, bool WIDE>
__global__ __launch_bounds__(1024) void tile_kernel(RunView v, uint64_t n_gens) {
  constexpr uint32_t L = (uint32_t)LC;
  constexpr uint32_t SW = (uint32_t)SWC;
  constexpr uint32_t N = 1u << L;
  constexpr bool kStr = Model::kString;
  // words per outbox entry (f, T, surface, header; with a string f, T, D0,
  // D1, P0, P1, header) and the header's word, as in the HBM outbox
  constexpr uint32_t obs = (SW == 1 && !kStr) ? 4u : 8u;
  constexpr uint32_t ob_hdr = kStr ? 6u : 2u + SW;
  const uint32_t tid = threadIdx.x, nthreads = blockDim.x;
  const uint32_t lane = __lane_id();
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nwaves = nthreads >> 6;
  const uint32_t W = v.width, H = v.height;

  // this workgroup's tile and its actual extent
  const uint32_t tile = xcd_band_group();
  const uint32_t tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const uint32_t x0 = tx * v.tile_w, y0 = ty * v.tile_h;
  const uint32_t w = min(v.tile_w, W - x0), h = min(v.tile_h, H - y0);
  const uint32_t ti = w * h;
  const uint32_t TI = v.tile_w * v.tile_h;
  const uint32_t TA = tile_agents_padded(TI, L);
  const uint32_t TR = TA + 2u;   // records: TA agents, scratch at TA (a pair keeps 16-byte alignment)
  const uint32_t TIP = TA >> L;  // islands covered by whole iterations
  const uint32_t n_iter = TA >> 6;
  const EdgePairs edges(w, h, W, H);

  uint4* pop = reinterpret_cast<uint4*>(tile_lds);         // [a]: f, T, D0, D1
  uint2* pstr = reinterpret_cast<uint2*>(pop + TR);        // [a]: P0, P1 (strings)
  uint32_t* lisl = tile_lds + TR * tile_agent_words(kStr);  // [li]: island id
  uint32_t* lxy = lisl + tile_table_words(TA, L);          // [li]: x | y << 16
  uint32_t* lob = lxy + tile_table_words(TA, L);           // [(p * TI + li) * obs + k]
  uint32_t* halo = lob + 2u * TI * obs;                    // [pair * obs + k]
  uint32_t* halo_isl = halo + 2u * (v.tile_w + v.tile_h) * obs;  // [pair]: neighbour island
  uint32_t* arrivals = halo_isl + 2u * (v.tile_w + v.tile_h);
  uint32_t* grab = arrivals + 1;  // [g & 1]: iterations handed out in generation g
  const uint32_t n_pairs = edges.count;
  // the HBM outbox entry (of plane `ob`) that edge pair p reads
  auto halo_src = [&](const uint32_t* ob, uint32_t p) {
    return ob + (size_t)halo_isl[p] * obs;
  };

  // ---- load: island table, population, pending outbox, halo ----------------
  for (uint32_t li = tid; li < TIP; li += nthreads) {
    const uint32_t r = li < ti ? li : 0u;
    const uint32_t ly = r / w, lx = r - ly * w;
    lxy[li] = (x0 + lx) | ((y0 + ly) << 16);
    lisl[li] = (y0 + ly) * W + x0 + lx;
  }
  for (uint32_t p = tid; p < n_pairs; p += nthreads) {
    uint32_t lx, ly, q, nx, ny;
    edges.of(p, &lx, &ly, &q);
    torus_xy(x0 + lx, y0 + ly, q, W, H, &nx, &ny);
    halo_isl[p] = ny * W + nx;
  }
  if (tid == 0u) {
    *arrivals = 0u;
    grab[0] = 0u;
    grab[1] = 0u;
  }
  __syncthreads();
  const uint64_t t0 = *v.gen;
  {
    const uint32_t* gpl[6] = {reinterpret_cast<const uint32_t*>(v.pop_f), v.pop_T, v.pop_D,
                              v.pop_D + v.agent_stride, v.pop_P, v.pop_P + v.agent_stride};
    for (uint32_t la = tid; la < TA; la += nthreads) {
      const uint32_t li = la >> L;
      const uint32_t a = (lisl[li] << L) + (la & (N - 1u));
      const bool ok = li < ti;
      pop[la] = ok ? make_uint4(gpl[0][a], gpl[1][a], gpl[2][a], SW > 1 ? gpl[3][a] : 0u)
                   : make_uint4(0u, 0u, 0u, 0u);
      if (kStr) pstr[la] = ok ? make_uint2(gpl[4][a], gpl[5][a]) : make_uint2(0u, 0u);
    }
    const uint32_t p_in = ((uint32_t)t0 & 1u) ^ 1u;
    const uint32_t* gob = v.ob[p_in];
    for (uint32_t k = tid; k < ti * obs; k += nthreads) {
      const uint32_t li = k / obs, j = k - li * obs;
      lob[(p_in * TI + li) * obs + j] = gob[(size_t)lisl[li] * obs + j];
    }
    for (uint32_t k = tid; k < n_pairs * obs; k += nthreads) {
      const uint32_t p = k / obs, j = k - p * obs;
      halo[k] = halo_src(gob, p)[j];
    }
  }
  __syncthreads();

  // neighbouring tiles this one waits on (lanes 0..3 of wavefront 0: N, E, S, W)
  uint32_t nb_tile = tile;
  if (lane < 4u) {
    const uint32_t gx = v.tiles_x, gy = v.tiles_y;
    const uint32_t ntx = lane == 1u ? (tx + 1u == gx ? 0u : tx + 1u)
                                    : (lane == 3u ? (tx == 0u ? gx : tx) - 1u : tx);
    const uint32_t nty = lane == 2u ? (ty + 1u == gy ? 0u : ty + 1u)
                                    : (lane == 0u ? (ty == 0u ? gy : ty) - 1u : ty);
    nb_tile = nty * gx + ntx;
  }
  const bool waits_on = lane < 4u && nb_tile != tile;
  uint32_t gave_up = 0u;
  // An island's place in the pass: its id, its place in the tile, and for
  // each direction the word offset in LDS of the entry it reads (the LDS
  // outbox entry of parity 0 for a neighbour in the tile, add TI * obs for
  // parity 1; the halo entry for one outside, whose bit in `inside` is 0).
  struct IslandGeom {
    uint32_t island, lx, ly, inside;
    uint32_t src[4];
  };
  auto geom = [&](uint32_t li) {
    const uint32_t xy = lxy[li];
    const uint32_t x = xy & 0xFFFFu, y = xy >> 16;
    IslandGeom gm;
    gm.island = y * W + x;
    gm.lx = x - x0;
    gm.ly = y - y0;
    gm.inside = 0u;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      uint32_t nx, ny;
      torus_xy(x, y, q, W, H, &nx, &ny);
      const bool in = nx - x0 < w && ny - y0 < h;
      gm.inside |= (in ? 1u : 0u) << q;
      gm.src[q] = in ? (uint32_t)(lob - tile_lds) + ((ny - y0) * w + (nx - x0)) * obs
                     : (uint32_t)(halo - tile_lds) + edges.index(gm.lx, gm.ly, q) * obs;
    }
    return gm;
  };
  // this thread's first island of the pass, fixed for the launch (most tiles
  // have no more islands than threads)
  const IslandGeom my_geom = geom(tid < ti ? tid : 0u);

  for (uint64_t g = 0; g < n_gens; ++g) {
    const uint64_t t = t0 + g;
    const uint32_t t_lo = (uint32_t)t;
    const uint32_t t_hi4 = (uint32_t)(t >> 32) << 2;
    const uint32_t p_out = t_lo & 1u, p_in = p_out ^ 1u;
    uint32_t* __restrict__ out_ob = v.ob[p_out];

    // ---- island pass: one thread per island ---------------------------------
    // (generation g - 1, the last user of the other counter, has passed its
    // closing barrier; generation g + 1 reads it after this one's)
    if (tid == 0u) grab[(g + 1u) & 1u] = 0u;
    auto island_pass = [&](const IslandGeom& gm, uint32_t li) {
      const uint32_t island = gm.island;
      const Block mig = philox10(0u, island, t_lo, t_hi4 | kStreamMigrate, v.seed, v.run_id);
      const uint32_t emig = L ? (mig.x >> (32u - L)) : 0u;
      // The four neighbours' entries: a neighbour in the tile gives its LDS
      // outbox entry of parity (t-1)&1, one outside the staged copy of its HBM
      // outbox entry. All four are read before any arrival is written (the
      // reads then go out together instead of each waiting on the previous
      // write), and every entry is written, an arrival to its drawn slot and
      // anything else to the scratch record, so there is no branch. Later
      // directions overwrite earlier ones.
      const bool edge = gm.inside != 15u;
      uint32_t e[4][obs];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t* src =
            tile_lds + gm.src[q] + (((gm.inside >> q) & 1u) ? p_in * TI * obs : 0u);
#pragma unroll
        for (uint32_t k = 0; k < obs; k += 4) {
          const uint4 u = *reinterpret_cast<const uint4*>(src + k);
          e[q][k] = u.x;
          e[q][k + 1] = u.y;
          e[q][k + 2] = u.z;
          e[q][k + 3] = u.w;
        }
      }
      // The emission is the drawn member after immigration: the last arrival
      // drawn into its slot, else the member there before the pass (read
      // now, ahead of the writes, so no read waits on them).
      const uint32_t a_em = (li << L) + emig;
      const uint4 pre = pop[a_em];
      uint32_t em[6] = {pre.x, pre.y, pre.z, pre.w, 0u, 0u};
      if (kStr) {
        const uint2 ps = pstr[a_em];
        em[4] = ps.x;
        em[5] = ps.y;
      }
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t slot = ((mig.z >> (8u * q)) & 0xFFu) >> (8u - L);
        const bool hit = e[q][ob_hdr] == (kMetaValid | (q ^ 2u));
        const uint32_t a = hit ? (li << L) + slot : TA;
        const uint32_t w3 = SW > 1 ? e[q][3] : 0u;
        pop[a] = make_uint4(e[q][0], e[q][1], e[q][2], w3);
        if (kStr) pstr[a] = make_uint2(e[q][4], e[q][5]);
        const bool takes = hit && slot == emig;
        em[0] = takes ? e[q][0] : em[0];
        em[1] = takes ? e[q][1] : em[1];
        em[2] = takes ? e[q][2] : em[2];
        em[3] = takes ? w3 : em[3];
        if (kStr) {
          em[4] = takes ? e[q][4] : em[4];
          em[5] = takes ? e[q][5] : em[5];
        }
      }
      uint32_t o[obs];
#pragma unroll
      for (uint32_t k = 0; k < obs; ++k) o[k] = 0u;
      o[0] = em[0];
      o[1] = em[1];
      o[2] = em[2];
      if (SW > 1) o[3] = em[3];
      if (kStr) {
        o[4] = em[4];
        o[5] = em[5];
      }
      o[ob_hdr] = v.migration ? (kMetaValid | (mig.y >> 30)) : 0u;
      uint4* dst = reinterpret_cast<uint4*>(lob + (p_out * TI + li) * obs);
#pragma unroll
      for (uint32_t k = 0; k < obs; k += 4) dst[k >> 2] = make_uint4(o[k], o[k + 1], o[k + 2], o[k + 3]);
      if (edge) {
        // completed (drained) before the tile's progress word moves on
        uint32_t* gdst = out_ob + (size_t)island * obs;
#pragma unroll
        for (uint32_t k = 0; k < obs; k += 2) store_agent2(gdst + k, o[k], o[k + 1]);
      }
    };
    if (tid < ti) island_pass(my_geom, tid);
    for (uint32_t li = tid + nthreads; li < ti; li += nthreads) island_pass(geom(li), li);
    __syncthreads();

    // ---- iterations: lanes are agent slots ----------------------------------
    // After its first iteration each wavefront drains its island-pass stores
    // and arrives on the LDS counter; the last to arrive publishes the tile's
    // progress (t + 1). Wavefront 0 meanwhile polls the neighbouring tiles'
    // progress and, once they have published t + 1, prefetches the halo of
    // generation t + 1 (their edge emissions of t) into registers, staged in
    // LDS after its last iteration.
    const bool next = g + 1u < n_gens;
    const uint32_t due = t_lo + 1u;
    uint32_t pf[obs];
    bool fetching = false;
    uint32_t polled = 0u, flag = 0u;
    const BreedLane bl = breed_lane<LC>(v, t);
    // Iterations are handed out from an LDS counter, one at a time: a
    // wavefront the SIMD favours takes more of them, so the tile's wavefronts
    // finish together instead of in age order (with a fixed share the
    // youngest ran last, alone on their SIMDs). Each grab is issued an
    // iteration ahead. Which wavefront computes an iteration does not change
    // its children.
    uint32_t* ctr = grab + (g & 1u);
    auto take = [&]() {
      uint32_t x = 0u;
      if (lane == 0u)
        x = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return x;
    };
    auto publish = [&]() {
      drain_memory();
      if (lane == 0u) {
        const uint32_t before = __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        if (before == (uint32_t)(g + 1u) * nwaves - 1u) store_agent(v.prog + tile, due);
      }
    };
    const uint32_t poll_from = n_iter / 2u;
    uint32_t k = 0;
    uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane(take());
    while (it < n_iter) {
      const uint32_t next_it = take();
      const uint32_t la = (it << 6) + lane;
      const uint32_t li = la >> L;
      const uint32_t island = lisl[li];
      const uint4 rec = pop[la];
      Genome gn;
      gn.f = __uint_as_float(rec.x);
      gn.T = rec.y;
      gn.D0 = rec.z;
      gn.D1 = rec.w;
      if (kStr) {
        const uint2 sr = pstr[la];
        gn.P0 = sr.x;
        gn.P1 = sr.y;
      }
      const Genome c = breed<LC, SWC, Model, WIDE>(v, bl, gn, island);
      if (li < ti) {
        pop[la] = make_uint4(__float_as_uint(c.f), c.T, c.D0, c.D1);
        if (kStr) pstr[la] = make_uint2(c.P0, c.P1);
      }
      if (k == 0u) publish();
      ++k;
      if (wave == 0u && next && !fetching && it >= poll_from) {
        // a poll issued one iteration ago is read now; a fresh one goes out
        if (polled) {
          drain_memory();
          if (__ballot(waits_on && (int32_t)(flag - due) < 0) == 0ull) {
            fetching = true;
            if (lane < n_pairs) {
              const uint32_t* src = halo_src(out_ob, lane);
#pragma unroll
              for (uint32_t j = 0; j < obs; j += 2) {
                const uint2 two = load_agent2(src + j);
                pf[j] = two.x;
                pf[j + 1] = two.y;
              }
            }
          }
        }
        if (!fetching) {
          flag = waits_on ? load_agent(v.prog + nb_tile) : due;
          polled = 1u;
        }
      }
      it = (uint32_t)__builtin_amdgcn_readfirstlane(next_it);
    }
    // a wavefront that got no iteration still drains its island-pass stores
    // and counts its arrival
    if (k == 0u) publish();

    // ---- wavefront 0: finish the wait and stage the halo of t + 1 ------------
    if (wave == 0u && next) {
      if (!fetching) {
        for (uint32_t spin = 0;; ++spin) {
          bool behind = false;
          if (waits_on) behind = (int32_t)(load_agent(v.prog + nb_tile) - due) < 0;
          if (__ballot(behind) == 0ull) break;
          if (spin == kLockSpins) {
            ++gave_up;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (lane < n_pairs) {
          const uint32_t* src = halo_src(out_ob, lane);
#pragma unroll
          for (uint32_t j = 0; j < obs; j += 2) {
            const uint2 two = load_agent2(src + j);
            pf[j] = two.x;
            pf[j + 1] = two.y;
          }
        }
      }
      drain_memory();
      if (lane < n_pairs) {
#pragma unroll
        for (uint32_t j = 0; j < obs; j += 4)
          *reinterpret_cast<uint4*>(halo + lane * obs + j) =
              make_uint4(pf[j], pf[j + 1], pf[j + 2], pf[j + 3]);
      }
      // pairs beyond the first 64, loaded and staged now
      for (uint32_t p = 64u + lane; p < n_pairs; p += 64u) {
        const uint32_t* src = halo_src(out_ob, p);
#pragma unroll
        for (uint32_t j = 0; j < obs; j += 2) {
          const uint2 two = load_agent2(src + j);
          halo[p * obs + j] = two.x;
          halo[p * obs + j + 1] = two.y;
        }
      }
    }
    __syncthreads();
  }

  // ---- store: population and the last generation's outbox -------------------
  {
    uint32_t* gpl[6] = {reinterpret_cast<uint32_t*>(v.pop_f), v.pop_T, v.pop_D,
                        v.pop_D + v.agent_stride, v.pop_P, v.pop_P + v.agent_stride};
    for (uint32_t la = tid; la < (ti << L); la += nthreads) {
      const uint32_t a = (lisl[la >> L] << L) + (la & (N - 1u));
      const uint4 rec = pop[la];
      gpl[0][a] = rec.x;
      gpl[1][a] = rec.y;
      gpl[2][a] = rec.z;
      if (SW > 1) gpl[3][a] = rec.w;
      if (kStr) {
        const uint2 sr = pstr[la];
        gpl[4][a] = sr.x;
        gpl[5][a] = sr.y;
      }
    }
    if (n_gens > 0) {
      const uint32_t p_last = (uint32_t)(t0 + n_gens - 1u) & 1u;
      uint32_t* gob = v.ob[p_last];
      for (uint32_t k = tid; k < ti * obs; k += nthreads) {
        const uint32_t li = k / obs, j = k - li * obs;
        gob[(size_t)lisl[li] * obs + j] = lob[(p_last * TI + li) * obs + j];
      }
    }
  }
  if (tid == 0u && gave_up)
    __hip_atomic_fetch_add(v.waits, (unsigned long long)gave_up, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

size_t tile_lds_bytes(uint32_t tile_w, uint32_t tile_h, uint32_t log2n, uint32_t words,
                      uint32_t model, uint32_t ob_stride) {
  (void)words;  // one 16-byte record per agent whatever the surface words
  const uint32_t TI = tile_w * tile_h;
  const uint32_t TA = tile_agents_padded(TI, log2n);
  return 4u * ((size_t)tile_agent_words(model_has_string(model)) * (TA + 2u) +
               2u * tile_table_words(TA, log2n) + 2u * (size_t)TI * ob_stride +
               2u * (size_t)(tile_w + tile_h) * (ob_stride + 1u) + 3u);
}

uint32_t tile_threads(uint32_t tile_w, uint32_t tile_h, uint32_t log2n) {
  const uint32_t iters = tile_agents_padded(tile_w * tile_h, log2n) >> 6;
  return 64u * (iters < 16u ? iters : 16u);
}

hipError_t tile_occupancy(const RunView& v, uint32_t threads, size_t lds, int* groups_per_cu) {
  return dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        groups_per_cu, tile_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)>, (int)threads, lds);
  });
}

hipError_t launch_tiles(const RunView& v, uint64_t n_gens, hipStream_t stream) {
  if (n_gens == 0) return hipSuccess;
  const uint32_t n_tiles = v.tiles_x * v.tiles_y;
  const uint32_t threads = tile_threads(v.tile_w, v.tile_h, v.log2n);
  const size_t lds = tile_lds_bytes(v.tile_w, v.tile_h, v.log2n, v.words, v.model, v.ob_stride);
  return dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    tile_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)><<<dim3(n_tiles), dim3(threads), lds, stream>>>(
        v, n_gens);
    return hipGetLastError();
  });
}

}  // namespace ga
