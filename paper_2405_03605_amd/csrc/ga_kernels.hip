// HIP kernels for the island-model GA generation step on gfx950 (CDNA4).
//
// Mapping. One wavefront owns a chunk of `ipw` consecutive islands and works
// through it in iterations of 64 agents: lanes are agent slots, an iteration
// covers 64/N islands, the tournament gathers and the parent copy are
// cross-lane permutes (ds_bpermute) inside the wavefront, and every genome is
// read from and written back to HBM exactly once per generation.
//
// Island pass. Before its iterations a wavefront handles the per-island work
// of its whole chunk at once, one island per lane: the migration draw (one
// Philox block per island), the four neighbour outbox headers, the arrivals
// (genomes loaded into a small LDS table, their slots packed into one
// register), and the emission, written to the outbox as consecutive entries.
// The iterations then only compare their slot against the packed arrival
// slots and read the LDS table in the rare case of a hit.
//
// Generation t (paper Sec. 2): absorb arrivals emitted during t-1 (outbox
// parity (t-1)&1), emit into parity t&1, then tournament, copy, mutation and
// one stratum deposit for every child. Islands are updated in place: a
// wavefront reads all of an island's agents before it writes any child, and no
// other wavefront reads them. Population and outbox planes are padded past the
// last island, so iterations never need a tail predicate.
#include "ga_device.hpp"

namespace ga {
namespace {

// Buffer of island i toward direction d for sending generations of parity p
// in the asynchronous mail plane, and island i's lockstep header there. Offsets
// are 64-bit: the mail plane (up to 256 bytes per island) outgrows 32-bit
// indexing long before the largest valid torus.
template <typename P>
__device__ __forceinline__ P* mail_entry(P* mail, uint32_t i, uint32_t d, uint32_t p,
                                         uint32_t stride) {
  return mail + ((size_t)i * 8u + d * 2u + p) * stride;
}
template <typename P>
__device__ __forceinline__ P* lock_header(P* lock, uint32_t i, uint32_t d, uint32_t p,
                                          uint32_t island_stride) {
  return lock + (size_t)(p * 4u + d) * island_stride + i;
}

__device__ __forceinline__ Genome load_genome(const float* pf, const uint32_t* pT,
                                              const uint32_t* pD0, const uint32_t* pD1,
                                              const uint32_t* pP0, const uint32_t* pP1,
                                              uint32_t off, uint32_t words, bool strings) {
  Genome g;
  g.f = *at_byte(pf, off);
  g.T = *at_byte(pT, off);
  g.D0 = *at_byte(pD0, off);
  if (words > 1) g.D1 = *at_byte(pD1, off);
  if (strings) {
    g.P0 = *at_byte(pP0, off);
    g.P1 = *at_byte(pP1, off);
  }
  return g;
}

// Per-wavefront state of the asynchronous schedule.
struct AsyncCtx {
  uint32_t lead;     // how many generations an island may run ahead of a neighbour
  uint32_t gave_up;  // waits for a neighbour that hit the spin limit
  uint32_t taken;    // this lane's islands: genomes absorbed (per lane)
};

// Flush a wavefront's asynchronous counters: give-ups to waits[0], genomes
// absorbed (summed over the lanes) to waits[1].
__device__ __forceinline__ void flush_async(const RunView& v, const AsyncCtx& ax) {
  uint32_t n = ax.taken;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) n += (uint32_t)__shfl_xor((int)n, m, 64);
  if (__lane_id() == 0u) {
    if (ax.gave_up)
      __hip_atomic_fetch_add(v.waits, (unsigned long long)ax.gave_up, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    if (n)
      __hip_atomic_fetch_add(v.waits + 1, (unsigned long long)n, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One generation for islands [base, base + v.ipw) of a run, by one wavefront.
// LC / SWC: log2 N and surface words fixed at compile time, or -1 to read them
// from the view. Model: the genome model. `lds` is this wavefront's table of
// 5 * ipw + 1 entries (16 bytes, 32 for a model with a string): arrivals
// [4 * local + q], emissions [4 * ipw + local], and one scratch entry read when
// a lane has no arrival.
template <int LC, int SWC, bool ASYNC = false, typename Model = FitnessModel, bool WIDE = false,
          bool LOCK = false>
__device__ __forceinline__ void chunk_generation(const RunView& v, uint32_t base, uint64_t t,
                                                 uint4* lds, AsyncCtx* ax = nullptr) {
  constexpr bool kStr = Model::kString;      // genomes carry a string
  constexpr uint32_t ES = kStr ? 2u : 1u;    // 16-byte units per LDS entry
  const uint32_t L = LC >= 0 ? (uint32_t)LC : v.log2n;
  const uint32_t SW = SWC >= 0 ? (uint32_t)SWC : v.words;
  const uint32_t lane = __lane_id();
  const uint32_t N = 1u << L;
  const uint32_t per_iter = 64u >> L;  // islands per wavefront iteration
  const uint32_t t_lo = (uint32_t)t;
  const uint32_t t_hi4 = (uint32_t)(t >> 32) << 2;
  const bool odd_gen = ((uint32_t)t & 1u) != 0u;  // emit into parity t&1, absorb the other
  const uint32_t W = v.width, H = v.height;
  const uint32_t* __restrict__ in_ob = odd_gen ? v.ob[0] : v.ob[1];
  uint32_t* __restrict__ out_ob = odd_gen ? v.ob[1] : v.ob[0];
  // words per outbox entry and header word: f, T, surface, header (model 0);
  // f, T, D0, D1, P0, P1, header (strings)
  const uint32_t ob_stride = (SW == 1 && !kStr) ? 4u : 8u;
  const uint32_t ob_hdr = kStr ? 6u : 2u + SW;

  // chunk base pointers (uniform) and this lane's byte offset in the chunk
  const uint32_t first_agent = base << L;
  float* __restrict__ pf = v.pop_f + first_agent;
  uint32_t* __restrict__ pT = v.pop_T + first_agent;
  uint32_t* __restrict__ pD0 = v.pop_D + first_agent;
  uint32_t* __restrict__ pD1 = v.pop_D + v.agent_stride + first_agent;
  uint32_t* __restrict__ pP0 = v.pop_P + first_agent;
  uint32_t* __restrict__ pP1 = v.pop_P + v.agent_stride + first_agent;
  const uint32_t n_iter = v.ipw >> (6u - L);
  uint32_t off = lane << 2;

  // the first iteration's genomes go in flight before the island pass, whose
  // own loads and draws then hide their latency
  Genome g = load_genome(pf, pT, pD0, pD1, pP0, pP1, off, SW, kStr);

  // ---- island pass: lane l handles island base + l ---------------------------
  const bool own_ok = lane < v.ipw && base + lane < v.islands;
  const uint32_t own = own_ok ? base + lane : base;
  const uint32_t ox = own % W, oy = own / W;
  const Block mig = philox10(0u, own, t_lo, t_hi4 | kStreamMigrate, v.seed, v.run_id);
  const uint32_t emig = L ? (mig.x >> (32u - L)) : 0u;
  // All four neighbour entries are loaded and parked in LDS whether they are
  // arrivals or not (for 32 sites the header rides in the same 16 bytes as the
  // genome; for 64 sites it is the next word), so the pass pays one memory
  // round trip; only the packed slots say which entries are arrivals.
  uint32_t desc = 0xFFFFFFFFu;  // byte q: slot taken by the arrival from direction q, or 0xFF
  uint32_t ready = 0u;          // lockstep: bit q set once the neighbour in direction q is done
  if constexpr (!ASYNC) {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t* e = in_ob + (size_t)torus_step(ox, oy, q, W, H) * ob_stride;
      const uint4 entry = *reinterpret_cast<const uint4*>(e);  // f, T, D0, header or D1
      uint4 more = make_uint4(0u, 0u, 0u, 0u);                  // P0, P1, header
      if (kStr) more = *reinterpret_cast<const uint4*>(e + 4);
      const uint32_t header = kStr ? more.z : (SW == 1 ? entry.w : e[ob_hdr]);
      const bool hit = own_ok && header == (kMetaValid | (q ^ 2u));
      const uint32_t slot = ((mig.z >> (8u * q)) & 0xFFu) >> (8u - L);
      desc = hit ? (desc & ~(0xFFu << (8u * q))) | (slot << (8u * q)) : desc;
      if (lane < v.ipw) {  // the table holds ipw islands
        lds[(lane * 4u + q) * ES] = entry;
        if (kStr) lds[(lane * 4u + q) * ES + 1u] = more;
      }
    }
  } else if constexpr (LOCK) {
    // Asynchronous schedule in lockstep (no lead). Every island writes, at the
    // end of generation g, the lockstep header of each of its four buffers of
    // parity g & 1: 2 (g + 1) toward the direction it sent a genome to,
    // 2 (g + 1) + 1 ("nothing") toward the others. So in generation t the
    // header of the neighbour's buffer of parity (t - 1) & 1 toward this
    // island says both that the neighbour has finished generation t - 1
    // (header >= 2t) and whether it sent a genome this way then (header ==
    // 2t). One wait on the four headers is the pacing, one read of the
    // payloads the exchange. The headers sit in a plane of their own, island
    // index fastest, so the headers a wavefront waits on share a few cache
    // lines. No re-read is needed: an island rewrites a buffer's payload only
    // after seeing that the neighbour it faces has finished the generation
    // that read the buffer's previous contents; after a wait that gave up it
    // sends nothing that way.
    const uint32_t due = 2u * t_lo;
    const uint32_t prev = (t_lo & 1u) ^ 1u;
    const uint32_t* mail = v.mail;
    const uint32_t* lock = v.lock;
    uint32_t hits = 0u;  // bit q: a genome was sent this way in generation t - 1
    for (uint32_t spin = 0;; ++spin) {
      uint32_t h[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q)
        h[q] = load_agent(
            lock_header(lock, torus_step(ox, oy, q, W, H), q ^ 2u, prev, v.island_stride));
      drain_memory();
      hits = 0u;
      ready = 0u;
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        hits |= (h[q] == due ? 1u : 0u) << q;
        ready |= ((int32_t)(h[q] - due) >= 0 ? 1u : 0u) << q;
      }
      if (__ballot(own_ok && ready != 15u) == 0ull) break;
      if (spin == kLockSpins) {
        ++ax->gave_up;
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    hits = own_ok ? hits : 0u;
    ax->taken += (uint32_t)__builtin_popcount(hits);
    // the entries, each with its stamp (the last one taken, as recorded)
    uint4 pay[4], pstr[4];
    uint32_t stamp[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      // the neighbour's buffer toward this island
      const uint32_t* e = mail_entry(mail, torus_step(ox, oy, q, W, H), q ^ 2u, prev, ob_stride);
      const uint2 lo = load_agent2(e);
      const uint2 hi = load_agent2(e + 2);  // D0, then D1 or the stamp
      pay[q] = make_uint4(lo.x, lo.y, hi.x, hi.y);
      pstr[q] = make_uint4(0u, 0u, 0u, 0u);
      stamp[q] = 0u;
      if (kStr) {
        const uint2 p = load_agent2(e + 4);
        const uint2 h2 = load_agent2(e + 6);  // stamp, padding
        pstr[q] = make_uint4(p.x, p.y, 0u, 0u);
        stamp[q] = h2.x;
      } else if (SW > 1) {
        stamp[q] = load_agent(e + 4);
      }
    }
    drain_memory();
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const bool hit = ((hits >> q) & 1u) != 0u;
      if (hit) v.seen[(size_t)own * 4u + q] = (SW == 1 && !kStr) ? pay[q].w : stamp[q];
      const uint32_t slot = ((mig.z >> (8u * q)) & 0xFFu) >> (8u - L);
      desc = hit ? (desc & ~(0xFFu << (8u * q))) | (slot << (8u * q)) : desc;
      if (lane < v.ipw) {
        lds[(lane * 4u + q) * ES] = pay[q];
        if (kStr) lds[(lane * 4u + q) * ES + 1u] = pstr[q];
      }
    }
  } else {
    // Asynchronous schedule. The neighbour in direction q keeps two buffers
    // toward this island (its buffers in direction q ^ 2), one per parity of
    // the sending generation, each with a stamp word 2 * (sending generation
    // + 1), odd while being rewritten. A genome is in flight during the
    // generation it was sent in, so in generation t a buffer is eligible if
    // its stamp is even, at most 2t, and newer than the last one taken from
    // that side; the newest eligible buffer is read, and its stamp read again
    // after the genome: the genome is taken if the two reads agree.
    uint32_t nb[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) nb[q] = torus_step(ox, oy, q, W, H);

    // Pacing: wait until every neighbouring chunk has completed at least
    // t - lead generations, checking at most kPaceSpins times, then go on
    // regardless (the exchange stays valid at any distance, only looser).
    if (ax->lead != kUnpaced) {
      uint32_t nbc[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) nbc[q] = nb[q] / v.ipw;
      for (uint32_t spin = 0;; ++spin) {
        bool behind = false;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q)
          behind |= (int32_t)(t_lo - ax->lead - load_agent(v.prog + nbc[q])) > 0;
        if (__ballot(own_ok && behind) == 0ull) break;
        if (spin == kPaceSpins) {
          ++ax->gave_up;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }

    uint32_t* seen_at = v.seen + (size_t)own * 4u;
    const uint4 seen4 = *reinterpret_cast<const uint4*>(seen_at);
    uint32_t seen_q[4] = {seen4.x, seen4.y, seen4.z, seen4.w};
    const uint32_t newest_ok = 2u * t_lo;  // stamp of a genome sent in t-1
    uint32_t* box[4];
    uint32_t stamp[4];
    bool ok[4];
    {
      uint32_t s0[4], s1[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        box[q] = mail_entry(v.mail, nb[q], q ^ 2u, 0u, ob_stride);
        s0[q] = load_agent(box[q] + ob_hdr);
        s1[q] = load_agent(box[q] + ob_stride + ob_hdr);
      }
      drain_memory();
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const bool e0 = (s0[q] & 1u) == 0u && (int32_t)(newest_ok - s0[q]) >= 0 &&
                        (int32_t)(s0[q] - seen_q[q]) > 0;
        const bool e1 = (s1[q] & 1u) == 0u && (int32_t)(newest_ok - s1[q]) >= 0 &&
                        (int32_t)(s1[q] - seen_q[q]) > 0;
        const bool take1 = e1 && (!e0 || (int32_t)(s1[q] - s0[q]) > 0);
        ok[q] = e0 || e1;
        stamp[q] = take1 ? s1[q] : s0[q];
        box[q] += take1 ? ob_stride : 0u;
      }
    }
    uint4 pay[4], pstr[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint2 lo = load_agent2(box[q]);
      const uint2 hi = load_agent2(box[q] + 2);  // D0, then D1 or the stamp
      pay[q] = make_uint4(lo.x, lo.y, hi.x, SW > 1 || kStr ? hi.y : 0u);
      pstr[q] = make_uint4(0u, 0u, 0u, 0u);
      if (kStr) {
        const uint2 p = load_agent2(box[q] + 4);
        pstr[q] = make_uint4(p.x, p.y, 0u, 0u);
      }
    }
    drain_memory();
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t again = load_agent(box[q] + ob_hdr);
      const bool hit = own_ok && ok[q] && again == stamp[q];
      ax->taken += hit ? 1u : 0u;
      seen_q[q] = hit ? stamp[q] : seen_q[q];
      const uint32_t slot = ((mig.z >> (8u * q)) & 0xFFu) >> (8u - L);
      desc = hit ? (desc & ~(0xFFu << (8u * q))) | (slot << (8u * q)) : desc;
      if (lane < v.ipw) {
        lds[(lane * 4u + q) * ES] = pay[q];
        if (kStr) lds[(lane * 4u + q) * ES + 1u] = pstr[q];
      }
    }
    if (own_ok)
      *reinterpret_cast<uint4*>(seen_at) = make_uint4(seen_q[0], seen_q[1], seen_q[2], seen_q[3]);
  }
  // emission: slot and header of what this island sends; the lane holding the
  // post-absorb member in that slot parks it in the LDS table during its
  // iteration, and the island's lane writes the outbox entry after the loop
  const uint32_t emit = own_ok ? (emig | ((v.migration ? (kMetaValid | (mig.y >> 30)) : 0u) << 8))
                               : 0xFFu;
  // hand the arrival table to the other lanes of this wavefront
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- iterations: lanes are agent slots ------------------------------------
  const BreedLane bl = breed_lane<LC>(v, t);
  const uint32_t slot = bl.slot;
  const uint32_t slot_bytes = slot * 0x01010101u;
  const uint32_t emit_base = 4u * v.ipw;
  const uint32_t scratch = 5u * v.ipw;

  // One iteration of loads stays in flight ahead of the compute. The wait
  // below settles the prologue loads once, so the loop body has no pending
  // load on its working registers and no divergent memory access: its only
  // wait is for the prefetched genomes, at the end of the iteration.
  __builtin_amdgcn_s_waitcnt(0);
  for (uint32_t it = 0; it < n_iter; ++it) {
    // next iteration's genomes; the last iteration reloads its own (cache
    // hits, values unused) rather than reaching into the next chunk, whose
    // lines often belong to another XCD's wavefront and would be fetched from
    // HBM a second time
    const uint32_t next_off = it + 1u < n_iter ? off + 256u : off;
    const Genome next = load_genome(pf, pT, pD0, pD1, pP0, pP1, next_off, SW, kStr);
    Genome cur = g;
    const uint32_t local = it * per_iter + (lane >> L);
    const uint32_t island = base + local;

    // 1. absorb: the last arriving direction whose drawn slot is mine wins.
    //    Bytes of x are zero exactly where the descriptor names my slot; z
    //    keeps the top bit of each such byte, and its highest set bit is the
    //    last direction.
    const uint32_t x = permute(desc, local << 2) ^ slot_bytes;
    const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    {
      // no branch: lanes without an arrival read the scratch entry and keep
      // their genome, so the loop carries no memory access under divergence
      const uint32_t q = (31u - __clz(z | 1u)) >> 3;
      const uint32_t at = (z ? local * 4u + q : scratch) * ES;
      const uint4 a = lds[at];
      cur.f = z ? __uint_as_float(a.x) : cur.f;
      cur.T = z ? a.y : cur.T;
      cur.D0 = z ? a.z : cur.D0;
      cur.D1 = z ? a.w : cur.D1;
      if (kStr) {
        const uint4 b = lds[at + 1u];
        cur.P0 = z ? b.x : cur.P0;
        cur.P1 = z ? b.y : cur.P1;
      }
    }

    // 2. the lane holding the island's drawn emigrant parks it in LDS
    if ((permute(emit, local << 2) & 0xFFu) == slot) {
      lds[(emit_base + local) * ES] = make_uint4(__float_as_uint(cur.f), cur.T, cur.D0, cur.D1);
      if (kStr) lds[(emit_base + local) * ES + 1u] = make_uint4(cur.P0, cur.P1, 0u, 0u);
    }

    // 3-7. tournament, copy, mutation, deposit
    const Genome c = breed<LC, SWC, Model, WIDE>(v, bl, cur, island);

    *at_byte(pf, off) = c.f;
    *at_byte(pT, off) = c.T;
    *at_byte(pD0, off) = c.D0;
    if (SW > 1) *at_byte(pD1, off) = c.D1;
    if (kStr) {
      *at_byte(pP0, off) = c.P0;
      *at_byte(pP1, off) = c.P1;
    }

    off += 256u;
    g = next;
  }

  // emissions: one 16-byte entry per island, consecutive across lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if constexpr (ASYNC && LOCK) {
    // the payload toward the drawn direction (if that neighbour is done with
    // the buffer) with its stamp in the entry's header word, as the general
    // exchange reads it; complete before the four lockstep headers
    const uint32_t hdr = emit >> 8;
    const uint32_t d = hdr & 3u;
    const bool sending = own_ok && hdr != 0u && ((ready >> d) & 1u) != 0u;
    const uint32_t stamp = 2u * (t_lo + 1u);
    if (sending) {
      uint32_t* box = mail_entry(v.mail, own, d, t_lo & 1u, ob_stride);
      const uint4 g = lds[(emit_base + lane) * ES];
      store_agent2(box, g.x, g.y);
      if (kStr) {
        const uint4 p = lds[(emit_base + lane) * ES + 1u];
        store_agent2(box + 2, g.z, g.w);
        store_agent2(box + 4, p.x, p.y);
        store_agent(box + 6, stamp);
      } else if (SW > 1) {
        store_agent2(box + 2, g.z, g.w);
        store_agent(box + 4, stamp);
      } else {
        store_agent2(box + 2, g.z, stamp);
      }
    }
    drain_memory();
    if (own_ok) {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q)
        store_agent(lock_header(v.lock, own, q, t_lo & 1u, v.island_stride),
                    (sending && q == d) ? stamp : stamp + 1u);
    }
  } else if constexpr (ASYNC) {
    // publish into this island's buffer toward the drawn direction for this
    // generation's parity: odd stamp, genome, even stamp, each step complete
    // before the next issues; then the chunk's progress
    const uint32_t hdr = emit >> 8;
    const bool sending = own_ok && hdr != 0u;
    uint32_t* box = mail_entry(v.mail, own, hdr & 3u, t_lo & 1u, ob_stride);
    const uint32_t stamp = 2u * (t_lo + 1u);
    if (sending) store_agent(box + ob_hdr, stamp - 1u);
    drain_memory();
    if (sending) {
      const uint4 g = lds[(emit_base + lane) * ES];
      store_agent2(box, g.x, g.y);
      if (SW > 1 || kStr) {
        store_agent2(box + 2, g.z, g.w);
      } else {
        store_agent(box + 2, g.z);
      }
      if (kStr) {
        const uint4 p = lds[(emit_base + lane) * ES + 1u];
        store_agent2(box + 4, p.x, p.y);
      }
    }
    drain_memory();
    if (sending) store_agent(box + ob_hdr, stamp);
    // complete before this wavefront's next chunk reads the buffers, and
    // before the progress word says the generation is done
    drain_memory();
    if (lane == 0u) store_agent(v.prog + base / v.ipw, t_lo + 1u);
  } else if (own_ok) {
    uint32_t* e = out_ob + (size_t)own * ob_stride;
    const uint32_t hdr = emit >> 8;
    if (hdr) {
      const uint4 g = lds[(emit_base + lane) * ES];
      if (kStr) {
        const uint4 p = lds[(emit_base + lane) * ES + 1u];
        *reinterpret_cast<uint4*>(e) = g;
        *reinterpret_cast<uint4*>(e + 4) = make_uint4(p.x, p.y, hdr, 0u);
      } else if (SW == 1) {
        *reinterpret_cast<uint4*>(e) = make_uint4(g.x, g.y, g.z, hdr);
      } else {
        *reinterpret_cast<uint4*>(e) = g;
        e[ob_hdr] = hdr;
      }
    } else {
      e[ob_hdr] = 0u;
    }
  }
}

// Dynamic LDS: a table of 5 * ipw + 1 entries per wavefront, each of `units`
// 16-byte units (1 for model 0, 2 for genomes with a string).
extern __shared__ uint4 ga_lds[];

__device__ __forceinline__ uint32_t lds_entries(uint32_t ipw) { return 5u * ipw + 1u; }

__device__ __forceinline__ uint4* wave_lds(uint32_t wave_in_group, uint32_t ipw, uint32_t units) {
  return ga_lds + wave_in_group * lds_entries(ipw) * units;
}

template <int LC, int SWC, typename Model, bool WIDE>
__global__ __launch_bounds__(1024) void generation_kernel(RunView v, uint32_t gen_offset) {
  const uint32_t wig = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wave = xcd_band_group() * (blockDim.x >> 6) + wig;
  const uint32_t base = wave * v.ipw;
  if (base >= v.islands) return;
  chunk_generation<LC, SWC, false, Model, WIDE>(v, base, *v.gen + gen_offset,
                                                wave_lds(wig, v.ipw, Model::kString ? 2u : 1u));
}

// Founders of a genome model that draws them (the initialize function): its
// initialize from the (slot, island) block of the sampling stream at
// generation 2^64 - 1, which no generation reaches.
template <typename Model>
__global__ void init_kernel(RunView v) {
  const uint32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= v.agents) return;
  const uint32_t island = a >> v.log2n, slot = a & ((1u << v.log2n) - 1u);
  const Block b = philox10(slot, island, 0xFFFFFFFFu, 0xFFFFFFFCu | kStreamSample, v.seed,
                           v.run_id);
  Genome g;
  g.f = v.pop_f[a];
  Model::initialize(g, b);
  v.pop_f[a] = g.f;
  if (Model::kString) {
    v.pop_P[a] = g.P0;
    v.pop_P[v.agent_stride + a] = g.P1;
  }
}

// Asynchronous schedule: each wavefront owns `chunks` consecutive chunks and
// runs n_gens generations over them with no barrier with any other wavefront;
// islands exchange genomes only through the stamped per-neighbour buffers,
// and an island waits (a bounded number of times) only while a neighbour is
// more than `lead` generations behind. Every wait ends, so the kernel ends
// however the wavefronts are scheduled; the grid is sized to the wavefronts
// the GPU holds at once, so all islands advance together.
// skew > 0 (one wavefront only): chunk c runs its generation g at step
// g + (c mod (skew + 1)), a reproducible interleaving with neighbours up to
// skew generations apart.
// eight wavefronts per SIMD: registers (scalar ones included) must fit, or the
// occupancy query would promise more resident wavefronts than the GPU holds
template <int LC, int SWC, typename Model, bool WIDE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void async_kernel(RunView v, uint32_t chunks, uint64_t n_gens, uint32_t lead, uint32_t skew) {
  const uint32_t wig = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + wig;
  const uint32_t first = wave * chunks * v.ipw;
  if (first >= v.islands) return;
  const uint32_t end = min(first + chunks * v.ipw, v.islands);
  const uint64_t t0 = *v.gen;
  uint4* lds = wave_lds(wig, v.ipw, Model::kString ? 2u : 1u);
  AsyncCtx ax{lead, 0u, 0u};
  for (uint64_t step = 0; step < n_gens + skew; ++step) {
    for (uint32_t base = first; base < end; base += v.ipw) {
      const uint64_t lag = skew ? (base / v.ipw) % (skew + 1u) : 0u;
      if (step < lag || step - lag >= n_gens) continue;
      chunk_generation<LC, SWC, true, Model, WIDE>(v, base, t0 + step - lag, lds, &ax);
    }
  }
  flush_async(v, ax);
}

// The asynchronous schedule with no lead and no skew: the lockstep exchange
// (same results as the synchronous schedule while no wait gives up), each
// wavefront over its `chunks` consecutive chunks as in async_kernel.
template <int LC, int SWC, typename Model, bool WIDE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void lockstep_kernel(RunView v, uint32_t chunks, uint64_t n_gens) {
  const uint32_t wig = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + wig;
  const uint32_t first = wave * chunks * v.ipw;
  if (first >= v.islands) return;
  const uint32_t end = min(first + chunks * v.ipw, v.islands);
  const uint64_t t0 = *v.gen;
  uint4* lds = wave_lds(wig, v.ipw, Model::kString ? 2u : 1u);
  AsyncCtx ax{0u, 0u, 0u};
  for (uint64_t step = 0; step < n_gens; ++step)
    for (uint32_t base = first; base < end; base += v.ipw)
      chunk_generation<LC, SWC, true, Model, WIDE, true>(v, base, t0 + step, lds, &ax);
  flush_async(v, ax);
}

// Before a lockstep launch at generation t0. After one generation under the
// lockstep headers, the genome sent in the previous generation is the only
// one the general rule could take (any older one was taken or passed over);
// in generation t0 itself, a launch with a lead or a skew before this one may
// have left an older genome pending. Thread (i, q) applies the general rule to
// the two buffers island i reads from direction q, once: the newest buffer
// whose stamp is even, at most 2 t0 and newer than the last one taken. If that
// is the buffer of parity t0 & 1, its entry (stamp included) is copied into
// the one of parity (t0 - 1) & 1, which the lockstep exchange reads in
// generation t0. The lockstep header of parity (t0 - 1) & 1 then reads 2 t0 if
// there is a genome to take, 2 t0 + 1 if not.
__global__ void lockstep_prologue_kernel(RunView v, uint32_t t0) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)v.islands * 4u) return;
  const uint32_t i = (uint32_t)(k >> 2), q = (uint32_t)k & 3u, d = q ^ 2u, p = (t0 & 1u) ^ 1u;
  const uint32_t ob_hdr = model_has_string(v.model) ? 6u : 2u + v.words;
  const uint32_t j = torus_step(i % v.width, i / v.width, q, v.width, v.height);
  uint32_t* read = mail_entry(v.mail, j, d, p, v.ob_stride);
  const uint32_t* other = mail_entry(v.mail, j, d, p ^ 1u, v.ob_stride);
  const uint32_t due = 2u * t0, seen = v.seen[k];
  const uint32_t s0 = read[ob_hdr], s1 = other[ob_hdr];
  const bool e0 = (s0 & 1u) == 0u && (int32_t)(due - s0) >= 0 && (int32_t)(s0 - seen) > 0;
  const bool e1 = (s1 & 1u) == 0u && (int32_t)(due - s1) >= 0 && (int32_t)(s1 - seen) > 0;
  if (e1 && (!e0 || (int32_t)(s1 - s0) > 0))
    for (uint32_t w = 0; w < v.ob_stride; ++w) read[w] = other[w];
  *lock_header(v.lock, j, d, p, v.island_stride) = (e0 || e1) ? due : due + 1u;
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
  for (uint32_t w = 0; w < v.words; ++w)
    D_out[(size_t)w * n + j] = v.pop_D[(size_t)w * v.agent_stride + a];
}

// The member table holds each run's pointers as byte offsets from the table
// itself: rebuilt from the kernel's table argument they are known to address
// global memory, so the bodies use global (not flat) loads and stores.
template <typename T>
__device__ __forceinline__ T* table_ptr(const RunView* table, T* off) {
  return reinterpret_cast<T*>(const_cast<char*>(reinterpret_cast<const char*>(table)) +
                              reinterpret_cast<uintptr_t>(off));
}
__device__ __forceinline__ void from_table(RunView& v, const RunView* table) {
  v.pop_f = table_ptr(table, v.pop_f);
  v.pop_T = table_ptr(table, v.pop_T);
  v.pop_D = table_ptr(table, v.pop_D);
  v.ob[0] = table_ptr(table, v.ob[0]);
  v.ob[1] = table_ptr(table, v.ob[1]);
  v.gen = table_ptr(table, v.gen);
  v.left = table_ptr(table, v.left);
}

// Memory that stays unchanged for a whole launch (the member table, a
// member's counters) is read through the constant address space, which the
// compiler issues as scalar loads straight into scalar registers: the batched
// form's member pointers then stay scalar (and global) through the
// generation's loop, as a plain launch's kernel arguments do, and a
// wavefront's start waits on no vector memory round trip for them.
typedef __attribute__((address_space(4))) const uint32_t ConstWord;
__device__ __forceinline__ uint32_t const_word(const void* p) {
  return *(ConstWord*)p;
}
__device__ __forceinline__ uint64_t const_u64(const void* p) {
  return (uint64_t)const_word(p) | ((uint64_t)const_word((const char*)p + 4) << 32);
}
// Member `run` of the table, one word at a time (an aggregate copy would be
// turned back into vector loads).
__device__ __forceinline__ RunView load_member(const RunView* table, uint32_t run) {
  RunView v;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(table + run);
#pragma unroll
  for (uint32_t i = 0; i < sizeof(RunView) / 4; ++i) dst[i] = const_word(src + i);
  from_table(v, table);
  return v;
}

// Every view word a synchronous body reads, requested before the member's
// counters are read (and both counters before they are tested): left to
// itself the compiler issues them after that test, a few at a time, and a
// starting wavefront waits on one scalar round trip after another before its
// first genome load.
__device__ __forceinline__ void view_ready(const RunView& v) {
  asm volatile("" ::"s"(v.pop_f), "s"(v.pop_T), "s"(v.pop_D), "s"(v.ob[0]), "s"(v.ob[1]),
               "s"(v.width), "s"(v.height), "s"(v.islands), "s"(v.agent_stride), "s"(v.ipw),
               "s"(v.seed), "s"(v.run_id), "s"(v.migration), "s"(v.k), "s"(v.selection),
               "s"(v.p32), "s"(v.law), "s"(v.p_ben), "s"(v.p_any), "s"(v.s_log), "s"(v.dlog),
               "s"(v.policy));
}

// Batched form, one launch per generation over every member's tiles (sorted by
// class, so neighbouring wavefronts run the same shape). Wavefront w runs the
// tile in slot w of the table, which the host lays out so that each XCD's
// workgroups (the dispatcher hands workgroup g to XCD g mod 8) take a
// contiguous stretch of tiles of about equal bytes; slots past the live tiles
// are empty, so a captured launch follows membership changes. Each wavefront
// branches (uniformly) to the body compiled for its member's log2 N and
// surface words.
__global__ __launch_bounds__(1024) void batch_all_kernel(const RunView* __restrict__ views,
                                                         const Tile* __restrict__ tiles,
                                                         uint32_t gen_offset, uint32_t max_ipw) {
  const uint32_t wig = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + wig;
  const uint32_t run = const_word(&tiles[wave].run), first = const_word(&tiles[wave].first);
  uint4* lds = wave_lds(wig, max_ipw, 1u);
  // only the tile is read before the branch; each body loads the member's
  // view itself (nothing of it stays live across the branch), then its two
  // counters side by side (the budget left follows the generation counter)
  switch (const_word(&tiles[wave].cls)) {
#define GA_BATCH_CASE(L, S)                                  \
  case L * 2 + S - 1: {                                      \
    const RunView v = load_member(views, run);               \
    view_ready(v);                                           \
    const uint64_t t0 = const_u64(v.gen), left = const_u64(v.gen + 1); \
    asm volatile("" ::"s"(t0), "s"(left));                   \
    if (left <= gen_offset) return;                          \
    chunk_generation<L, S>(v, first, t0 + gen_offset, lds);  \
    break;                                                   \
  }
    GA_BATCH_CASE(0, 1) GA_BATCH_CASE(0, 2) GA_BATCH_CASE(1, 1) GA_BATCH_CASE(1, 2)
    GA_BATCH_CASE(2, 1) GA_BATCH_CASE(2, 2) GA_BATCH_CASE(3, 1) GA_BATCH_CASE(3, 2)
    GA_BATCH_CASE(4, 1) GA_BATCH_CASE(4, 2) GA_BATCH_CASE(5, 1) GA_BATCH_CASE(5, 2)
    GA_BATCH_CASE(6, 1) GA_BATCH_CASE(6, 2)
#undef GA_BATCH_CASE
    default: break;  // an empty slot (members' classes are validated on admission)
  }
}

__global__ void store_u64_kernel(unsigned long long* p, unsigned long long value) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

// Close a block: each member's counter advances by what it ran of the block.
// The member count lives in device memory (the grid covers the table's capacity).
__global__ void batch_advance_kernel(const RunView* views, const uint32_t* n_runs, uint64_t block) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_runs) return;
  RunView v = views[i];
  from_table(v, views);
  const unsigned long long left = *v.left;
  const unsigned long long done = left < block ? left : block;
  *v.gen = *v.gen + done;
  *v.left = left - done;
}

}  // namespace

size_t lds_bytes(uint32_t ipw, uint32_t waves, uint32_t model) {
  return (5u * ipw + 1u) * sizeof(uint4) * (model_has_string(model) ? 2u : 1u) * waves;
}

hipError_t launch_generation(const RunView& v, uint32_t gen_offset, uint32_t waves,
                             uint32_t waves_per_group, hipStream_t stream) {
  if (waves == 0) return hipSuccess;
  const uint32_t groups = (waves + waves_per_group - 1) / waves_per_group;
  const dim3 grid(groups), block(64 * waves_per_group);
  const size_t lds = lds_bytes(v.ipw, waves_per_group, v.model);
  return dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    generation_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)><<<grid, block, lds, stream>>>(v, gen_offset);
    return hipGetLastError();
  });
}

hipError_t launch_async(const RunView& v, uint64_t n_gens, uint32_t waves, uint32_t chunks,
                        uint32_t waves_per_group, uint32_t lead, uint32_t skew,
                        hipStream_t stream) {
  if (waves == 0 || n_gens == 0) return hipSuccess;
  const uint32_t groups = (waves + waves_per_group - 1) / waves_per_group;
  const dim3 grid(groups), block(64 * waves_per_group);
  const size_t lds = lds_bytes(v.ipw, waves_per_group, v.model);
  return dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    async_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)><<<grid, block, lds, stream>>>(v, chunks, n_gens,
                                                                           lead, skew);
    return hipGetLastError();
  });
}

hipError_t launch_lockstep(const RunView& v, uint64_t gen, uint64_t n_gens, uint32_t waves,
                           uint32_t chunks, uint32_t waves_per_group, hipStream_t stream) {
  if (waves == 0 || n_gens == 0) return hipSuccess;
  const size_t fix = (size_t)v.islands * 4u;
  lockstep_prologue_kernel<<<dim3((uint32_t)((fix + 255u) / 256u)), dim3(256), 0, stream>>>(
      v, (uint32_t)gen);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t groups = (waves + waves_per_group - 1) / waves_per_group;
  const dim3 grid(groups), block(64 * waves_per_group);
  const size_t lds = lds_bytes(v.ipw, waves_per_group, v.model);
  return dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    lockstep_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)><<<grid, block, lds, stream>>>(v, chunks, n_gens);
    return hipGetLastError();
  });
}

hipError_t async_capacity(const RunView& v, uint32_t waves_per_group, bool lockstep,
                          uint32_t* waves) {
  int device = 0, cus = 0, groups = 0;
  hipError_t e = hipGetDevice(&device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  const int block = 64 * (int)waves_per_group;
  const size_t lds = lds_bytes(v.ipw, waves_per_group, v.model);
  e = dispatch(v, [&](auto LC, auto SWC, auto M, auto WD) {
    return lockstep ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &groups, lockstep_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)>, block, lds)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &groups, async_kernel<GA_SHAPE_ARGS(LC, SWC, M, WD)>, block, lds);
  });
  if (e != hipSuccess) return e;
  *waves = (uint32_t)groups * (uint32_t)cus * waves_per_group;
  return hipSuccess;
}

bool model_has_string_host(uint32_t id) { return model_has_string(id); }
uint32_t model_count() { return kModelCount; }

hipError_t launch_init(const RunView& v, hipStream_t stream) {
  if (v.agents == 0) return hipSuccess;
  const dim3 grid((v.agents + 255) / 256), block(256);
#define GA_INIT_CASE(ID, M)                                \
  case ID:                                                 \
    init_kernel<M><<<grid, block, 0, stream>>>(v);         \
    break;
  switch (v.model) {
    GA_FOR_EACH_MODEL(GA_INIT_CASE)
    default: return hipErrorInvalidValue;
  }
#undef GA_INIT_CASE
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

hipError_t launch_batch_all(const RunView* views, const Tile* tiles, uint32_t grid_waves,
                            uint32_t gen_offset, uint32_t max_ipw, uint32_t waves_per_group,
                            hipStream_t stream) {
  if (grid_waves == 0) return hipSuccess;
  if (waves_per_group == 0 || grid_waves % waves_per_group) return hipErrorInvalidValue;
  const uint32_t groups = grid_waves / waves_per_group;
  const size_t lds = lds_bytes(max_ipw, waves_per_group, 0u);
  batch_all_kernel<<<dim3(groups), dim3(64 * waves_per_group), lds, stream>>>(
      views, tiles, gen_offset, max_ipw);
  return hipGetLastError();
}

hipError_t launch_store_u64(unsigned long long* p, unsigned long long value, hipStream_t stream) {
  store_u64_kernel<<<1, 64, 0, stream>>>(p, value);
  return hipGetLastError();
}

hipError_t launch_batch_advance(const RunView* views, const uint32_t* n_runs, uint32_t cap,
                                uint64_t block, hipStream_t stream) {
  if (cap == 0) return hipSuccess;
  batch_advance_kernel<<<dim3((cap + 255) / 256), dim3(256), 0, stream>>>(views, n_runs, block);
  return hipGetLastError();
}

}  // namespace ga
