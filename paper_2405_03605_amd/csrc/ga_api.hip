// C ABI of libga_hip: configuration checks, device layout, launch planning,
// HIP-graph capture of generation blocks, state I/O and the batched form.
// Declarations and semantics: include/ga.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/ga.h"
#include "ga_internal.hpp"

namespace {

thread_local std::string g_last_error;

// A roctx range (recorded by rocprofv3 --marker-trace) over host work that
// submits generations: a step call, and inside it each graph block. Ranges
// time the submission on the host thread; the kernels run after it.
struct Range {
  Range(const char* what, uint64_t gens) {
    char name[64];
    std::snprintf(name, sizeof name, "%s %llu", what, (unsigned long long)gens);
    roctxRangePushA(name);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return GA_EDEVICE;
}

#define GA_HIP(call, what)                      \
  do {                                          \
    hipError_t _e = (call);                     \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

constexpr size_t kAlign = 256;
// Most tiles of the LDS-resident form (one workgroup each, all resident at once).
constexpr uint32_t kMaxTiles = 8192;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sizes of earlier configuration layouts: before mutation_law /
// beneficial_threshold, and before schedule.
constexpr uint32_t kConfigV1Size = (uint32_t)offsetof(ga_config, mutation_law);
constexpr uint32_t kConfigV2Size = (uint32_t)offsetof(ga_config, schedule);
constexpr uint32_t kConfigV3Size = (uint32_t)offsetof(ga_config, genome_model);
constexpr uint32_t kConfigV4Size = (uint32_t)offsetof(ga_config, differentia_bits);
constexpr uint32_t kConfigV5Size = (uint32_t)offsetof(ga_config, surface_policy);

bool is_pow2(uint32_t v) { return v != 0 && (v & (v - 1)) == 0; }
uint32_t log2u(uint32_t v) {
  uint32_t l = 0;
  while ((1u << l) < v) ++l;
  return l;
}

uint32_t dbits_of(const ga_config* c) {
  return c->struct_size > kConfigV4Size ? c->differentia_bits : 1u;
}

uint32_t policy_of(const ga_config* c) {
  return c->struct_size > kConfigV5Size ? c->surface_policy : GA_POLICY_STEADY;
}

// S sites of b-bit differentia filling one or two 32-bit words
bool surface_ok(uint32_t sites, uint32_t b) {
  if (b != 1 && b != 2 && b != 4 && b != 8) return false;
  if (!is_pow2(sites) || sites < 4 || sites > 64) return false;
  return sites * b == 32 || sites * b == 64;
}

bool policy_ok(uint32_t policy, uint32_t sites, uint32_t b, std::string* why) {
  const char* m = nullptr;
  if (policy > GA_POLICY_HYBRID) m = "surface_policy must be 0 (steady), 1 (tilted) or 2 (hybrid)";
  else if (policy == GA_POLICY_TILTED && sites != 32 && sites != 64)
    m = "the tilted policy needs 32 or 64 sites";
  else if (policy == GA_POLICY_HYBRID && (sites != 64 || b != 1))
    m = "the hybrid policy needs 64 one-bit sites";
  if (m && why) *why = m;
  return m == nullptr;
}

size_t surface_words(const ga_config* c) { return c->surface_sites * dbits_of(c) / 32; }

bool config_ok(const ga_config* c, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (!c) return no("config is NULL");
  if (c->struct_size != sizeof(ga_config) && c->struct_size != kConfigV1Size &&
      c->struct_size != kConfigV2Size && c->struct_size != kConfigV3Size &&
      c->struct_size != kConfigV4Size && c->struct_size != kConfigV5Size)
    return no("struct_size must be sizeof(ga_config)");
  if (c->width < 1 || c->width > 65535) return no("width must be in [1, 65535]");
  if (c->height < 1 || c->height > 65535) return no("height must be in [1, 65535]");
  if (!is_pow2(c->pop_per_island) || c->pop_per_island > 64)
    return no("pop_per_island must be a power of two in [1, 64]");
  if (!surface_ok(c->surface_sites, dbits_of(c)))
    return no("surface_sites x differentia_bits must be 32 or 64 bits, differentia_bits 1, 2, "
              "4 or 8, surface_sites a power of two >= 4");
  if (c->tournament_size < 1 || c->tournament_size > 8) return no("tournament_size must be in [1, 8]");
  if (c->selection > 1) return no("selection must be 0 or 1");
  if (c->migration > 1) return no("migration must be 0 or 1");
  if (!policy_ok(policy_of(c), c->surface_sites, dbits_of(c), why)) return false;
  if (c->struct_size > kConfigV2Size && c->schedule > GA_SCHEDULE_ASYNC)
    return no("schedule must be 0 (synchronous) or 1 (asynchronous)");
  if (c->struct_size > kConfigV3Size) {
    if (c->genome_model >= ga::model_count())
      return no("genome_model must name a compiled-in model (0 fitness, 1 OneMax, 2 Trap-4)");
    if (ga::model_has_string_host(c->genome_model) && c->mutation_law != 0)
      return no("a genome model with a string uses mutation_law 0");
  }
  if (c->struct_size >= kConfigV2Size) {
    if (c->mutation_law > 1) return no("mutation_law must be 0 or 1");
    if (c->mutation_law == 1 &&
        (uint64_t)c->beneficial_threshold + c->mutation_threshold > 0xFFFFFFFFull)
      return no("beneficial_threshold + mutation_threshold must be < 2^32");
  }
  const uint64_t agents = (uint64_t)c->width * c->height * c->pop_per_island;
  if (agents >= (1ull << 30)) return no("width * height * pop_per_island must be < 2^30");
  return true;
}

// Byte offsets of every plane inside a run's device buffer.
struct Layout {
  size_t pop_f, pop_T, pop_D, pop_P;
  size_t ob[2];     // synchronous schedule
  size_t mail, seen, prog, lock;  // asynchronous schedule
  size_t counters;  // generation counter, batch budget
  size_t st_ids, st_T, st_D;
  size_t total;
};

bool is_async(const ga_config* c) {
  return c->struct_size > kConfigV2Size && c->schedule == GA_SCHEDULE_ASYNC;
}

uint32_t model_of(const ga_config* c) {
  return c->struct_size > kConfigV3Size ? c->genome_model : GA_MODEL_FITNESS;
}

// words per AoS outbox entry: fitness, T, surface words, header, padding to 16 B;
// with a string: fitness, T, two surface words, two string words, header, pad
size_t outbox_stride(const ga_config* c) {
  return surface_words(c) == 1 && !ga::model_has_string_host(model_of(c)) ? 4 : 8;
}

// Planes run 128 islands past the last 64-island boundary: a wavefront's last
// chunk may end up to 63 islands past the last island (the rest is slack).
size_t padded_islands(const ga_config* c) {
  const size_t islands = (size_t)c->width * c->height;
  return (islands + 63) / 64 * 64 + 128;
}

Layout layout_of(const ga_config* c) {
  const size_t islands = padded_islands(c);
  const size_t agents = islands * c->pop_per_island;
  const size_t words = surface_words(c);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.pop_f = take(agents * 4);
  L.pop_T = take(agents * 4);
  L.pop_D = take(agents * 4 * words);
  if (ga::model_has_string_host(model_of(c))) L.pop_P = take(agents * 4 * 2);
  if (is_async(c)) {
    // eight buffers per island (direction x parity), four stamps, one
    // progress word per possible chunk, and the lockstep headers (eight per
    // island)
    L.mail = take(islands * 8 * 4 * outbox_stride(c));
    L.seen = take(islands * 4 * 4);
    L.prog = take(islands * 4);
    L.lock = take(islands * 8 * 4);
  } else {
    for (int p = 0; p < 2; ++p) L.ob[p] = take(islands * 4 * outbox_stride(c));
    // LDS-resident tiles: a progress word per tile (never more tiles than islands)
    L.prog = take(std::min<size_t>(kMaxTiles, (size_t)c->width * c->height) * 4);
  }
  L.counters = take(32);  // generation, batch budget, async give-ups, async genomes taken
  L.st_ids = take(islands * 4);
  L.st_T = take(islands * 4);
  L.st_D = take(islands * 4 * words);
  L.total = o;
  return L;
}

}  // namespace

struct ga_run {
  ga_config cfg{};
  ga::RunView view{};
  Layout lay{};
  hipStream_t stream = nullptr;
  uint8_t* base = nullptr;
  uint64_t gen_host = 0;
  uint32_t ipw = 64;
  bool ipw_set = false;  // islands per wavefront chosen by the caller (not the default)
  uint32_t wpg = 4;
  uint32_t form = GA_FORM_AUTO;
  uint32_t graph_block = 100;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  uint32_t graph_key_ipw = 0, graph_key_wpg = 0, graph_key_block = 0;
  ga_batch* batch = nullptr;
  uint32_t async_max_waves = 0;  // 0: as many as the GPU holds at once
  uint32_t async_lead = 0;       // pacing bound (ga::kUnpaced: none)
  uint32_t async_skew = 0;       // reproducible skewed interleaving (one wavefront)
  uint32_t want_tile_w = 0, want_tile_h = 0;  // caller's tile shape (0: chosen here)
  int tile_state = 0;            // 0 not planned, 1 planned (view.tile_*), -1 no tiling fits
  std::string tile_why;          // why no tiling fits
};

// Per-class settings of a batch: one class per (log2 N, surface words).
struct BatchClass {
  uint32_t ipw = 0;      // islands per wavefront (0: the batch's default rule)
  uint32_t n_tiles = 0;  // tiles of the current members
};

struct ga_batch {
  hipStream_t stream = nullptr;
  std::vector<ga_run*> members;
  std::vector<uint64_t> remaining;
  std::vector<uint64_t> finished_step;  // step call at which the member's budget ran out
  // device tables: [views: view_cap RunViews][tiles: tile_cap slots][tile count, member count]
  uint8_t* d_tab = nullptr;
  uint32_t view_cap = 0, tile_cap = 0;
  // pinned staging for the table uploads, two buffers used in turn, each free
  // again once its copy's event has completed
  uint8_t* h_stage[2] = {nullptr, nullptr};
  hipEvent_t stage_done[2] = {nullptr, nullptr};
  size_t stage_bytes = 0;
  int stage_next = 0;
  BatchClass cls[ga::kBatchClasses];
  uint32_t wpg = 4;            // wavefronts per group of the batch launch
  uint32_t ipw_override = 0;   // default islands per wavefront (0: about 512 agents per wavefront)
  uint32_t graph_block = 100;
  // the launch the graph was captured with: wavefronts covered (with
  // headroom), largest islands per wavefront (sizes the LDS), group size
  uint32_t grid_waves = 0, use_max_ipw = 0, use_wpg = 0;
  bool dirty = true;           // membership or shapes changed since the last upload
  bool graph_stale = true;     // the captured graph no longer matches
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  // one event per step call (ring; step_of[i] the call whose event slot i
  // holds): a member whose budget ran out at step s is settled once step s
  // has completed. At most kStepsInFlight calls are left in flight (a call
  // waits for the one kStepsInFlight before it), so the host cannot run
  // ahead of the GPU by more than that, and a slot is reused only after its
  // step is known complete (done_through: every step up to it has run).
  static constexpr int kStepEvents = 8;
  static constexpr uint64_t kStepsInFlight = 2;
  hipEvent_t step_done[kStepEvents] = {};
  uint64_t step_of[kStepEvents] = {};
  uint64_t done_through = 0;
  uint64_t steps = 0;          // step calls so far
};

// A run pool: runs sub-allocated from one caller-owned device buffer and
// advanced together as one batch. Free space is a map offset -> size of
// disjoint, non-adjacent blocks (adjacent ones are merged on release); runs
// take the first block that fits.
struct ga_pool {
  uint8_t* base = nullptr;
  size_t bytes = 0;
  uint32_t max_slots = 0;
  ga_batch* batch = nullptr;
  std::map<size_t, size_t> free_blocks;
  struct Member {
    ga_run* run;
    size_t off, size;
  };
  std::map<uint64_t, Member> members;
  uint64_t next_ticket = 1;
  size_t used = 0;
  // retirement samples a finished run on a stream of its own, so the batch
  // stream keeps running the next block meanwhile
  hipStream_t side = nullptr;
  hipEvent_t batch_mark = nullptr, side_mark = nullptr;
};

namespace {

// First block of the pool's free space that holds `size` bytes; SIZE_MAX if none.
size_t pool_take(ga_pool* p, size_t size) {
  for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
    if (it->second < size) continue;
    const size_t off = it->first, left = it->second - size;
    p->free_blocks.erase(it);
    if (left) p->free_blocks.emplace(off + size, left);
    return off;
  }
  return SIZE_MAX;
}

// Return [off, off + size) to the pool's free space, merging with neighbours.
void pool_give(ga_pool* p, size_t off, size_t size) {
  auto next = p->free_blocks.lower_bound(off);
  if (next != p->free_blocks.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      off = prev->first;
      size += prev->second;
      p->free_blocks.erase(prev);
    }
  }
  if (next != p->free_blocks.end() && off + size == next->first) {
    size += next->second;
    p->free_blocks.erase(next);
  }
  p->free_blocks.emplace(off, size);
}

uint32_t per_iter(const ga_run* r) { return 64u >> r->view.log2n; }

// Default islands per wavefront: 16 (measured best for large grids on
// MI355X), fewer when that leaves under 4 wavefronts per SIMD (1024 SIMDs),
// never fewer than one iteration's worth (64/N islands).
uint32_t default_ipw(const ga::RunView& v) {
  const uint32_t g = 64u >> v.log2n;
  uint32_t ipw = 16;
  while (ipw > g && (v.islands + ipw - 1) / ipw < 4096) ipw >>= 1;
  return std::max(g, std::min(64u, ipw));
}

uint32_t waves_for(const ga_run* r, uint32_t ipw) {
  return (r->view.islands + ipw - 1) / ipw;
}

// LDS of one CU (gfx950), the most a workgroup can take.
constexpr size_t kMaxGroupLds = 160 * 1024;

// Default lower bound on a tile's agents: below it the per-generation
// exchange between tiles costs more than the work it spreads.
constexpr uint32_t kMinTileAgents = 2048;

uint32_t ceil_div(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

struct TileCand {
  uint32_t tw, th, gx, gy;
  size_t lds;
  uint32_t threads;
};

TileCand tile_cand(const ga::RunView& v, uint32_t tw, uint32_t th) {
  TileCand c{tw, th, ceil_div(v.width, tw), ceil_div(v.height, th), 0, 0};
  c.lds = ga::tile_lds_bytes(tw, th, v.log2n, v.words, v.model, v.ob_stride);
  c.threads = ga::tile_threads(tw, th, v.log2n);
  return c;
}

// Whether every tile's workgroup of candidate c can be resident at once:
// first a bound from LDS and threads per CU alone, then the occupancy query.
int tile_fits(const ga::RunView& v, const TileCand& c, uint32_t cus, bool* fits) {
  *fits = false;
  if (c.lds > kMaxGroupLds || (size_t)c.gx * c.gy > kMaxTiles) return GA_OK;
  const uint64_t bound = std::min<uint64_t>(kMaxGroupLds / c.lds, 2048u / c.threads);
  if ((uint64_t)c.gx * c.gy > bound * cus) return GA_OK;
  int groups = 0;
  GA_HIP(ga::tile_occupancy(v, c.threads, c.lds, &groups), "occupancy query");
  *fits = (uint64_t)c.gx * c.gy <= (uint64_t)groups * (uint64_t)cus;
  return GA_OK;
}

// The tiling of the LDS-resident form: the caller's tile shape, or the one
// that spreads the run over the most CUs (smallest tiles, but not below
// kMinTileAgents agents), then the fewest tiles, then the squarest; every
// tile's workgroup must be resident at once. Sets view.tile_* and tile_state.
int plan_tiles(ga_run* r) {
  if (r->tile_state != 0) return GA_OK;
  ga::RunView& v = r->view;
  const uint32_t W = v.width, H = v.height, N = 1u << v.log2n;
  std::vector<TileCand> cands;
  if (r->want_tile_w) {
    cands.push_back(tile_cand(v, std::min(r->want_tile_w, W), std::min(r->want_tile_h, H)));
  } else {
    // distinct tile widths ceil(W / k) and heights ceil(H / k)
    std::vector<uint32_t> ws, hs;
    for (uint32_t k = 1; k <= W; ++k)
      if (ws.empty() || ws.back() != ceil_div(W, k)) ws.push_back(ceil_div(W, k));
    for (uint32_t k = 1; k <= H; ++k)
      if (hs.empty() || hs.back() != ceil_div(H, k)) hs.push_back(ceil_div(H, k));
    const uint64_t floor_agents = std::min<uint64_t>((uint64_t)v.agents, kMinTileAgents);
    for (uint32_t tw : ws)
      for (uint32_t th : hs) {
        const TileCand c = tile_cand(v, tw, th);
        if (c.lds > kMaxGroupLds || (uint64_t)c.gx * c.gy > kMaxTiles) continue;
        cands.push_back(c);
      }
    auto key = [&](const TileCand& c) {
      const uint64_t agents = (uint64_t)c.tw * c.th * N;
      return std::make_tuple(std::max(agents, floor_agents), (uint64_t)c.gx * c.gy,
                             c.tw + c.th, c.tw);
    };
    std::sort(cands.begin(), cands.end(),
              [&](const TileCand& a, const TileCand& b) { return key(a) < key(b); });
  }
  int device = 0, cus = 0;
  GA_HIP(hipGetDevice(&device), "get device");
  GA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "CU count");
  for (const TileCand& c : cands) {
    bool fits = false;
    const int rc = tile_fits(v, c, (uint32_t)cus, &fits);
    if (rc != GA_OK) return rc;
    if (!fits) continue;
    v.tile_w = c.tw;
    v.tile_h = c.th;
    v.tiles_x = c.gx;
    v.tiles_y = c.gy;
    r->tile_state = 1;
    return GA_OK;
  }
  r->tile_state = -1;
  r->tile_why = r->want_tile_w ? "the tile shape needs more LDS than a CU has, or more "
                                 "workgroups than the GPU holds at once"
                               : "no tiling of the run fits the GPU's LDS";
  return GA_OK;
}

// Whether ga_step runs the LDS-resident tile form.
int use_tiles(ga_run* r, bool* yes) {
  *yes = false;
  if (r->form == GA_FORM_STREAMING) return GA_OK;
  const int rc = plan_tiles(r);
  if (rc != GA_OK) return rc;
  if (r->tile_state == 1) {
    *yes = true;
    return GA_OK;
  }
  if (r->form == GA_FORM_RESIDENT) return fail(GA_EINVAL, "resident form: " + r->tile_why);
  return GA_OK;
}

// A tile's wait that gave up leaves the state invalid (its workgroups were
// not all resident at once); reported when the state is read.
int check_tile_waits(ga_run* r) {
  if (r->cfg.schedule == GA_SCHEDULE_ASYNC) return GA_OK;
  unsigned long long n = 0;
  GA_HIP(hipMemcpy(&n, r->view.waits, sizeof(n), hipMemcpyDeviceToHost), "read waits");
  if (n) return fail(GA_EDEVICE, "an LDS-resident tile stopped waiting for a neighbouring tile "
                                 "(not every tile was resident at once): the state is invalid");
  return GA_OK;
}

int step_tiles(ga_run* r, uint64_t n) {
  const ga::RunView& v = r->view;
  const uint32_t n_tiles = v.tiles_x * v.tiles_y;
  // about 2^34 agent-generations, at most 2^16 generations, per launch
  const uint64_t slice_max =
      std::max<uint64_t>(1, std::min<uint64_t>(1u << 16, (1ull << 34) / std::max(1u, v.agents)));
  uint64_t left = n;
  while (left > 0) {
    const uint64_t slice = std::min(left, slice_max);
    GA_HIP(ga::launch_fill(v.prog, (uint32_t)r->gen_host, n_tiles, r->stream), "progress reset");
    GA_HIP(ga::launch_tiles(v, slice, r->stream), "tile launch");
    GA_HIP(ga::launch_advance(v.gen, slice, r->stream), "advance launch");
    left -= slice;
    r->gen_host += slice;
  }
  return GA_OK;
}

// Destroy the run's graph once its stream has finished any launch of it.
void drop_graph(ga_run* r) {
  if (r->graph) {
    (void)hipStreamSynchronize(r->stream);
    (void)hipGraphExecDestroy(r->graph);
    r->graph = nullptr;
  }
}

int enqueue_direct(ga_run* r, uint64_t n) {
  // Streaming launches in slices whose generation offsets fit a 32-bit argument.
  ga::RunView v = r->view;
  v.ipw = r->ipw;
  const uint32_t waves = waves_for(r, r->ipw);
  while (n > 0) {
    const uint64_t slice = std::min<uint64_t>(n, 1u << 20);
    for (uint64_t g = 0; g < slice; ++g)
      GA_HIP(ga::launch_generation(v, (uint32_t)g, waves, r->wpg, r->stream), "generation launch");
    GA_HIP(ga::launch_advance(v.gen, slice, r->stream), "advance launch");
    n -= slice;
  }
  return GA_OK;
}

int ensure_graph(ga_run* r) {
  if (r->graph && r->graph_key_ipw == r->ipw && r->graph_key_wpg == r->wpg &&
      r->graph_key_block == r->graph_block)
    return GA_OK;
  drop_graph(r);
  if (!r->capture_stream)
    GA_HIP(hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking), "capture stream");
  ga::RunView v = r->view;
  v.ipw = r->ipw;
  const uint32_t waves = waves_for(r, r->ipw);
  GA_HIP(hipStreamBeginCapture(r->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t err = hipSuccess;
  for (uint32_t g = 0; g < r->graph_block && err == hipSuccess; ++g)
    err = ga::launch_generation(v, g, waves, r->wpg, r->capture_stream);
  if (err == hipSuccess) err = ga::launch_advance(v.gen, r->graph_block, r->capture_stream);
  hipGraph_t graph = nullptr;
  hipError_t end = hipStreamEndCapture(r->capture_stream, &graph);
  if (err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(err, "launch during capture");
  }
  if (end != hipSuccess) return hip_fail(end, "end capture");
  hipGraphExec_t exec = nullptr;
  err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (err != hipSuccess) return hip_fail(err, "graph instantiate");
  r->graph = exec;
  r->graph_key_ipw = r->ipw;
  r->graph_key_wpg = r->wpg;
  r->graph_key_block = r->graph_block;
  return GA_OK;
}

// Asynchronous schedule: one persistent launch per slice of generations, the
// chunks spread over as many wavefronts as the GPU holds at once (or over the
// caller's cap), each wavefront owning consecutive chunks.
int step_async(ga_run* r, uint64_t n) {
  ga::RunView v = r->view;
  v.ipw = r->ipw;
  // no lead and no skew: the lockstep exchange
  const bool lockstep = r->async_lead == 0u && r->async_skew == 0u;
  uint32_t cap = 0;
  GA_HIP(ga::async_capacity(v, r->wpg, lockstep, &cap), "occupancy query");
  // With the default chunk size (and no skew, whose one-wavefront
  // interleavings name their chunks): while each resident wavefront would run
  // more than two chunks in turn (waiting out each one's exchange), take
  // chunks twice as large. Measured at 1024 x 512 x 32, four 16-island chunks
  // per wavefront against two 32-island ones: lockstep 127 against 123 us per
  // generation (one 64-island chunk, at lower occupancy: 130), max_lead 2 158
  // against 142, unpaced 150 against 136. Lockstep results do not depend on it.
  while (r->async_skew == 0u && !r->ipw_set && waves_for(r, v.ipw) > 2u * cap &&
         v.ipw * 2u <= 64u && ga::lds_bytes(v.ipw * 2u, r->wpg, v.model) <= kMaxGroupLds) {
    v.ipw *= 2u;
    GA_HIP(ga::async_capacity(v, r->wpg, lockstep, &cap), "occupancy query");
  }
  const uint32_t chunks = waves_for(r, v.ipw);
  uint32_t waves = std::max(1u, std::min(chunks, cap));
  if (r->async_max_waves) waves = std::min(waves, r->async_max_waves);
  const uint32_t per_wave = (chunks + waves - 1) / waves;
  waves = (chunks + per_wave - 1) / per_wave;
  // bound one launch to about 2^34 agent-generations; with a skew, one call
  // is one interleaving block, so it is never split
  const uint64_t slice_max =
      r->async_skew ? n
                    : std::max<uint64_t>(1, std::min<uint64_t>(1u << 16,
                                                               (1ull << 34) / std::max(1u, v.agents)));
  uint64_t left = n;
  while (left > 0) {
    const uint64_t slice = std::min(left, slice_max);
    if (lockstep) {
      GA_HIP(ga::launch_lockstep(v, r->gen_host, slice, waves, per_wave, r->wpg, r->stream),
             "lockstep launch");
    } else {
      // every chunk starts the launch having completed the current generation
      GA_HIP(ga::launch_fill(v.prog, (uint32_t)r->gen_host, v.island_stride, r->stream),
             "progress reset");
      GA_HIP(ga::launch_async(v, slice, waves, per_wave, r->wpg, r->async_lead, r->async_skew,
                              r->stream), "async launch");
    }
    GA_HIP(ga::launch_advance(v.gen, slice, r->stream), "advance launch");
    left -= slice;
    r->gen_host += slice;
  }
  return GA_OK;
}

}  // namespace

extern "C" {

const char* ga_strerror(int code) {
  switch (code) {
    case GA_OK: return "success";
    case GA_EINVAL: return "invalid argument";
    case GA_ENOMEM: return "device buffer too small";
    case GA_EDEVICE: return "HIP runtime error";
    case GA_ESTATE: return "handle in the wrong state";
    default: return "unknown error";
  }
}

const char* ga_last_error(void) { return g_last_error.c_str(); }

size_t ga_state_bytes(const ga_config* cfg) {
  if (!config_ok(cfg, nullptr)) return 0;
  return layout_of(cfg).total;
}

int ga_init(const ga_config* cfg, void* dev_mem, size_t bytes, void* hip_stream, ga_run** out) {
  std::string why;
  if (!out) return fail(GA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!config_ok(cfg, &why)) return fail(GA_EINVAL, why);
  if (!dev_mem) return fail(GA_EINVAL, "dev_mem is NULL");
  if (reinterpret_cast<uintptr_t>(dev_mem) % kAlign) return fail(GA_EINVAL, "dev_mem must be 256-byte aligned");
  const Layout lay = layout_of(cfg);
  if (bytes < lay.total) return fail(GA_ENOMEM, "dev_mem smaller than ga_state_bytes(cfg)");

  ga_run* r = new (std::nothrow) ga_run();
  if (!r) return fail(GA_EINVAL, "host allocation failed");
  std::memcpy(&r->cfg, cfg, cfg->struct_size);
  const bool async = is_async(cfg);
  const uint32_t model = model_of(cfg);
  r->cfg.struct_size = sizeof(ga_config);  // fields past the caller's size stay 0
  r->lay = lay;
  r->stream = static_cast<hipStream_t>(hip_stream);
  r->base = static_cast<uint8_t*>(dev_mem);
  ga::RunView& v = r->view;
  uint8_t* b = r->base;
  v.pop_f = reinterpret_cast<float*>(b + lay.pop_f);
  v.pop_T = reinterpret_cast<uint32_t*>(b + lay.pop_T);
  v.pop_D = reinterpret_cast<uint32_t*>(b + lay.pop_D);
  v.model = model;
  v.pop_P = ga::model_has_string_host(model) ? reinterpret_cast<uint32_t*>(b + lay.pop_P) : nullptr;
  for (int p = 0; p < 2; ++p) v.ob[p] = async ? nullptr : reinterpret_cast<uint32_t*>(b + lay.ob[p]);
  v.mail = async ? reinterpret_cast<uint32_t*>(b + lay.mail) : nullptr;
  v.seen = async ? reinterpret_cast<uint32_t*>(b + lay.seen) : nullptr;
  v.prog = reinterpret_cast<uint32_t*>(b + lay.prog);
  v.lock = async ? reinterpret_cast<uint32_t*>(b + lay.lock) : nullptr;
  v.ob_stride = (uint32_t)outbox_stride(cfg);
  v.gen = reinterpret_cast<unsigned long long*>(b + lay.counters);
  v.left = v.gen + 1;
  v.waits = v.gen + 2;
  v.width = cfg->width;
  v.height = cfg->height;
  v.islands = cfg->width * cfg->height;
  v.agents = v.islands * cfg->pop_per_island;
  v.island_stride = (uint32_t)padded_islands(cfg);
  v.agent_stride = v.island_stride * cfg->pop_per_island;
  v.log2n = log2u(cfg->pop_per_island);
  v.words = (uint32_t)surface_words(cfg);
  v.s_log = log2u(cfg->surface_sites);
  v.dlog = log2u(dbits_of(cfg));
  v.policy = policy_of(cfg);
  v.k = cfg->tournament_size;
  v.selection = cfg->selection;
  v.p32 = cfg->mutation_threshold;
  v.migration = cfg->migration;
  v.seed = cfg->seed;
  v.run_id = cfg->run_id;
  v.law = r->cfg.mutation_law;
  v.p_ben = v.law ? r->cfg.beneficial_threshold : 0u;
  v.p_any = v.law ? r->cfg.beneficial_threshold + r->cfg.mutation_threshold : 0u;
  r->ipw = default_ipw(v);
  v.ipw = r->ipw;

  // Founders: all-zero bits are +0 fitness, T = 0, blank surfaces, invalid
  // outbox headers, generation 0.
  hipError_t e = ga::launch_fill(reinterpret_cast<uint32_t*>(b), 0u, lay.total / 4, r->stream);
  if (e == hipSuccess) e = ga::launch_init(v, r->stream);
  if (e != hipSuccess) {
    delete r;
    return hip_fail(e, "init fill");
  }
  *out = r;
  return GA_OK;
}

uint64_t ga_generation(const ga_run* r) { return r ? r->gen_host : 0; }

int ga_set_launch(ga_run* r, uint32_t ipw, uint32_t wpg, uint32_t form) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  const uint32_t g = per_iter(r);
  uint32_t new_ipw = ipw ? ipw : r->ipw;
  uint32_t new_wpg = wpg ? wpg : r->wpg;
  if (new_ipw < g || new_ipw > 64 || new_ipw % g)
    return fail(GA_EINVAL, "islands_per_wave must be a multiple of 64/N in [64/N, 64]");
  if (new_wpg < 1 || new_wpg > (uint32_t)ga::kMaxWavesPerGroup)
    return fail(GA_EINVAL, "waves_per_group must be in [1, 16]");
  if (ga::lds_bytes(new_ipw, new_wpg, r->view.model) > kMaxGroupLds)
    return fail(GA_EINVAL, "islands_per_wave x waves_per_group needs more LDS than a CU has");
  if (form > GA_FORM_RESIDENT) return fail(GA_EINVAL, "unknown form");
  if (form == GA_FORM_RESIDENT && r->cfg.schedule == GA_SCHEDULE_ASYNC)
    return fail(GA_EINVAL, "the resident form is synchronous");
  if (form == GA_FORM_RESIDENT && r->cfg.schedule != GA_SCHEDULE_ASYNC) {
    const int rc = plan_tiles(r);
    if (rc != GA_OK) return rc;
    if (r->tile_state != 1) return fail(GA_EINVAL, "resident form: " + r->tile_why);
  }
  r->ipw = new_ipw;
  r->ipw_set = r->ipw_set || ipw != 0;
  r->wpg = new_wpg;
  r->form = form;
  return GA_OK;
}

int ga_set_tiles(ga_run* r, uint32_t tile_w, uint32_t tile_h) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (r->cfg.schedule == GA_SCHEDULE_ASYNC) return fail(GA_EINVAL, "tiles are synchronous");
  if ((tile_w == 0) != (tile_h == 0)) return fail(GA_EINVAL, "give both tile sides or neither");
  const uint32_t old_w = r->want_tile_w, old_h = r->want_tile_h;
  const ga::RunView old_view = r->view;
  const int old_state = r->tile_state;
  const std::string old_why = r->tile_why;
  r->want_tile_w = std::min(tile_w, r->view.width);
  r->want_tile_h = std::min(tile_h, r->view.height);
  r->tile_state = 0;
  int rc = plan_tiles(r);
  if (rc == GA_OK && r->tile_state != 1) rc = fail(GA_EINVAL, "tiles: " + r->tile_why);
  if (rc != GA_OK) {  // a failed call leaves the run as it was
    r->want_tile_w = old_w;
    r->want_tile_h = old_h;
    r->view = old_view;
    r->tile_state = old_state;
    r->tile_why = old_why;
  }
  return rc;
}

int ga_get_tiles(ga_run* r, uint32_t* tile_w, uint32_t* tile_h, uint32_t* tiles) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  bool yes = false;
  if (r->cfg.schedule != GA_SCHEDULE_ASYNC && !r->batch) {
    const int rc = use_tiles(r, &yes);
    if (rc != GA_OK) return rc;
  }
  if (tile_w) *tile_w = yes ? r->view.tile_w : 0u;
  if (tile_h) *tile_h = yes ? r->view.tile_h : 0u;
  if (tiles) *tiles = yes ? r->view.tiles_x * r->view.tiles_y : 0u;
  return GA_OK;
}

int ga_set_async(ga_run* r, uint32_t max_wavefronts, uint32_t max_lead, uint32_t skew) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (r->cfg.schedule != GA_SCHEDULE_ASYNC) return fail(GA_EINVAL, "run is not asynchronous");
  if (skew && (max_wavefronts != 1 || max_lead != GA_ASYNC_UNPACED))
    return fail(GA_EINVAL, "a skewed interleaving needs one wavefront and no pacing");
  if (skew > 1024) return fail(GA_EINVAL, "skew must be <= 1024");
  r->async_max_waves = max_wavefronts;
  r->async_lead = max_lead;
  r->async_skew = skew;
  return GA_OK;
}

int ga_async_last_taken(ga_run* r, int64_t* sent) {
  if (!r || !sent) return fail(GA_EINVAL, "run or sent is NULL");
  if (r->cfg.schedule != GA_SCHEDULE_ASYNC) return fail(GA_EINVAL, "run is not asynchronous");
  GA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  const size_t I = r->view.islands;
  std::vector<uint32_t> stamps(I * 4);
  unsigned long long t = 0;
  GA_HIP(hipMemcpy(&t, r->view.gen, sizeof(t), hipMemcpyDeviceToHost), "read generation");
  GA_HIP(hipMemcpy(stamps.data(), r->view.seen, I * 16, hipMemcpyDeviceToHost), "read stamps");
  // stamp = 2 * (sending generation + 1) mod 2^32; a taken genome was sent
  // less than 2^31 generations before t
  for (size_t k = 0; k < I * 4; ++k) {
    const uint32_t back = (uint32_t)(2u * (uint32_t)t) - stamps[k];
    sent[k] = (int64_t)t - 1 - (int64_t)(back / 2u);
  }
  return GA_OK;
}

int ga_async_waits(ga_run* r, uint64_t* gave_up) {
  if (!r || !gave_up) return fail(GA_EINVAL, "run or gave_up is NULL");
  if (r->cfg.schedule != GA_SCHEDULE_ASYNC) return fail(GA_EINVAL, "run is not asynchronous");
  GA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  unsigned long long n = 0;
  GA_HIP(hipMemcpy(&n, r->view.waits, sizeof(n), hipMemcpyDeviceToHost), "read waits");
  *gave_up = n;
  return GA_OK;
}

int ga_async_taken(ga_run* r, uint64_t* taken) {
  if (!r || !taken) return fail(GA_EINVAL, "run or taken is NULL");
  if (r->cfg.schedule != GA_SCHEDULE_ASYNC) return fail(GA_EINVAL, "run is not asynchronous");
  GA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  unsigned long long n = 0;
  GA_HIP(hipMemcpy(&n, r->view.waits + 1, sizeof(n), hipMemcpyDeviceToHost), "read taken");
  *taken = n;
  return GA_OK;
}

int ga_set_graph_block(ga_run* r, uint32_t gens) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (gens > 100000) return fail(GA_EINVAL, "graph block too long");
  r->graph_block = gens;
  return GA_OK;
}

int ga_step(ga_run* r, uint64_t n) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (r->batch) return fail(GA_ESTATE, "run is a batch member; advance it with ga_batch_step");
  if (n == 0) return GA_OK;
  const Range range("ga_step", n);
  if (r->cfg.schedule == GA_SCHEDULE_ASYNC) return step_async(r, n);
  bool tiles = false;
  int rc0 = use_tiles(r, &tiles);
  if (rc0 != GA_OK) return rc0;
  if (tiles) return step_tiles(r, n);
  uint64_t left = n;
  if (r->graph_block > 0 && left >= r->graph_block) {
    int rc = ensure_graph(r);
    if (rc != GA_OK) return rc;
    while (left >= r->graph_block) {
      const Range block("block", r->graph_block);
      GA_HIP(hipGraphLaunch(r->graph, r->stream), "graph launch");
      left -= r->graph_block;
    }
  }
  int rc = enqueue_direct(r, left);
  if (rc != GA_OK) return rc;
  r->gen_host += n;
  return GA_OK;
}

int ga_read_population(ga_run* r, float* fitness, uint32_t* T, uint32_t* surface_words,
                       ga_outbox_entry* outbox, uint64_t* generation) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (outbox && r->cfg.schedule == GA_SCHEDULE_ASYNC)
    return fail(GA_EINVAL, "an asynchronous run has no synchronous outbox");
  if (outbox && ga::model_has_string_host(r->view.model))
    return fail(GA_EINVAL, "the outbox of a genome model with a string is not exchanged");
  hipStream_t s = r->batch ? r->batch->stream : r->stream;
  GA_HIP(hipStreamSynchronize(s), "stream sync");
  const int waited = check_tile_waits(r);
  if (waited != GA_OK) return waited;
  const ga::RunView& v = r->view;
  const size_t A = v.agents, I = v.islands, W = v.words;
  unsigned long long t = 0;
  GA_HIP(hipMemcpy(&t, v.gen, sizeof(t), hipMemcpyDeviceToHost), "read generation");
  if (fitness) GA_HIP(hipMemcpy(fitness, v.pop_f, A * 4, hipMemcpyDeviceToHost), "read fitness");
  if (T) GA_HIP(hipMemcpy(T, v.pop_T, A * 4, hipMemcpyDeviceToHost), "read T");
  if (surface_words) {
    if (W == 1) {
      GA_HIP(hipMemcpy(surface_words, v.pop_D, A * 4, hipMemcpyDeviceToHost), "read surfaces");
    } else {
      std::vector<uint32_t> planes(A * W);
      for (size_t w = 0; w < W; ++w)
        GA_HIP(hipMemcpy(planes.data() + w * A, v.pop_D + w * v.agent_stride, A * 4,
                         hipMemcpyDeviceToHost), "read surfaces");
      for (size_t a = 0; a < A; ++a)
        for (size_t w = 0; w < W; ++w) surface_words[a * W + w] = planes[w * A + a];
    }
  }
  if (outbox) {
    const int p = (int)((t & 1) ^ 1);
    const size_t st = v.ob_stride;
    std::vector<uint32_t> ob(I * st);
    GA_HIP(hipMemcpy(ob.data(), v.ob[p], I * st * 4, hipMemcpyDeviceToHost), "read outbox");
    for (size_t i = 0; i < I; ++i) {
      const uint32_t* src = &ob[i * st];
      const uint32_t hdr = src[2 + W];
      ga_outbox_entry& e = outbox[i];
      e.valid = (hdr & ga::kMetaValid) ? 1u : 0u;
      e.dir = hdr & 3u;
      std::memcpy(&e.fitness, &src[0], 4);
      e.T = src[1];
      e.surface[0] = src[2];
      e.surface[1] = W > 1 ? src[3] : 0u;
    }
  }
  if (generation) *generation = t;
  if (!r->batch) r->gen_host = t;
  return GA_OK;
}

int ga_write_population(ga_run* r, const float* fitness, const uint32_t* T,
                        const uint32_t* surface_words, const ga_outbox_entry* outbox,
                        uint64_t generation) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  if (r->batch) return fail(GA_ESTATE, "run is a batch member");
  const bool async = r->cfg.schedule == GA_SCHEDULE_ASYNC;
  if (outbox && async) return fail(GA_EINVAL, "an asynchronous run has no synchronous outbox");
  if (outbox && ga::model_has_string_host(r->view.model))
    return fail(GA_EINVAL, "the outbox of a genome model with a string is not exchanged");
  if (outbox) {
    for (size_t i = 0; i < r->view.islands; ++i)
      if (outbox[i].valid > 1 || outbox[i].dir > 3) return fail(GA_EINVAL, "outbox entry out of range");
  }
  hipStream_t s = r->stream;
  GA_HIP(hipStreamSynchronize(s), "stream sync");
  const ga::RunView& v = r->view;
  const size_t A = v.agents, I = v.islands, W = v.words;
  unsigned long long t_old = 0;
  GA_HIP(hipMemcpy(&t_old, v.gen, sizeof(t_old), hipMemcpyDeviceToHost), "read generation");
  const hipMemcpyKind h2d = hipMemcpyHostToDevice, d2d = hipMemcpyDeviceToDevice;
  if (fitness) GA_HIP(hipMemcpyAsync(v.pop_f, fitness, A * 4, h2d, s), "write fitness");
  if (T) GA_HIP(hipMemcpyAsync(v.pop_T, T, A * 4, h2d, s), "write T");
  std::vector<uint32_t> planes;
  if (surface_words) {
    planes.resize(A * W);
    for (size_t a = 0; a < A; ++a)
      for (size_t w = 0; w < W; ++w) planes[w * A + a] = surface_words[a * W + w];
    for (size_t w = 0; w < W; ++w)
      GA_HIP(hipMemcpyAsync(v.pop_D + w * v.agent_stride, planes.data() + w * A, A * 4, h2d, s),
             "write surfaces");
  }
  const int p_old = (int)((t_old & 1) ^ 1);
  const int p_new = (int)((generation & 1) ^ 1);
  const size_t st = v.ob_stride;
  std::vector<uint32_t> ob;
  if (outbox) {
    ob.assign(I * st, 0u);
    for (size_t i = 0; i < I; ++i) {
      uint32_t* dst = &ob[i * st];
      std::memcpy(&dst[0], &outbox[i].fitness, 4);
      dst[1] = outbox[i].T;
      for (size_t w = 0; w < W; ++w) dst[2 + w] = outbox[i].surface[w];
      dst[2 + W] = outbox[i].valid ? (ga::kMetaValid | outbox[i].dir) : 0u;
    }
    GA_HIP(hipMemcpyAsync(v.ob[p_new], ob.data(), I * st * 4, h2d, s), "write outbox");
  } else if (async) {
    // empty buffers: every stamp reads as already taken at the new generation
    const uint32_t taken = (uint32_t)(2u * (uint32_t)generation);
    GA_HIP(ga::launch_fill(v.mail, taken, (size_t)v.island_stride * 8 * st, s), "reset buffers");
    GA_HIP(ga::launch_fill(v.seen, taken, (size_t)v.island_stride * 4, s), "reset stamps");
  } else if (p_new != p_old) {
    // keep the pending emissions readable at the new generation's parity
    GA_HIP(hipMemcpyAsync(v.ob[p_new], v.ob[p_old], (size_t)v.island_stride * st * 4, d2d, s),
           "move outbox");
  }
  unsigned long long t = generation;
  GA_HIP(hipMemcpyAsync(v.gen, &t, sizeof(t), h2d, s), "write generation");
  GA_HIP(hipStreamSynchronize(s), "stream sync");
  r->gen_host = generation;
  return GA_OK;
}

int ga_read_strings(ga_run* r, uint32_t* words) {
  if (!r || !words) return fail(GA_EINVAL, "run or words is NULL");
  if (!ga::model_has_string_host(r->view.model))
    return fail(GA_EINVAL, "the genome model has no string");
  hipStream_t s = r->batch ? r->batch->stream : r->stream;
  GA_HIP(hipStreamSynchronize(s), "stream sync");
  const size_t A = r->view.agents;
  std::vector<uint32_t> planes(A * 2);
  for (size_t w = 0; w < 2; ++w)
    GA_HIP(hipMemcpy(planes.data() + w * A, r->view.pop_P + w * r->view.agent_stride, A * 4,
                     hipMemcpyDeviceToHost), "read strings");
  for (size_t a = 0; a < A; ++a) {
    words[a * 2] = planes[a];
    words[a * 2 + 1] = planes[A + a];
  }
  return GA_OK;
}

int ga_write_strings(ga_run* r, const uint32_t* words) {
  if (!r || !words) return fail(GA_EINVAL, "run or words is NULL");
  if (!ga::model_has_string_host(r->view.model))
    return fail(GA_EINVAL, "the genome model has no string");
  if (r->batch) return fail(GA_ESTATE, "run is a batch member");
  GA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  const size_t A = r->view.agents;
  std::vector<uint32_t> planes(A * 2);
  for (size_t a = 0; a < A; ++a) {
    planes[a] = words[a * 2];
    planes[A + a] = words[a * 2 + 1];
  }
  for (size_t w = 0; w < 2; ++w)
    GA_HIP(hipMemcpy(r->view.pop_P + w * r->view.agent_stride, planes.data() + w * A, A * 4,
                     hipMemcpyHostToDevice), "write strings");
  return GA_OK;
}

int ga_extract_surfaces(ga_run* r, const uint64_t* agent_ids, size_t n, uint64_t* ids_out,
                        uint32_t* T_out, uint32_t* surface_words_out) {
  if (!r) return fail(GA_EINVAL, "run is NULL");
  const ga::RunView& v = r->view;
  const size_t I = v.islands, W = v.words;
  if (!agent_ids && n != I) return fail(GA_EINVAL, "n must equal the island count when agent_ids is NULL");
  if (agent_ids)
    for (size_t j = 0; j < n; ++j)
      if (agent_ids[j] >= v.agents) return fail(GA_EINVAL, "agent id out of range");
  if (n == 0) return GA_OK;
  hipStream_t s = r->batch ? r->batch->stream : r->stream;
  GA_HIP(hipStreamSynchronize(s), "stream sync");
  const int waited = check_tile_waits(r);
  if (waited != GA_OK) return waited;
  uint32_t* st_ids = reinterpret_cast<uint32_t*>(r->base + r->lay.st_ids);
  uint32_t* st_T = reinterpret_cast<uint32_t*>(r->base + r->lay.st_T);
  uint32_t* st_D = reinterpret_cast<uint32_t*>(r->base + r->lay.st_D);
  std::vector<uint32_t> ids32(std::min(n, I)), tT(std::min(n, I)), tD(std::min(n, I) * W);
  for (size_t done = 0; done < n;) {
    const size_t m = std::min(n - done, I);
    if (agent_ids) {
      for (size_t j = 0; j < m; ++j) ids32[j] = (uint32_t)agent_ids[done + j];
      GA_HIP(hipMemcpyAsync(st_ids, ids32.data(), m * 4, hipMemcpyHostToDevice, s), "write ids");
    } else {
      GA_HIP(ga::launch_sample(v, st_ids, s), "sample launch");
    }
    GA_HIP(ga::launch_gather(v, st_ids, (uint32_t)m, st_T, st_D, s), "gather launch");
    GA_HIP(hipMemcpyAsync(ids32.data(), st_ids, m * 4, hipMemcpyDeviceToHost, s), "read ids");
    GA_HIP(hipMemcpyAsync(tT.data(), st_T, m * 4, hipMemcpyDeviceToHost, s), "read T");
    GA_HIP(hipMemcpyAsync(tD.data(), st_D, m * W * 4, hipMemcpyDeviceToHost, s), "read surfaces");
    GA_HIP(hipStreamSynchronize(s), "stream sync");
    for (size_t j = 0; j < m; ++j) {
      if (ids_out) ids_out[done + j] = ids32[j];
      if (T_out) T_out[done + j] = tT[j];
      if (surface_words_out)
        for (size_t w = 0; w < W; ++w) surface_words_out[(done + j) * W + w] = tD[w * m + j];
    }
    done += m;
  }
  return GA_OK;
}

void ga_destroy(ga_run* r) {
  if (!r) return;
  if (r->batch) ga_batch_remove(r->batch, r);
  (void)hipStreamSynchronize(r->stream);
  drop_graph(r);
  if (r->capture_stream) (void)hipStreamDestroy(r->capture_stream);
  delete r;
}

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------

int ga_batch_create(void* hip_stream, ga_batch** out) {
  if (!out) return fail(GA_EINVAL, "out is NULL");
  ga_batch* b = new (std::nothrow) ga_batch();
  if (!b) return fail(GA_EINVAL, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  *out = b;
  return GA_OK;
}

size_t ga_batch_size(const ga_batch* b) { return b ? b->members.size() : 0; }

int ga_batch_set_graph_block(ga_batch* b, uint32_t gens) {
  if (!b) return fail(GA_EINVAL, "batch is NULL");
  if (gens > 100000) return fail(GA_EINVAL, "graph block too long");
  if (gens != b->graph_block) b->graph_stale = true;
  b->graph_block = gens;
  return GA_OK;
}

int ga_batch_set_launch(ga_batch* b, uint32_t ipw, uint32_t wpg) {
  if (!b) return fail(GA_EINVAL, "batch is NULL");
  if (ipw > 64) return fail(GA_EINVAL, "islands_per_wave must be <= 64");
  if (wpg > (uint32_t)ga::kMaxWavesPerGroup) return fail(GA_EINVAL, "waves_per_group must be in [1, 16]");
  b->ipw_override = ipw;
  if (wpg) b->wpg = wpg;
  b->dirty = true;
  return GA_OK;
}

int ga_batch_set_class_launch(ga_batch* b, uint32_t log2n, uint32_t words, uint32_t ipw) {
  if (!b) return fail(GA_EINVAL, "batch is NULL");
  if (log2n > 6 || words < 1 || words > 2) return fail(GA_EINVAL, "no such class");
  const uint32_t g = 64u >> log2n;
  if (ipw && (ipw < g || ipw > 64 || ipw % g))
    return fail(GA_EINVAL, "islands_per_wave must be 0 or a multiple of 64/N in [64/N, 64]");
  b->cls[log2n * 2 + words - 1].ipw = ipw;
  b->dirty = true;
  return GA_OK;
}

int ga_batch_add(ga_batch* b, ga_run* r, uint64_t budget) {
  if (!b || !r) return fail(GA_EINVAL, "batch or run is NULL");
  if (r->cfg.schedule == GA_SCHEDULE_ASYNC)
    return fail(GA_EINVAL, "a batch advances synchronous runs only");
  if (r->view.model != GA_MODEL_FITNESS)
    return fail(GA_EINVAL, "a batch advances fitness-valued genomes only");
  if (r->view.dlog != 0u || r->view.policy != GA_POLICY_STEADY)
    return fail(GA_EINVAL, "a batch advances one-bit differentia on the steady policy only");
  if (r->batch) return fail(GA_ESTATE, "run is already in a batch");
  // the run's own work (its founders, earlier steps) comes first in the
  // batch's stream order; then its budget is set on the device
  if (r->stream != b->stream) {
    hipEvent_t ev = nullptr;
    GA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    hipError_t e = hipEventRecord(ev, r->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
    (void)hipEventDestroy(ev);
    GA_HIP(e, "order the run before the batch");
  }
  GA_HIP(ga::launch_store_u64(r->view.left, budget, b->stream), "write budget");
  r->batch = b;
  b->members.push_back(r);
  b->remaining.push_back(budget);
  b->finished_step.push_back(budget == 0 ? b->steps : UINT64_MAX);
  b->dirty = true;
  return GA_OK;
}

int ga_batch_remove(ga_batch* b, ga_run* r) {
  if (!b || !r) return fail(GA_EINVAL, "batch or run is NULL");
  auto it = std::find(b->members.begin(), b->members.end(), r);
  if (it == b->members.end()) return fail(GA_EINVAL, "run is not a member");
  const size_t idx = (size_t)(it - b->members.begin());
  b->members.erase(it);
  b->remaining.erase(b->remaining.begin() + (long)idx);
  b->finished_step.erase(b->finished_step.begin() + (long)idx);
  // later work on the run's own stream follows the batch's work so far
  if (r->stream != b->stream) {
    hipEvent_t ev = nullptr;
    GA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    hipError_t e = hipEventRecord(ev, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(r->stream, ev, 0);
    (void)hipEventDestroy(ev);
    GA_HIP(e, "order the batch before the run");
  }
  r->batch = nullptr;
  b->dirty = true;
  return GA_OK;
}

uint64_t ga_batch_remaining(const ga_batch* b, const ga_run* r) {
  if (!b) return 0;
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->members[i] == r) return b->remaining[i];
  return 0;
}

namespace {

// Whether step call s of the batch has completed (wait: block until it has).
// Steps complete in stream order, so step s implies every earlier one.
int step_complete(ga_batch* b, uint64_t s, bool wait, bool* done) {
  *done = false;
  if (s <= b->done_through) {
    *done = true;
    return GA_OK;
  }
  const int slot = (int)((s - 1) % ga_batch::kStepEvents);
  const hipEvent_t ev = b->step_done[slot];
  if (!ev || b->step_of[slot] < s) return fail(GA_ESTATE, "step not enqueued");
  // a slot holding a later step is only reused after step s was known complete
  if (b->step_of[slot] > s) {
    b->done_through = std::max(b->done_through, s);
    *done = true;
    return GA_OK;
  }
  const hipError_t q = wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
  if (q == hipSuccess) {
    b->done_through = std::max(b->done_through, s);
    *done = true;
  } else if (q != hipErrorNotReady) {
    return hip_fail(q, "step event");
  }
  return GA_OK;
}

}  // namespace

int ga_batch_settled(ga_batch* b, const ga_run* r, int* settled) {
  if (!b || !settled) return fail(GA_EINVAL, "batch or settled is NULL");
  for (size_t i = 0; i < b->members.size(); ++i) {
    if (b->members[i] != r) continue;
    const uint64_t s = b->finished_step[i];
    *settled = 0;
    if (s == UINT64_MAX) return GA_OK;
    if (s == 0) {  // never advanced
      *settled = 1;
      return GA_OK;
    }
    bool done = false;
    const int rc = step_complete(b, s, false, &done);
    if (rc != GA_OK) return rc;
    *settled = done ? 1 : 0;
    return GA_OK;
  }
  return fail(GA_EINVAL, "run is not a member");
}

namespace {

// Islands per wavefront of a class: its own setting, else the batch's, else
// about 512 agents per wavefront whatever the island size (a batch has
// wavefronts enough, so small members need no finer chunks, and short
// wavefronts would spend their time in the per-wavefront set-up).
uint32_t class_ipw(const ga_batch* b, uint32_t c) {
  const uint32_t log2n = c / 2;
  const uint32_t g = 64u >> log2n;
  uint32_t ipw = b->cls[c].ipw ? b->cls[c].ipw
                               : (b->ipw_override ? b->ipw_override : std::max(1u, 512u >> log2n));
  ipw = std::max(g, ipw / g * g);
  return std::min(64u, ipw);
}

uint32_t class_of(const ga::RunView& v) { return v.log2n * 2u + v.words - 1u; }

extern "C++" {
namespace {
template <typename T>
T* table_offset(T* p, const void* table) {
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) - reinterpret_cast<uintptr_t>(table));
}

// The pointers the batch kernels follow, as byte offsets from the device table
// (the kernels add them back to the table's address).
void to_table(ga::RunView& v, const void* table) {
  v.pop_f = table_offset(v.pop_f, table);
  v.pop_T = table_offset(v.pop_T, table);
  v.pop_D = table_offset(v.pop_D, table);
  v.ob[0] = table_offset(v.ob[0], table);
  v.ob[1] = table_offset(v.ob[1], table);
  v.gen = table_offset(v.gen, table);
  v.left = table_offset(v.left, table);
}
}  // namespace
}  // extern "C++"

size_t tab_tiles_off(const ga_batch* b) { return align_up((size_t)b->view_cap * sizeof(ga::RunView)); }
size_t tab_counts_off(const ga_batch* b) {
  return tab_tiles_off(b) + align_up((size_t)b->tile_cap * sizeof(ga::Tile));
}
// the counts: live tiles, then members
size_t tab_bytes(const ga_batch* b) { return tab_counts_off(b) + align_up(2 * 4); }

uint32_t pow2_at_least(uint32_t v) {
  uint32_t p = 256;
  while (p < v) p <<= 1;
  return p;
}

// Algorithmic bytes a tile moves in one generation: each agent's fitness,
// lineage counter and surface read and written, each island's outbox entry
// read and written.
uint64_t tile_bytes(const ga::RunView& v, uint32_t islands) {
  const uint64_t agent = 2u * (8u + 4u * v.words), island = 2u * (12u + 4u * v.words);
  return (uint64_t)islands * (((uint64_t)1 << v.log2n) * agent + island);
}

// Place the tiles (in class order) in the launch's wavefront slots. The
// dispatcher hands workgroup g to XCD g mod 8, each XCD with its own L2: the
// tiles are cut into eight contiguous stretches of about equal weight, a
// tile's bytes plus a wavefront's fixed cost (wavefronts of different classes
// move different amounts), stretch x fills
// XCD x's workgroups x, x + 8, x + 16, ... wpg tiles each, in order, so a
// member's neighbouring tiles share an L2 and no XCD is left with a heavier
// share to finish alone. Returns the slots the placement spans (a multiple of
// 8 wpg); slot[i] is tile i's slot.
uint32_t place_tiles(const std::vector<ga::RunView>& views, const std::vector<ga::Tile>& tiles,
                     uint32_t wpg, std::vector<uint32_t>& slot) {
  slot.assign(tiles.size(), 0u);
  if (tiles.empty()) return 0;
  std::vector<uint64_t> w(tiles.size());
  uint64_t total = 0;
  for (size_t i = 0; i < tiles.size(); ++i) {
    const ga::RunView& v = views[tiles[i].run];
    w[i] = tile_bytes(v, std::min(v.ipw, v.islands - tiles[i].first)) + ga::kWaveFixedBytes;
    total += w[i];
  }
  // tile i goes to the XCD whose eighth of the bytes holds its midpoint
  uint32_t count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint64_t before = 0;
  uint32_t groups = 0;
  for (size_t i = 0; i < tiles.size(); ++i) {
    const uint64_t mid2 = 2 * before + w[i];  // twice the midpoint
    const uint32_t x = (uint32_t)std::min<uint64_t>(7, mid2 * 8 / (2 * total));
    const uint32_t k = count[x]++;
    slot[i] = ((k / wpg) * 8u + x) * wpg + k % wpg;
    groups = std::max(groups, k / wpg + 1);
    before += w[i];
  }
  return groups * 8u * wpg;
}

// Rebuild the device tables for the current members and upload them in the
// batch's stream order (no wait: a kernel already enqueued keeps reading the
// old contents until the copy runs after it). Capacities grow (with a wait
// for the stream and a new graph) only when the members outgrow them.
int rebuild_tables(ga_batch* b) {
  std::vector<ga::RunView> views;
  std::vector<ga::Tile> tiles;
  views.reserve(b->members.size());
  uint32_t max_ipw = 1;
  for (uint32_t m = 0; m < b->members.size(); ++m) {
    ga::RunView v = b->members[m]->view;
    v.ipw = class_ipw(b, class_of(v));
    max_ipw = std::max(max_ipw, v.ipw);
    views.push_back(v);
    for (uint32_t first = 0; first < v.islands; first += v.ipw)
      tiles.push_back({m, first, class_of(v), 0u});
  }
  // wavefronts of one class side by side: neighbouring wavefronts on a CU
  // then run the same shape and share instruction-cache lines
  std::stable_sort(tiles.begin(), tiles.end(),
                   [](const ga::Tile& a, const ga::Tile& c) { return a.cls < c.cls; });
  for (BatchClass& k : b->cls) k.n_tiles = 0;
  for (const ga::Tile& t : tiles) b->cls[t.cls].n_tiles += 1;
  std::vector<uint32_t> slot;
  const uint32_t span = place_tiles(views, tiles, b->wpg, slot);
  // the graph's grid covers the placement with headroom; it is captured
  // again only when a placement outgrows it or the launch shape changes (the
  // largest islands per wavefront sizes each wavefront's LDS)
  const uint32_t unit = 8u * b->wpg;  // whole groups on every XCD
  uint32_t grid = b->grid_waves;
  if (span > grid || b->wpg != b->use_wpg)
    grid = ceil_div(std::max(grid, pow2_at_least(span)), unit) * unit;
  if (views.size() > b->view_cap || grid > b->tile_cap || !b->d_tab) {
    GA_HIP(hipStreamSynchronize(b->stream), "stream sync");
    if (b->d_tab) GA_HIP(hipFree(b->d_tab), "free tables");
    b->d_tab = nullptr;
    b->view_cap = std::max<uint32_t>({64u, b->view_cap, (uint32_t)views.size() * 2});
    b->tile_cap = std::max<uint32_t>({4096u, b->tile_cap, grid * 2});
    GA_HIP(hipMalloc(&b->d_tab, tab_bytes(b)), "alloc tables");
    for (int i = 0; i < 2; ++i) {
      if (b->h_stage[i]) GA_HIP(hipHostFree(b->h_stage[i]), "free staging");
      b->h_stage[i] = nullptr;
      GA_HIP(hipHostMalloc(reinterpret_cast<void**>(&b->h_stage[i]), tab_bytes(b)), "alloc staging");
      if (!b->stage_done[i])
        GA_HIP(hipEventCreateWithFlags(&b->stage_done[i], hipEventDisableTiming), "event");
    }
    b->stage_bytes = tab_bytes(b);
    b->graph_stale = true;
  }
  // a staging buffer is reused once its previous copy has completed
  uint8_t* st = b->h_stage[b->stage_next];
  GA_HIP(hipEventSynchronize(b->stage_done[b->stage_next]), "staging free");
  std::memset(st, 0, b->stage_bytes);
  for (ga::RunView& v : views) to_table(v, b->d_tab);
  if (!views.empty()) std::memcpy(st, views.data(), views.size() * sizeof(ga::RunView));
  ga::Tile* tab = reinterpret_cast<ga::Tile*>(st + tab_tiles_off(b));
  for (uint32_t i = 0; i < b->tile_cap; ++i) tab[i] = {0u, 0u, ga::kNoTile, 0u};
  for (size_t i = 0; i < tiles.size(); ++i) tab[slot[i]] = tiles[i];
  uint32_t* counts = reinterpret_cast<uint32_t*>(st + tab_counts_off(b));
  counts[0] = (uint32_t)tiles.size();
  counts[1] = (uint32_t)views.size();
  if (grid != b->grid_waves) b->graph_stale = true;
  b->grid_waves = grid;
  if (max_ipw != b->use_max_ipw || b->wpg != b->use_wpg) b->graph_stale = true;
  b->use_max_ipw = max_ipw;
  b->use_wpg = b->wpg;
  GA_HIP(hipMemcpyAsync(b->d_tab, st, b->stage_bytes, hipMemcpyHostToDevice, b->stream),
         "upload tables");
  GA_HIP(hipEventRecord(b->stage_done[b->stage_next], b->stream), "staging event");
  b->stage_next ^= 1;
  b->dirty = false;
  return GA_OK;
}

const ga::RunView* tab_views(const ga_batch* b) {
  return reinterpret_cast<const ga::RunView*>(b->d_tab);
}
const ga::Tile* tab_tiles(const ga_batch* b) {
  return reinterpret_cast<const ga::Tile*>(b->d_tab + tab_tiles_off(b));
}
const uint32_t* tab_count(const ga_batch* b, uint32_t i) {
  return reinterpret_cast<const uint32_t*>(b->d_tab + tab_counts_off(b)) + i;
}

hipError_t launch_gen(ga_batch* b, uint32_t gen_offset, hipStream_t s) {
  return ga::launch_batch_all(tab_views(b), tab_tiles(b), b->grid_waves, gen_offset,
                              b->use_max_ipw, b->use_wpg, s);
}

int batch_direct(ga_batch* b, uint64_t n) {
  while (n > 0) {
    const uint64_t slice = std::min<uint64_t>(n, 1u << 20);
    for (uint64_t g = 0; g < slice; ++g)
      GA_HIP(launch_gen(b, (uint32_t)g, b->stream), "batch launch");
    GA_HIP(ga::launch_batch_advance(tab_views(b), tab_count(b, 1), b->view_cap, slice, b->stream),
           "batch advance");
    n -= slice;
  }
  return GA_OK;
}

// One block of graph_block generations: one launch per generation over every
// member's tiles, then the block's advance. Members are read from the device
// tables at run time, so the graph outlives membership changes.
int batch_graph(ga_batch* b) {
  if (b->graph && !b->graph_stale) return GA_OK;
  if (b->graph) {
    // the graph may still be running its last launch: it is destroyed only
    // once the stream has finished it
    GA_HIP(hipStreamSynchronize(b->stream), "stream sync");
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  if (!b->capture_stream)
    GA_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking), "capture stream");
  GA_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t err = hipSuccess;
  for (uint32_t g = 0; g < b->graph_block && err == hipSuccess; ++g)
    err = launch_gen(b, g, b->capture_stream);
  if (err == hipSuccess)
    err = ga::launch_batch_advance(tab_views(b), tab_count(b, 1), b->view_cap, b->graph_block,
                                   b->capture_stream);
  hipGraph_t graph = nullptr;
  hipError_t end = hipStreamEndCapture(b->capture_stream, &graph);
  if (err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(err, "launch during capture");
  }
  if (end != hipSuccess) return hip_fail(end, "end capture");
  hipGraphExec_t exec = nullptr;
  err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (err != hipSuccess) return hip_fail(err, "graph instantiate");
  b->graph = exec;
  b->graph_stale = false;
  return GA_OK;
}

}  // namespace

int ga_batch_class_launch(ga_batch* b, uint32_t log2n, uint32_t words, uint32_t* ipw,
                          uint32_t* tiles) {
  if (!b) return fail(GA_EINVAL, "batch is NULL");
  if (log2n > 6 || words < 1 || words > 2) return fail(GA_EINVAL, "no such class");
  const uint32_t c = log2n * 2 + words - 1;
  uint32_t n = 0;
  for (const ga_run* r : b->members)
    if (class_of(r->view) == c) n += ceil_div(r->view.islands, class_ipw(b, c));
  if (ipw) *ipw = class_ipw(b, c);
  if (tiles) *tiles = n;
  return GA_OK;
}

int ga_batch_step(ga_batch* b, uint64_t n) {
  if (!b) return fail(GA_EINVAL, "batch is NULL");
  if (n == 0 || b->members.empty()) return GA_OK;
  const Range range("ga_batch_step", n);
  if (b->dirty) {
    int rc = rebuild_tables(b);
    if (rc != GA_OK) return rc;
  }
  uint64_t left = n;
  if (b->graph_block > 0 && left >= b->graph_block) {
    int rc = batch_graph(b);
    if (rc != GA_OK) return rc;
    while (left >= b->graph_block) {
      const Range block("batch block", b->graph_block);
      GA_HIP(hipGraphLaunch(b->graph, b->stream), "graph launch");
      left -= b->graph_block;
    }
  }
  int rc = batch_direct(b, left);
  if (rc != GA_OK) return rc;
  // host mirrors: however the n generations are split into blocks, each
  // member advances by min(n, its remaining budget)
  b->steps += 1;
  const int slot = (int)((b->steps - 1) % ga_batch::kStepEvents);
  hipEvent_t& ev = b->step_done[slot];
  if (!ev) GA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  GA_HIP(hipEventRecord(ev, b->stream), "step event");
  b->step_of[slot] = b->steps;
  // the work just enqueued keeps the GPU busy while the host waits for the
  // call kStepsInFlight before this one
  if (b->steps > ga_batch::kStepsInFlight) {
    bool done = false;
    const int rc = step_complete(b, b->steps - ga_batch::kStepsInFlight, true, &done);
    if (rc != GA_OK) return rc;
  }
  for (size_t i = 0; i < b->members.size(); ++i) {
    const uint64_t adv = std::min<uint64_t>(b->remaining[i], n);
    b->members[i]->gen_host += adv;
    b->remaining[i] -= adv;
    if (adv && b->remaining[i] == 0) b->finished_step[i] = b->steps;
  }
  return GA_OK;
}

void ga_batch_destroy(ga_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (ga_run* r : b->members) r->batch = nullptr;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (hipEvent_t e : b->step_done)
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < 2; ++i) {
    if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
    if (b->stage_done[i]) (void)hipEventDestroy(b->stage_done[i]);
  }
  if (b->d_tab) (void)hipFree(b->d_tab);
  delete b;
}

// ---------------------------------------------------------------------------
// Run pool (served form)
// ---------------------------------------------------------------------------

int ga_pool_create(void* dev_mem, size_t bytes, uint32_t max_slots, void* hip_stream,
                   ga_pool** out) {
  if (!out) return fail(GA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!dev_mem) return fail(GA_EINVAL, "dev_mem is NULL");
  if (reinterpret_cast<uintptr_t>(dev_mem) % kAlign) return fail(GA_EINVAL, "dev_mem must be 256-byte aligned");
  if (max_slots == 0) return fail(GA_EINVAL, "max_slots must be >= 1");
  ga_pool* p = new (std::nothrow) ga_pool();
  if (!p) return fail(GA_EINVAL, "host allocation failed");
  p->base = static_cast<uint8_t*>(dev_mem);
  p->bytes = bytes / kAlign * kAlign;
  p->max_slots = max_slots;
  if (p->bytes) p->free_blocks.emplace(0, p->bytes);
  const int rc = ga_batch_create(hip_stream, &p->batch);
  if (rc != GA_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return GA_OK;
}

int ga_pool_admit(ga_pool* p, const ga_config* cfg, uint64_t n_gens, uint64_t* ticket) {
  if (!p || !ticket) return fail(GA_EINVAL, "pool or ticket is NULL");
  const size_t need = align_up(ga_state_bytes(cfg));
  if (need == 0) return fail(GA_EINVAL, "invalid configuration");
  if (need > p->bytes) return fail(GA_EINVAL, "run larger than the whole pool");
  if (p->members.size() >= p->max_slots) return fail(GA_ENOMEM, "every slot is taken");
  const size_t off = pool_take(p, need);
  if (off == SIZE_MAX) return fail(GA_ENOMEM, "no free block holds the run");
  ga_run* r = nullptr;
  int rc = ga_init(cfg, p->base + off, need, p->batch->stream, &r);
  if (rc == GA_OK) {
    rc = ga_batch_add(p->batch, r, n_gens);
    if (rc != GA_OK) ga_destroy(r);
  }
  if (rc != GA_OK) {
    pool_give(p, off, need);
    return rc;
  }
  *ticket = p->next_ticket++;
  p->members.emplace(*ticket, ga_pool::Member{r, off, need});
  p->used += need;
  return GA_OK;
}

int ga_pool_step(ga_pool* p, uint64_t n_gens) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  return ga_batch_step(p->batch, n_gens);
}

int ga_pool_set_graph_block(ga_pool* p, uint32_t gens_per_block) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  return ga_batch_set_graph_block(p->batch, gens_per_block);
}

int ga_pool_set_launch(ga_pool* p, uint32_t islands_per_wave, uint32_t waves_per_group) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  return ga_batch_set_launch(p->batch, islands_per_wave, waves_per_group);
}

int ga_pool_set_class_launch(ga_pool* p, uint32_t log2n, uint32_t words,
                             uint32_t islands_per_wave) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  return ga_batch_set_class_launch(p->batch, log2n, words, islands_per_wave);
}

int ga_pool_remaining(const ga_pool* p, uint64_t ticket, uint64_t* left) {
  if (!p || !left) return fail(GA_EINVAL, "pool or left is NULL");
  auto it = p->members.find(ticket);
  if (it == p->members.end()) return fail(GA_EINVAL, "unknown ticket");
  *left = ga_batch_remaining(p->batch, it->second.run);
  return GA_OK;
}

int ga_pool_poll(const ga_pool* p, uint64_t* tickets, size_t cap, size_t* n_done) {
  return ga_pool_poll_settled(p, tickets, cap, n_done, 0);
}

int ga_pool_poll_settled(const ga_pool* p, uint64_t* tickets, size_t cap, size_t* n_done,
                         int settled_only) {
  if (!p || !n_done) return fail(GA_EINVAL, "pool or n_done is NULL");
  size_t n = 0;
  for (const auto& m : p->members) {
    if (ga_batch_remaining(p->batch, m.second.run) != 0) continue;
    if (settled_only) {
      int settled = 0;
      const int rc = ga_batch_settled(p->batch, m.second.run, &settled);
      if (rc != GA_OK) return rc;
      if (!settled) continue;
    }
    if (tickets && n < cap) tickets[n] = m.first;
    ++n;
  }
  *n_done = n;
  return GA_OK;
}

namespace {

// One agent per island of run r (sampling stream at its current generation),
// on the pool's side stream; waits for the side stream only. A settled run
// (its last generation has run) is sampled at once: the batch's later work
// only reads its counters and skips it. Otherwise the sampling follows
// everything enqueued so far on the batch stream.
int pool_sample(ga_pool* p, ga_run* r, bool settled, uint64_t* ids_out, uint32_t* T_out,
                uint32_t* surface_words_out) {
  if (!p->side) GA_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking), "side stream");
  if (!p->batch_mark) GA_HIP(hipEventCreateWithFlags(&p->batch_mark, hipEventDisableTiming), "event");
  if (!p->side_mark) GA_HIP(hipEventCreateWithFlags(&p->side_mark, hipEventDisableTiming), "event");
  if (!settled) {
    GA_HIP(hipEventRecord(p->batch_mark, p->batch->stream), "mark batch");
    GA_HIP(hipStreamWaitEvent(p->side, p->batch_mark, 0), "side waits");
  }
  const ga::RunView& v = r->view;
  const size_t I = v.islands, W = v.words;
  uint32_t* st_ids = reinterpret_cast<uint32_t*>(r->base + r->lay.st_ids);
  uint32_t* st_T = reinterpret_cast<uint32_t*>(r->base + r->lay.st_T);
  uint32_t* st_D = reinterpret_cast<uint32_t*>(r->base + r->lay.st_D);
  std::vector<uint32_t> ids32(I), tT(I), tD(I * W);
  GA_HIP(ga::launch_sample(v, st_ids, p->side), "sample launch");
  GA_HIP(ga::launch_gather(v, st_ids, (uint32_t)I, st_T, st_D, p->side), "gather launch");
  GA_HIP(hipMemcpyAsync(ids32.data(), st_ids, I * 4, hipMemcpyDeviceToHost, p->side), "read ids");
  GA_HIP(hipMemcpyAsync(tT.data(), st_T, I * 4, hipMemcpyDeviceToHost, p->side), "read T");
  GA_HIP(hipMemcpyAsync(tD.data(), st_D, I * W * 4, hipMemcpyDeviceToHost, p->side), "read surfaces");
  GA_HIP(hipStreamSynchronize(p->side), "side sync");
  for (size_t j = 0; j < I; ++j) {
    if (ids_out) ids_out[j] = ids32[j];
    if (T_out) T_out[j] = tT[j];
    if (surface_words_out)
      for (size_t w = 0; w < W; ++w) surface_words_out[j * W + w] = tD[w * I + j];
  }
  return GA_OK;
}

}  // namespace

int ga_pool_retire(ga_pool* p, uint64_t ticket, uint64_t* ids_out, uint32_t* T_out,
                   uint32_t* surface_words_out) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  auto it = p->members.find(ticket);
  if (it == p->members.end()) return fail(GA_EINVAL, "unknown ticket");
  ga_run* r = it->second.run;
  // sample while the run is still a member (a failure leaves the pool as it was)
  const bool sampled = ids_out || T_out || surface_words_out;
  if (sampled) {
    int settled = 0;
    int rc = ga_batch_settled(p->batch, r, &settled);
    if (rc == GA_OK) rc = pool_sample(p, r, settled != 0, ids_out, T_out, surface_words_out);
    if (rc != GA_OK) return rc;
  }
  const int rc = ga_batch_remove(p->batch, r);
  if (rc != GA_OK) return rc;
  // the run's block returns to the pool; whatever the batch stream runs next
  // (a new run's founders in that block) follows the sampling
  if (sampled) {
    GA_HIP(hipEventRecord(p->side_mark, p->side), "mark side");
    GA_HIP(hipStreamWaitEvent(p->batch->stream, p->side_mark, 0), "batch waits");
  }
  // no wait for the run's stream (the batch stream): the memory is not freed,
  // and every later use of it is ordered after the batch's work by the stream
  drop_graph(r);
  if (r->capture_stream) (void)hipStreamDestroy(r->capture_stream);
  delete r;
  pool_give(p, it->second.off, it->second.size);
  p->used -= it->second.size;
  p->members.erase(it);
  return GA_OK;
}

int ga_pool_usage(const ga_pool* p, size_t* used, size_t* largest_free, uint32_t* live) {
  if (!p) return fail(GA_EINVAL, "pool is NULL");
  if (used) *used = p->used;
  if (largest_free) {
    size_t big = 0;
    for (const auto& b : p->free_blocks) big = std::max(big, b.second);
    *largest_free = big;
  }
  if (live) *live = (uint32_t)p->members.size();
  return GA_OK;
}

void ga_pool_destroy(ga_pool* p) {
  if (!p) return;
  for (auto& m : p->members) {
    (void)ga_batch_remove(p->batch, m.second.run);
    ga_destroy(m.second.run);
  }
  ga_batch_destroy(p->batch);
  if (p->side) {
    (void)hipStreamSynchronize(p->side);
    (void)hipStreamDestroy(p->side);
  }
  if (p->batch_mark) (void)hipEventDestroy(p->batch_mark);
  if (p->side_mark) (void)hipEventDestroy(p->side_mark);
  delete p;
}

// ---------------------------------------------------------------------------
// Roof microbenchmarks
// ---------------------------------------------------------------------------

int ga_roof_inplace(void* planes, size_t words_per_plane, uint32_t n_planes, void* hip_stream) {
  if (!planes) return fail(GA_EINVAL, "planes is NULL");
  if (reinterpret_cast<uintptr_t>(planes) % 16 || words_per_plane % 4)
    return fail(GA_EINVAL, "planes must be 16-byte aligned and words_per_plane a multiple of 4");
  if (n_planes < 1 || n_planes > 8) return fail(GA_EINVAL, "n_planes must be in [1, 8]");
  GA_HIP(ga::launch_roof_inplace(planes, words_per_plane, n_planes,
                                 static_cast<hipStream_t>(hip_stream)), "roof launch");
  return GA_OK;
}

int ga_roof_philox(uint32_t* out, uint32_t threads, uint32_t blocks_per_thread, void* hip_stream) {
  if (!out) return fail(GA_EINVAL, "out is NULL");
  if (threads % 256) return fail(GA_EINVAL, "threads must be a multiple of 256");
  GA_HIP(ga::launch_roof_philox(out, threads, blocks_per_thread,
                                static_cast<hipStream_t>(hip_stream)), "roof launch");
  return GA_OK;
}

int ga_roof_valu(uint32_t* out, uint32_t threads, uint32_t iters, uint32_t kind, void* hip_stream) {
  if (!out) return fail(GA_EINVAL, "out is NULL");
  if (threads % 256) return fail(GA_EINVAL, "threads must be a multiple of 256");
  if (kind > 1) return fail(GA_EINVAL, "kind must be 0 (three-input XOR) or 1 (64-bit multiply-add)");
  GA_HIP(ga::launch_roof_valu(out, threads, iters, kind, static_cast<hipStream_t>(hip_stream)),
         "roof launch");
  return GA_OK;
}

// ---------------------------------------------------------------------------
// Post hoc relatedness
// ---------------------------------------------------------------------------

size_t ga_mrca_workspace_bytes(size_t n) { return ga::mrca_workspace_bytes(n); }

namespace {

// Argument checks shared by the relatedness calls.
int mrca_args_ok(const uint32_t* T, const uint32_t* surface_words, size_t n,
                 uint32_t surface_sites, uint32_t differentia_bits, uint32_t surface_policy,
                 uint32_t kc, const uint32_t* L, const uint32_t* U) {
  if (n > 65535) return fail(GA_EINVAL, "n must be <= 65535");
  if (!surface_ok(surface_sites, differentia_bits))
    return fail(GA_EINVAL, "surface_sites x differentia_bits must be 32 or 64 bits");
  std::string why;
  if (!policy_ok(surface_policy, surface_sites, differentia_bits, &why))
    return fail(GA_EINVAL, why);
  if (kc < 1) return fail(GA_EINVAL, "kc must be >= 1");
  if (!T || !surface_words || !L || !U) return fail(GA_EINVAL, "NULL pointer");
  return GA_OK;
}

}  // namespace

int ga_mrca_matrix_ex(const uint32_t* T, const uint32_t* surface_words, size_t n,
                      uint32_t surface_sites, uint32_t differentia_bits, uint32_t surface_policy,
                      uint32_t kc, void* workspace, size_t workspace_bytes, uint32_t* L,
                      uint32_t* U, void* hip_stream) {
  if (n == 0) return GA_OK;
  const int rc = mrca_args_ok(T, surface_words, n, surface_sites, differentia_bits,
                              surface_policy, kc, L, U);
  if (rc != GA_OK) return rc;
  if (surface_policy == GA_POLICY_STEADY) {
    if (!workspace) return fail(GA_EINVAL, "NULL workspace");
    if (workspace_bytes < ga::mrca_workspace_bytes(n)) return fail(GA_ENOMEM, "workspace too small");
  }
  GA_HIP(ga::launch_mrca_matrix(T, surface_words, (uint32_t)n, log2u(surface_sites),
                                log2u(differentia_bits), surface_policy, kc, workspace, L, U,
                                static_cast<hipStream_t>(hip_stream)),
         "mrca launch");
  return GA_OK;
}

int ga_mrca_matrix_noalloc(const uint32_t* T, const uint32_t* surface_words, size_t n,
                           uint32_t surface_sites, uint32_t differentia_bits,
                           uint32_t surface_policy, uint32_t kc, uint32_t* L, uint32_t* U,
                           void* hip_stream) {
  if (n == 0) return GA_OK;
  if (n > ga::kScratchSurfaces)
    return fail(GA_EINVAL, "n exceeds the 65,536 surfaces of the static workspace");
  const int rc = mrca_args_ok(T, surface_words, n, surface_sites, differentia_bits,
                              surface_policy, kc, L, U);
  if (rc != GA_OK) return rc;
  GA_HIP(ga::launch_mrca_matrix_noalloc(T, surface_words, (uint32_t)n, log2u(surface_sites),
                                        log2u(differentia_bits), surface_policy, kc, L, U,
                                        static_cast<hipStream_t>(hip_stream)),
         "mrca launch (static workspace)");
  return GA_OK;
}

int ga_mrca_matrix(const uint32_t* T, const uint32_t* surface_words, size_t n,
                   uint32_t surface_sites, uint32_t kc, void* workspace, size_t workspace_bytes,
                   uint32_t* L, uint32_t* U, void* hip_stream) {
  if (n != 0 && surface_sites != 32 && surface_sites != 64)
    return fail(GA_EINVAL, "surface_sites must be 32 or 64");
  return ga_mrca_matrix_ex(T, surface_words, n, surface_sites, 1, GA_POLICY_STEADY, kc,
                           workspace, workspace_bytes, L, U, hip_stream);
}

}  // extern "C"
