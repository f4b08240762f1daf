// Internal definitions shared by the kernels and the C ABI of libga_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ga {

// Device view of one run's state. The population is SoA planes so a
// wavefront touches 256 contiguous bytes per field; outbox entries are AoS so
// one 16-byte load brings an arrival's genome (and, for 32-site surfaces, its
// header):
//   pop_f[a], pop_T[a], pop_D[w * agent_stride + a]      a = island * N + slot
//   ob[p][i * ob_stride + k], k = 0 fitness, 1 T, 2.. surface words,
//   2 + words header (bit 2 valid, bits 0-1 direction); ob_stride = 4 or 8
//   words; p = generation parity.
// Planes are padded to island_stride = roundup(islands, 64) + 128 islands
// (agent_stride = island_stride * N agents): a wavefront's last chunk may run
// up to 63 islands past the last island and then only touches padding (the
// rest is slack).
struct RunView {
  float* pop_f;
  uint32_t* pop_T;
  uint32_t* pop_D;
  uint32_t* ob[2];
  unsigned long long* gen;   // generation counter t (device)
  unsigned long long* left;  // generations still owed in the current batch block (batch
                             // only); always the word after *gen
  uint32_t width, height, islands, agents;
  uint32_t island_stride, agent_stride;
  uint32_t log2n, words, k, selection;
  uint32_t p32, migration, seed, run_id;
  uint32_t ipw;              // islands per wavefront
  uint32_t ob_stride;        // words per outbox entry
  uint32_t law;              // 0 discrete delta, 1 treatments (normal sizes)
  uint32_t p_ben;            // law 1: beneficial iff draw < p_ben
  uint32_t p_any;            // law 1: deleterious iff p_ben <= draw < p_any
  uint32_t pad;
  // asynchronous schedule only (NULL otherwise):
  //   mail[((i * 4 + d) * 2 + p) * ob_stride + k]: island i's buffer toward
  //     direction d for sending generations of parity p, k as in an outbox
  //     entry, the header word holding the stamp 2 * (sending generation + 1),
  //     odd while being rewritten;
  //   seen[i * 4 + q]: stamp of the last genome island i took from direction q;
  //   prog[c]: generations chunk c (islands c * ipw ...) has completed, low word;
  //   lock[(p * 4 + d) * island_stride + i]: lockstep header of island i's
  //     buffer toward direction d for sending generations of parity p:
  //     2 * (g + 1) if it sent a genome that way in generation g, else
  //     2 * (g + 1) + 1;
  //   waits[0]: how often a wavefront stopped waiting for a neighbour and went
  //     on; waits[1]: genomes absorbed from the buffers.
  uint32_t* mail;
  uint32_t* seen;
  uint32_t* prog;
  uint32_t* lock;
  unsigned long long* waits;
  // genome model (an id of GA_FOR_EACH_MODEL) and, for a model with a
  // string, its two word planes pop_P[w * agent_stride + a]
  uint32_t model;
  uint32_t* pop_P;
  // surface: S = 2^s_log sites of 2^dlog-bit differentia in `words` words,
  // policy 0 "doubling steady", 1 "tilted", 2 "hybrid"
  uint32_t s_log, dlog, policy;
  // LDS-resident tiles (synchronous schedule): tiles of tile_w x tile_h
  // islands, tiles_x across and tiles_y down (the last ones ragged); tile c's
  // progress word is prog[c]
  uint32_t tile_w, tile_h, tiles_x, tiles_y;
};

// Asynchronous pacing: no bound on how far an island may run ahead, and the
// number of progress checks before an island goes on regardless.
constexpr uint32_t kUnpaced = 0xFFFFFFFFu;
constexpr uint32_t kPaceSpins = 2048;
// The lockstep exchange waits only on its neighbours' real progress, so its
// bound (about 70 ms of checks) only has to end waits on a wavefront that
// never runs; shorter bounds gave up on wavefronts held back a few
// milliseconds (first touches of a multi-GB mail plane).
constexpr uint32_t kLockSpins = 32768;

// One wavefront's share of a batched launch: islands [first, first + ipw) of
// member `run`, whose class is `cls` (read with the tile, so the wavefront
// branches to its body before it reads anything of the member). The table
// has one slot per wavefront of the launch; a slot no tile takes has class
// kNoTile.
// Batch classes: one per (log2 N, surface words), index log2 N * 2 + words - 1.
constexpr uint32_t kBatchClasses = 14;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
// A batched wavefront's fixed cost (its start, the island pass) in the units
// the tiles are balanced over the XCDs in, algorithmic bytes: measured on the
// 64-run workload, weights of 2 to 8 KiB per wavefront balance best.
constexpr uint64_t kWaveFixedBytes = 4096;
struct Tile {
  uint32_t run;
  uint32_t first;
  uint32_t cls;
  uint32_t pad;
};

constexpr uint32_t kMetaValid = 4u;
constexpr uint32_t kDiscard = 0xFFFFFFFFu;
constexpr int kMaxWavesPerGroup = 16;

// Launch wrappers (defined in ga_kernels.hip). All enqueue on `stream`.
hipError_t launch_generation(const RunView& v, uint32_t gen_offset, uint32_t waves,
                             uint32_t waves_per_group, hipStream_t stream);
// The LDS-resident tile form: one persistent launch of n_gens generations,
// one workgroup per tile (v.tile_* set; v.prog holds a word per tile, equal to
// the generation counter's low word before the launch).
hipError_t launch_tiles(const RunView& v, uint64_t n_gens, hipStream_t stream);
// LDS bytes and threads of a tile's workgroup, and how many such workgroups
// one CU holds at once.
size_t tile_lds_bytes(uint32_t tile_w, uint32_t tile_h, uint32_t log2n, uint32_t words,
                      uint32_t model, uint32_t ob_stride);
uint32_t tile_threads(uint32_t tile_w, uint32_t tile_h, uint32_t log2n);
hipError_t tile_occupancy(const RunView& v, uint32_t threads, size_t lds, int* groups_per_cu);
hipError_t launch_async(const RunView& v, uint64_t n_gens, uint32_t waves, uint32_t chunks,
                        uint32_t waves_per_group, uint32_t lead, uint32_t skew,
                        hipStream_t stream);
// The lockstep asynchronous launch (no lead, no skew) at generation `gen`:
// its header prologue, then the persistent kernel.
hipError_t launch_lockstep(const RunView& v, uint64_t gen, uint64_t n_gens, uint32_t waves,
                           uint32_t chunks, uint32_t waves_per_group, hipStream_t stream);
// Wavefronts of the async (or lockstep) kernel the current device holds at once.
hipError_t async_capacity(const RunView& v, uint32_t waves_per_group, bool lockstep,
                          uint32_t* waves);
hipError_t launch_advance(unsigned long long* gen, uint64_t n, hipStream_t stream);
// Founders of the run's genome model (its initialize function).
hipError_t launch_init(const RunView& v, hipStream_t stream);
// Whether genome model `id` carries a 64-bit string, and how many models there are.
bool model_has_string_host(uint32_t id);
uint32_t model_count();
// Dynamic LDS bytes of a launch.
size_t lds_bytes(uint32_t ipw, uint32_t waves, uint32_t model);
hipError_t launch_fill(uint32_t* p, uint32_t value, size_t words, hipStream_t stream);
hipError_t launch_sample(const RunView& v, uint32_t* ids, hipStream_t stream);
hipError_t launch_gather(const RunView& v, const uint32_t* ids, uint32_t n, uint32_t* T_out,
                         uint32_t* D_out, hipStream_t stream);
// One generation of a batch: grid_waves wavefronts, wavefront w running
// tiles[w] (the table holds grid_waves slots; an empty one has class
// kNoTile); LDS sized for max_ipw.
hipError_t launch_batch_all(const RunView* views, const Tile* tiles, uint32_t grid_waves,
                            uint32_t gen_offset, uint32_t max_ipw, uint32_t waves_per_group,
                            hipStream_t stream);
hipError_t launch_store_u64(unsigned long long* p, unsigned long long value, hipStream_t stream);
// Close a block of a batch: *n_runs members (device count), a grid for cap.
hipError_t launch_batch_advance(const RunView* views, const uint32_t* n_runs, uint32_t cap,
                                uint64_t block, hipStream_t stream);

// Roof microbenchmarks (ga_roofs.hip).
hipError_t launch_roof_inplace(void* base, size_t words_per_plane, uint32_t planes,
                               hipStream_t stream);
hipError_t launch_roof_philox(uint32_t* out, uint32_t threads, uint32_t blocks, hipStream_t stream);
hipError_t launch_roof_valu(uint32_t* out, uint32_t threads, uint32_t iters, uint32_t kind,
                            hipStream_t stream);

size_t mrca_workspace_bytes(size_t n);
// Most surfaces the allocation-free relatedness call takes (its workspace is a
// static device array of this many normalised surfaces, 16 bytes each).
constexpr uint32_t kScratchSurfaces = 65536;
// launch_mrca_matrix with that static array as its workspace.
hipError_t launch_mrca_matrix_noalloc(const uint32_t* T, const uint32_t* D, uint32_t n,
                                      uint32_t s_log, uint32_t dlog, uint32_t policy, uint32_t kc,
                                      uint32_t* L, uint32_t* U, hipStream_t stream);
hipError_t launch_mrca_matrix(const uint32_t* T, const uint32_t* D, uint32_t n, uint32_t s_log,
                              uint32_t dlog, uint32_t policy, uint32_t kc, void* workspace,
                              uint32_t* L, uint32_t* U, hipStream_t stream);

}  // namespace ga
