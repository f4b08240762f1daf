/*
 * ga.h - C ABI of the MI355X island-model GA library (libga_hip.so).
 *
 * The library runs the generation step of a tracking-enabled island-model
 * genetic algorithm (Moreno, Yang, Dolson, Zaman, "Trackable Island-model
 * Genetic Algorithms at Wafer Scale", GECCO '24 Companion) as HIP kernels on
 * one gfx950 GPU. Islands sit on a W x H torus, each holding N agents; every
 * generation handles migration first, then evaluation, tournament selection,
 * mutation of the whole next population and one hereditary-stratigraphy
 * deposit per agent, and the run halts at a generation count (Sec. 2,
 * Methods). The genome is a float32 fitness followed by tracking annotation
 * (Sec. 3): here a uint32 deposit counter T and an S-site surface of 1-bit
 * differentia.
 *
 * Semantics of one generation t (synchronous; every island finishes t before
 * any island starts t+1):
 *   1. absorb: for q = N, E, S, W (0..3), if the neighbour in direction q
 *      emitted toward this island during t-1, its genome overwrites the slot
 *      this island draws for q; a later q wins a clash (Sec. 2, immigration);
 *   2. emit: a copy of one random member (post-absorb) is sent to one random
 *      cardinal neighbour, delivered at t+1 (Sec. 2, emigration);
 *   3-5. every child slot takes the fittest of k entrants drawn with
 *      replacement, the first in draw order on ties (tournament with random
 *      tie-break, Sec. 2), or entrant 0 under neutral selection;
 *   6. with probability p the child's fitness gains a delta drawn uniformly
 *      from {-1, -1/2, 0, 1/2, 1} (binary32, round to nearest even) (Sec. 2,
 *      mutation operator);
 *   7. the child writes one random differentia bit at the site the
 *      "doubling steady" surface policy gives for rank T (or writes nothing),
 *      then T += 1 (Sec. 2, stratigraphy update once per generation).
 * Every random draw is one Philox4x32-10 block (Salmon et al., SC'11) keyed
 * by (seed, run_id) with counter (slot or 0, island, generation low word,
 * generation high word * 4 + stream), stream 0 selection, 1 migration,
 * 2 sampling, 3 mutation sizes (law 1). Results are therefore bit-identical for any launch
 * shape and with or without batching; the asynchronous schedule (below) changes only the
 * moment a migrant is read, and with its default pacing not even that.
 *
 * Conventions for every entry point:
 *   - Return value: GA_OK (0) or a negative GA_E* code; ga_last_error()
 *     gives a message for the calling thread's last failure. A call that
 *     fails leaves the run's state unchanged. No C++ exception crosses the ABI.
 *   - Device memory for a run's state is allocated by the caller and is never
 *     freed by the library. Host buffers are owned by the caller.
 *   - A run is bound to one HIP stream. Calls on one handle must not overlap
 *     from several host threads.
 *   - Agent a = island * N + slot, island = y * W + x.
 */
#ifndef GA_H
#define GA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GA_OK 0
#define GA_EINVAL (-1)   /* invalid argument or configuration */
#define GA_ENOMEM (-2)   /* caller's device buffer smaller than ga_state_bytes */
#define GA_EDEVICE (-3)  /* a HIP runtime call failed */
#define GA_ESTATE (-4)   /* handle in the wrong state for this call */

/* Run configuration. All fields are validated by ga_init. */
typedef struct ga_config {
  uint32_t struct_size;        /* sizeof(ga_config) */
  uint32_t width;              /* islands per row, 1..65535 */
  uint32_t height;             /* rows, 1..65535; width * height * N < 2^30 */
  uint32_t pop_per_island;     /* N: power of two, 1..64 (Sec. 2 uses 32) */
  uint32_t surface_sites;      /* S sites: 32 or 64 one-bit differentia (or, with
                                * differentia_bits b > 1, a power of two with
                                * S * b = 32 or 64) */
  uint32_t tournament_size;    /* k: 1..8 (Sec. 2 uses 5) */
  uint32_t selection;          /* 1 tournament, 0 neutral (uniform parent) */
  uint32_t mutation_threshold; /* p * 2^32: mutate iff a 32-bit draw < this */
  uint32_t migration;          /* 1 one emigrant per island per generation, 0 none */
  uint32_t seed;               /* RNG key word 0 */
  uint32_t run_id;             /* RNG key word 1 */
  /* Fields below were added after the first release; a caller passing
   * struct_size = offsetof(ga_config, mutation_law) gets law 0. */
  uint32_t mutation_law;       /* 0: with probability p the delta above;
                                * 1: the paper's treatments (Sec. 3): with
                                * probability b fitness gains |Z|, else with
                                * probability p it loses |Z|; Z ~ N(0,1)
                                * approximated by the variance-matched sum of
                                * eight uniform 16-bit draws (stream 3) */
  uint32_t beneficial_threshold; /* b * 2^32 (law 1); b + p <= 1 */
  /* Added later still; struct_size = offsetof(ga_config, schedule) gets the
   * synchronous schedule. */
  uint32_t schedule;           /* GA_SCHEDULE_SYNC or GA_SCHEDULE_ASYNC */
  /* Added later; struct_size = offsetof(ga_config, genome_model) gets model 0. */
  uint32_t genome_model;       /* GA_MODEL_* below */
  /* Added later; struct_size = offsetof(ga_config, differentia_bits) gets 1. */
  uint32_t differentia_bits;   /* b: bits per differentia, 1, 2, 4 or 8, with
                                * S * b = 32 or 64 (the surface keeps its 32- or
                                * 64-bit footprint; wider differentia make a
                                * spurious match at a common rank a 2^-b event
                                * but leave fewer sites). A deposit writes the top
                                * b bits of word 0 of the Philox block with
                                * counter (slot + 256, island, t low word,
                                * t high word * 4 + 3); b = 1 writes the top bit
                                * of the selection block's word 3 as always. */
  /* Added last; struct_size = offsetof(ga_config, surface_policy) gets steady. */
  uint32_t surface_policy;     /* GA_POLICY_STEADY, GA_POLICY_TILTED or GA_POLICY_HYBRID */
} ga_config;

/* Surface policies (ga_config.surface_policy): which site a deposit of rank r
 * overwrites.
 * GA_POLICY_STEADY ("doubling steady"): after n deposits the multiples of
 * 2^e(n) below n are kept, e(n) = max(0, ceil(log2 n) - log2 S); evenly spaced
 * over the whole history.
 * GA_POLICY_TILTED (recency-proportional; S = 32 or 64, m = S / 32): rank r
 * with k trailing zero bits (k capped at 31; rank 0 counts as 31) overwrites
 * slot (r >> (k+1)) mod m ((r >> 31) mod m for k = 31) of level k, site
 * k * m + slot. Each level keeps its m most recent ranks, so about m ranks per
 * doubling of age survive: recent ancestry is resolved finely, old ancestry
 * coarsely. Every deposit is written.
 * GA_POLICY_HYBRID (64 one-bit sites): even ranks 2q go to a 32-site steady
 * half (sites 0..31) as its rank q, odd ranks 2q + 1 to a 32-site tilted half
 * (sites 32..63) as its rank q: even coverage of the whole history beside fine
 * recent resolution. */
#define GA_POLICY_STEADY 0
#define GA_POLICY_TILTED 1
#define GA_POLICY_HYBRID 2

/* Genome models (ga_config.genome_model). The paper's kernel serves any
 * fixed-length genome through three functions, initialize, mutate and
 * evaluate (Sec. 2 Methods); here a model is a type with those three device
 * functions (one header each, listed with its id in the library's model
 * registry) compiled into every generation kernel as a template argument.
 * Ids not in the registry are GA_EINVAL.
 *
 * GA_MODEL_FITNESS: the genome is its fitness value (the paper's runs):
 * founders +0, mutation as mutation_law says.
 * GA_MODEL_ONEMAX, GA_MODEL_TRAP4: a 64-bit string carried with the genome
 * (bit b is bit b % 32 of word b / 32). Founders take words 0 and 1 of the
 * sampling stream's block for (slot, island) at generation 2^64 - 1; with
 * probability p (mutation_threshold; mutation_law must be 0) a child's string
 * has bit (draw mod 64) flipped, the draw being the one the fitness delta would
 * use; the fitness is then re-evaluated: OneMax counts the one bits; Trap-4
 * (Deb and Goldberg's deceptive trap of order 4) splits the string into 16
 * four-bit blocks and scores a block with u one bits 4 if u = 4, else 3 - u.
 * Strings travel with migrants. ga_read_strings / ga_write_strings move them;
 * the outbox arguments of ga_read_population and ga_write_population must be
 * NULL for such a run, and it cannot join a batch. */
#define GA_MODEL_FITNESS 0
#define GA_MODEL_ONEMAX 1
#define GA_MODEL_TRAP4 2

/* Schedules (ga_config.schedule).
 *
 * GA_SCHEDULE_SYNC: the deterministic schedule described at the top of this
 * file; results do not depend on the launch shape.
 *
 * GA_SCHEDULE_ASYNC: the paper's asynchronous exchange (Sec. 2 Methods): each
 * island keeps emigration buffers per cardinal neighbour (two, by parity of
 * the sending generation); at the start of each generation it takes from each
 * side the newest genome sent before this generation that it has not taken
 * yet (a genome is in flight during the generation it was sent in), and after
 * updating it writes its emigrant into the buffer toward the drawn direction.
 * There is no barrier across the grid: wavefronts of one persistent launch
 * each own a range of islands and run the generations, an island waiting only
 * while a neighbour is more than a set number of generations behind (see
 * ga_set_async). Every random draw is the same as in the synchronous schedule;
 * only the moment a genome is read differs. With the default pacing, or
 * migration off, the results equal the synchronous schedule's unless a wait
 * gave up; looser pacing lets genomes arrive late or be overwritten unread,
 * and the results then depend on timing, except in the reproducible skewed
 * interleaving of ga_set_async. An asynchronous run has no synchronous outbox:
 * the outbox arguments of ga_read_population and ga_write_population must be
 * NULL, ga_write_population empties the buffers, and it cannot join a batch. */
#define GA_SCHEDULE_SYNC 0
#define GA_SCHEDULE_ASYNC 1

/* Outbox entry as exchanged with the host (ga_read/ga_write_population):
 * the genome an island emitted in the last generation and its direction. */
typedef struct ga_outbox_entry {
  uint32_t valid;              /* 1 if the island emitted, else 0 */
  uint32_t dir;                /* 0 N, 1 E, 2 S, 3 W */
  float fitness;
  uint32_t T;
  uint32_t surface[2];         /* word 1 unused when S = 32 */
} ga_outbox_entry;

typedef struct ga_run ga_run;

/* Device bytes a run needs (population planes, double-buffered outboxes or,
 * for the asynchronous schedule, per island eight buffers (direction x parity),
 * four last-taken stamps, a progress word and eight lockstep headers; the
 * generation counter and extraction staging). 0 for an invalid configuration. */
size_t ga_state_bytes(const ga_config* cfg);

/* Create a run in caller-owned device memory dev_mem (>= ga_state_bytes(cfg),
 * 256-byte aligned) on hip_stream (a hipStream_t; NULL = default stream).
 * Founders: fitness +0, T = 0, blank surfaces, no emission pending,
 * generation 0 (the paper leaves initialisation to the genome model, Sec. 2).
 * Initialisation is enqueued on the stream. *out receives the handle. */
int ga_init(const ga_config* cfg, void* dev_mem, size_t bytes, void* hip_stream,
            ga_run** out);

/* Enqueue n_gens generations on the run's stream (asynchronous; Sec. 2
 * generation cycle with a generation-count halt). n_gens = 0 is a no-op. */
int ga_step(ga_run* run, uint64_t n_gens);

/* Copy the population at the start of the current generation to the host,
 * after waiting for the run's stream. fitness[agents], T[agents] and
 * surface_words[agents * S*b/32] (agent-major) may each be NULL; outbox, if not
 * NULL, receives one ga_outbox_entry per island (the emissions the next
 * generation will absorb); generation, if not NULL, receives t.
 * GA_EDEVICE if a resident-form tile ever stopped waiting for a neighbouring
 * tile (its workgroups were not all resident at once): the state is then not
 * the synchronous schedule's (the same check guards ga_extract_surfaces). */
int ga_read_population(ga_run* run, float* fitness, uint32_t* T,
                       uint32_t* surface_words, ga_outbox_entry* outbox,
                       uint64_t* generation);

/* Overwrite the state (checkpoint resume). Same layouts as
 * ga_read_population; NULL leaves that part unchanged. Synchronous. */
int ga_write_population(ga_run* run, const float* fitness, const uint32_t* T,
                        const uint32_t* surface_words,
                        const ga_outbox_entry* outbox, uint64_t generation);

/* Genome models with a string: copy every agent's 64-bit string to the host
 * (words[agents * 2], agent-major), after waiting for the run's stream, or
 * overwrite them from the host (synchronous; the caller keeps fitness
 * consistent with ga_write_population). GA_EINVAL for GA_MODEL_FITNESS. */
int ga_read_strings(ga_run* run, uint32_t* words);
int ga_write_strings(ga_run* run, const uint32_t* words);

/* Sample end-state genomes for post hoc reconstruction (Sec. 3: one genome
 * sampled per island). agent_ids == NULL picks one agent per island from the
 * sampling stream at the current generation (n must equal the island count);
 * otherwise the n listed agents are gathered. Writes ids_out[n] (may be NULL),
 * T_out[n] and surface_words_out[n * S*b/32]. Synchronous. */
int ga_extract_surfaces(ga_run* run, const uint64_t* agent_ids, size_t n,
                        uint64_t* ids_out, uint32_t* T_out,
                        uint32_t* surface_words_out);

/* Generation counter as enqueued so far (host mirror; no synchronisation). */
uint64_t ga_generation(const ga_run* run);

/* Release the handle (waits for the run's stream). Device memory stays with
 * the caller. NULL is allowed. */
void ga_destroy(ga_run* run);

/* Launch forms for ga_step (synchronous runs).
 * GA_FORM_STREAMING: one kernel per generation over all islands, the
 * population read from and written back to HBM every generation.
 * GA_FORM_RESIDENT: the population held in LDS across generations, as each
 * processing element of the paper's design holds its island in local memory
 * (Sec. 2 Methods). The torus is cut into tiles of tile_w x tile_h islands
 * (the last column and row of tiles ragged); one workgroup per tile runs every
 * generation of a launch, all tiles' workgroups resident at once. Between
 * generations tiles exchange only their edge islands' emissions through the
 * HBM outbox, each tile waiting (a bounded number of times) until its four
 * neighbouring tiles have published generation t - 1. HBM carries the
 * population only at the start and end of a launch (at most 2^16 generations
 * or about 2^34 agent-generations each). Needs a tiling whose tiles fit the
 * LDS of a CU (160 KiB: per agent 4 bytes each of fitness, T, the surface
 * words and any string words; per island two outbox entries) with every
 * workgroup resident at once. The launch needs the GPU's CUs to itself: kernels
 * running at the same time (another stream's, another process's) hold CUs,
 * tiles then wait for neighbours that are not scheduled until their bounded
 * waits give up, and reading the state reports GA_EDEVICE. Runs stepped on one
 * stream are safe; choose GA_FORM_STREAMING for runs stepped on streams that
 * run concurrently or on a GPU shared with other work.
 * GA_FORM_AUTO (default): the resident form when such a tiling exists, else
 * streaming. Results do not depend on the form. */
#define GA_FORM_AUTO 0
#define GA_FORM_STREAMING 1
#define GA_FORM_RESIDENT 2

/* Launch tuning for one run: islands per wavefront (a multiple of 64/N, at
 * most 64; default 16, or fewer for small grids) and wavefronts per workgroup
 * (1..16; default 4) of the streaming form, and the launch form. 0 keeps the
 * current value of the first two. Results do not depend on any of these.
 * GA_EINVAL if a streaming workgroup's LDS table (5 * islands_per_wave + 1
 * entries of 16 bytes, 32 with a genome string, per wavefront) would exceed
 * the 160 KiB of a CU, or if the resident form is asked for a run with no
 * tiling that fits (or for an asynchronous run). */
int ga_set_launch(ga_run* run, uint32_t islands_per_wave, uint32_t waves_per_group,
                  uint32_t form);

/* Tile shape of the resident form: tile_w x tile_h islands (clamped to the
 * torus), or 0, 0 to let the library choose (the default: the smallest tiles,
 * but not under 2,048 agents, whose workgroups all fit the GPU at once; then
 * the fewest and squarest). GA_EINVAL for an asynchronous run, for one side
 * given without the other, or if the tiles do not fit (LDS of a CU, or more
 * workgroups than the GPU holds at once); the run then keeps its tiling.
 * Results do not depend on the tile shape. */
int ga_set_tiles(ga_run* run, uint32_t tile_w, uint32_t tile_h);

/* The tiling ga_step uses for this run: tile sides and tile count, all 0 when
 * it runs the streaming form (or is asynchronous or a batch member). */
int ga_get_tiles(ga_run* run, uint32_t* tile_w, uint32_t* tile_h, uint32_t* tiles);
/* Asynchronous runs only (GA_EINVAL for a synchronous run).
 *
 * max_wavefronts caps the wavefronts of a launch (0, the default: as many as
 * the GPU holds at once, from the occupancy of the kernel).
 *
 * max_lead bounds how many generations an island may run ahead of a
 * neighbour: before generation t an island waits until each neighbour has
 * completed t - max_lead generations, checking a bounded number of times and
 * then going on regardless (ga_async_waits counts those). Default 0: each
 * island waits for its neighbours to finish the previous generation, which
 * makes the results equal to the synchronous schedule's whenever no wait gave
 * up, with no barrier across the grid. GA_ASYNC_UNPACED: no waiting at all.
 * With max_lead 0 and no skew the launch uses the lockstep exchange: each
 * island publishes, every generation, one header per side saying whether it
 * sent a genome that way, and a neighbour's header doubles as its progress, so
 * one wait and one read replace the stamped reads; its first generation
 * applies the general rule above, so it takes what any other launch would. A
 * wait that gives up in lockstep drops the genome toward the late neighbour
 * (its buffer may still be in use) rather than overwrite it.
 *
 * skew > 0 (needs max_wavefronts 1 and GA_ASYNC_UNPACED): the reproducible
 * interleaving in which chunk c (islands c*ipw ...) runs its generation g of a
 * ga_step call at step g + (c mod (skew + 1)), the chunks in order within a
 * step; neighbours are then up to skew generations apart, so genomes arrive
 * late or are overwritten unread. skew <= 1024. */
#define GA_ASYNC_UNPACED 0xFFFFFFFFu
int ga_set_async(ga_run* run, uint32_t max_wavefronts, uint32_t max_lead, uint32_t skew);
/* Asynchronous runs: how many times so far an island stopped waiting for a
 * neighbour and went on (0 means every pacing wait was met). Synchronous. */
int ga_async_waits(ga_run* run, uint64_t* gave_up);
/* Asynchronous runs: genomes the islands have absorbed from their neighbours'
 * buffers since the run was created (Sec. 2 Methods: an island takes what
 * has arrived and goes on). With migration on, every island sends one genome
 * per generation and generation 0 has nothing to take, so after g
 * generations 1 - taken / (islands * (g - 1)) is the share of genomes
 * overwritten before they were read (0 in lockstep).
 * GA_EINVAL for a synchronous run (which absorbs every genome sent).
 * Synchronous. */
int ga_async_taken(ga_run* run, uint64_t* taken);
/* Asynchronous runs: for island i and direction q, sent[i*4 + q] receives the
 * generation in which the last genome island i took from that side was sent
 * (t - 1 where t is the generation of the run or of the last
 * ga_write_population if it took none since; -1 at the start). The gap to
 * the current generation shows how fresh the exchange is. Synchronous. */
int ga_async_last_taken(ga_run* run, int64_t* sent);

/* Generations per captured HIP graph replay (0 disables graphs). */
int ga_set_graph_block(ga_run* run, uint32_t gens_per_block);

/* ---------------------------------------------------------------------- */
/* Batched form: many independent runs of uneven shape advanced together  */
/* (Sec. 3 runs replicates and treatments as independent runs): one       */
/* kernel launch per generation over every member's islands, each         */
/* wavefront running the body compiled for its member's class (island     */
/* size, surface words), blocks of generations replayed from a HIP graph. */
/* Members and their budgets live in device tables that the graph reads,  */
/* so members come and go without a new graph or a wait for the stream    */
/* (a new graph only when the tiles outgrow the launch's headroom or the  */
/* launch shape changes). Each member gives the bits it would give alone. */
/* ---------------------------------------------------------------------- */
typedef struct ga_batch ga_batch;

/* Create an empty batch bound to hip_stream. The batch allocates its own
 * small descriptor tables in device memory (and pinned host staging for
 * them), growing them, with a wait for the stream, when the members outgrow
 * them. */
int ga_batch_create(void* hip_stream, ga_batch** out);
/* Add a run (created by ga_init, bound to any stream; from now on it is
 * advanced only through the batch) with a generation budget: the batch stops
 * advancing it after budget more generations. Enqueued: the run's earlier
 * work on its own stream comes first. Returns GA_OK; GA_EINVAL for an
 * asynchronous run, a genome model with a string, differentia_bits > 1 or a
 * surface policy other than steady; GA_ESTATE if the run is already in a batch. */
int ga_batch_add(ga_batch* batch, ga_run* run, uint64_t budget);
/* Remove a member. Enqueued, no wait: work later enqueued on the run's own
 * stream follows the batch's work so far; ga_generation is exact at once
 * (the batch keeps the host mirror). */
int ga_batch_remove(ga_batch* batch, ga_run* run);
/* Enqueue up to n_gens generations for every member with budget left. At
 * most two step calls stay in flight: a call returns once the call two before
 * it has run on the GPU (the one just enqueued keeps the GPU busy meanwhile). */
int ga_batch_step(ga_batch* batch, uint64_t n_gens);
/* Generations still owed to a member (host mirror). */
uint64_t ga_batch_remaining(const ga_batch* batch, const ga_run* run);
/* Whether a member's last generation has run on the GPU (*settled 1), not
 * only been enqueued (0; also 0 while it has budget left). Waits for nothing.
 * GA_EINVAL for a run that is not a member. */
int ga_batch_settled(ga_batch* batch, const ga_run* run, int* settled);
/* Members; waits for nothing. */
size_t ga_batch_size(const ga_batch* batch);
/* Generations per graph replay for the batch (default 100; 0 disables). */
int ga_batch_set_graph_block(ga_batch* batch, uint32_t gens_per_block);
/* Launch shape for the whole batch: islands per wavefront for every member
 * (0 = the default, 512/N for each member: about 512 agents per wavefront;
 * rounded down to a multiple of 64/N, at most 64) and
 * wavefronts per workgroup (1..16; 0 keeps the current value, default 4).
 * Results do not depend on either. */
int ga_batch_set_launch(ga_batch* batch, uint32_t islands_per_wave, uint32_t waves_per_group);
/* Islands per wavefront of one class of members (log2 N in 0..6, surface
 * words 1 or 2), overriding ga_batch_set_launch for it: 0 = the batch's
 * rule, else a multiple of 64/N in [64/N, 64]. Results do not depend on it. */
int ga_batch_set_class_launch(ga_batch* batch, uint32_t log2n, uint32_t words,
                              uint32_t islands_per_wave);
/* The islands per wavefront a class uses and how many wavefront tiles its
 * current members make (either output may be NULL). */
int ga_batch_class_launch(ga_batch* batch, uint32_t log2n, uint32_t words,
                          uint32_t* islands_per_wave, uint32_t* tiles);
void ga_batch_destroy(ga_batch* batch);

/* ---------------------------------------------------------------------- */
/* Run pool: the served form's runtime. Runs are created inside one       */
/* caller-owned device buffer (first fit, 256-byte aligned; a released     */
/* run's block merges with free neighbours) and advanced together as one   */
/* batch; each run gives the bits it would give alone. Arrival order and   */
/* admission policy stay with the caller.                                  */
/* ---------------------------------------------------------------------- */
typedef struct ga_pool ga_pool;

/* Create a pool over dev_mem[0, bytes) (device memory owned by the caller,
 * 256-byte aligned, never freed by the library) holding at most max_slots
 * runs, bound to hip_stream. */
int ga_pool_create(void* dev_mem, size_t bytes, uint32_t max_slots, void* hip_stream,
                   ga_pool** out);
/* Create a run from cfg in the pool with a budget of n_gens generations and
 * give it a ticket (> 0). GA_ENOMEM if every slot is taken or no free block
 * holds ga_state_bytes(cfg) now (retiring runs makes room); GA_EINVAL for an
 * invalid configuration, one larger than the whole pool, or one a batch does
 * not take (see ga_batch_add). Founders as ga_init; enqueued on the stream. */
int ga_pool_admit(ga_pool* pool, const ga_config* cfg, uint64_t n_gens, uint64_t* ticket);
/* Enqueue up to n_gens generations for every run with budget left. */
int ga_pool_step(ga_pool* pool, uint64_t n_gens);
/* Generations per graph replay (as ga_batch_set_graph_block). */
int ga_pool_set_graph_block(ga_pool* pool, uint32_t gens_per_block);
/* Launch shape of the pool's batch, as ga_batch_set_launch and
 * ga_batch_set_class_launch (for the classes its runs may fall in; results do
 * not depend on it). */
int ga_pool_set_launch(ga_pool* pool, uint32_t islands_per_wave, uint32_t waves_per_group);
int ga_pool_set_class_launch(ga_pool* pool, uint32_t log2n, uint32_t words,
                             uint32_t islands_per_wave);
/* Generations still owed to a run (host mirror). GA_EINVAL for an unknown ticket. */
int ga_pool_remaining(const ga_pool* pool, uint64_t ticket, uint64_t* left);
/* Tickets of the runs whose budget is spent: up to cap of them in tickets
 * (may be NULL), in ticket order; *n_done receives how many there are. */
int ga_pool_poll(const ga_pool* pool, uint64_t* tickets, size_t cap, size_t* n_done);
/* ga_pool_poll restricted, if settled_only, to runs whose last generation has
 * already run on the GPU (ga_batch_settled): retiring those waits for no
 * block still running. */
int ga_pool_poll_settled(const ga_pool* pool, uint64_t* tickets, size_t cap, size_t* n_done,
                         int settled_only);
/* Remove a run (finished or not) and release its memory. Unless all three
 * outputs are NULL, first sample its end population as ga_extract_surfaces
 * does with agent_ids NULL: one agent per island from the sampling stream,
 * ids_out[islands], T_out[islands], surface_words_out[islands * S*b/32]
 * (Sec. 3: one genome sampled per island). The sample is taken on a stream of
 * the pool's own after the work enqueued so far, and the call waits for that
 * stream only, so blocks already enqueued keep running; later work on the
 * pool's stream (a run admitted into the freed memory) follows the sampling.
 * A failure leaves the run in the pool. */
int ga_pool_retire(ga_pool* pool, uint64_t ticket, uint64_t* ids_out, uint32_t* T_out,
                   uint32_t* surface_words_out);
/* Bytes held by runs, the largest free block, and the number of runs; any
 * pointer may be NULL. */
int ga_pool_usage(const ga_pool* pool, size_t* used, size_t* largest_free, uint32_t* live);
/* Release every run and the pool (waits for the stream). NULL is allowed. */
void ga_pool_destroy(ga_pool* pool);

/* ---------------------------------------------------------------------- */
/* Post hoc relatedness (Fig. 1: markers on genomes support estimating how */
/* related two lineages are after the run; Sec. 3 reconstructs phylogenies */
/* from 10k sampled end-state genomes).                                    */
/* ---------------------------------------------------------------------- */

/* Device bytes of the workspace ga_mrca_matrix needs for n surfaces. */
size_t ga_mrca_workspace_bytes(size_t n);

/* MRCA intervals for every pair of n sampled surfaces, on the GPU. All
 * pointers are DEVICE pointers owned by the caller: T[n] deposit counters,
 * surface_words[n * S/32] (agent-major, as ga_extract_surfaces returns them),
 * workspace of at least ga_mrca_workspace_bytes(n) bytes, and outputs
 * L[n * n], U[n * n] (row x, column y). For the pair (x, y), the counter g of
 * the most recent common ancestor satisfies g <= U[x*n+y] always, and
 * g < L[x*n+y] with probability at most 2^-kc: the ranks both surfaces
 * retain are compared oldest first, U is the first whose bits differ (or
 * min(Tx, Ty)), and L sits kc common ranks below U (0 if there are fewer).
 * n <= 65535, kc >= 1, surface_sites 32 or 64. Enqueued on hip_stream. */
int ga_mrca_matrix(const uint32_t* T, const uint32_t* surface_words, size_t n,
                   uint32_t surface_sites, uint32_t kc, void* workspace,
                   size_t workspace_bytes, uint32_t* L, uint32_t* U, void* hip_stream);
/* The same for surfaces of b = differentia_bits bits per site (S * b = 32 or
 * 64; surface_words holds S * b / 32 words per surface) under either surface
 * policy. The ranks both surfaces still hold, c_0 < c_1 < ..., are compared
 * oldest first as b-bit fields: U is the first that differs (or min(Tx, Ty)),
 * L = c_{j-kc} + 1 for its index j (0 if j < kc), so g < L has probability at
 * most 2^-(b kc). The tilted and hybrid policies need no workspace (NULL is
 * accepted). */
int ga_mrca_matrix_ex(const uint32_t* T, const uint32_t* surface_words, size_t n,
                      uint32_t surface_sites, uint32_t differentia_bits, uint32_t surface_policy,
                      uint32_t kc, void* workspace, size_t workspace_bytes, uint32_t* L,
                      uint32_t* U, void* hip_stream);

/* ga_mrca_matrix_ex without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the steady policy's normalised surfaces
 * go to a static device array inside the library (65,536 entries of 16 bytes:
 * 1 MiB per GPU the library runs on, held until the process ends). Nothing is allocated and nothing needs clearing: every entry
 * the call reads it has written first. All calls on one GPU share that array,
 * so calls that overlap on one GPU (on different streams or host threads)
 * race and must be serialised by the caller. The current device must be the
 * one the pointers and the stream belong to. n <= 65,535 as for
 * ga_mrca_matrix_ex (GA_EINVAL above, and for every argument that call
 * rejects). Same results as ga_mrca_matrix_ex. */
int ga_mrca_matrix_noalloc(const uint32_t* T, const uint32_t* surface_words, size_t n,
                           uint32_t surface_sites, uint32_t differentia_bits,
                           uint32_t surface_policy, uint32_t kc, uint32_t* L, uint32_t* U,
                           void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Roof microbenchmarks: the limits the generation step is measured       */
/* against (measurement only; all enqueued on hip_stream, device buffers  */
/* owned by the caller).                                                  */
/* ---------------------------------------------------------------------- */

/* HBM roof of the streaming form: n_planes (1..8) planes of words_per_plane
 * u32 each (a multiple of 4; 16-byte aligned, consecutive) are read and
 * written back incremented, 16 bytes per access: 8 * n_planes * words bytes
 * moved, the traffic of a generation that updates the population planes in
 * place. */
int ga_roof_inplace(void* planes, size_t words_per_plane, uint32_t n_planes, void* hip_stream);
/* RNG roof: `threads` threads (a multiple of 256) each draw blocks_per_thread
 * full Philox4x32-10 blocks (the block every child of a generation draws,
 * Sec. 2's selection and mutation randomness) and write one folded word to
 * out[thread]. */
int ga_roof_philox(uint32_t* out, uint32_t threads, uint32_t blocks_per_thread, void* hip_stream);
/* Issue rate of one instruction kind: `threads` threads (a multiple of 256)
 * run eight coupled chains of `iters` steps: kind 0 one three-input XOR per
 * step, kind 1 one 32x32->64 multiply-add plus one XOR per step. One word per
 * thread to out[thread]. */
int ga_roof_valu(uint32_t* out, uint32_t threads, uint32_t iters, uint32_t kind, void* hip_stream);

/* Message for a return code, and the calling thread's last error message. */
const char* ga_strerror(int code);
const char* ga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GA_H */
