/*
 * CPU oracle for the tracking-enabled island-model GA generation step.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, single-threaded reference
 * that the GPU library is checked against. Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or helper with the GPU library; the two meet only in the seeded run
 * configuration they are both given.
 *
 * The method (paper: Moreno, Yang, Dolson, Zaman, "Trackable Island-model
 * Genetic Algorithms at Wafer Scale", GECCO '24 Companion):
 *   - islands on a 2D lattice each host an independent, fixed-size population
 *     and exchange genomes with their cardinal neighbours (Sec. 2 Methods);
 *   - each generation handles migration first, then evaluation, tournament
 *     selection with random tie-breaks, mutation of the whole next population,
 *     and one hereditary-stratigraphy update, until a generation count is met
 *     (Sec. 2 Methods);
 *   - the genome carries a float fitness first, the rest is tracking
 *     annotation (Sec. 3 Results and Discussion).
 * Where the paper is silent (schedule, RNG, surface policy, mutation law) the
 * readings below are the project's conventions; the GPU library follows the
 * same readings, written separately.
 */
#ifndef GA_ORACLE_H
#define GA_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_DISCARD 0xFFFFFFFFu

typedef struct orc_config {
  uint32_t width;       /* islands per row (x extent) */
  uint32_t height;      /* rows (y extent); island id = y*width + x */
  uint32_t pop;         /* agents per island, power of two, 1..256 */
  uint32_t sites;       /* surface sites S, a power of two in 4..64 */
  uint32_t k;           /* tournament size, 1..8 */
  uint32_t selection;   /* 1 tournament, 0 neutral (uniform parent) */
  uint32_t p32;         /* mutate iff a 32-bit draw is below this */
  uint32_t migration;   /* 1 one emigrant per island per generation, 0 off */
  uint32_t seed;        /* RNG key word 0 */
  uint32_t run_id;      /* RNG key word 1 */
  uint32_t law;         /* 0 discrete delta with probability p32;
                           1 treatments: beneficial (+|Z|) if draw < p_ben32,
                           else deleterious (-|Z|) if draw < p_ben32 + p32 */
  uint32_t p_ben32;     /* beneficial probability times 2^32 (law 1) */
  uint32_t model;       /* genome model: 0 the genome is its fitness (law 0 or 1);
                           1 OneMax, 2 Trap-4, both on a 64-bit string (law 0's
                           probability p flips one bit) */
  uint32_t dbits;       /* bits per differentia: 1, 2, 4 or 8; sites * dbits is 32
                           or 64 (the surface fills one or two words) */
  uint32_t policy;      /* surface policy: 0 "doubling steady", 1 "tilted"
                           (recency-proportional; sites 32 or 64), 2 "hybrid"
                           (64 one-bit sites: steady and tilted halves) */
} orc_config;

typedef struct orc_run orc_run;

/* Philox4x32 with 10 rounds (Salmon et al., SC'11): one 128-bit block. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Surface policy: site written by the deposit of stratum rank r, or ORC_DISCARD. */
uint32_t orc_site_of(uint64_t rank, uint32_t sites);
/* Epoch after n deposits: max(0, ceil(log2 n) - log2 S). */
uint32_t orc_epoch(uint64_t n, uint32_t sites);
/* Tilted policy (S = 32 m sites, 32 levels of m slots): rank r with k
 * trailing zeros (capped at 31; rank 0 counts as 31) takes slot
 * (r >> (k+1)) mod m of level k ((r >> 31) mod m on level 31), site k m + slot.
 * Every deposit is written. */
uint32_t orc_site_of_tilted(uint64_t rank, uint32_t sites);
/* Hybrid policy (64 sites): even rank 2q at steady site orc_site_of(q, 32)
 * (or nowhere), odd rank 2q + 1 at 32 + orc_site_of_tilted(q, 32). */
uint32_t orc_site_of_hybrid(uint64_t rank);
/* Site of a deposit under policy 0 (steady), 1 (tilted) or 2 (hybrid). */
uint32_t orc_site_of_policy(uint64_t rank, uint32_t sites, uint32_t policy);
/* Ranks a surface holds after n deposits, ascending (at most S); returns the
 * count. */
size_t orc_retained(uint64_t n, uint32_t sites, uint32_t policy, uint64_t* out);
/* MRCA interval for any policy from the common retained ranks c_0 < c_1 < ...:
 * U = the first with differing differentia (or min T), L = c_{j-kc} + 1 (0 if
 * j < kc); P(g < L) <= 2^-(dbits kc). */
void orc_mrca_interval_policy(uint32_t Ta, const uint32_t* Da, uint32_t Tb, const uint32_t* Db,
                              uint32_t sites, uint32_t dbits, uint32_t policy, uint32_t kc,
                              uint32_t* L, uint32_t* U);
void orc_mrca_interval_matrix_policy(const uint32_t* T, const uint32_t* D, size_t n,
                                     uint32_t sites, uint32_t dbits, uint32_t policy, uint32_t kc,
                                     uint32_t* L, uint32_t* U);
/* Bulk form for tests: out[i] = orc_site_of(first + i, sites). */
void orc_site_of_range(uint64_t first, size_t count, uint32_t sites, uint32_t* out);

/* 0 on success, -1 for an invalid configuration. */
int orc_validate(const orc_config* cfg);
/* record_lineage != 0 keeps every child's tournament winner (1 byte each). */
orc_run* orc_create(const orc_config* cfg, int record_lineage);
void orc_free(orc_run* run);
/* Reserve lineage storage for gens generations in one allocation. */
int orc_reserve_lineage(orc_run* run, uint64_t gens);
/* Advance n generations. Returns 0, or -1 when the lineage buffer cannot grow. */
int orc_step(orc_run* run, uint64_t n);
uint64_t orc_generation(const orc_run* run);
/* Asynchronous schedule in a reproducible interleaving: n generations in
 * which islands go in consecutive groups of `group`; group c runs its
 * generation t at step t + (c mod (skew + 1)), groups in order within a step,
 * each reading its arrivals, updating, then publishing. Per neighbour and per
 * parity of the sending generation a buffer holds the latest genome sent; in
 * generation t a receiver takes, from each side, the newest buffer sent before
 * t and not taken yet. skew 0 gives the synchronous schedule's results.
 * Buffers start empty and are separate from the synchronous outbox. Returns
 * -1 with lineage on, group == 0, or no memory. */
int orc_step_async(orc_run* run, uint64_t n, uint64_t group, uint32_t skew);
/* Empty every asynchronous buffer and forget what was taken from them. */
void orc_clear_mailboxes(orc_run* run);
/* Asynchronous buffers, entry b = (i*4 + d)*2 + p (island i's buffer toward
 * d for sending generations of parity p): stamp[b] (sending generation + 1,
 * 0 if empty) and the genome; seen[i*4 + q] is the stamp of the last arrival
 * island i took from its neighbour in direction q. Any pointer may be NULL. */
void orc_get_mailboxes(const orc_run* run, uint64_t* stamp, uint64_t* seen, float* f,
                       uint32_t* T, uint32_t* D);

uint64_t orc_agents(const orc_run* run);

/* Genome payload of models 1 and 2, two words per agent (agent-major); zero
 * for model 0. */
void orc_get_payload(const orc_run* run, uint32_t* P);
void orc_set_payload(orc_run* run, const uint32_t* P);
/* Fitness a model gives a 64-bit string (words p0, p1); 0 for model 0. */
float orc_evaluate(uint32_t model, uint32_t p0, uint32_t p1);

/* Population at the start of the current generation. D is agent-major:
 * D[a*W + w] with W = sites/32 words per agent. Any pointer may be NULL. */
void orc_get_population(const orc_run* run, float* f, uint32_t* T, uint32_t* D);
void orc_set_population(orc_run* run, const float* f, const uint32_t* T, const uint32_t* D);
/* The outbox the next generation will absorb from (one entry per island). */
void orc_get_outbox(const orc_run* run, uint8_t* valid, uint8_t* dir, float* f,
                    uint32_t* T, uint32_t* D);
void orc_set_outbox(orc_run* run, const uint8_t* valid, const uint8_t* dir,
                    const float* f, const uint32_t* T, const uint32_t* D);
/* Jump the generation counter (state is kept as is; lineage must be off). */
int orc_set_generation(orc_run* run, uint64_t t);

/* One agent per island, drawn from the SAMPLE stream at the current
 * generation: ids[i] = i*pop + slot. */
void orc_sample_one_per_island(const orc_run* run, uint64_t* ids);

/* True lineage (needs record_lineage from generation 0). For two agents of
 * the current population, the generation counter T of their most recent
 * common ancestor, or -1 when they descend from different founders. */
int64_t orc_true_mrca(const orc_run* run, uint64_t agent_a, uint64_t agent_b);
/* Lineage walk: writes up to max_len (generation, island, slot) triples of
 * the ancestors of one agent, newest first; returns the chain length. */
size_t orc_ancestry(const orc_run* run, uint64_t agent, uint64_t* gen,
                    uint32_t* island, uint32_t* slot, size_t max_len);

/* Pairwise true MRCA for n agents of the current population:
 * out[x*n + y] = T of the MRCA of ids[x] and ids[y], or -1 for different
 * founders. Each agent's ancestor chain is walked once; pairs merge chains.
 * Returns 0, or -1 if lineage was not recorded or memory ran out. */
int orc_true_mrca_matrix(const orc_run* run, const uint64_t* ids, size_t n, int32_t* out);

/* MRCA intervals for all pairs of n surfaces (T[n], D[n * S/32]):
 * L[x*n + y], U[x*n + y] as orc_mrca_interval gives them. */
void orc_mrca_interval_matrix(const uint32_t* T, const uint32_t* D, size_t n, uint32_t sites,
                              uint32_t kc, uint32_t* L, uint32_t* U);

/* MRCA interval from two surfaces: g (the MRCA's T) is always <= *U, and
 * g < *L has probability at most 2^-kc. */
void orc_mrca_interval(uint32_t Ta, const uint32_t* Da, uint32_t Tb,
                       const uint32_t* Db, uint32_t sites, uint32_t kc,
                       uint32_t* L, uint32_t* U);
/* The same for dbits-bit differentia (sites * dbits = 32 or 64 bits of
 * surface); g < *L then has probability at most 2^-(dbits * kc). */
void orc_mrca_interval_bits(uint32_t Ta, const uint32_t* Da, uint32_t Tb, const uint32_t* Db,
                            uint32_t sites, uint32_t dbits, uint32_t kc, uint32_t* L,
                            uint32_t* U);
void orc_mrca_interval_matrix_bits(const uint32_t* T, const uint32_t* D, size_t n,
                                   uint32_t sites, uint32_t dbits, uint32_t kc, uint32_t* L,
                                   uint32_t* U);

#ifdef __cplusplus
}
#endif
#endif
