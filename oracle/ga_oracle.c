/*
 * CPU oracle for the tracking-enabled island-model GA generation step.
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded, written for reading
 * against the paper, not for speed. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may use it. It shares no code with the GPU
 * library.
 *
 * Paper: Moreno, Yang, Dolson, Zaman, "Trackable Island-model Genetic
 * Algorithms at Wafer Scale" (GECCO '24 Companion).
 *
 * Readings taken where the paper is silent (the GPU library follows the same
 * readings in its own code):
 *   schedule   synchronous; every island finishes generation t before any
 *              starts t+1; an emigrant sent in generation t is absorbed in
 *              generation t+1 (Sec. 2: immigration consumes buffers filled
 *              earlier, emigration refills them afterwards).
 *   migration  one emigrant per island per generation, copied (the sender keeps
 *              it), sent to one random cardinal neighbour; the receiver draws
 *              the slot it overwrites; up to 4 arrivals are applied in
 *              direction order N, E, S, W, the later one winning a slot clash.
 *   selection  k entrants drawn with replacement; the first entrant (in draw
 *              order) with the strictly greatest fitness wins, which breaks
 *              ties uniformly at random as the paper asks (Sec. 2).
 *   mutation   with probability p the fitness gains a delta drawn uniformly
 *              from {-1, -1/2, 0, 1/2, 1}, added in binary32 with
 *              round-to-nearest-even.
 *   tracking   a hereditary-stratigraphy surface of S one-bit differentia plus
 *              a deposit counter T; one deposit per generation (Sec. 2), at
 *              the site chosen by the "doubling steady" policy below.
 *   RNG        Philox4x32-10 keyed by (seed, run_id), counter
 *              (slot or 0, island, generation low word,
 *               generation high word * 4 + stream tag).
 */
#include "ga_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------- */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel Random      */
/* Numbers: As Easy as 1, 2, 3" (SC'11). Each round multiplies counter      */
/* words 0 and 2 by fixed odd constants, keeps both halves of each 64-bit   */
/* product, and mixes the high halves with the other two words and the key; */
/* the key grows by the Weyl increments between rounds.                     */
/* ----------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { TAG_SELECT = 0, TAG_MIGRATE = 1, TAG_SAMPLE = 2, TAG_MUTATE = 3 };

static void draw(const orc_config* cfg, uint32_t slot, uint32_t island, uint64_t t,
                 uint32_t tag, uint32_t out[4]) {
  uint32_t ctr[4];
  uint32_t key[2];
  ctr[0] = slot;
  ctr[1] = island;
  ctr[2] = (uint32_t)t;
  ctr[3] = (uint32_t)(t >> 32) * 4u + tag;
  key[0] = cfg->seed;
  key[1] = cfg->run_id;
  orc_philox(ctr, key, out);
}

/* ----------------------------------------------------------------------- */
/* Surface policy ("doubling steady").                                      */
/* With S sites and n deposits made, the epoch is e(n) = max(0, ceil(log2 n) */
/* - log2 S) and the retained ranks are the multiples of 2^e(n) below n.    */
/* A deposit of rank r is written only if r is a multiple of 2^e(r+1);      */
/* ranks below S get site r; the j-th rank written during epoch e >= 1     */
/* reuses the site of the j-th smallest rank that left the retained set     */
/* when epoch e began, i.e. rank (2j+1) * 2^(e-1).                          */
/* ----------------------------------------------------------------------- */
static uint32_t log2_exact(uint32_t v) {
  uint32_t l = 0;
  while ((1u << l) < v) ++l;
  return l;
}

uint32_t orc_epoch(uint64_t n, uint32_t sites) {
  uint32_t s = log2_exact(sites);
  uint32_t c = 0; /* ceil(log2 n) for n >= 1; 0 for n <= 1 */
  while (c < 64 && ((uint64_t)1 << c) < n) ++c;
  return c > s ? c - s : 0;
}

uint32_t orc_site_of(uint64_t rank, uint32_t sites) {
  uint64_t r = rank;
  int first = 1;
  for (;;) {
    if (r < sites) return (uint32_t)r;
    uint32_t e = orc_epoch(r + 1, sites);
    if (r % ((uint64_t)1 << e) != 0) {
      /* Only the deposit itself can be a discard: every rank reached by the
       * recursion below was written in its own time. */
      if (first) return ORC_DISCARD;
      abort();
    }
    uint64_t m = r >> e;              /* in [S/2, S) */
    uint64_t j = m - sites / 2;       /* j-th rank written in epoch e */
    r = (2 * j + 1) << (e - 1);       /* j-th rank dropped when e began */
    first = 0;
  }
}

/* ----------------------------------------------------------------------- */
/* Surface policy "tilted" (recency-proportional resolution), S = 32 m      */
/* sites as 32 levels of m slots. A rank with k trailing zero bits (k       */
/* capped at 31; rank 0 counts as 31) belongs to level k and overwrites     */
/* slot (r >> (k + 1)) mod m of it (slot (r >> 31) mod m on level 31), so   */
/* each level holds its m most recent ranks. Ranks with k trailing zeros    */
/* come once every 2^(k+1) deposits, so level k's ranks are under about     */
/* m 2^(k+1) deposits old: the retained ranks thin out in proportion to    */
/* their age, and every deposit is written (no discards).                   */
/* ----------------------------------------------------------------------- */
uint32_t orc_site_of_tilted(uint64_t rank, uint32_t sites) {
  const uint32_t m = sites / 32;
  uint32_t k = 0;
  while (k < 31 && ((rank >> k) & 1u) == 0) ++k;
  const uint64_t slot = k < 31 ? (rank >> (k + 1)) % m : (rank >> 31) % m;
  return k * m + (uint32_t)slot;
}

/* ----------------------------------------------------------------------- */
/* Surface policy "hybrid" (64 sites): the ranks alternate between two      */
/* 32-site halves, even ranks 2q into a steady surface (sites 0..31, as its */
/* rank q) and odd ranks 2q + 1 into a tilted one (sites 32..63, as its     */
/* rank q): even coverage of the whole history beside fine recent ranks.    */
/* ----------------------------------------------------------------------- */
uint32_t orc_site_of_hybrid(uint64_t rank) {
  if ((rank & 1u) == 0) return orc_site_of(rank >> 1, 32);
  return 32u + orc_site_of_tilted(rank >> 1, 32);
}

uint32_t orc_site_of_policy(uint64_t rank, uint32_t sites, uint32_t policy) {
  if (policy == 2) return orc_site_of_hybrid(rank);
  return policy == 1 ? orc_site_of_tilted(rank, sites) : orc_site_of(rank, sites);
}

static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Ranks whose differentia a surface holds after n deposits, ascending;
 * returns their count (at most S). Steady: the multiples of 2^e(n) below n.
 * Tilted: per level, its m most recent ranks below n. */
size_t orc_retained(uint64_t n, uint32_t sites, uint32_t policy, uint64_t* out) {
  size_t c = 0;
  if (n == 0) return 0;
  if (policy == 2) {
    /* n deposits: ceil(n/2) even ranks (steady half), floor(n/2) odd ones */
    uint64_t half[64];
    const size_t ne = orc_retained((n + 1) / 2, 32, 0, half);
    for (size_t i = 0; i < ne; ++i) out[c++] = 2 * half[i];
    const size_t no = orc_retained(n / 2, 32, 1, half);
    for (size_t i = 0; i < no; ++i) out[c++] = 2 * half[i] + 1;
    qsort(out, c, sizeof(uint64_t), cmp_u64);
    return c;
  }
  if (policy == 0) {
    const uint64_t step = (uint64_t)1 << orc_epoch(n, sites);
    for (uint64_t r = 0; r < n; r += step) out[c++] = r;
    return c;
  }
  const uint32_t m = sites / 32;
  for (uint32_t k = 0; k < 31; ++k) {
    /* odd multiples 2^k (2j + 1) <= n - 1 */
    const uint64_t q = (n - 1) >> k;
    if (q == 0) continue;
    const uint64_t jmax = (q - 1) / 2;
    for (uint64_t i = 0; i < m && i <= jmax; ++i) out[c++] = ((2 * (jmax - i) + 1) << k);
  }
  const uint64_t imax = (n - 1) >> 31; /* multiples of 2^31 below n */
  for (uint64_t i = 0; i < m && i <= imax; ++i) out[c++] = (imax - i) << 31;
  qsort(out, c, sizeof(uint64_t), cmp_u64);
  return c;
}

void orc_site_of_range(uint64_t first, size_t count, uint32_t sites, uint32_t* out) {
  for (size_t i = 0; i < count; ++i) out[i] = orc_site_of(first + i, sites);
}

/* ----------------------------------------------------------------------- */
/* Run state.                                                               */
/* ----------------------------------------------------------------------- */
typedef struct outbox_entry {
  uint8_t valid;
  uint8_t dir;
  float f;
  uint32_t T;
  uint32_t D[2];
  uint32_t P[2];       /* genome payload (bitstring models) */
} outbox_entry;

/* One emigration buffer of the asynchronous schedule: the latest genome an
 * island sent toward one neighbour in a generation of one parity, stamped with
 * that generation + 1 (0: none). */
typedef struct mail_entry {
  uint64_t stamp;
  float f;
  uint32_t T;
  uint32_t D[2];
  uint32_t P[2];
} mail_entry;

struct orc_run {
  orc_config cfg;
  uint32_t log2pop;
  uint32_t words;      /* surface words per agent */
  uint64_t islands;
  uint64_t agents;
  uint64_t t;
  float* f;            /* population at the start of generation t */
  uint32_t* T;
  uint32_t* D;
  float* nf;           /* next population, built during a generation */
  uint32_t* nT;
  uint32_t* nD;
  uint32_t* P;         /* genome payload, 2 words per agent (zero for model 0) */
  uint32_t* nP;
  outbox_entry* prev;  /* emitted during t-1, absorbed during t */
  outbox_entry* next;  /* emitted during t */
  mail_entry* mail;    /* asynchronous schedule: mail[(i*4 + d)*2 + p], island i's buffer
                          toward d for sending generations of parity p */
  uint64_t* seen;      /* seen[i*4 + q]: stamp of the last arrival island i took from q */
  int lineage;
  uint8_t* winners;    /* winners[g*agents + a]: tournament winner of child a in generation g */
  uint64_t lineage_gens;
  uint64_t lineage_cap;  /* generations the winners buffer can hold */
};

static int is_pow2(uint32_t v) { return v != 0 && (v & (v - 1)) == 0; }
uint32_t orc_site_of_policy(uint64_t rank, uint32_t sites, uint32_t policy);

static int model_known(uint32_t model);

int orc_validate(const orc_config* cfg) {
  if (!cfg) return -1;
  if (cfg->width == 0 || cfg->height == 0) return -1;
  if (!is_pow2(cfg->pop) || cfg->pop > 256) return -1;
  /* S sites of dbits-bit differentia in one or two 32-bit words */
  if (cfg->dbits != 1 && cfg->dbits != 2 && cfg->dbits != 4 && cfg->dbits != 8) return -1;
  if (!is_pow2(cfg->sites) || cfg->sites < 4 || cfg->sites > 64) return -1;
  if (cfg->sites * cfg->dbits != 32 && cfg->sites * cfg->dbits != 64) return -1;
  if (cfg->policy > 2) return -1;
  if (cfg->policy == 1 && cfg->sites != 32 && cfg->sites != 64) return -1;
  if (cfg->policy == 2 && (cfg->sites != 64 || cfg->dbits != 1)) return -1;
  if (cfg->k < 1 || cfg->k > 8) return -1;
  if (cfg->selection > 1 || cfg->migration > 1) return -1;
  if (cfg->law > 1) return -1;
  if (cfg->law == 1 && (uint64_t)cfg->p_ben32 + cfg->p32 > 0xFFFFFFFFull) return -1;
  if (!model_known(cfg->model)) return -1;
  if (cfg->model != 0 && cfg->law != 0) return -1;
  return 0;
}

/* ----------------------------------------------------------------------- */
/* Normally distributed mutation sizes for the paper's two treatments       */
/* (Sec. 3: deleterious Normal decrements in 33% of replications; beneficial */
/* Normal increments in 0.3%). Z is the variance-matched sum of eight       */
/* uniform 16-bit draws (Irwin-Hall, n = 8): mean 0, variance 1 - 2^-32,     */
/* excess kurtosis -0.15, |Z| < 4.9. Only integer sums and one rounded      */
/* binary32 product are involved, so the value is exactly reproducible.     */
/* ----------------------------------------------------------------------- */
static float normal_draw(const uint32_t m[4]) {
  uint32_t sum = 0;
  for (int j = 0; j < 8; ++j) sum += (m[j / 2] >> (16 * (j % 2))) & 0xFFFFu;
  /* E[sum] = 8 * 65535 / 2; Var[sum] = 8 * (65536^2 - 1) / 12 */
  const float scale = (float)(sqrt(1.5) / 65536.0);
  return (float)((int32_t)sum - 262140) * scale;
}

/* ----------------------------------------------------------------------- */
/* Genome models (Sec. 2 Methods: the kernel takes any fixed-length genome  */
/* through three functions, initialize, mutate and evaluate). Each model   */
/* below is those three functions and one row of the table MODELS; the     */
/* generation cycle calls only the table.                                  */
/*   model 0  the genome is its fitness value (the paper's own runs): no    */
/*            payload; mutation changes the fitness (law 0 or 1).           */
/*   model 1  OneMax on a 64-bit string (payload words P0, P1): fitness is  */
/*            the number of one bits.                                       */
/*   model 2  Trap-4 on a 64-bit string (Deb and Goldberg's deceptive trap  */
/*            of order 4): the string is 16 four-bit blocks, block b with u  */
/*            one bits scores 4 if u = 4, else 3 - u; fitness is the sum.   */
/* Models 1 and 2 share initialize and mutate: initialize draws the         */
/* founder's string as words 0 and 1 of one block of the sampling stream at */
/* the counter's last generation (2^64 - 1, never a real one); mutate, with */
/* the same probability p as model 0, flips bit (w3 mod 64) of the child's  */
/* string, bit b of the string being bit b mod 32 of word b / 32, and then  */
/* evaluates the string, so the stored fitness always equals                */
/* evaluate(string).                                                        */
/* ----------------------------------------------------------------------- */
typedef struct orc_model orc_model;
struct orc_model {
  /* founder in slot `slot` of island `island`: its payload P[0..1] and fitness */
  void (*initialize)(const orc_model* m, const orc_config* cfg, uint32_t slot, uint32_t island,
                     uint32_t* P, float* f);
  /* the child in slot `slot` of island `island` at generation t, a copy of its
   * parent: w is the child's selection block (words 2 and 3 are the mutation
   * test and its detail) */
  void (*mutate)(const orc_model* m, const orc_config* cfg, const uint32_t w[4], uint32_t slot,
                 uint32_t island, uint64_t t, uint32_t* P, float* f);
  /* fitness of a payload (NULL: the genome is its fitness) */
  float (*evaluate)(const uint32_t P[2]);
};

/* model 0: founders +0; law 0 adds a delta from {-1, -0.5, 0, 0.5, 1}; law 1
 * adds or subtracts a Normal size drawn from the mutation stream */
static void fitness_initialize(const orc_model* m, const orc_config* cfg, uint32_t slot,
                               uint32_t island, uint32_t* P, float* f) {
  (void)m, (void)cfg, (void)slot, (void)island, (void)P;
  *f = 0.0f;
}

static void fitness_mutate(const orc_model* m, const orc_config* cfg, const uint32_t w[4],
                           uint32_t slot, uint32_t island, uint64_t t, uint32_t* P, float* f) {
  (void)m, (void)P;
  if (cfg->law == 0) {
    if (w[2] < cfg->p32) {
      uint32_t idx = (uint32_t)(((uint64_t)(w[3] & 0x7FFFFFFFu) * 5u) >> 31);
      float delta = 0.5f * (float)((int)idx - 2);
      *f = *f + delta;
    }
  } else {
    int beneficial = w[2] < cfg->p_ben32;
    int deleterious = !beneficial && (uint64_t)w[2] < (uint64_t)cfg->p_ben32 + cfg->p32;
    if (beneficial || deleterious) {
      uint32_t d[4];
      draw(cfg, slot, island, t, TAG_MUTATE, d);
      float size = fabsf(normal_draw(d));
      *f = beneficial ? *f + size : *f - size;
    }
  }
}

static uint32_t ones_in(uint32_t v) {
  uint32_t n = 0;
  for (int b = 0; b < 32; ++b) n += (v >> b) & 1u;
  return n;
}

static void string_initialize(const orc_model* m, const orc_config* cfg, uint32_t slot,
                              uint32_t island, uint32_t* P, float* f) {
  uint32_t w[4];
  draw(cfg, slot, island, UINT64_MAX, TAG_SAMPLE, w);
  P[0] = w[0];
  P[1] = w[1];
  *f = m->evaluate(P);
}

static void string_mutate(const orc_model* m, const orc_config* cfg, const uint32_t w[4],
                          uint32_t slot, uint32_t island, uint64_t t, uint32_t* P, float* f) {
  (void)slot, (void)island, (void)t;
  if (w[2] < cfg->p32) {
    const uint32_t bit = w[3] & 63u;
    P[bit / 32] ^= 1u << (bit % 32);
    *f = m->evaluate(P);
  }
}

static float onemax_evaluate(const uint32_t P[2]) {
  return (float)(ones_in(P[0]) + ones_in(P[1]));
}

static float trap4_evaluate(const uint32_t P[2]) {
  uint32_t sum = 0;
  for (int b = 0; b < 16; ++b) {
    const uint32_t u = ones_in((P[b / 8] >> (4 * (b % 8))) & 0xFu);
    sum += u == 4 ? 4u : 3u - u;
  }
  return (float)sum;
}

static const orc_model MODELS[] = {
    {fitness_initialize, fitness_mutate, NULL},           /* 0: fitness-valued */
    {string_initialize, string_mutate, onemax_evaluate},  /* 1: OneMax */
    {string_initialize, string_mutate, trap4_evaluate},   /* 2: Trap-4 */
};
#define N_MODELS (sizeof(MODELS) / sizeof(MODELS[0]))

static int model_known(uint32_t model) { return model < N_MODELS; }

static void initialize_founders(orc_run* r) {
  const orc_model* m = &MODELS[r->cfg.model];
  for (uint64_t i = 0; i < r->islands; ++i)
    for (uint64_t s = 0; s < r->cfg.pop; ++s) {
      const uint64_t a = i * r->cfg.pop + s;
      m->initialize(m, &r->cfg, (uint32_t)s, (uint32_t)i, &r->P[a * 2], &r->f[a]);
    }
}

orc_run* orc_create(const orc_config* cfg, int record_lineage) {
  if (orc_validate(cfg) != 0) return NULL;
  orc_run* r = (orc_run*)calloc(1, sizeof(orc_run));
  if (!r) return NULL;
  r->cfg = *cfg;
  r->log2pop = log2_exact(cfg->pop);
  r->words = cfg->sites * cfg->dbits / 32;
  r->islands = (uint64_t)cfg->width * cfg->height;
  r->agents = r->islands * cfg->pop;
  r->t = 0;
  /* Founders: fitness +0, no deposits, blank surface (Sec. 2 leaves the
   * initial genome to the model's initialize function). */
  r->f = (float*)calloc(r->agents, sizeof(float));
  r->T = (uint32_t*)calloc(r->agents, sizeof(uint32_t));
  r->D = (uint32_t*)calloc(r->agents * r->words, sizeof(uint32_t));
  r->nf = (float*)calloc(r->agents, sizeof(float));
  r->nT = (uint32_t*)calloc(r->agents, sizeof(uint32_t));
  r->nD = (uint32_t*)calloc(r->agents * r->words, sizeof(uint32_t));
  r->P = (uint32_t*)calloc(r->agents * 2, sizeof(uint32_t));
  r->nP = (uint32_t*)calloc(r->agents * 2, sizeof(uint32_t));
  r->prev = (outbox_entry*)calloc(r->islands, sizeof(outbox_entry));
  r->next = (outbox_entry*)calloc(r->islands, sizeof(outbox_entry));
  r->lineage = record_lineage != 0;
  if (!r->f || !r->T || !r->D || !r->nf || !r->nT || !r->nD || !r->P || !r->nP || !r->prev ||
      !r->next) {
    orc_free(r);
    return NULL;
  }
  initialize_founders(r);
  return r;
}

void orc_free(orc_run* r) {
  if (!r) return;
  free(r->f); free(r->T); free(r->D);
  free(r->nf); free(r->nT); free(r->nD);
  free(r->P); free(r->nP);
  free(r->prev); free(r->next);
  free(r->mail); free(r->seen);
  free(r->winners);
  free(r);
}

uint64_t orc_generation(const orc_run* r) { return r->t; }
uint64_t orc_agents(const orc_run* r) { return r->agents; }

/* Torus neighbour of island i in direction d: 0 north (y-1), 1 east (x+1),
 * 2 south (y+1), 3 west (x-1). The opposite direction is d ^ 2. */
static uint64_t neighbour(const orc_config* cfg, uint64_t i, uint32_t d) {
  uint64_t x = i % cfg->width, y = i / cfg->width;
  uint64_t W = cfg->width, H = cfg->height;
  switch (d) {
    case 0: y = (y + H - 1) % H; break;
    case 1: x = (x + 1) % W; break;
    case 2: y = (y + 1) % H; break;
    default: x = (x + W - 1) % W; break;
  }
  return y * W + x;
}

/* Index in [0, 2^bits) from the top bits of an 8-bit or 32-bit draw. */
static uint32_t top_bits_of_byte(uint32_t byte, uint32_t bits) { return byte >> (8 - bits); }
static uint32_t top_bits_of_word(uint32_t word, uint32_t bits) {
  return (uint32_t)((uint64_t)word >> (32 - bits));
}

static uint32_t byte_of(const uint32_t w[4], uint32_t m) {
  /* byte m of the little-endian 64-bit pair (w[0], w[1]) */
  uint32_t word = m < 4 ? w[0] : w[1];
  return (word >> (8 * (m & 3))) & 0xFFu;
}

static void copy_agent(const orc_run* r, const float* sf, const uint32_t* sT,
                       const uint32_t* sD, const uint32_t* sP, uint64_t src, float* df,
                       uint32_t* dT, uint32_t* dD, uint32_t* dP, uint64_t dst) {
  df[dst] = sf[src];
  dT[dst] = sT[src];
  for (uint32_t w = 0; w < r->words; ++w) dD[dst * r->words + w] = sD[src * r->words + w];
  dP[dst * 2] = sP[src * 2];
  dP[dst * 2 + 1] = sP[src * 2 + 1];
}

static int grow_lineage(orc_run* r, uint64_t gens) {
  if (gens <= r->lineage_cap) return 0;
  size_t bytes = (size_t)(gens * r->agents);
  uint8_t* p = (uint8_t*)realloc(r->winners, bytes);
  if (!p) return -1;
  r->winners = p;
  r->lineage_cap = gens;
  return 0;
}

int orc_reserve_lineage(orc_run* r, uint64_t gens) {
  if (!r->lineage) return -1;
  return grow_lineage(r, gens);
}

/* Steps 3-7 of generation t for island i (Sec. 2): evaluation (reading the
 * fitness word), tournament, copy, mutation and one stratum deposit for every
 * child, read from the current population and written to the next one. */
static void reproduce_island(orc_run* r, uint64_t i, uint64_t t, uint8_t* win_row) {
  const orc_config* cfg = &r->cfg;
  const uint64_t N = cfg->pop;
  const uint32_t L = r->log2pop;
  uint32_t w[4];
  for (uint64_t s = 0; s < N; ++s) {
    draw(cfg, (uint32_t)s, (uint32_t)i, t, TAG_SELECT, w);
    /* Evaluation is reading the fitness word (Sec. 3 genome layout). */
    uint32_t best = top_bits_of_byte(byte_of(w, 0), L);
    if (cfg->selection) {
      for (uint32_t m = 1; m < cfg->k; ++m) {
        uint32_t cand = top_bits_of_byte(byte_of(w, m), L);
        if (r->f[i * N + cand] > r->f[i * N + best]) best = cand;
      }
    }
    uint64_t child = i * N + s;
    copy_agent(r, r->f, r->T, r->D, r->P, i * N + best, r->nf, r->nT, r->nD, r->nP, child);
    if (win_row) win_row[child] = (uint8_t)best;

    MODELS[cfg->model].mutate(&MODELS[cfg->model], cfg, w, (uint32_t)s, (uint32_t)i, t,
                              &r->nP[child * 2], &r->nf[child]);

    /* the differentia: one bit, the top bit of the selection block's word
     * 3; wider ones, the top dbits bits of word 0 of a block of their own
     * (mutation stream, counter word 0 = slot + 256) */
    uint32_t site = orc_site_of_policy(r->nT[child], cfg->sites, cfg->policy);
    if (site != ORC_DISCARD) {
      uint32_t value = w[3] >> 31;
      if (cfg->dbits > 1) {
        uint32_t d[4];
        draw(cfg, (uint32_t)s + 256u, (uint32_t)i, t, TAG_MUTATE, d);
        value = d[0] >> (32 - cfg->dbits);
      }
      const uint32_t pos = site * cfg->dbits;
      const uint32_t field = cfg->dbits == 32 ? ~0u : (1u << cfg->dbits) - 1u;
      uint32_t* word = &r->nD[child * r->words + (pos >> 5)];
      *word = (*word & ~(field << (pos & 31))) | (value << (pos & 31));
    }
    r->nT[child] = r->nT[child] + 1;
  }
}

static void one_generation(orc_run* r) {
  const orc_config* cfg = &r->cfg;
  const uint64_t N = cfg->pop;
  const uint32_t L = r->log2pop;
  const uint64_t t = r->t;
  uint32_t w[4];

  /* 1. Migration, immigration half (Sec. 2): arrivals overwrite receiver-drawn
   *    slots, applied in direction order so the later direction wins a clash. */
  for (uint64_t i = 0; i < r->islands; ++i) {
    draw(cfg, 0, (uint32_t)i, t, TAG_MIGRATE, w);
    for (uint32_t q = 0; q < 4; ++q) {
      uint64_t j = neighbour(cfg, i, q);
      const outbox_entry* in = &r->prev[j];
      if (!in->valid || in->dir != (q ^ 2u)) continue;
      uint32_t slot = top_bits_of_byte((w[2] >> (8 * q)) & 0xFFu, L);
      uint64_t a = i * N + slot;
      r->f[a] = in->f;
      r->T[a] = in->T;
      for (uint32_t k = 0; k < r->words; ++k) r->D[a * r->words + k] = in->D[k];
      r->P[a * 2] = in->P[0];
      r->P[a * 2 + 1] = in->P[1];
    }
  }

  /* 2. Migration, emigration half (Sec. 2): a copy of one random member goes to
   *    one random neighbour; it is absorbed in the next generation. */
  for (uint64_t i = 0; i < r->islands; ++i) {
    outbox_entry* out = &r->next[i];
    memset(out, 0, sizeof(*out));
    if (!cfg->migration) continue;
    draw(cfg, 0, (uint32_t)i, t, TAG_MIGRATE, w);
    uint32_t e = top_bits_of_word(w[0], L);
    uint64_t a = i * N + e;
    out->valid = 1;
    out->dir = (uint8_t)(w[1] >> 30);
    out->f = r->f[a];
    out->T = r->T[a];
    for (uint32_t k = 0; k < r->words; ++k) out->D[k] = r->D[a * r->words + k];
    out->P[0] = r->P[a * 2];
    out->P[1] = r->P[a * 2 + 1];
  }

  /* 3-7. Evaluation, tournament, copy, mutation, stratum deposit (Sec. 2). */
  uint8_t* win_row = r->lineage ? r->winners + (size_t)(t * r->agents) : NULL;
  for (uint64_t i = 0; i < r->islands; ++i) reproduce_island(r, i, t, win_row);

  /* 8. Generational replacement; the fresh outbox becomes next generation's input. */
  float* tf = r->f; r->f = r->nf; r->nf = tf;
  uint32_t* tT = r->T; r->T = r->nT; r->nT = tT;
  uint32_t* tD = r->D; r->D = r->nD; r->nD = tD;
  uint32_t* tP = r->P; r->P = r->nP; r->nP = tP;
  outbox_entry* to = r->prev; r->prev = r->next; r->next = to;
  r->t = t + 1;
}

int orc_step(orc_run* r, uint64_t n) {
  if (r->lineage) {
    if (r->lineage_gens != r->t) return -1; /* lineage must start at generation 0 */
    if (grow_lineage(r, r->t + n) != 0) return -1;
  }
  for (uint64_t g = 0; g < n; ++g) {
    one_generation(r);
    if (r->lineage) r->lineage_gens = r->t;
  }
  return 0;
}

/* ----------------------------------------------------------------------- */
/* Asynchronous schedule (Sec. 2 Methods): every island keeps an            */
/* immigration and an emigration buffer per cardinal neighbour and, at the  */
/* start of each pass of its update loop, takes in whatever has arrived and */
/* refills the buffers it sends from. Here each island keeps, per           */
/* direction, two buffers told apart by the parity of the sending           */
/* generation; a buffer holds the latest genome sent that way in a          */
/* generation of its parity, stamped with that generation + 1. A send       */
/* starts as its sender's pass begins and is read when the receiver begins  */
/* a pass, so a genome is still in flight during the generation it was     */
/* sent in: in generation t a receiver takes, from each side, the newest    */
/* buffer sent before t that is newer than the last one it took from there  */
/* (if any). A genome overwritten before it was taken is lost, as a send    */
/* that never completed would be. Arrivals go to the receiver-drawn slots   */
/* in direction order N, E, S, W and the emission is drawn from the         */
/* post-absorb population, exactly as in the synchronous schedule; only the */
/* moment a genome is read differs.                                         */
/*                                                                          */
/* On hardware the islands interleave freely. This function runs one        */
/* reproducible interleaving: islands go in consecutive groups of `group`;  */
/* group c runs its generation t at step t + (c mod (skew + 1)), and within */
/* a step the groups go in order, each reading all of its arrivals, then    */
/* updating, then publishing. While every island's neighbours are between   */
/* the end of its previous generation and the start of its next one (skew   */
/* 0), this is exactly the synchronous schedule; larger skews put           */
/* neighbours generations apart, so genomes arrive late or are overwritten. */
/* ----------------------------------------------------------------------- */
static int ensure_mail(orc_run* r) {
  if (r->mail) return 0;
  r->mail = (mail_entry*)calloc(r->islands * 8, sizeof(mail_entry));
  r->seen = (uint64_t*)calloc(r->islands * 4, sizeof(uint64_t));
  if (!r->mail || !r->seen) {
    free(r->mail); free(r->seen);
    r->mail = NULL; r->seen = NULL;
    return -1;
  }
  return 0;
}

void orc_clear_mailboxes(orc_run* r) {
  if (!r->mail) return;
  memset(r->mail, 0, r->islands * 8 * sizeof(mail_entry));
  memset(r->seen, 0, r->islands * 4 * sizeof(uint64_t));
}

/* Generation t for the islands [lo, hi), as one group of the interleaving. */
static void group_generation_async(orc_run* r, uint64_t lo, uint64_t hi, uint64_t t) {
  const orc_config* cfg = &r->cfg;
  const uint64_t N = cfg->pop;
  const uint32_t L = r->log2pop;
  uint32_t w[4];
  /* immigration: the buffers neighbour j keeps toward i are j's buffers in
   * direction q ^ 2 */
  for (uint64_t i = lo; i < hi; ++i) {
    draw(cfg, 0, (uint32_t)i, t, TAG_MIGRATE, w);
    for (uint32_t q = 0; q < 4; ++q) {
      const mail_entry* pick = NULL;
      for (uint32_t p = 0; p < 2; ++p) {
        const mail_entry* in = &r->mail[(neighbour(cfg, i, q) * 4 + (q ^ 2u)) * 2 + p];
        if (in->stamp > t || in->stamp <= r->seen[i * 4 + q]) continue;
        if (!pick || in->stamp > pick->stamp) pick = in;
      }
      if (!pick) continue;
      r->seen[i * 4 + q] = pick->stamp;
      uint64_t a = i * N + top_bits_of_byte((w[2] >> (8 * q)) & 0xFFu, L);
      r->f[a] = pick->f;
      r->T[a] = pick->T;
      for (uint32_t k = 0; k < r->words; ++k) r->D[a * r->words + k] = pick->D[k];
      r->P[a * 2] = pick->P[0];
      r->P[a * 2 + 1] = pick->P[1];
    }
  }
  /* emigration choice from the post-absorb population, held back until the
   * group is done */
  for (uint64_t i = lo; i < hi; ++i) {
    outbox_entry* out = &r->next[i];
    memset(out, 0, sizeof(*out));
    if (!cfg->migration) continue;
    draw(cfg, 0, (uint32_t)i, t, TAG_MIGRATE, w);
    uint64_t a = i * N + top_bits_of_word(w[0], L);
    out->valid = 1;
    out->dir = (uint8_t)(w[1] >> 30);
    out->f = r->f[a];
    out->T = r->T[a];
    for (uint32_t k = 0; k < r->words; ++k) out->D[k] = r->D[a * r->words + k];
    out->P[0] = r->P[a * 2];
    out->P[1] = r->P[a * 2 + 1];
  }
  /* update: the group's next population replaces its current one */
  for (uint64_t i = lo; i < hi; ++i) {
    reproduce_island(r, i, t, NULL);
    for (uint64_t s = 0; s < N; ++s)
      copy_agent(r, r->nf, r->nT, r->nD, r->nP, i * N + s, r->f, r->T, r->D, r->P, i * N + s);
  }
  for (uint64_t i = lo; i < hi; ++i) {
    const outbox_entry* out = &r->next[i];
    if (!out->valid) continue;
    mail_entry* m = &r->mail[(i * 4 + out->dir) * 2 + (t & 1)];
    m->stamp = t + 1;
    m->f = out->f;
    m->T = out->T;
    for (uint32_t k = 0; k < r->words; ++k) m->D[k] = out->D[k];
    m->P[0] = out->P[0];
    m->P[1] = out->P[1];
  }
}

int orc_step_async(orc_run* r, uint64_t n, uint64_t group, uint32_t skew) {
  if (r->lineage || group == 0) return -1;
  if (ensure_mail(r) != 0) return -1;
  const uint64_t t0 = r->t;
  for (uint64_t step = 0; step < n + skew; ++step) {
    uint64_t c = 0;
    for (uint64_t lo = 0; lo < r->islands; lo += group, ++c) {
      const uint64_t lag = c % ((uint64_t)skew + 1);
      if (step < lag || step - lag >= n) continue;
      const uint64_t hi = lo + group < r->islands ? lo + group : r->islands;
      group_generation_async(r, lo, hi, t0 + step - lag);
    }
  }
  r->t = t0 + n;
  return 0;
}

void orc_get_mailboxes(const orc_run* r, uint64_t* stamp, uint64_t* seen, float* f,
                       uint32_t* T, uint32_t* D) {
  for (uint64_t b = 0; b < r->islands * 8; ++b) {
    const mail_entry* m = r->mail ? &r->mail[b] : NULL;
    if (stamp) stamp[b] = m ? m->stamp : 0;
    if (f) f[b] = m ? m->f : 0.0f;
    if (T) T[b] = m ? m->T : 0;
    if (D) for (uint32_t k = 0; k < r->words; ++k) D[b * r->words + k] = m ? m->D[k] : 0;
  }
  if (seen)
    for (uint64_t b = 0; b < r->islands * 4; ++b) seen[b] = r->seen ? r->seen[b] : 0;
}

void orc_get_payload(const orc_run* r, uint32_t* P) {
  memcpy(P, r->P, r->agents * 2 * sizeof(uint32_t));
}

void orc_set_payload(orc_run* r, const uint32_t* P) {
  memcpy(r->P, P, r->agents * 2 * sizeof(uint32_t));
}

float orc_evaluate(uint32_t model, uint32_t p0, uint32_t p1) {
  const uint32_t P[2] = {p0, p1};
  return model < N_MODELS && MODELS[model].evaluate ? MODELS[model].evaluate(P) : 0.0f;
}

void orc_get_population(const orc_run* r, float* f, uint32_t* T, uint32_t* D) {
  if (f) memcpy(f, r->f, r->agents * sizeof(float));
  if (T) memcpy(T, r->T, r->agents * sizeof(uint32_t));
  if (D) memcpy(D, r->D, r->agents * r->words * sizeof(uint32_t));
}

void orc_set_population(orc_run* r, const float* f, const uint32_t* T, const uint32_t* D) {
  if (f) memcpy(r->f, f, r->agents * sizeof(float));
  if (T) memcpy(r->T, T, r->agents * sizeof(uint32_t));
  if (D) memcpy(r->D, D, r->agents * r->words * sizeof(uint32_t));
}

void orc_get_outbox(const orc_run* r, uint8_t* valid, uint8_t* dir, float* f,
                    uint32_t* T, uint32_t* D) {
  for (uint64_t i = 0; i < r->islands; ++i) {
    const outbox_entry* e = &r->prev[i];
    if (valid) valid[i] = e->valid;
    if (dir) dir[i] = e->dir;
    if (f) f[i] = e->f;
    if (T) T[i] = e->T;
    if (D) for (uint32_t k = 0; k < r->words; ++k) D[i * r->words + k] = e->D[k];
  }
}

void orc_set_outbox(orc_run* r, const uint8_t* valid, const uint8_t* dir,
                    const float* f, const uint32_t* T, const uint32_t* D) {
  for (uint64_t i = 0; i < r->islands; ++i) {
    outbox_entry* e = &r->prev[i];
    if (valid) e->valid = valid[i] ? 1 : 0;
    if (dir) e->dir = dir[i] & 3u;
    if (f) e->f = f[i];
    if (T) e->T = T[i];
    if (D) for (uint32_t k = 0; k < r->words; ++k) e->D[k] = D[i * r->words + k];
  }
}

int orc_set_generation(orc_run* r, uint64_t t) {
  if (r->lineage) return -1;
  r->t = t;
  return 0;
}

void orc_sample_one_per_island(const orc_run* r, uint64_t* ids) {
  uint32_t w[4];
  for (uint64_t i = 0; i < r->islands; ++i) {
    draw(&r->cfg, 0, (uint32_t)i, r->t, TAG_SAMPLE, w);
    ids[i] = i * r->cfg.pop + top_bits_of_word(w[0], r->log2pop);
  }
}

/* ----------------------------------------------------------------------- */
/* True lineage. An individual is named by where it was born: generation b  */
/* (it is a member of the population at the start of b; b = 0 for founders), */
/* island and slot. Migration copies keep the name of what they copy.       */
/* ----------------------------------------------------------------------- */

/* Who occupies slot w of island i right after generation t's immigration. */
static void post_absorb(const orc_run* r, uint64_t t, uint64_t i, uint32_t w,
                        uint64_t* bt, uint64_t* bi, uint32_t* bs) {
  const orc_config* cfg = &r->cfg;
  uint32_t blk[4], nb[4];
  for (;;) {
    int moved = 0;
    if (cfg->migration && t >= 1) {
      draw(cfg, 0, (uint32_t)i, t, TAG_MIGRATE, blk);
      for (int q = 3; q >= 0 && !moved; --q) {
        uint32_t slot = top_bits_of_byte((blk[2] >> (8 * q)) & 0xFFu, r->log2pop);
        if (slot != w) continue;
        uint64_t j = neighbour(cfg, i, (uint32_t)q);
        draw(cfg, 0, (uint32_t)j, t - 1, TAG_MIGRATE, nb);
        if ((nb[1] >> 30) != ((uint32_t)q ^ 2u)) continue;
        /* The arrival is the copy j emitted during t-1 of its own slot. */
        i = j;
        w = top_bits_of_word(nb[0], r->log2pop);
        t = t - 1;
        moved = 1;
      }
    }
    if (!moved) break;
  }
  *bt = t; *bi = i; *bs = w;
}

size_t orc_ancestry(const orc_run* r, uint64_t agent, uint64_t* gen, uint32_t* island,
                    uint32_t* slot, size_t max_len) {
  uint64_t t = r->t, i = agent / r->cfg.pop;
  uint32_t s = (uint32_t)(agent % r->cfg.pop);
  size_t n = 0;
  for (;;) {
    if (n < max_len) { gen[n] = t; island[n] = (uint32_t)i; slot[n] = s; }
    ++n;
    if (t == 0) break;
    uint32_t w = r->winners[(size_t)((t - 1) * r->agents + i * r->cfg.pop + s)];
    post_absorb(r, t - 1, i, w, &t, &i, &s);
  }
  return n;
}

int64_t orc_true_mrca(const orc_run* r, uint64_t agent_a, uint64_t agent_b) {
  if (!r->lineage || r->lineage_gens != r->t) return -2;
  uint64_t ta = r->t, tb = r->t;
  uint64_t ia = agent_a / r->cfg.pop, ib = agent_b / r->cfg.pop;
  uint32_t sa = (uint32_t)(agent_a % r->cfg.pop), sb = (uint32_t)(agent_b % r->cfg.pop);
  uint64_t steps_a = 0;
  /* Walk both chains back in birth order until they name the same individual. */
  for (;;) {
    if (ta == tb && ia == ib && sa == sb) return (int64_t)r->T[agent_a] - (int64_t)steps_a;
    if (ta == 0 && tb == 0) return -1;
    if (ta >= tb) {
      uint32_t w = r->winners[(size_t)((ta - 1) * r->agents + ia * r->cfg.pop + sa)];
      post_absorb(r, ta - 1, ia, w, &ta, &ia, &sa);
      ++steps_a;
    } else {
      uint32_t w = r->winners[(size_t)((tb - 1) * r->agents + ib * r->cfg.pop + sb)];
      post_absorb(r, tb - 1, ib, w, &tb, &ib, &sb);
    }
  }
}

/* ----------------------------------------------------------------------- */
/* MRCA interval from two surfaces (post hoc relatedness estimation,        */
/* Fig. 1). Ranks retained by both are the multiples of 2^max(ea, eb)       */
/* below min(Ta, Tb). Strata older than the MRCA are inherited identically, */
/* so the first mismatching common rank bounds the MRCA's T from above;     */
/* each common rank at or after the MRCA matches by chance with probability */
/* 1/2, so kc matches in a row below that bound leave the MRCA earlier than */
/* them with probability at most 2^-kc.                                     */
/* ----------------------------------------------------------------------- */
/* The dbits-bit differentia held at a site. */
static uint32_t field_at(const uint32_t* D, uint32_t site, uint32_t dbits) {
  const uint32_t pos = site * dbits;
  return (D[pos >> 5] >> (pos & 31)) & ((1u << dbits) - 1u);
}

void orc_mrca_interval_bits(uint32_t Ta, const uint32_t* Da, uint32_t Tb, const uint32_t* Db,
                            uint32_t sites, uint32_t dbits, uint32_t kc, uint32_t* L, uint32_t* U) {
  uint32_t ea = orc_epoch(Ta, sites), eb = orc_epoch(Tb, sites);
  uint64_t step = (uint64_t)1 << (ea > eb ? ea : eb);
  uint64_t n = Ta < Tb ? Ta : Tb;
  uint64_t first_mismatch = n;
  for (uint64_t r = 0; r < n; r += step) {
    uint32_t site = orc_site_of(r, sites);
    if (field_at(Da, site, dbits) != field_at(Db, site, dbits)) { first_mismatch = r; break; }
  }
  *U = (uint32_t)first_mismatch;
  uint64_t below = (first_mismatch + step - 1) / step; /* common ranks below the bound */
  *L = below < kc ? 0u : (uint32_t)((below - kc) * step + 1);
}

void orc_mrca_interval(uint32_t Ta, const uint32_t* Da, uint32_t Tb, const uint32_t* Db,
                       uint32_t sites, uint32_t kc, uint32_t* L, uint32_t* U) {
  orc_mrca_interval_bits(Ta, Da, Tb, Db, sites, 1, kc, L, U);
}

/* MRCA interval for any policy, from the retained ranks: the common ranks
 * c_0 < c_1 < ... are compared oldest first; U is the first whose
 * differentia differ (or min(Ta, Tb)); L = c_{j - kc} + 1 for the first
 * mismatch index j, or 0 if fewer than kc common ranks lie below it. */
void orc_mrca_interval_policy(uint32_t Ta, const uint32_t* Da, uint32_t Tb, const uint32_t* Db,
                              uint32_t sites, uint32_t dbits, uint32_t policy, uint32_t kc,
                              uint32_t* L, uint32_t* U) {
  uint64_t ra[64], rb[64], common[64];
  const size_t na = orc_retained(Ta, sites, policy, ra);
  const size_t nb = orc_retained(Tb, sites, policy, rb);
  size_t n = 0, x = 0, y = 0;
  while (x < na && y < nb) {
    if (ra[x] == rb[y]) { common[n++] = ra[x]; ++x; ++y; }
    else if (ra[x] < rb[y]) ++x;
    else ++y;
  }
  size_t j = n;
  for (size_t i = 0; i < n; ++i) {
    const uint32_t site = orc_site_of_policy(common[i], sites, policy);
    if (field_at(Da, site, dbits) != field_at(Db, site, dbits)) { j = i; break; }
  }
  *U = j < n ? (uint32_t)common[j] : (Ta < Tb ? Ta : Tb);
  *L = j >= kc ? (uint32_t)(common[j - kc] + 1) : 0u;
}

void orc_mrca_interval_matrix_policy(const uint32_t* T, const uint32_t* D, size_t n,
                                     uint32_t sites, uint32_t dbits, uint32_t policy, uint32_t kc,
                                     uint32_t* L, uint32_t* U) {
  const uint32_t words = sites * dbits / 32;
  for (size_t x = 0; x < n; ++x)
    for (size_t y = 0; y < n; ++y)
      orc_mrca_interval_policy(T[x], D + x * words, T[y], D + y * words, sites, dbits, policy,
                               kc, &L[x * n + y], &U[x * n + y]);
}

int orc_true_mrca_matrix(const orc_run* r, const uint64_t* ids, size_t n, int32_t* out) {
  if (!r->lineage || r->lineage_gens != r->t) return -1;
  const size_t cap = (size_t)r->t + 1;
  uint64_t* gen = (uint64_t*)malloc(n * cap * sizeof(uint64_t));
  uint32_t* isl = (uint32_t*)malloc(n * cap * sizeof(uint32_t));
  uint32_t* slt = (uint32_t*)malloc(n * cap * sizeof(uint32_t));
  size_t* len = (size_t*)malloc(n * sizeof(size_t));
  if (!gen || !isl || !slt || !len) {
    free(gen); free(isl); free(slt); free(len);
    return -1;
  }
  for (size_t x = 0; x < n; ++x)
    len[x] = orc_ancestry(r, ids[x], gen + x * cap, isl + x * cap, slt + x * cap, cap);
  for (size_t x = 0; x < n; ++x) {
    out[x * n + x] = (int32_t)r->T[ids[x]];
    for (size_t y = x + 1; y < n; ++y) {
      /* Both chains list ancestors newest first with strictly decreasing
       * birth generations: walk them together until they name one individual. */
      const uint64_t* ga = gen + x * cap; const uint64_t* gb = gen + y * cap;
      const uint32_t* ia = isl + x * cap; const uint32_t* ib = isl + y * cap;
      const uint32_t* sa = slt + x * cap; const uint32_t* sb = slt + y * cap;
      size_t pa = 0, pb = 0;
      int32_t g = -1;
      while (pa < len[x] && pb < len[y]) {
        if (ga[pa] == gb[pb]) {
          if (ia[pa] == ib[pb] && sa[pa] == sb[pb]) {
            g = (int32_t)r->T[ids[x]] - (int32_t)pa;
            break;
          }
          ++pa;
          ++pb;
        } else if (ga[pa] > gb[pb]) {
          ++pa;
        } else {
          ++pb;
        }
      }
      out[x * n + y] = g;
      out[y * n + x] = g;
    }
  }
  free(gen); free(isl); free(slt); free(len);
  return 0;
}

void orc_mrca_interval_matrix_bits(const uint32_t* T, const uint32_t* D, size_t n,
                                   uint32_t sites, uint32_t dbits, uint32_t kc, uint32_t* L,
                                   uint32_t* U) {
  const uint32_t words = sites * dbits / 32;
  for (size_t x = 0; x < n; ++x)
    for (size_t y = 0; y < n; ++y)
      orc_mrca_interval_bits(T[x], D + x * words, T[y], D + y * words, sites, dbits, kc,
                             &L[x * n + y], &U[x * n + y]);
}

void orc_mrca_interval_matrix(const uint32_t* T, const uint32_t* D, size_t n, uint32_t sites,
                              uint32_t kc, uint32_t* L, uint32_t* U) {
  orc_mrca_interval_matrix_bits(T, D, n, sites, 1, kc, L, U);
}
