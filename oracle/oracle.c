/*
 * oracle.c -- plain, slow CPU reference of the polymerization reaction step of
 * de Buyl & Nies, "A parallel algorithm for step- and chain-growth
 * polymerization in Molecular Dynamics" (arXiv:1409.7498).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link
 * or call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP implementation: both are written independently from
 * the paper and from the arithmetic contract stated in the design notes.
 *
 * What it computes, in the paper's order (Sec. III, Table I, steps 1-9):
 *   1. candidates: every (A, T) pair whose type and state match the rule and
 *      whose distance is below the reaction cutoff (Sec. II, Eq. (2) and the
 *      text after it), found by brute force over all pairs -- no cell list;
 *   2. acceptance of each candidate with probability p = k*dt*Theta
 *      (Sec. II, Eqs. (3)-(4): u < k dt Theta, u uniform in [0,1));
 *   3-5. for each active particle A, one accepted target T chosen at random;
 *   6-7. for each target T, one of the A's that chose it, chosen at random;
 *   9. bond creation and state update of both partners (Eq. (2): t -> t+dt,
 *      a -> a+da), simultaneously after all selections.
 * The communication steps (4, 6, 8) have no counterpart in a shared-memory run.
 *
 * Randomness.  The paper only asks for uniform u and "random" selection.  To
 * make one outcome the correct one, each (step, id_A, id_T) pair draws one
 * Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3"); word 0 decides acceptance, word 1 ranks the
 * A-side choice, word 2 ranks the T-side choice.  The minimum of i.i.d.
 * uniform keys is a uniform choice, ties (impossible within one A or one T,
 * since the low 32 bits carry the partner id) go to the lower id.
 *
 * Floating point: positions are FP32; the squared minimum-image distance is
 * evaluated as ((dx*dx + dy*dy) + dz*dz) with every operation rounded to
 * FP32 and no fused multiply-add (this file must be built with
 * -ffp-contract=off and without -ffast-math; see build.py).  The pair is in range iff
 * r2 < rc2 with rc2 = fl32(rc*rc) (strict).
 *
 * Enumeration order.  The whole step (or_react_step) visits every (A, T)
 * pair exactly once, by brute force, in tiles: OR_TILE active particles
 * against every particle j.  The tiling only reorders the visits so that the
 * particle arrays stream from memory once per tile instead of once per A;
 * each pair's arithmetic is the one above, and every reduction (the minimum
 * over 64-bit keys, integer counts) is exact and independent of order.  The
 * sampled form (or_sample_bonds) visits pairs one A at a time, in the plain
 * loop order, and a test shows both give the same bonds.
 *
 * Pins of every function are in tests/pins.py and tests/test_oracle_*.py
 * (hand cases, closed forms, statistics, planted mistakes).
 */
#include <math.h>
#include <stdint.h>
/* OR_MUTANT (default 0) plants one known mistake per value; only the mutation
 * tests build such variants, to show that the pins catch each mistake. */
#ifndef OR_MUTANT
#define OR_MUTANT 0
#endif
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* error codes, same numeric meaning as the library's */
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERULE_AMBIGUOUS (-2)
#define OR_ECAP (-3)
#define OR_ENOMEM (-4)

/* ----------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the Philox S-P network  */
/* on a 128-bit counter with a 64-bit key; between rounds the key is       */
/* bumped by the Weyl constants (golden ratio, sqrt(3)-1).                 */
/* ----------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], uint64_t key, uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)prod1;
    uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)prod0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* bulk form for the tests: n counters (4 words each) -> n outputs */
void or_philox_bulk(int64_t n, const uint32_t* ctr, const uint64_t* key, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key[i], out + 4 * i);
}

/* ----------------------------------------------------------------------- */
/* Rule and helpers                                                          */
/* ----------------------------------------------------------------------- */
typedef struct {
  int32_t type_a, a_min, a_max, d_a;  /* active role A: type, state window, delta */
  int32_t type_t, t_min, t_max, d_t;  /* target role T */
  float rc;                           /* reaction cutoff */
  double p;                           /* acceptance probability k*dt*Theta */
  int32_t exclude_bonded;             /* 1: already bonded pairs are not candidates */
} or_rule;

static int is_active(const or_rule* r, int32_t type, int32_t state) {
  return type == r->type_a && state >= r->a_min && state <= r->a_max;
}
static int is_target(const or_rule* r, int32_t type, int32_t state) {
  return type == r->type_t && state >= r->t_min && state <= r->t_max;
}

/* acceptance threshold: w0 < ceil(p * 2^32)  <=>  w0 * 2^-32 < p */
uint64_t or_threshold(double p) {
  double t = ceil(p * 4294967296.0);
  if (t < 0.0) t = 0.0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (uint64_t)t;
}

/* minimum-image component: one conditional wrap, as fixed by the contract */
static float min_image(float d, float L, float halfL) {
#if OR_MUTANT == 2 /* mutant: no periodic wrap */
  return d;
#endif
  const float dn = d - L, up = d + L;
  return d > halfL ? dn : (d < -halfL ? up : d);
}

/* squared distance of T at (xt, yt, zt) relative to A at (xa, ya, za), every
 * op rounded to FP32: differences T - A, minimum image, ((dx^2 + dy^2) + dz^2) */
static inline float pair_r2(float xt, float yt, float zt, float xa, float ya, float za,
                            float L, float halfL) {
  float dx = min_image(xt - xa, L, halfL);
  float dy = min_image(yt - ya, L, halfL);
  float dz = min_image(zt - za, L, halfL);
  float sx = dx * dx;
  float sy = dy * dy;
  float sz = dz * dz;
  float sxy = sx + sy;
#if OR_MUTANT == 1 /* mutant: dropped z term */
  return sxy + 0.0f * sz;
#endif
  return sxy + sz;
}

static float dist2(const float* x, const float* y, const float* z, int64_t i, int64_t j,
                   float L, float halfL) {
  return pair_r2(x[j], y[j], z[j], x[i], y[i], z[i], L, halfL);
}

/* the cutoff test of step 1: strictly inside */
static inline int in_cutoff(float r2, float rc2) {
#if OR_MUTANT == 3 /* mutant: inclusive cutoff */
  return r2 <= rc2;
#else
  return r2 < rc2;
#endif
}

static int bonded(const int32_t* adj, int32_t B, int64_t i, int64_t j) {
  for (int32_t k = 0; k < B; ++k)
    if (adj[i * B + k] == (int32_t)j) return 1;
  return 0;
}

static int validate(int32_t n, float L, const float* x, const float* y, const float* z,
                    int32_t B, const or_rule* r) {
  if (n < 0 || B < 1) return OR_EINVAL;
  if (!(r->rc > 0.0f) || !(L > 2.0f * r->rc) || !isfinite(L)) return OR_EINVAL;
  if (!(r->p >= 0.0 && r->p <= 1.0)) return OR_EINVAL;
  if (r->type_a == r->type_t && r->a_min <= r->t_max && r->t_min <= r->a_max)
    return OR_ERULE_AMBIGUOUS;
  for (int64_t i = 0; i < n; ++i) {
    if (!(x[i] >= 0.0f && x[i] < L) || !(y[i] >= 0.0f && y[i] < L) ||
        !(z[i] >= 0.0f && z[i] < L))
      return OR_EINVAL;
  }
  return OR_OK;
}

/* per-step counters (int64 x 9):
 *   a_elig, t_elig  particles eligible for the A and T roles
 *   in_rc           eligible (A, T) pairs with r2 < rc2
 *   drawn           in-range pairs whose draw passes u < p
 *   excluded        drawn pairs that are already bonded (not candidates)
 *   accepted        drawn and not bonded: the retained candidates
 *   proposals       A's with at least one retained candidate
 *   bonds           bonds created
 *   adj_overflow    adjacency appends that found the row full */
enum {
  ST_A_ELIG = 0, ST_T_ELIG, ST_IN_RC, ST_DRAWN, ST_EXCLUDED, ST_ACCEPTED,
  ST_PROPOSALS, ST_BONDS, ST_ADJ_OVERFLOW, ST_COUNT
};

/* Steps 1-2 and the A side of step 5 for one in-range (A = i, T = j) pair:
 * bonded exclusion, the draw u < k dt Theta, and the running minimum of the
 * (w1, id_T) keys of i.  cnt += {in range, drawn, excluded, accepted}. */
static void take_pair(const int32_t* adj, int32_t B, const or_rule* R, uint64_t thresh,
                      uint64_t seed, uint32_t step, int64_t i, int64_t j, uint64_t* best,
                      int64_t cnt[4]) {
  cnt[0]++;
#if OR_MUTANT == 9 /* mutant: bonded pairs not excluded */
  const int already = 0;
#else
  const int already = R->exclude_bonded && bonded(adj, B, i, j); /* step 1: not yet bonded */
#endif
  uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, 0u}, w[4];
  or_philox4x32_10(ctr, seed, w);
  if (!((uint64_t)w[0] < thresh)) return;        /* step 2: u < k dt Theta */
  cnt[1]++;
  if (already) {
    cnt[2]++;
    return;
  }
  cnt[3]++;
  uint64_t key = ((uint64_t)w[1] << 32) | (uint64_t)(uint32_t)j;
  if (key < *best) *best = key;                   /* step 5: one T per A */
}

/* Steps 1-5 for one active particle i: brute force over all particles, keep
 * the in-range, target-eligible, not yet bonded, accepted ones (Table I, steps
 * 1-2) and return the smallest (w1, id_T) key among them, or UINT64_MAX when
 * there is none (steps 3-5).  cnt += {in range, drawn, excluded, accepted}. */
static uint64_t choose_target(int32_t n, float L, const float* x, const float* y,
                              const float* z, const uint8_t* is_t, const int32_t* adj,
                              int32_t B, const or_rule* R, uint64_t thresh, uint64_t seed,
                              uint32_t step, int64_t i, int64_t cnt[4]) {
  const float halfL = 0.5f * L;
  const float rc2 = R->rc * R->rc;
  uint64_t best = UINT64_MAX;
  for (int64_t j = 0; j < n; ++j) {
    if (!is_t[j] || j == i) continue;
    if (!in_cutoff(dist2(x, y, z, i, j, L, halfL), rc2)) continue;  /* step 1: cutoff */
    take_pair(adj, B, R, thresh, seed, step, i, j, &best, cnt);
  }
  return best;
}

/* Steps 1-5 for a tile of m <= OR_TILE active particles ids[0..m-1], every
 * particle j tested against each of them: the same pairs, arithmetic and
 * keys as choose_target for each, visited j-major so that the particle
 * arrays are read once per tile.  best[k] receives the key of ids[k]. */
#define OR_TILE 64
__attribute__((target_clones("avx512f", "avx2", "default")))
static void choose_targets_tile(int32_t n, float L, const float* x, const float* y,
                                const float* z, const uint8_t* is_t, const int32_t* adj,
                                int32_t B, const or_rule* R, uint64_t thresh, uint64_t seed,
                                uint32_t step, const int64_t* ids, int m, uint64_t* best,
                                int64_t cnt[4]) {
  const float halfL = 0.5f * L;
  const float rc2 = R->rc * R->rc;
  float ax[OR_TILE], ay[OR_TILE], az[OR_TILE], r2[OR_TILE];
  for (int k = 0; k < OR_TILE; ++k) {  /* unused slots repeat the last A */
    const int64_t i = ids[k < m ? k : m - 1];
    ax[k] = x[i];
    ay[k] = y[i];
    az[k] = z[i];
  }
  for (int k = 0; k < m; ++k) best[k] = UINT64_MAX;
  for (int64_t j = 0; j < n; ++j) {
    if (!is_t[j]) continue;
    const float xj = x[j], yj = y[j], zj = z[j];
    int any = 0;
    for (int k = 0; k < OR_TILE; ++k) {
      r2[k] = pair_r2(xj, yj, zj, ax[k], ay[k], az[k], L, halfL);
      any |= in_cutoff(r2[k], rc2);
    }
    if (!any) continue;
    for (int k = 0; k < m; ++k) {
      if (ids[k] == j || !in_cutoff(r2[k], rc2)) continue;            /* step 1: cutoff */
      take_pair(adj, B, R, thresh, seed, step, ids[k], j, &best[k], cnt);
    }
  }
}

/* ----------------------------------------------------------------------- */
/* One reaction step (Table I, steps 1-9).                                   */
/* bonds: 2*cap int32 (id_A, id_T), written in increasing id_A order.        */
/* ----------------------------------------------------------------------- */
int or_react_step(int32_t n, float L, const float* x, const float* y, const float* z,
                  const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                  int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
                  int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
                  float rc, double p, int32_t exclude_bonded,
                  uint64_t seed, uint32_t step,
                  int32_t* bonds, int64_t cap, int64_t* n_bonds, int64_t* stats) {
  or_rule R = {type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t, rc, p, exclude_bonded};
  int err = validate(n, L, x, y, z, B, &R);
  if (err) return err;
  if (cap < (int64_t)n / 2) return OR_ECAP;

#if OR_MUTANT == 7 /* mutant: doubled acceptance probability */
  const uint64_t thresh = or_threshold(p > 0.5 ? 1.0 : 2.0 * p);
#else
  const uint64_t thresh = or_threshold(p);
#endif
  const uint64_t EMPTY = UINT64_MAX;

  /* roles from the pre-step state (all predicates use the state before the step) */
  int64_t* alist = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* is_t = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  uint64_t* a_choice = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  uint64_t* t_best = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  if (!alist || !is_t || !a_choice || !t_best) {
    free(alist); free(is_t); free(a_choice); free(t_best);
    return OR_ENOMEM;
  }
  int64_t na = 0, nt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (is_active(&R, type[i], state[i])) alist[na++] = i;
    is_t[i] = (uint8_t)is_target(&R, type[i], state[i]);
    nt += is_t[i];
    t_best[i] = EMPTY;
  }

  /* Steps 1-5: every particle is tested against every A (brute force, in
   * tiles of OR_TILE A's); each A keeps the in-range, eligible, non-bonded,
   * accepted targets and picks one of them: the smallest (w1, id_T) key. */
  int64_t in_rc = 0, drawn = 0, excluded = 0, accepted = 0, proposals = 0;
  const int64_t ntile = (na + OR_TILE - 1) / OR_TILE;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : in_rc, drawn, excluded, accepted, proposals)
  for (int64_t t = 0; t < ntile; ++t) {
    int64_t cnt[4] = {0, 0, 0, 0};
    const int64_t k0 = t * OR_TILE;
    const int m = (int)(na - k0 < OR_TILE ? na - k0 : OR_TILE);
    choose_targets_tile(n, L, x, y, z, is_t, adj, B, &R, thresh, seed, step, alist + k0, m,
                        a_choice + k0, cnt);
    in_rc += cnt[0];
    drawn += cnt[1];
    excluded += cnt[2];
    accepted += cnt[3];
    for (int k = 0; k < m; ++k) proposals += a_choice[k0 + k] != EMPTY;
  }

  /* Steps 6-7: each chosen T keeps the A with the smallest (w2, id_A). */
  for (int64_t k = 0; k < na; ++k) {
    if (a_choice[k] == EMPTY) continue;
    const int64_t i = alist[k];
    const int64_t j = (int64_t)(a_choice[k] & 0xFFFFFFFFu);
    uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, 0u}, w[4];
    or_philox4x32_10(ctr, seed, w);
    uint64_t key2 = ((uint64_t)w[2] << 32) | (uint64_t)(uint32_t)i;
    if (key2 < t_best[j]) t_best[j] = key2;
  }

  /* Step 9: bonds in increasing id_A order; states updated simultaneously
   * (every selection above used the pre-step states). */
  int64_t nb = 0, overflow = 0;
  for (int64_t k = 0; k < na; ++k) {
    if (a_choice[k] == EMPTY) continue;
    const int64_t i = alist[k];
    const int64_t j = (int64_t)(a_choice[k] & 0xFFFFFFFFu);
#if OR_MUTANT != 5 /* mutant 5: no one-A-per-T selection */
    if ((t_best[j] & 0xFFFFFFFFu) != (uint64_t)(uint32_t)i) continue;
#endif
    bonds[2 * nb] = (int32_t)i;
    bonds[2 * nb + 1] = (int32_t)j;
    nb++;
  }
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
#if OR_MUTANT == 10 /* mutant: deltas swapped between roles */
    state[i] += d_t;
    state[j] += d_a;
#else
    state[i] += d_a;
    state[j] += d_t;
#endif
    int placed = 0;
    for (int32_t s = 0; s < B && !placed; ++s)
      if (adj[i * B + s] < 0) { adj[i * B + s] = (int32_t)j; placed = 1; }
    if (!placed) overflow++;
    placed = 0;
    for (int32_t s = 0; s < B && !placed; ++s)
      if (adj[j * B + s] < 0) { adj[j * B + s] = (int32_t)i; placed = 1; }
    if (!placed) overflow++;
  }
  *n_bonds = nb;
  if (stats) {
    stats[ST_A_ELIG] = na;
    stats[ST_T_ELIG] = nt;
    stats[ST_IN_RC] = in_rc;
    stats[ST_DRAWN] = drawn;
    stats[ST_EXCLUDED] = excluded;
    stats[ST_ACCEPTED] = accepted;
    stats[ST_PROPOSALS] = proposals;
    stats[ST_BONDS] = nb;
    stats[ST_ADJ_OVERFLOW] = overflow;
  }
  free(alist); free(is_t); free(a_choice); free(t_best);
  return overflow ? OR_ECAP : OR_OK;
}

/* ----------------------------------------------------------------------- */
/* The "nearest" selection of LAMMPS fix bond/create (Sec. IV A), one step:  */
/*  1. every candidate pair -- eligible A and T (same windows as the rule),  */
/*     in range (r2 < rc2, FP32 as above), not already bonded when           */
/*     exclude_bonded -- is visited; each particle records its closest       */
/*     partner, by the key (r2, partner id): r2's FP32 bits above the id,    */
/*     so equal distances go to the lower id;                                */
/*  2. the consolidation across processors has nothing to do on one memory; */
/*  3. a pair whose partners record each other is evaluated once: the       */
/*     probability test u < p with the pair's draw (counter (step, id_A,     */
/*     id_T, 0), word 0, the same draw as above: one draw per pair, which is */
/*     what evaluating it on one particle of the pair amounts to);           */
/*  then bonds and states as in step 9 of the random selection.             */
/* A pair whose draw fails does not bond, and neither partner falls back to */
/* another one in that step.                                                */
/* Counters: in_rc and excluded count in-range pairs (excluded: bonded);    */
/* drawn counts the mutual pairs, accepted and bonds those that pass;       */
/* proposals counts A's with a closest partner.                             */
/* ----------------------------------------------------------------------- */
typedef struct {
  int64_t i, j;
  float r2;
} or_cand;

static uint64_t near_key(float r2, int64_t partner) {
  uint32_t bits;
  memcpy(&bits, &r2, sizeof bits);  /* r2 >= 0: its bits order like the value */
  return ((uint64_t)bits << 32) | (uint64_t)(uint32_t)partner;
}

int or_react_step_nearest(int32_t n, float L, const float* x, const float* y, const float* z,
                          const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                          int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
                          int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
                          float rc, double p, int32_t exclude_bonded,
                          uint64_t seed, uint32_t step,
                          int32_t* bonds, int64_t cap, int64_t* n_bonds, int64_t* stats) {
  or_rule R = {type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t, rc, p, exclude_bonded};
  int err = validate(n, L, x, y, z, B, &R);
  if (err) return err;
  if (cap < (int64_t)n / 2) return OR_ECAP;
  const uint64_t thresh = or_threshold(p);
  const float halfL = 0.5f * L, rc2 = rc * rc;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int64_t* alist = (int64_t*)malloc(sizeof(int64_t) * nn);
  uint8_t* is_t = (uint8_t*)malloc(nn);
  uint64_t* nearA = (uint64_t*)malloc(sizeof(uint64_t) * nn);
  uint64_t* nearT = (uint64_t*)malloc(sizeof(uint64_t) * nn);
  if (!alist || !is_t || !nearA || !nearT) {
    free(alist); free(is_t); free(nearA); free(nearT);
    return OR_ENOMEM;
  }
  int64_t na = 0, nt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (is_active(&R, type[i], state[i])) alist[na++] = i;
    is_t[i] = (uint8_t)is_target(&R, type[i], state[i]);
    nt += is_t[i];
    nearA[i] = nearT[i] = UINT64_MAX;
  }
  /* Step 1, brute force over all (A, T) pairs in tiles of OR_TILE A's: the
   * in-range pairs of each tile are collected, then every candidate updates
   * the closest-partner keys of both of its particles. */
  const int64_t ntile = (na + OR_TILE - 1) / OR_TILE;
  or_cand** found = (or_cand**)calloc((size_t)(ntile > 0 ? ntile : 1), sizeof(or_cand*));
  int64_t* nfound = (int64_t*)calloc((size_t)(ntile > 0 ? ntile : 1), sizeof(int64_t));
  int oom = !found || !nfound;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < ntile; ++t) {
    if (oom) continue;
    const int64_t k0 = t * OR_TILE;
    const int m = (int)(na - k0 < OR_TILE ? na - k0 : OR_TILE);
    int64_t cap_t = 256, cnt = 0;
    or_cand* buf = (or_cand*)malloc(sizeof(or_cand) * (size_t)cap_t);
    for (int64_t j = 0; j < n && buf; ++j) {
      if (!is_t[j]) continue;
      for (int k = 0; k < m; ++k) {
        const int64_t i = alist[k0 + k];
        if (i == j) continue;
        const float r2 = dist2(x, y, z, i, j, L, halfL);
        if (!in_cutoff(r2, rc2)) continue;
        if (cnt == cap_t) {
          cap_t *= 2;
          or_cand* nb = (or_cand*)realloc(buf, sizeof(or_cand) * (size_t)cap_t);
          if (!nb) { free(buf); buf = NULL; break; }
          buf = nb;
        }
        buf[cnt].i = i;
        buf[cnt].j = j;
        buf[cnt].r2 = r2;
        cnt++;
      }
    }
    if (!buf) oom = 1;
    found[t] = buf;
    nfound[t] = cnt;
  }
  int64_t in_rc = 0, excluded = 0;
  for (int64_t t = 0; t < ntile && !oom; ++t) {
    for (int64_t c = 0; c < nfound[t]; ++c) {
      const or_cand q = found[t][c];
      in_rc++;
#if OR_MUTANT == 18 /* mutant: bonded pairs stay candidates */
      const int already = 0;
#else
      const int already = exclude_bonded && bonded(adj, B, q.i, q.j);
#endif
      if (already) {
        excluded++;
        continue;
      }
      const uint64_t ka = near_key(q.r2, q.j), kt = near_key(q.r2, q.i);
      if (ka < nearA[q.i]) nearA[q.i] = ka;
      if (kt < nearT[q.j]) nearT[q.j] = kt;
    }
  }
  for (int64_t t = 0; t < ntile && found; ++t) free(found[t]);
  free(found);
  free(nfound);
  if (oom) {
    free(alist); free(is_t); free(nearA); free(nearT);
    return OR_ENOMEM;
  }
  /* Step 3: mutual pairs, one draw each, bonds in increasing id_A order */
  int64_t proposals = 0, mutual = 0, nb = 0;
  for (int64_t k = 0; k < na; ++k) {
    const int64_t i = alist[k];
    if (nearA[i] == UINT64_MAX) continue;
    proposals++;
    const int64_t j = (int64_t)(nearA[i] & 0xFFFFFFFFu);
#if OR_MUTANT == 19 /* mutant: the T side's choice ignored */
    const int mutual_pair = 1;
#else
    const int mutual_pair = (int64_t)(nearT[j] & 0xFFFFFFFFu) == i;
#endif
    if (!mutual_pair) continue;
    mutual++;
    uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, 0u}, w[4];
    or_philox4x32_10(ctr, seed, w);
    if (!((uint64_t)w[0] < thresh)) continue;
    bonds[2 * nb] = (int32_t)i;
    bonds[2 * nb + 1] = (int32_t)j;
    nb++;
  }
  /* bonds and states (Table I, step 9), simultaneously */
  int64_t overflow = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
    state[i] += d_a;
    state[j] += d_t;
    int placed = 0;
    for (int32_t s2 = 0; s2 < B && !placed; ++s2)
      if (adj[i * B + s2] < 0) { adj[i * B + s2] = (int32_t)j; placed = 1; }
    if (!placed) overflow++;
    placed = 0;
    for (int32_t s2 = 0; s2 < B && !placed; ++s2)
      if (adj[j * B + s2] < 0) { adj[j * B + s2] = (int32_t)i; placed = 1; }
    if (!placed) overflow++;
  }
  *n_bonds = nb;
  if (stats) {
    stats[ST_A_ELIG] = na;
    stats[ST_T_ELIG] = nt;
    stats[ST_IN_RC] = in_rc;
    stats[ST_DRAWN] = mutual;
    stats[ST_EXCLUDED] = excluded;
    stats[ST_ACCEPTED] = nb;
    stats[ST_PROPOSALS] = proposals;
    stats[ST_BONDS] = nb;
    stats[ST_ADJ_OVERFLOW] = overflow;
  }
  free(alist); free(is_t); free(nearA); free(nearT);
  return overflow ? OR_ECAP : OR_OK;
}

/* ----------------------------------------------------------------------- */
/* Several concurrent rules in one step (the extension Sec. III B and the    */
/* conclusions propose; the paper gives no procedure, so this is the        */
/* generalisation of Table I the library implements):                       */
/*  1-2. every rule r contributes its candidates (A and T eligible under r, */
/*       in range of r's cutoff, not bonded when r excludes bonded pairs),  */
/*       each with its own draw: counter (step, id_A, id_T, tag(r)), tag 0  */
/*       for rule 0 and 0x100 + r otherwise, accepted iff w0 < thresh(p_r); */
/*  3-5. each particle, as an A, picks among all its accepted candidates    */
/*       (any rule) the smallest (w1, id_T), the lower rule on a tie;       */
/*  6-7. each T keeps, among the A's that picked it, the smallest (w2,      */
/*       id_A) of the picked pairs;                                         */
/*  8.   a particle can now hold two winning pairs (as the A of one rule    */
/*       and the T of another): it keeps the one with the smaller (w3,      */
/*       partner id, rule), and a pair is bonded only if both of its        */
/*       particles keep it (losers wait for a later step, as in step 7);    */
/*  9.   bonds in increasing id_A order, each with its rule's deltas.       */
/* With one rule no particle can hold two roles (the windows of a rule do   */
/* not overlap), step 8 never acts and the result is or_react_step's.       */
/* rules: nrules records of 10 int32 (type_a, a_min, a_max, d_a, type_t,    */
/* t_min, t_max, d_t, exclude_bonded, unused), rc[nrules], p[nrules].       */
/* bonds: 3 * cap int32 (id_A, id_T, rule).  Counters summed over rules.    */
/* ----------------------------------------------------------------------- */
#define OR_MAX_RULES 4

static float wrap_box(float v, float L);
void or_ih4_offsets(uint32_t step, uint32_t id, uint32_t tag, uint64_t seed, int32_t S[3]);

void or_jitter(int32_t n, float L, float* x, float* y, float* z, uint64_t seed, uint32_t step,
               double sigma);

uint32_t or_rule_tag(int32_t r) { return r == 0 ? 0u : 0x100u + (uint32_t)r; }

typedef struct {
  uint64_t key;  /* (w1, id_T) */
  int32_t rule;
} or_pick;

static int pick_less(uint64_t k1, int32_t r1, uint64_t k2, int32_t r2) {
  return k1 < k2 || (k1 == k2 && r1 < r2);
}

int or_react_step_multi(int32_t n, float L, const float* x, const float* y, const float* z,
                        const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                        const int32_t* rules, const float* rc, const double* p, int32_t nrules,
                        uint64_t seed, uint32_t step,
                        int32_t* bonds, int64_t cap, int64_t* n_bonds, int64_t* stats) {
  if (nrules < 1 || nrules > OR_MAX_RULES) return OR_EINVAL;
  or_rule R[OR_MAX_RULES];
  uint64_t thresh[OR_MAX_RULES];
  for (int32_t r = 0; r < nrules; ++r) {
    const int32_t* q = rules + 10 * r;
    or_rule rr = {q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], rc[r], p[r], q[8]};
    R[r] = rr;
    int err = validate(n, L, x, y, z, B, &R[r]);
    if (err) return err;
    thresh[r] = or_threshold(p[r]);
  }
  if (cap < (int64_t)n / 2) return OR_ECAP;
  const float halfL = 0.5f * L;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  or_pick* pickA = (or_pick*)malloc(sizeof(or_pick) * nn);   /* steps 3-5, per A */
  uint64_t* bestT = (uint64_t*)malloc(sizeof(uint64_t) * nn); /* steps 6-7, per T */
  uint64_t* keep = (uint64_t*)malloc(sizeof(uint64_t) * nn);  /* step 8, per particle */
  int32_t* keep_rule = (int32_t*)malloc(sizeof(int32_t) * nn);
  if (!pickA || !bestT || !keep || !keep_rule) {
    free(pickA); free(bestT); free(keep); free(keep_rule);
    return OR_ENOMEM;
  }
  int64_t na = 0, nt = 0;
  for (int64_t i = 0; i < n; ++i) {
    int a = 0, t = 0;
    for (int32_t r = 0; r < nrules; ++r) {
      a |= is_active(&R[r], type[i], state[i]);
      t |= is_target(&R[r], type[i], state[i]);
    }
    na += a;
    nt += t;
    pickA[i].key = UINT64_MAX;
    pickA[i].rule = -1;
    bestT[i] = keep[i] = UINT64_MAX;
    keep_rule[i] = -1;
  }
  /* steps 1-5: brute force over all pairs and rules */
  int64_t in_rc = 0, drawn = 0, excluded = 0, accepted = 0, proposals = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : in_rc, drawn, excluded, accepted)
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t r = 0; r < nrules; ++r) {
      if (!is_active(&R[r], type[i], state[i])) continue;
      const float rc2 = rc[r] * rc[r];
      for (int64_t j = 0; j < n; ++j) {
        if (j == i || !is_target(&R[r], type[j], state[j])) continue;
        if (!in_cutoff(dist2(x, y, z, i, j, L, halfL), rc2)) continue;
        in_rc++;
        const int already = R[r].exclude_bonded && bonded(adj, B, i, j);
        uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, or_rule_tag(r)}, w[4];
        or_philox4x32_10(ctr, seed, w);
        if (!((uint64_t)w[0] < thresh[r])) continue;
        drawn++;
        if (already) {
          excluded++;
          continue;
        }
        accepted++;
        const uint64_t key = ((uint64_t)w[1] << 32) | (uint64_t)(uint32_t)j;
        if (pick_less(key, r, pickA[i].key, pickA[i].rule)) {
          pickA[i].key = key;
          pickA[i].rule = r;
        }
      }
    }
  }
  /* steps 6-7 */
  for (int64_t i = 0; i < n; ++i) {
    if (pickA[i].rule < 0) continue;
    proposals++;
    const int64_t j = (int64_t)(pickA[i].key & 0xFFFFFFFFu);
    uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, or_rule_tag(pickA[i].rule)}, w[4];
    or_philox4x32_10(ctr, seed, w);
    const uint64_t key2 = ((uint64_t)w[2] << 32) | (uint64_t)(uint32_t)i;
    if (key2 < bestT[j]) bestT[j] = key2;
  }
  /* step 8: every winning pair offers itself to both of its particles */
  for (int64_t i = 0; i < n; ++i) {
    if (pickA[i].rule < 0) continue;
    const int64_t j = (int64_t)(pickA[i].key & 0xFFFFFFFFu);
    if ((bestT[j] & 0xFFFFFFFFu) != (uint64_t)(uint32_t)i) continue;
    const int32_t r = pickA[i].rule;
    uint32_t ctr[4] = {step, (uint32_t)i, (uint32_t)j, or_rule_tag(r)}, w[4];
    or_philox4x32_10(ctr, seed, w);
    const uint64_t ki = ((uint64_t)w[3] << 32) | (uint64_t)(uint32_t)j;  /* at i */
    const uint64_t kj = ((uint64_t)w[3] << 32) | (uint64_t)(uint32_t)i;  /* at j */
    if (pick_less(ki, r, keep[i], keep_rule[i])) { keep[i] = ki; keep_rule[i] = r; }
    if (pick_less(kj, r, keep[j], keep_rule[j])) { keep[j] = kj; keep_rule[j] = r; }
  }
  /* step 9 */
  int64_t nb = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (pickA[i].rule < 0) continue;
    const int64_t j = (int64_t)(pickA[i].key & 0xFFFFFFFFu);
    if ((bestT[j] & 0xFFFFFFFFu) != (uint64_t)(uint32_t)i) continue;
    const int32_t r = pickA[i].rule;
#if OR_MUTANT != 21 /* mutant 21: no step 8 */
    if (keep_rule[i] != r || (keep[i] & 0xFFFFFFFFu) != (uint64_t)(uint32_t)j) continue;
    if (keep_rule[j] != r || (keep[j] & 0xFFFFFFFFu) != (uint64_t)(uint32_t)i) continue;
#endif
    bonds[3 * nb] = (int32_t)i;
    bonds[3 * nb + 1] = (int32_t)j;
    bonds[3 * nb + 2] = r;
    nb++;
  }
  int64_t overflow = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t i = bonds[3 * b], j = bonds[3 * b + 1];
    const int32_t r = bonds[3 * b + 2];
    state[i] += R[r].d_a;
    state[j] += R[r].d_t;
    int placed = 0;
    for (int32_t s2 = 0; s2 < B && !placed; ++s2)
      if (adj[i * B + s2] < 0) { adj[i * B + s2] = (int32_t)j; placed = 1; }
    if (!placed) overflow++;
    placed = 0;
    for (int32_t s2 = 0; s2 < B && !placed; ++s2)
      if (adj[j * B + s2] < 0) { adj[j * B + s2] = (int32_t)i; placed = 1; }
    if (!placed) overflow++;
  }
  *n_bonds = nb;
  if (stats) {
    stats[ST_A_ELIG] = na;
    stats[ST_T_ELIG] = nt;
    stats[ST_IN_RC] = in_rc;
    stats[ST_DRAWN] = drawn;
    stats[ST_EXCLUDED] = excluded;
    stats[ST_ACCEPTED] = accepted;
    stats[ST_PROPOSALS] = proposals;
    stats[ST_BONDS] = nb;
    stats[ST_ADJ_OVERFLOW] = overflow;
  }
  free(pickA); free(bestT); free(keep); free(keep_rule);
  return overflow ? OR_ECAP : OR_OK;
}

/* Steps first_step .. with several rules: each step re-jitters (sigma > 0)
 * and runs or_react_step_multi.  Log rows: (step, id_A, id_T, rule). */
int or_run_multi(int32_t n, float L, float* x, float* y, float* z, const int32_t* type,
                 int32_t* state, int32_t* adj, int32_t B, const int32_t* rules, const float* rc,
                 const double* p, int32_t nrules, uint64_t seed, uint32_t first_step,
                 uint32_t n_steps, double sigma, int32_t* log, int64_t log_cap, int64_t* n_log,
                 int64_t* stats_per_step) {
  int32_t* sb = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n / 2 + 1));
  if (!sb) return OR_ENOMEM;
  int64_t total = 0;
  int code = OR_OK;
  for (uint32_t k = 0; k < n_steps; ++k) {
    const uint32_t st = first_step + k;
    if (sigma > 0.0) or_jitter(n, L, x, y, z, seed, st, sigma);
    int64_t nb = 0;
    int e = or_react_step_multi(n, L, x, y, z, type, state, adj, B, rules, rc, p, nrules, seed,
                                st, sb, n / 2 + 1, &nb,
                                stats_per_step ? stats_per_step + (int64_t)k * ST_COUNT : NULL);
    if (e != OR_OK && e != OR_ECAP) { code = e; break; }
    if (e == OR_ECAP) code = OR_ECAP;
    for (int64_t b = 0; b < nb; ++b, ++total) {
      if (total < log_cap) {
        log[4 * total] = (int32_t)st;
        log[4 * total + 1] = sb[3 * b];
        log[4 * total + 2] = sb[3 * b + 1];
        log[4 * total + 3] = sb[3 * b + 2];
      }
    }
  }
  *n_log = total;
  free(sb);
  if (code == OR_OK && total > log_cap) return OR_ECAP;
  return code;
}

/* ----------------------------------------------------------------------- */
/* Sampled form of steps 1-7, for checks at sizes where a whole step is too  */
/* slow: for each sampled particle ids[k], out[k] = the id of the target it  */
/* bonds with in this step, or -1.  Its choice (steps 1-5) is computed by    */
/* brute force; the T side (steps 6-7) by computing the choice of every      */
/* active particle within the cutoff of that target.                          */
/* ----------------------------------------------------------------------- */
int or_sample_bonds(int32_t n, float L, const float* x, const float* y, const float* z,
                    const int32_t* type, const int32_t* state, const int32_t* adj, int32_t B,
                    int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
                    int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
                    float rc, double p, int32_t exclude_bonded, uint64_t seed, uint32_t step,
                    const int64_t* ids, int64_t m, int32_t* out) {
  or_rule R = {type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t, rc, p, exclude_bonded};
  int err = validate(n, L, x, y, z, B, &R);
  if (err) return err;
  const uint64_t thresh = or_threshold(p);
  const float halfL = 0.5f * L, rc2 = rc * rc;
  uint8_t* is_t = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  if (!is_t) return OR_ENOMEM;
  for (int64_t i = 0; i < n; ++i) is_t[i] = (uint8_t)is_target(&R, type[i], state[i]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < m; ++k) {
    const int64_t i = ids[k];
    int64_t cnt[4] = {0, 0, 0, 0};
    out[k] = -1;
    if (!is_active(&R, type[i], state[i])) continue;
    const uint64_t key = choose_target(n, L, x, y, z, is_t, adj, B, &R, thresh, seed, step, i, cnt);
    if (key == UINT64_MAX) continue;
    const int64_t j = (int64_t)(key & 0xFFFFFFFFu);
    uint64_t best = UINT64_MAX;
    for (int64_t i2 = 0; i2 < n; ++i2) {
      if (!is_active(&R, type[i2], state[i2])) continue;
      if (!(dist2(x, y, z, i2, j, L, halfL) < rc2)) continue;
      const uint64_t k2 = choose_target(n, L, x, y, z, is_t, adj, B, &R, thresh, seed, step, i2, cnt);
      if (k2 == UINT64_MAX || (int64_t)(k2 & 0xFFFFFFFFu) != j) continue;
      uint32_t ctr[4] = {step, (uint32_t)i2, (uint32_t)j, 0u}, w[4];
      or_philox4x32_10(ctr, seed, w);
      const uint64_t bid = ((uint64_t)w[2] << 32) | (uint64_t)(uint32_t)i2;
      if (bid < best) best = bid;
    }
    if ((best & 0xFFFFFFFFu) == (uint64_t)(uint32_t)i) out[k] = (int32_t)j;
  }
  free(is_t);
  return OR_OK;
}

/* ----------------------------------------------------------------------- */
/* FP64 recheck of the cutoff decision (diagnostic only; Sec. II gives the  */
/* cutoff as a distance, the contract decides it in FP32 on r^2).            */
/* Over every pair of an A-eligible i and a T-eligible j != i, from the same */
/* FP32 coordinates converted to double: r64 = sqrt of the FP64 squared      */
/* minimum-image distance.  near counts |r64 - rc| < tol (rc the FP32 cutoff */
/* as a double), disagree counts pairs whose FP64 decision r64 < rc differs  */
/* from the FP32 decision of the step (pair_r2 < fl32(rc*rc)).  Pairs with   */
/* r64 >= rc + 1 can be neither (the FP32 value is within a few ulps of the  */
/* FP64 one) and are skipped after their FP64 r^2.  Brute force, in tiles of */
/* OR_TILE A's like the step.                                                */
/* ----------------------------------------------------------------------- */
static inline double min_image64(double d, double L, double halfL) {
#if OR_MUTANT == 14 /* mutant: no periodic wrap in the FP64 recheck */
  return d;
#endif
  const double dn = d - L, up = d + L;
  return d > halfL ? dn : (d < -halfL ? up : d);
}

__attribute__((target_clones("avx512f", "avx2", "default")))
static void near_tile(int32_t n, float L, const float* x, const float* y, const float* z,
                      const uint8_t* is_t, const int64_t* ids, int m, float rc, double tol,
                      int64_t* near, int64_t* disagree) {
  const double Ld = (double)L, halfd = 0.5 * Ld, rcd = (double)rc;
  const double lim2 = (rcd + 1.0) * (rcd + 1.0);
  const float halfL = 0.5f * L, rc2 = rc * rc;
  double ax[OR_TILE], ay[OR_TILE], az[OR_TILE], r2[OR_TILE];
  for (int k = 0; k < OR_TILE; ++k) {
    const int64_t i = ids[k < m ? k : m - 1];
    ax[k] = (double)x[i];
    ay[k] = (double)y[i];
    az[k] = (double)z[i];
  }
  int64_t cn = 0, cd = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (!is_t[j]) continue;
    const double xj = (double)x[j], yj = (double)y[j], zj = (double)z[j];
    int any = 0;
    for (int k = 0; k < OR_TILE; ++k) {
      const double dx = min_image64(xj - ax[k], Ld, halfd);
      const double dy = min_image64(yj - ay[k], Ld, halfd);
      const double dz = min_image64(zj - az[k], Ld, halfd);
      r2[k] = dx * dx + dy * dy + dz * dz;
      any |= r2[k] < lim2;
    }
    if (!any) continue;
    for (int k = 0; k < m; ++k) {
      if (ids[k] == j || !(r2[k] < lim2)) continue;
      const double r = sqrt(r2[k]);
#if OR_MUTANT == 15 /* mutant: tolerance applied to r^2 instead of r */
      cn += fabs(r2[k] - rcd * rcd) < tol;
#else
      cn += fabs(r - rcd) < tol;
#endif
      const int64_t i = ids[k];
#if OR_MUTANT == 17 /* mutant: the FP32 side taken in FP64 (never disagrees) */
      const int in32 = r2[k] < (double)rc2;
#else
      const int in32 = pair_r2(x[j], y[j], z[j], x[i], y[i], z[i], L, halfL) < rc2;
#endif
      const int in64 = r < rcd;
      cd += in32 != in64;
    }
  }
  *near += cn;
  *disagree += cd;
}

int or_near_cutoff(int32_t n, float L, const float* x, const float* y, const float* z,
                   const int32_t* type, const int32_t* state,
                   int32_t type_a, int32_t a_min, int32_t a_max,
                   int32_t type_t, int32_t t_min, int32_t t_max,
                   float rc, double tol, int64_t* near, int64_t* disagree) {
  or_rule R = {type_a, a_min, a_max, 0, type_t, t_min, t_max, 0, rc, 0.0, 0};
  int64_t* alist = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint8_t* is_t = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  if (!alist || !is_t) {
    free(alist); free(is_t);
    return OR_ENOMEM;
  }
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i) {
#if OR_MUTANT == 16 /* mutant: every particle counted as an A */
    alist[na++] = i;
#else
    if (is_active(&R, type[i], state[i])) alist[na++] = i;
#endif
    is_t[i] = (uint8_t)is_target(&R, type[i], state[i]);
  }
  int64_t cnt_near = 0, cnt_dis = 0;
  const int64_t ntile = (na + OR_TILE - 1) / OR_TILE;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : cnt_near, cnt_dis)
  for (int64_t t = 0; t < ntile; ++t) {
    const int64_t k0 = t * OR_TILE;
    const int m = (int)(na - k0 < OR_TILE ? na - k0 : OR_TILE);
    int64_t a = 0, d = 0;
    near_tile(n, L, x, y, z, is_t, alist + k0, m, rc, tol, &a, &d);
    cnt_near += a;
    cnt_dis += d;
  }
  *near = cnt_near;
  *disagree = cnt_dis;
  free(alist);
  free(is_t);
  return OR_OK;
}

/* ----------------------------------------------------------------------- */
/* Kinetics counters of a configuration (Sec. II B-C): the quantities the    */
/* rate equations are built from.                                           */
/*  pop[s]   particles of type type_a in state s, s = 0 .. nstate-1 (the    */
/*           populations [X_s] of Eq. (12), [M], [P*] of Eqs. (5)-(10));    */
/*  pairs[s] over the A-eligible particles in state s, the number of        */
/*           T-eligible particles within the cutoff (FP32 r2 < fl32(rc^2),  */
/*           the step's own test) that are not bonded to them when the rule */
/*           excludes bonded pairs: pairs[s] / pop[s] is <N_{X^s E^0}>      */
/*           (Eq. (13)) or <N_{P* M}> (k_c of Eq. (6));                     */
/*  hist[b]  the same pairs by distance, b = 0 .. nbins-1: the pair is in   */
/*           bin b iff e2[b] <= r2 < e2[b + 1] with e2[b] = fl32((rc b /    */
/*           nbins)^2) evaluated in double (e2[nbins] is the cutoff rc2).   */
/*           hist[b] / pop / (rho_T shell volume) is g(r), whose integral   */
/*           up to rc gives <N>.                                            */
/* Brute force over all (A, T) pairs in tiles of OR_TILE A's.               */
/* ----------------------------------------------------------------------- */
float or_kin_edge2(float rc, int32_t b, int32_t nbins) {
  const double r = (double)rc * (double)b / (double)nbins;
  return (float)(r * r);
}

int or_kinetics(int32_t n, float L, const float* x, const float* y, const float* z,
                const int32_t* type, const int32_t* state, const int32_t* adj, int32_t B,
                int32_t type_a, int32_t a_min, int32_t a_max,
                int32_t type_t, int32_t t_min, int32_t t_max, float rc, int32_t exclude_bonded,
                int32_t nstate, int64_t* pop, int64_t* pairs, int32_t nbins, int64_t* hist) {
  or_rule R = {type_a, a_min, a_max, 0, type_t, t_min, t_max, 0, rc, 0.0, exclude_bonded};
  if (nstate < 1 || nbins < 0) return OR_EINVAL;
  for (int32_t q = 0; q < nstate; ++q) pop[q] = pairs[q] = 0;
  for (int32_t b = 0; b < nbins; ++b) hist[b] = 0;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int64_t* alist = (int64_t*)malloc(sizeof(int64_t) * nn);
  uint8_t* is_t = (uint8_t*)malloc(nn);
  float* e2 = (float*)malloc(sizeof(float) * (size_t)(nbins + 1));
  if (!alist || !is_t || !e2) {
    free(alist); free(is_t); free(e2);
    return OR_ENOMEM;
  }
  for (int32_t b = 0; b <= nbins; ++b) e2[b] = or_kin_edge2(rc, b, nbins);
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (type[i] == type_a && state[i] >= 0 && state[i] < nstate) pop[state[i]]++;
    if (is_active(&R, type[i], state[i])) alist[na++] = i;
    is_t[i] = (uint8_t)is_target(&R, type[i], state[i]);
  }
  const float halfL = 0.5f * L, rc2 = rc * rc;
  const int64_t ntile = (na + OR_TILE - 1) / OR_TILE;
#pragma omp parallel
  {
    int64_t* lp = (int64_t*)calloc((size_t)nstate, sizeof(int64_t));
    int64_t* lh = (int64_t*)calloc((size_t)(nbins > 0 ? nbins : 1), sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < ntile; ++t) {
      const int64_t k0 = t * OR_TILE;
      const int m = (int)(na - k0 < OR_TILE ? na - k0 : OR_TILE);
      for (int64_t j = 0; j < n && lp && lh; ++j) {
        if (!is_t[j]) continue;
        for (int k = 0; k < m; ++k) {
          const int64_t i = alist[k0 + k];
          if (i == j) continue;
          const float r2 = dist2(x, y, z, i, j, L, halfL);
          if (!in_cutoff(r2, rc2)) continue;
          if (exclude_bonded && bonded(adj, B, i, j)) continue;
#if OR_MUTANT == 20 /* mutant: partners counted for the T's state */
          const int32_t s = state[j];
#else
          const int32_t s = state[i];
#endif
          if (s >= 0 && s < nstate) lp[s]++;
          int32_t b = 0;
          while (b + 1 < nbins && !(r2 < e2[b + 1])) b++;
          if (nbins > 0) lh[b]++;
        }
      }
    }
#pragma omp critical
    {
      for (int32_t q = 0; q < nstate && lp; ++q) pairs[q] += lp[q];
      for (int32_t b = 0; b < nbins && lh; ++b) hist[b] += lh[b];
    }
    free(lp);
    free(lh);
  }
  free(alist); free(is_t); free(e2);
  return OR_OK;
}

/* ----------------------------------------------------------------------- */
/* Bonded-force coupling: velocity-Verlet MD with the mirror Lennard-Jones   */
/* bond potential (Sec. II D, Eq. (mirror LJ); Ref. Akkermans et al.):       */
/*   V_b(r) = 4 eps ((sig/(2 sc - r))^12 - (sig/(2 sc - r))^6 + 1/4)         */
/*   for sc < r < 2 sc, 0 otherwise (sc = 2^(1/6) sig, the LJ cutoff),       */
/* over every bond of the adjacency table; unit masses; no other force (the  */
/* minimal loop that moves particles between reaction steps instead of the  */
/* re-jitter).  Bonds are made at r < rc = 1.12 < sc, where V_b and its      */
/* force vanish: bonding adds no energy (the paper's thermoneutral          */
/* reaction), and the total energy is conserved by the integrator.          */
/* FP32 contract (identical on the device): for the bond (i, j) at i,       */
/*   d = min_image(x_j - x_i) per component, r2 = (dx dx + dy dy) + dz dz;  */
/*   if r2 > sc^2 (FP32 of the double product):                             */
/*     r = sqrt(r2), s = 2sc - r, q = sig / s, q2 = q q, q6 = (q2 q2) q2,   */
/*     q12 = q6 q6, c = ((24 eps) ((q12 + q12) - q6) / s) / r,              */
/*     F_i += c d (component-wise, bonds in adjacency-row order);           */
/*   r >= 2 sc (a bond torn apart) is an error.                             */
/* One MD step: v += h F; x = wrap(x + dt v); F = F(x); v += h F, with     */
/* h = fl32(dt / 2), each particle's forces taken from the positions of the */
/* same instant.                                                            */
/* ----------------------------------------------------------------------- */
typedef struct {
  float dt, h, sc, sc2, two_sc, sig, e24;
} or_md;

static or_md md_params(double dt, double sig, double eps) {
  or_md m;
  m.dt = (float)dt;
  m.h = (float)(0.5 * dt);
  m.sc = (float)(pow(2.0, 1.0 / 6.0) * sig);
  m.sc2 = (float)((double)m.sc * (double)m.sc);
  m.two_sc = (float)(2.0 * (double)m.sc);
  m.sig = (float)sig;
  m.e24 = (float)(24.0 * eps);
  return m;
}

/* forces on every particle from its bonds (rows of adj, -1 = empty) */
static int md_forces(int32_t n, float L, const float* x, const float* y, const float* z,
                     const int32_t* adj, int32_t B, const or_md* m, float* fx, float* fy,
                     float* fz) {
  const float halfL = 0.5f * L;
  int torn = 0;
#pragma omp parallel for schedule(static) reduction(| : torn)
  for (int64_t i = 0; i < n; ++i) {
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (int32_t b = 0; b < B; ++b) {
      const int32_t j = adj[i * B + b];
      if (j < 0) continue;
      const float dx = min_image(x[j] - x[i], L, halfL);
      const float dy = min_image(y[j] - y[i], L, halfL);
      const float dz = min_image(z[j] - z[i], L, halfL);
      const float r2 = (dx * dx + dy * dy) + dz * dz;
      if (!(r2 > m->sc2)) continue;                 /* V_b = 0 up to sc */
      const float r = sqrtf(r2);
      const float sgap = m->two_sc - r;
      if (!(sgap > 0.0f)) { torn = 1; continue; }
      const float q = m->sig / sgap;
      const float q2 = q * q;
      const float q6 = (q2 * q2) * q2;
      const float q12 = q6 * q6;
#if OR_MUTANT == 22 /* mutant: repulsive sign */
      const float c = -((m->e24 * ((q12 + q12) - q6)) / sgap) / r;
#else
      const float c = ((m->e24 * ((q12 + q12) - q6)) / sgap) / r;
#endif
      ax = ax + c * dx;
      ay = ay + c * dy;
      az = az + c * dz;
    }
    fx[i] = ax;
    fy[i] = ay;
    fz[i] = az;
  }
  return torn ? OR_EINVAL : OR_OK;
}

/* theta MD steps (velocity Verlet) in place. */
int or_md_block(int32_t n, float L, float* x, float* y, float* z, float* vx, float* vy,
                float* vz, const int32_t* adj, int32_t B, double dt, double sig, double eps,
                int32_t theta) {
  const or_md m = md_params(dt, sig, eps);
  const size_t nn = (size_t)(n > 0 ? n : 1);
  float* f = (float*)malloc(sizeof(float) * 3 * nn);
  if (!f) return OR_ENOMEM;
  float *fx = f, *fy = f + nn, *fz = f + 2 * nn;
  int e = md_forces(n, L, x, y, z, adj, B, &m, fx, fy, fz);
  for (int32_t k = 0; k < theta && !e; ++k) {
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] + m.h * fx[i];
      vy[i] = vy[i] + m.h * fy[i];
      vz[i] = vz[i] + m.h * fz[i];
      x[i] = wrap_box(x[i] + m.dt * vx[i], L);
      y[i] = wrap_box(y[i] + m.dt * vy[i], L);
      z[i] = wrap_box(z[i] + m.dt * vz[i], L);
    }
    e = md_forces(n, L, x, y, z, adj, B, &m, fx, fy, fz);
    for (int64_t i = 0; i < n; ++i) {
      vx[i] = vx[i] + m.h * fx[i];
      vy[i] = vy[i] + m.h * fy[i];
      vz[i] = vz[i] + m.h * fz[i];
    }
  }
  free(f);
  return e;
}

/* Total energy in FP64 from the FP32 state: sum v^2 / 2 + sum over bonds
 * (each once) of V_b(r). */
double or_md_energy(int32_t n, float L, const float* x, const float* y, const float* z,
                    const float* vx, const float* vy, const float* vz, const int32_t* adj,
                    int32_t B, double sig, double eps) {
  const double sc = pow(2.0, 1.0 / 6.0) * sig, Ld = L, hl = 0.5 * Ld;
  double e = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    e += 0.5 * ((double)vx[i] * vx[i] + (double)vy[i] * vy[i] + (double)vz[i] * vz[i]);
    for (int32_t b = 0; b < B; ++b) {
      const int32_t j = adj[i * B + b];
      if (j <= i) continue;
      double d[3] = {(double)x[j] - x[i], (double)y[j] - y[i], (double)z[j] - z[i]};
      double r2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        if (d[c] > hl) d[c] -= Ld;
        else if (d[c] < -hl) d[c] += Ld;
        r2 += d[c] * d[c];
      }
      const double r = sqrt(r2);
      if (r <= sc) continue;
      const double q = sig / (2.0 * sc - r), q6 = pow(q, 6.0);
      e += 4.0 * eps * (q6 * q6 - q6 + 0.25);
    }
  }
  return e;
}

/* Initial velocities at temperature temp (unit mass): per component an
 * Irwin-Hall(4) offset of the bytes of word d of the Philox block (0, id, 0,
 * 6) times fl32(sqrt(temp / 21845)) (unit variance per offset). */
void or_md_velocities(int32_t n, float* vx, float* vy, float* vz, uint64_t seed, double temp) {
  const float c = (float)sqrt(temp / 21845.0);
  for (int64_t i = 0; i < n; ++i) {
    int32_t S[3];
    or_ih4_offsets(0u, (uint32_t)i, 6u, seed, S);
    vx[i] = (float)S[0] * c;
    vy[i] = (float)S[1] * c;
    vz[i] = (float)S[2] * c;
  }
}

/* Reaction steps with the MD in between: step s runs theta MD steps and
 * then the reaction step s (random selection).  Log rows (step, id_A, id_T). */
int or_run_md(int32_t n, float L, float* x, float* y, float* z, float* vx, float* vy, float* vz,
              const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
              int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
              int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
              float rc, double p, int32_t exclude_bonded, uint64_t seed,
              uint32_t first_step, uint32_t n_steps, double dt, double sig, double eps,
              int32_t theta, int32_t* log, int64_t log_cap, int64_t* n_log,
              int64_t* stats_per_step) {
  int32_t* sb = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n / 2 + 1));
  if (!sb) return OR_ENOMEM;
  int64_t total = 0;
  int code = OR_OK;
  for (uint32_t k = 0; k < n_steps; ++k) {
    const uint32_t st = first_step + k;
    int e = or_md_block(n, L, x, y, z, vx, vy, vz, adj, B, dt, sig, eps, theta);
    if (e) { code = e; break; }
    int64_t nb = 0;
    e = or_react_step(n, L, x, y, z, type, state, adj, B, type_a, a_min, a_max, d_a, type_t,
                      t_min, t_max, d_t, rc, p, exclude_bonded, seed, st, sb, n / 2 + 1, &nb,
                      stats_per_step ? stats_per_step + (int64_t)k * ST_COUNT : NULL);
    if (e != OR_OK && e != OR_ECAP) { code = e; break; }
    if (e == OR_ECAP) code = OR_ECAP;
    for (int64_t b = 0; b < nb; ++b, ++total)
      if (total < log_cap) {
        log[3 * total] = (int32_t)st;
        log[3 * total + 1] = sb[2 * b];
        log[3 * total + 2] = sb[2 * b + 1];
      }
  }
  *n_log = total;
  free(sb);
  if (code == OR_OK && total > log_cap) return OR_ECAP;
  return code;
}

/* ----------------------------------------------------------------------- */
/* Integer Irwin-Hall(12) offsets of the synthetic initial configuration:    */
/* per dimension S = (sum of 12 uniform bytes) - 1530 (mean 0, variance     */
/* 65535); the bytes come from three Philox blocks with counter              */
/* (step, id, blk, tag), blk = 0..2, words 3d..3d+2 for dimension d.         */
/* ----------------------------------------------------------------------- */
void or_ih12_offsets(uint32_t step, uint32_t id, uint32_t tag, uint64_t seed, int32_t S[3]) {
  uint32_t words[12];
  for (uint32_t blk = 0; blk < 3; ++blk) {
    uint32_t ctr[4] = {step, id, blk, tag};
    or_philox4x32_10(ctr, seed, words + 4 * blk);
  }
  for (int d = 0; d < 3; ++d) {
    int32_t sum = 0;
    for (int w = 0; w < 3; ++w) {
      uint32_t v = words[3 * d + w];
      for (int b = 0; b < 4; ++b) sum += (int32_t)((v >> (8 * b)) & 0xFFu);
    }
    S[d] = sum - 1530;
  }
}

/* ----------------------------------------------------------------------- */
/* Re-jitter between reaction steps: the synthetic stand-in for the MD       */
/* integration that the paper runs between reaction steps (Sec. III: the     */
/* reaction runs every Theta MD steps).  Not part of the paper's method.     */
/* Displacement per dimension d: S = (sum of the 4 bytes of word d) - 510,   */
/* an Irwin-Hall(4) variable on an integer grid with mean 0 and variance     */
/* 21845, scaled by c = fl32(sigma / sqrt(21845)); the words come from one   */
/* Philox block with counter (step, id, 0, tag).                             */
/* ----------------------------------------------------------------------- */
void or_ih4_offsets(uint32_t step, uint32_t id, uint32_t tag, uint64_t seed, int32_t S[3]) {
  uint32_t words[4];
  uint32_t ctr[4] = {step, id, 0u, tag};
  or_philox4x32_10(ctr, seed, words);
  for (int d = 0; d < 3; ++d) {
    int32_t sum = 0;
    for (int b = 0; b < 4; ++b) sum += (int32_t)((words[d] >> (8 * b)) & 0xFFu);
#if OR_MUTANT == 12 /* mutant: off-centre jitter */
    S[d] = sum - 512;
#else
    S[d] = sum - 510;
#endif
  }
}

/* The displacement scale of the re-jitter for a given sigma. */
float or_jitter_scale(double sigma) { return (float)(sigma / sqrt(21845.0)); }

static float wrap_box(float v, float L) {
  if (v < 0.0f) v = v + L;
  if (v >= L) v = v - L;
  return v;
}

void or_jitter(int32_t n, float L, float* x, float* y, float* z, uint64_t seed,
               uint32_t step, double sigma) {
  const float c = or_jitter_scale(sigma);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int32_t S[3];
    or_ih4_offsets(step, (uint32_t)i, 1u, seed, S);
    float dx = (float)S[0] * c, dy = (float)S[1] * c, dz = (float)S[2] * c;
    x[i] = wrap_box(x[i] + dx, L);
    y[i] = wrap_box(y[i] + dy, L);
    z[i] = wrap_box(z[i] + dz, L);
  }
}

/* ----------------------------------------------------------------------- */
/* A run of reaction steps first_step .. first_step+n_steps-1.  Each step s  */
/* jitters the positions with step index s (if sigma > 0) and then reacts.   */
/* Bond log rows: (step, id_A, id_T).  stats_per_step: n_steps x ST_COUNT.   */
/* ----------------------------------------------------------------------- */
static int run_policy(int policy, int32_t n, float L, float* x, float* y, float* z,
                      const int32_t* type,
           int32_t* state, int32_t* adj, int32_t B,
           int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
           int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
           float rc, double p, int32_t exclude_bonded, uint64_t seed,
           uint32_t first_step, uint32_t n_steps, double sigma,
           int32_t* log, int64_t log_cap, int64_t* n_log, int64_t* stats_per_step) {
  int32_t* step_bonds = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n / 2 + 1));
  if (!step_bonds) return OR_ENOMEM;
  int64_t total = 0;
  int rc_code = OR_OK;
  for (uint32_t k = 0; k < n_steps; ++k) {
    uint32_t s = first_step + k;
    if (sigma > 0.0) or_jitter(n, L, x, y, z, seed, s, sigma);
    int64_t nb = 0;
    int64_t* st = stats_per_step ? stats_per_step + (int64_t)k * ST_COUNT : NULL;
    int e = (policy == 1 ? or_react_step_nearest : or_react_step)(
        n, L, x, y, z, type, state, adj, B, type_a, a_min, a_max, d_a, type_t, t_min, t_max,
        d_t, rc, p, exclude_bonded, seed, s, step_bonds, n / 2 + 1, &nb, st);
    if (e != OR_OK && e != OR_ECAP) { rc_code = e; break; }
    if (e == OR_ECAP) rc_code = OR_ECAP;
    for (int64_t b = 0; b < nb; ++b) {
      if (total < log_cap) {
        log[3 * total] = (int32_t)s;
        log[3 * total + 1] = step_bonds[2 * b];
        log[3 * total + 2] = step_bonds[2 * b + 1];
      }
      total++;
    }
  }
  *n_log = total;
  free(step_bonds);
  if (rc_code == OR_OK && total > log_cap) return OR_ECAP;
  return rc_code;
}

int or_run(int32_t n, float L, float* x, float* y, float* z, const int32_t* type,
           int32_t* state, int32_t* adj, int32_t B,
           int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
           int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
           float rc, double p, int32_t exclude_bonded, uint64_t seed,
           uint32_t first_step, uint32_t n_steps, double sigma,
           int32_t* log, int64_t log_cap, int64_t* n_log, int64_t* stats_per_step) {
  return run_policy(0, n, L, x, y, z, type, state, adj, B, type_a, a_min, a_max, d_a, type_t,
                    t_min, t_max, d_t, rc, p, exclude_bonded, seed, first_step, n_steps, sigma,
                    log, log_cap, n_log, stats_per_step);
}

/* or_run with the "nearest" selection of or_react_step_nearest. */
int or_run_nearest(int32_t n, float L, float* x, float* y, float* z, const int32_t* type,
                   int32_t* state, int32_t* adj, int32_t B,
                   int32_t type_a, int32_t a_min, int32_t a_max, int32_t d_a,
                   int32_t type_t, int32_t t_min, int32_t t_max, int32_t d_t,
                   float rc, double p, int32_t exclude_bonded, uint64_t seed,
                   uint32_t first_step, uint32_t n_steps, double sigma,
                   int32_t* log, int64_t log_cap, int64_t* n_log, int64_t* stats_per_step) {
  return run_policy(1, n, L, x, y, z, type, state, adj, B, type_a, a_min, a_max, d_a, type_t,
                    t_min, t_max, d_t, rc, p, exclude_bonded, seed, first_step, n_steps, sigma,
                    log, log_cap, n_log, stats_per_step);
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
