/*
 * polyreact.h -- C ABI of the MI355X (gfx950) reaction-step library.
 *
 * The library implements the bond-creation step of de Buyl & Nies, "A
 * parallel algorithm for step- and chain-growth polymerization in Molecular
 * Dynamics" (arXiv:1409.7498): particles of given type and state that are
 * closer than a cutoff react pairwise with probability p = k*dt*Theta per
 * reaction step; every particle takes at most one new bond per step; bonded
 * partners update their states.  All compute runs in HIP kernels built for
 * gfx950; there is no CPU fallback.
 *
 * Conventions (every entry point):
 *   - returns PR_OK (0) or a negative PR_E* code and never aborts; the text of
 *     the last error of the calling thread is available from pr_last_error();
 *   - argument validation that needs no device data happens before any launch
 *     and leaves every buffer untouched;
 *   - "device" pointers are HIP device allocations (e.g. torch tensors'
 *     data_ptr()), "host" pointers ordinary host memory; sizes are in elements;
 *   - stream arguments are hipStream_t passed as void*; NULL is the default
 *     stream.  Calls that return host-visible results synchronise that stream.
 *
 * Arithmetic contract (identical on every path; the CPU oracle in the test
 * suite implements the same contract independently):
 *   - min-image component: d = p_T - p_A; if (d > L/2) d -= L; else if
 *     (d < -L/2) d += L;  r2 = (dx*dx + dy*dy) + dz*dz, each operation rounded
 *     to FP32, no fused multiply-add; in range iff r2 < fl32(rc*rc);
 *   - draw: Philox4x32-10 (Salmon et al., SC'11) with counter
 *     (step, id_A, id_T, 0) and key seed -> words (w0, w1, w2, w3); accepted
 *     iff w0 < ceil(p * 2^32), i.e. u = w0 * 2^-32 < p (Sec. II, Eq. (4));
 *   - one T per A: the smallest (w1, id_T) among A's retained candidates
 *     (Table I, steps 3-5); one A per T: the smallest (w2, id_A) among the A's
 *     that chose it (Table I, steps 6-7); states updated simultaneously after
 *     all choices (Table I, step 9; Eq. (2));
 *   - bonds of one step are reported in increasing id_A order.
 */
#ifndef POLYREACT_H
#define POLYREACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_OK 0
#define PR_EINVAL (-1)          /* bad size, box, cutoff, probability or position */
#define PR_ERULE_AMBIGUOUS (-2) /* type_a == type_t and the two state windows overlap */
#define PR_ECAP (-3)            /* an output or adjacency capacity was too small */
#define PR_ENOMEM (-4)          /* device allocation failed */
#define PR_EHIP (-5)            /* a HIP runtime call failed (the handle is unusable) */
#define PR_EBUSY (-6)           /* serving: request does not fit the memory budget now */
#define PR_ENOTFOUND (-7)       /* serving: unknown ticket */
#define PR_ECANCELED (-8)       /* serving: the request was cancelled */

/* Selection policies of a rule.
 * PR_POLICY_RANDOM: the paper's algorithm (Sec. III, Table I): every
 *   candidate pair is accepted with probability p, each A picks one accepted
 *   T at random, each T one of the A's that picked it.
 * PR_POLICY_NEAREST: the selection of LAMMPS fix bond/create (Sec. IV A):
 *   every particle keeps its closest candidate partner (key (r^2, partner id):
 *   equal distances go to the lower id); a pair whose particles keep each
 *   other is tested once, u < p with the pair's draw (word 0 of the counter
 *   (step, id_A, id_T, 0)), and bonds if it passes.  Already bonded pairs
 *   (exclude_bonded) are no candidates at all.  Counters: drawn = mutual
 *   pairs tested, accepted = bonds, excluded = in-range pairs already bonded. */
#define PR_POLICY_RANDOM 0
#define PR_POLICY_NEAREST 1

/* One reaction rule, T^t + A^a -> T^(t+d_t)-A^(a+d_a) (Sec. II, Eq. (2)).
 * A particle is eligible for the A role iff type == type_a and
 * a_min <= state <= a_max (the paper's s_min^A, Sec. III); for the T role iff
 * type == type_t and t_min <= state <= t_max.  Roles are decided on the state
 * before the step.  rc: reaction cutoff (strict, r < rc).  p = k*dt*Theta in
 * [0, 1] (Sec. II, Eqs. (3)-(4)).  exclude_bonded = 1: a pair that is already
 * bonded (id_T present in the A's adjacency row) is never a candidate.
 * policy: PR_POLICY_RANDOM (0) or PR_POLICY_NEAREST (1), else PR_EINVAL. */
typedef struct pr_rule {
  int32_t type_a, a_min, a_max, d_a;
  int32_t type_t, t_min, t_max, d_t;
  float rc;
  int32_t exclude_bonded;
  double p;
  int32_t policy;
} pr_rule;

/* Per-step counters.  in_rc: eligible (A, T) pairs with r2 < rc2; drawn: of
 * those, pairs whose draw passed; excluded: drawn pairs already bonded;
 * accepted = drawn - excluded (the retained candidates); proposals: A's with a
 * retained candidate; bonds: bonds created; adj_overflow: adjacency appends
 * that found the row full (the bond and the states are still applied). */
typedef struct pr_stats {
  int64_t a_elig, t_elig, in_rc, drawn, excluded, accepted, proposals, bonds, adj_overflow;
} pr_stats;

/* Text of the calling thread's last error (static storage, never NULL). */
const char* pr_last_error(void);

/* Library version string. */
const char* pr_version(void);

/* The per-pair, per-step acceptance probability p = k * dt * Theta of a rate
 * constant k, an MD time step dt and a reaction interval of Theta MD steps
 * (Sec. II, Eqs. (3)-(4)); the method assumes p << 1.  *warn (may be NULL)
 * receives 1 when p > 0.1 (then the single draw per pair and interval is a
 * coarse stand-in for the rate: two reactive events in one interval are no
 * longer rare), else 0.  Negative or non-finite inputs return -1.  Host
 * only. */
double pr_p_from_rate(double k, double dt, double theta, int32_t* warn);

/* The library's draws: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11)
 * of n counters under one key, computed on the device by the same code as
 * the acceptance test of Eq. (4) (counter (step, id_A, id_T, 0), key = the
 * system's seed) and the re-jitter.  ctr, out: device arrays of 4 n uint32
 * (counter words 0-3, output words 0-3; out may equal ctr).  0 <= n <= 2^30
 * (else PR_EINVAL).  Asynchronous on stream. */
int pr_draws(const uint32_t* ctr, int64_t n, uint64_t key, uint32_t* out, void* stream);

/* ------------------------------------------------------------------------ */
/* One reaction step on caller-owned device arrays (Table I, steps 1-9).     */
/*                                                                          */
/* n particles in the periodic cube [0, L)^3.  Device arrays, indexed by     */
/* particle id 0..n-1: x, y, z (FP32, each in [0, L)), type, state (in/out),  */
/* adj (in/out, n x B row-major, -1 = empty slot; new partners are written   */
/* into the first empty slot of each row).  step and seed key the draws.     */
/* bonds (device, 2*cap int32): (id_A, id_T) pairs in increasing id_A order; */
/* cap >= n/2 is required (at most one bond per particle).  n_bonds (host)   */
/* receives the count; st (host, may be NULL) the counters.                  */
/* Errors: PR_EINVAL (n < 0 or n > 2^30, B < 1, rc <= 0, L <= 2 rc, p outside */
/* [0,1], or a                                                              */
/* position that is NaN or outside [0, L) -- detected on the device before   */
/* any write), PR_ERULE_AMBIGUOUS, PR_ECAP (cap < n/2: nothing written; or    */
/* an adjacency row was full: the step is complete except for the missing     */
/* adjacency entries, counted in st->adj_overflow).  Synchronises stream.    */
/* ------------------------------------------------------------------------ */
int pr_react_step(int32_t n, float L, const float* x, const float* y, const float* z,
                  const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                  const pr_rule* rule, uint64_t seed, uint32_t step, int32_t* bonds,
                  int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream);

/* Several concurrent rules in one step (1 <= nrules <= 4, each validated as
 * for pr_react_step, all with PR_POLICY_RANDOM).  The paper proposes such
 * concurrent reactions without a procedure (Sec. III B); the library
 * generalises Table I: every rule contributes its candidates, each with its
 * own draw (counter (step, id_A, id_T, tag), tag 0 for rule 0 and 0x100 + r
 * for rule r); each particle, as an A, picks among its accepted candidates of
 * all rules the smallest (w1, id_T) (the lower rule on a tie); each T keeps
 * the smallest (w2, id_A) of the pairs that picked it; a particle that then
 * wins both as the A of one pair and the T of another keeps the pair with
 * the smaller (w3, partner id, rule), and a pair bonds only if both of its
 * particles keep it.  Every particle still takes at most one new bond.  With
 * one rule the result is pr_react_step's.  A particle may hold the A role of
 * one rule and the T role of another.  bonds: 3 * cap int32 (id_A, id_T,
 * rule) in increasing id_A order; the rest as pr_react_step. */
int pr_react_step_multi(int32_t n, float L, const float* x, const float* y, const float* z,
                        const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                        const pr_rule* rules, int32_t nrules, uint64_t seed, uint32_t step,
                        int32_t* bonds, int32_t cap, int32_t* n_bonds, pr_stats* st,
                        void* stream);

/* pr_react_step for callers that cannot allocate device memory: tight serving
 * loops and harnesses that forbid hipMalloc (like pr_react_step it
 * synchronises its stream, so it is not itself meant for graph capture).  Same
 * arguments, arithmetic, results and errors as pr_react_step, but no call to
 * hipMalloc, hipFree or any allocating routine: the step's scratch is one
 * fixed region of device memory per GPU (24 MiB, a file-scope device array
 * of the library, held until the process ends).  n is limited to 32768
 * particles (PR_EINVAL beyond, with nothing written); every such call on one
 * GPU shares the region and clears what it needs at its start.  Calls on one
 * GPU are serialised by the library for the duration of the call (it
 * synchronises stream before returning); launches that other code makes into
 * the region concurrently would race.  Synchronises stream. */
int pr_react_step_noalloc(int32_t n, float L, const float* x, const float* y, const float* z,
                          const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                          const pr_rule* rule, uint64_t seed, uint32_t step, int32_t* bonds,
                          int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream);

/* ------------------------------------------------------------------------ */
/* Resident system: particle state kept in device memory across steps.      */
/* ------------------------------------------------------------------------ */
typedef struct pr_sys pr_sys;

/* Creates a system of n particles (1 <= n <= 2^30) in the cube [0, L)^3 with
 * adjacency width B, reaction rule and draw seed.  log_cap: capacity of the device bond log
 * in bonds (0 = n).  The handle owns all its device memory; stream (may be
 * NULL) is the stream every later call on the handle uses. */
int pr_sys_create(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule,
                  uint64_t seed, int64_t log_cap, void* stream);

/* As pr_sys_create, with the brick edge chosen: the storage is sorted by
 * bricks of brick^3 coarse cells (brick in 1..6, 0 = 4; clamped to nc - 2
 * for small boxes, nc = coarse cells per side) and the sweep runs one
 * workgroup per brick.  Larger bricks mean fewer workgroups (each staging a
 * larger region); they suit large systems with few A's.  A tuning parameter
 * only: every result is identical for every brick.  PR_EINVAL for brick
 * outside 0..6. */
int pr_sys_create_ex(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule,
                     uint64_t seed, int64_t log_cap, void* stream, int32_t brick);

/* A resident system with several concurrent rules (as pr_react_step_multi;
 * the coarse grid is sized for the largest cutoff).  The bond log rows stay
 * (step, id_A, id_T).  Checkpoints and kinetics counters take one rule
 * (PR_EINVAL here); batches and the server take one rule per replica. */
int pr_sys_create_multi(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rules,
                        int32_t nrules, uint64_t seed, int64_t log_cap, void* stream,
                        int32_t brick);

/* The handle's geometry: coarse cells per side, effective brick edge and
 * number of bricks (= sweep workgroups once sorted).  Any output may be NULL. */
int pr_sys_geometry(pr_sys* s, int32_t* nc, int32_t* brick, int32_t* nbricks);
void pr_sys_destroy(pr_sys* s);

/* Loads a configuration indexed by particle id: x, y, z, type, state and adj
 * (n x B).  on_device = 1: the pointers are device memory, 0: host memory.
 * Clears the bond log and the counters.  PR_EINVAL on a position outside
 * [0, L) or NaN (detected on the device, nothing loaded).  Synchronises. */
int pr_sys_load(pr_sys* s, const float* x, const float* y, const float* z, const int32_t* type,
                const int32_t* state, const int32_t* adj, int32_t on_device);

/* Generates the synthetic jittered-lattice configuration on the device:
 * kind 0 = step growth (5% crosslinkers type 1 state 4, else type 0 state 2),
 * kind 1 = chain growth (0.1% active ends state 2, else free monomers state 0);
 * lattice displacement sigma0; gen_seed keys the draws.  Same recipe as the
 * host generator of the package.  Clears the bond log and counters. */
int pr_sys_generate(pr_sys* s, int32_t kind, uint64_t gen_seed, double sigma0);

/* Runs reaction steps first_step .. first_step + n_steps - 1.  Each step
 * first moves every particle by the re-jitter (when sigma > 0) -- the
 * stand-in for the MD integration between reaction steps: per dimension an
 * Irwin-Hall(4) offset (the four bytes of one Philox4x32-10 word of the block
 * (step, id, 0, 1), summed, minus 510) times fl32(sigma / sqrt(21845)), then
 * a single periodic wrap -- and then reacts.
 * Bonds are appended to the device bond log as (step, id_A, id_T) rows and
 * counters to the per-step counter log.  Asynchronous on the handle's stream;
 * errors found on the device are reported by the next synchronising call. */
int pr_sys_run(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma);

/* Phase timing: like pr_sys_run, but every step is launched directly (no
 * graph) and the call synchronises; ms[0..4] receive the summed GPU time from
 * the start of each step to the start of its pair sweep (the binning of the
 * A particles), of whole steps (a spatial sort excluded), of the pair-sweep
 * kernels alone (their own start and end, stamped by hipExtLaunchKernel), of
 * the spatial sorts that fell due during the run, and (as a float) the number
 * of those sorts, measured with HIP events on the handle's stream. */
int pr_sys_run_timed(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma, float* ms);

/* Captures, without running anything, the HIP graphs that a following
 * pr_sys_run of n_steps steps with this sigma will replay, so that the run
 * itself pays no capture (a latency-sensitive caller, a timed region).  A run
 * of any length replays graphs: one per segment of steps between spatial
 * sorts, cached by shape.  No effect when graphs are off.  Synchronous. */
int pr_sys_prepare(pr_sys* s, uint32_t n_steps, double sigma);

/* Bonded-force coupling: instead of the re-jitter, every reaction step of
 * pr_sys_run is preceded by theta steps of velocity-Verlet MD (time step dt,
 * unit masses) under the mirror Lennard-Jones bond potential of every bond in
 * the adjacency table (Sec. II D, Eq. (mirror LJ)):
 *   V_b(r) = 4 eps ((sig / (2 sc - r))^12 - (sig / (2 sc - r))^6 + 1/4) for
 *   sc < r < 2 sc, sc = 2^(1/6) sig, and 0 below sc,
 * and no other force.  Bonds are made at r < rc <= sc, where V_b vanishes,
 * so a reaction step adds no energy (the paper's thermoneutral bonding).
 * FP32 arithmetic in a fixed order (forces in adjacency-row order; per MD
 * step v += (dt/2) F, x = wrap(x + dt v), F = F(x), v += (dt/2) F).
 * Velocities are (re)initialised at temperature temp: per component an
 * Irwin-Hall(4) offset of the bytes of word d of the Philox block (0, id,
 * 0, 6) under vseed, times fl32(sqrt(temp / 21845)).  pr_sys_run then needs
 * sigma = 0.  theta = 0 switches back to the re-jitter.  A bond stretched to
 * 2 sc or beyond is reported as PR_EINVAL by the next synchronising call.
 * Call after pr_sys_load / pr_sys_generate.  Synchronises. */
int pr_sys_set_md(pr_sys* s, int32_t theta, double dt, double sig, double eps, double temp,
                  uint64_t vseed);

/* The bonded-force kernel's FP32 square root (correctly rounded, as IEEE
 * sqrt) on n device values, each positive and normal (others: unspecified).
 * in, out: device arrays (may be equal); 0 <= n <= 2^30.  Asynchronous. */
int pr_sqrt_rn(const float* in, float* out, int64_t n, void* stream);

/* Velocities in particle-id order (host arrays of n floats; PR_EINVAL when
 * pr_sys_set_md was never called).  Synchronises. */
int pr_sys_read_velocities(pr_sys* s, float* vx, float* vy, float* vz);

/* The re-jitter alone for steps first_step .. first_step + n_steps - 1: every
 * particle moves exactly as the re-jitter of pr_sys_run's steps would move it
 * (the stand-in for the MD integration between reaction steps), and no
 * reaction happens (nothing is logged; a later run continues from the moved
 * configuration with the next step numbers).  kernel_ms (host, may be NULL):
 * receives the summed GPU time of the re-jitter kernels, stamped at each
 * kernel's own start and end (the call then synchronises).  Used to separate
 * the reaction step's own cost from the fused step's. */
int pr_sys_jitter(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma,
                  float* kernel_ms);

/* Kinetics counters of the current configuration: the quantities the
 * paper's rate equations are built from (Sec. II B-C), counted on the device
 * so that they can be followed at any system size.
 *   pop[s]   particles of type type_a in state s, s = 0 .. nstate-1 (the
 *            populations [X_s] of Eq. (12); [M], [P*] of Eqs. (5)-(10) when
 *            A and T share a type); other states are not counted;
 *   pairs[s] summed over the A-eligible particles in state s: the T-eligible
 *            particles within the cutoff (the step's own FP32 test) that are
 *            not bonded to them when the rule excludes bonded pairs, so that
 *            pairs[s] / pop[s] is <N_{X^s E^0}> of Eq. (13), or <N_{P* M}>
 *            of the chain-growth rate k_c;
 *   hist[b]  those pairs by distance: bin b holds e2[b] <= r2 < e2[b + 1],
 *            e2[b] = fl32((rc b / nbins)^2) with the product in double, the
 *            last bin ending at the cutoff (a pair distribution function up
 *            to rc, whose integral is <N>).
 * Host arrays of nstate (1..64) and nbins (0..256; hist may be NULL when 0)
 * elements.  Nothing of the system changes.  Synchronises. */
int pr_sys_kinetics(pr_sys* s, int32_t nstate, int64_t* pop, int64_t* pairs, int32_t nbins,
                    int64_t* hist);

/* Copies the current configuration out in particle-id order (host or device
 * pointers per on_device; any pointer may be NULL to skip).  Synchronises;
 * returns a pending device error, if any. */
int pr_sys_read(pr_sys* s, float* x, float* y, float* z, int32_t* state, int32_t* adj,
                int32_t on_device);

/* Copies the bond log out: up to cap rows of (step, id_A, id_T) int32 into
 * host memory, ordered by step and, within a step, by id_A (Table I, step 9);
 * *n receives the total logged (PR_ECAP if it exceeded the log capacity; rows
 * beyond it were dropped).  The order is made on the device, in place: the
 * log in HBM stays in that order and later steps append after it.  Takes
 * temporary device memory (about 24 bytes per logged row) from the stream's
 * memory pool.  Synchronises. */
int pr_sys_bonds(pr_sys* s, int32_t* out, int64_t cap, int64_t* n);

/* Copies the per-step counters of the steps run since the last load (at most
 * cap records) into host memory; *n receives their number.  Synchronises. */
int pr_sys_stats(pr_sys* s, pr_stats* out, int64_t cap, int64_t* n);

/* Checkpoint of a resident system into host memory: the configuration in
 * particle-id order (x, y, z, type, state, adjacency), the bond log and the
 * per-step counters, with the handle's n, B, L, rule and seed.  *bytes
 * receives the size needed; buf == NULL only asks for it.  PR_ECAP when cap
 * is smaller (nothing written) or when the bond log has overflowed its
 * capacity (a checkpoint would be incomplete).  Synchronises. */
int pr_sys_checkpoint(pr_sys* s, void* buf, int64_t cap, int64_t* bytes);

/* Restores a checkpoint into a handle created with the same n, B, L, rule
 * and seed (brick edge, sort period and log capacity may differ).  Runs
 * continued from it give the bonds, counters and configuration of the
 * uninterrupted run: the draws depend only on (step, ids) and the seed.
 * PR_EINVAL for another system's or a malformed checkpoint, PR_ECAP if its
 * bonds exceed the log capacity (in these cases the handle is unchanged);
 * PR_EINVAL for a position outside [0, L) (the handle then holds no valid
 * configuration).  Synchronises. */
int pr_sys_restore(pr_sys* s, const void* buf, int64_t bytes);

/* Dense-pass tuning of a handle: sort_period = steps between spatial re-sorts
 * of the particle storage (default 64; 0 = never sort).  Results never depend
 * on it: every selection is a minimum over keys, whatever the storage order. */
int pr_sys_set_sort_period(pr_sys* s, int32_t sort_period);

/* on = 1 (default): pr_sys_run replays its steps from captured HIP graphs,
 * one per segment (a spatial sort when one is due, then the steps up to the
 * next sort; 32 steps at a time without sorting), cached by segment shape;
 * on = 0: every kernel is launched directly.  Results are identical. */
int pr_sys_set_graphs(pr_sys* s, int32_t on);

/* Fused binning (Table I step 1, the candidate search): enable = 1 (default)
 * lets a handle on sorted storage with one rule, the random selection and no
 * MD skip the binning kernel: each step's sweep bins the A's of the next step
 * (at their positions re-jittered once more) into cell buckets of its own,
 * and the resolve drops or adds the A's whose roles its bonds change, so a
 * step is two kernels.  The buckets are allocated on the first run that can
 * use them (about 2 x 160 bytes per cell and 40 per particle) and filled by
 * the spatial sort; they hold the A's of one reaction step, so a run that
 * does not continue the previous one (another first_step or sigma, after
 * pr_sys_jitter or pr_sys_set_md) sorts first.  enable = 0: the binning
 * kernel runs before every sweep.  Results are identical.  PR_EINVAL for
 * enable outside {0, 1}. */
int pr_sys_set_fused_binning(pr_sys* s, int32_t enable);

/* *active = 1 when the handle's next step uses fused binning (as the last run
 * left it), else 0. */
int pr_sys_fused_binning(pr_sys* s, int32_t* active);


/* Bandwidth probe: copies bytes from src to dst (device memory, bytes a
 * multiple of width) with the library's own copy kernel, each lane moving
 * one element of width 4, 8 or 16 bytes per iteration (a wavefront reads and
 * writes 64 * width contiguous bytes), 2048 workgroups striding over the
 * buffer.  kernel_ms (host, may be NULL): the kernel's own duration (the call
 * then synchronises).  Measures the HBM ceiling the reaction kernels are
 * compared with and calibrates the profiler's byte counters.  PR_EINVAL for
 * another width, a negative or unaligned size, or NULL buffers. */
int pr_stream_copy(const void* src, void* dst, int64_t bytes, int32_t width, void* stream,
                   float* kernel_ms);

/* ------------------------------------------------------------------------ */
/* Batched ensemble: many independent replicas (uneven sizes, step or chain  */
/* growth, each with its own rule, seed and rate) stepped in lockstep.  Each */
/* kernel launch covers every replica (a map spreads one grid over them) and */
/* blocks of steps -- one spatial sort and then sort_period steps -- replay  */
/* from one captured HIP graph.  Every replica's bonds, states, positions    */
/* and counters equal those of a pr_sys run of that replica alone (the same  */
/* arithmetic contract; results never depend on launch grouping).            */
/* ------------------------------------------------------------------------ */
typedef struct pr_replica_desc {
  int32_t n;          /* particles (>= 1) */
  float L;            /* periodic cube [0, L)^3 */
  int32_t B;          /* adjacency width */
  pr_rule rule;       /* reaction rule */
  uint64_t seed;      /* draw seed of the reaction steps and the re-jitter */
  int32_t gen_kind;   /* synthetic start: 0 step growth, 1 chain growth (as pr_sys_generate) */
  uint64_t gen_seed;  /* generator seed */
  double gen_sigma0;  /* lattice displacement of the generator */
  int64_t log_cap;    /* bond-log capacity in bonds (0 = n) */
  int32_t brick;      /* brick edge in cells, 1..6 (0 = 4): see pr_sys_create_ex */
} pr_replica_desc;

typedef struct pr_batch pr_batch;

/* Creates n_rep replicas (each validated like pr_sys_create) and generates
 * their configurations on the device.  The handle owns all device memory;
 * stream (may be NULL) is used by every later call.  Synchronises. */
int pr_batch_create(pr_batch** out, const pr_replica_desc* reps, int32_t n_rep, void* stream);
void pr_batch_destroy(pr_batch* b);

/* Runs steps first_step .. first_step + n_steps - 1 of every replica (each
 * step: re-jitter with sigma, then the reaction step), all replicas in the
 * same launches, blocks of sort_period (64) steps replayed from one graph.
 * Asynchronous on the handle's stream. */
int pr_batch_run(pr_batch* b, uint32_t first_step, uint32_t n_steps, double sigma);

/* The same steps as a plain per-replica launch loop: replica after replica,
 * every kernel launched directly from the host (no graph, no batching).
 * The reference point for the batched run; results are identical. */
int pr_batch_run_loop(pr_batch* b, uint32_t first_step, uint32_t n_steps, double sigma);

/* Per-replica results, as pr_sys_bonds, pr_sys_read and pr_sys_stats
 * (rep in [0, n_rep), else PR_EINVAL).  Synchronise. */
int pr_batch_bonds(pr_batch* b, int32_t rep, int32_t* out, int64_t cap, int64_t* n);
int pr_batch_read(pr_batch* b, int32_t rep, float* x, float* y, float* z, int32_t* state,
                  int32_t* adj, int32_t on_device);
int pr_batch_stats(pr_batch* b, int32_t rep, pr_stats* out, int64_t cap, int64_t* n);
/* pr_sys_kinetics of one replica. */
int pr_batch_kinetics(pr_batch* b, int32_t rep, int32_t nstate, int64_t* pop, int64_t* pairs,
                      int32_t nbins, int64_t* hist);


/* Device bytes a resident system of this description allocates for a run of
 * n_steps steps (the admission measure of the server).  PR_EINVAL as
 * pr_sys_create. */
int pr_footprint(const pr_replica_desc* r, uint32_t n_steps, int64_t* bytes);

/* Autotuner of the brick edge: for every brick edge 1..6 that gives a
 * distinct brick count, creates the replica with that edge -- copies = 1: one
 * system (pr_sys_create_ex); copies > 1: a batch of `copies` identical
 * replicas (pr_batch_create), the context of a replica in a full batch --
 * generates it, runs one untimed block of 64 steps (first sort, graph
 * capture) and times n_steps more steps (use a multiple of 64) with HIP
 * events on stream.  *best receives the fastest edge, us[0..5] (may be NULL)
 * the microseconds per replica-step of edges 1..6 (-1 where not timed).
 * Allocates and frees one candidate at a time; synchronises stream.  Errors
 * as pr_sys_create_ex / pr_batch_create and the runs. */
int pr_autotune(const pr_replica_desc* r, uint32_t n_steps, double sigma, int32_t copies,
                void* stream, int32_t* best, float* us);

/* pr_autotune with a cache file (host text, one line per tuned geometry: the
 * coarse cells per side, copies and adjacency width, the choice and the
 * times).  A hit returns the stored choice and times without running
 * anything; a miss tunes and appends a line.  cache_path NULL: no cache.
 * PR_EINVAL if the file cannot be appended to. */
int pr_autotune_cached(const pr_replica_desc* r, uint32_t n_steps, double sigma, int32_t copies,
                       void* stream, const char* cache_path, int32_t* best, float* us);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with continuous batching.  Requests (a replica   */
/* description, a number of steps and the re-jitter sigma) queue in arrival */
/* order; a worker thread admits the head of the queue as soon as a slot and */
/* its HBM footprint (pr_footprint) are free, keeps the admitted replicas    */
/* resident, and advances all of them together, rounds of up to 64 steps in */
/* the batched launches (each replica takes part in the steps it has left). */
/* A finished replica is retired by a second thread on its own stream (its  */
/* results moved to host memory through pinned staging, its device memory  */
/* freed) while the worker launches the next round, so later requests are  */
/* admitted while others still run.                                         */
/* Each result equals the replica run alone (pr_sys_run).                    */
/* ------------------------------------------------------------------------ */
typedef struct pr_server pr_server;

typedef struct pr_server_info {
  int64_t budget, used;            /* HBM budget and bytes held by admitted replicas */
  int64_t queued, active, done, failed;
  int64_t rounds;                  /* batched rounds launched */
  double busy_s;                   /* GPU time of those rounds (HIP events) */
  double admit_s, finish_s;        /* time creating replicas (worker) / retiring them (finisher) */
  double launch_s, wait_s;         /* worker time launching rounds / waiting for their end */
} pr_server_info;

/* hbm_budget: bytes the admitted replicas may hold together; max_slots:
 * replicas resident at once.  stream: NULL = the server creates its own.
 * Starts the worker and finisher threads (on the calling thread's current
 * device). */
int pr_server_create(pr_server** out, int64_t hbm_budget, int32_t max_slots, void* stream);
/* Stops admitting, lets the worker finish its current round, cancels what
 * is queued, frees everything. */
void pr_server_destroy(pr_server* s);

/* Queues a request and returns its ticket.  PR_EINVAL on an invalid
 * description; PR_EBUSY if its footprint exceeds the whole budget (it could
 * never be admitted).  Thread-safe. */
int pr_server_submit(pr_server* s, const pr_replica_desc* r, uint32_t n_steps, double sigma,
                     uint64_t* ticket);

/* Request status: 0 queued, 1 running, 2 done, 3 failed (*code: its error);
 * latency_s: completion minus submission time (seconds, steady clock; valid
 * when done).  timeout_s > 0 waits up to that long for completion, 0 does
 * not wait.  PR_ENOTFOUND for an unknown or released ticket. */
int pr_server_wait(pr_server* s, uint64_t ticket, double timeout_s, int32_t* status,
                   int32_t* code, double* latency_s);

/* pr_server_wait without waiting. */
int pr_server_poll(pr_server* s, uint64_t ticket, int32_t* status, int32_t* code,
                   double* latency_s);

/* Cancels a request.  A queued one fails at once with code PR_ECANCELED; a
 * running one is retired, without results, when its current round of steps
 * ends (then status 3, code PR_ECANCELED).  PR_EBUSY if it has already
 * finished (its results stand), PR_ENOTFOUND for an unknown ticket.
 * Thread-safe. */
int pr_server_cancel(pr_server* s, uint64_t ticket);

/* Results of a finished request (host memory), as pr_sys_bonds, pr_sys_read
 * (on_device = 0) and pr_sys_stats; PR_EBUSY while it is not done. */
int pr_server_bonds(pr_server* s, uint64_t ticket, int32_t* out, int64_t cap, int64_t* n);
int pr_server_read(pr_server* s, uint64_t ticket, float* x, float* y, float* z, int32_t* state,
                   int32_t* adj);
int pr_server_stats(pr_server* s, uint64_t ticket, pr_stats* out, int64_t cap, int64_t* n);
/* Forgets a finished request (frees its host results). */
int pr_server_release(pr_server* s, uint64_t ticket);
int pr_server_info_get(pr_server* s, pr_server_info* out);

#ifdef __cplusplus
}
#endif
#endif /* POLYREACT_H */
