// common.hpp -- device-side data layout shared by the kernels and the host
// runtime of the reaction-step library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pr {

// A-role particles are binned into a coarse grid whose cell width is at least
// twice the cutoff, so that the partners of a particle lie in the 2x2x2 block
// of cells nearest to it.  Each cell keeps up to kCellCap records in a fixed
// bucket; records beyond that go to an overflow list every sweep also scans.
constexpr int kCellCap = 8;
constexpr unsigned long long kEmpty = ~0ull;
constexpr int kThreads = 256;       // workgroup size of the per-particle kernels
constexpr int kPrepRoles = 16;      // role bytes a prep thread scans for A's
constexpr int kFinThreads = 1024;   // the single-workgroup finishing kernels
constexpr int kSortLds = 4096;      // bonds of a stateless step sorted in LDS up to this
constexpr int kStatsPerStep = 9;    // pr_stats fields
constexpr int kGroup = 256;         // sweep workgroups closed by one closing workgroup
constexpr int kPart = 8;            // partial counters per closing workgroup and step
constexpr int kWgOut = 9;           // per sweep workgroup counters (see WgOut)
constexpr int kRetCap = 32;         // retained pairs a sweep workgroup hands to the resolve
constexpr int kWinCap = 16;         // bonds a resolve workgroup stages in place
constexpr int kAdjStage = 4;        // adjacency rows up to this width travel with A records
// Spatially sorted storage: particles are kept ordered by "brick" (a block of
// bs^3 coarse cells); one sweep workgroup owns a brick and stages the A
// records of the brick plus one halo cell layer in LDS.
constexpr int kMaxBrick = 6;
constexpr int kDefaultBrick = 4;
constexpr int kStageCells = (kMaxBrick + 2) * (kMaxBrick + 2) * (kMaxBrick + 2);
static_assert(kStageCells <= 2 * kThreads, "the sweep stages two region cells per thread");
// bricks up to this edge take the sweep variant with one region cell per thread
constexpr int kOneCellBrick = 4;
constexpr int kStageCells1 = (kOneCellBrick + 2) * (kOneCellBrick + 2) * (kOneCellBrick + 2);
static_assert(kStageCells1 <= kThreads, "one region cell per thread");
static_assert((kMaxBrick + 1) * (kMaxBrick + 1) * (kMaxBrick + 1) + 1 <= 6 * 64,
              "the per-brick sort scan takes up to six bins per lane");
constexpr int kStageRecs = 256;
constexpr int kTPass = 768;         // particles a sweep workgroup holds per pass (3 per thread)
constexpr int kQueue = 512;         // in-range pairs queued per pass
constexpr int32_t kMaxParticles = 1 << 30;  // byte offsets of 4-byte fields fit in 32 bits
constexpr int kMaxRules = 4;        // concurrent rules of one system
constexpr int kKinMaxState = 64;    // kinetics counters: states per call
constexpr int kKinMaxBins = 256;    // kinetics counters: distance bins per call
constexpr int kKinStride = 2 * kKinMaxState + kKinMaxBins;  // one slice of kinetics counters
constexpr int kKinSlices = 64;      // slices the kinetics workgroups spread their sums over

enum WgOut { kOutTElig = 0, kOutInRc, kOutDrawn, kOutExcl, kOutRet, kOutProp, kOutBonds, kOutLost,
             kOutAElig };

// Device control block.  Steps are launched in blocks of K steps; the kernels
// of step k of a block use step0 + k and parity (par0 + k) & 1, so a captured
// graph of a block can be replayed: its last kernel advances step0 and par0.
struct Ctl {
  uint32_t step0;      // reaction step of the block's first step (draw counter word 0)
  uint32_t par0;       // parity of the block's first step (buffers used per step)
  int32_t err;         // first device-detected error (0 = none)
  uint32_t set;        // which of the two storage sets holds the particles
  uint32_t ovf_n[2];   // A records beyond their cell bucket, by parity
  uint32_t ret_ovf[2];    // retained pairs beyond kRetCap (the resolve then re-enumerates)
  uint32_t nwin_ovf[2];   // bonds beyond kWinCap, by parity
  uint32_t stats_n0;   // counter-log index of the block's first step
  uint64_t log_n;      // rows appended to the bond log (may exceed capacity)
  uint32_t fovf_n[3];  // fused binning: A records beyond their bucket, by step mod 3
};

struct RuleD {
  int32_t type_a, a_min, a_max, d_a;
  int32_t type_t, t_min, t_max, d_t;
  int32_t exclude;
  int32_t policy;  // PR_POLICY_RANDOM / PR_POLICY_NEAREST
};

// One of several concurrent rules: its windows and deltas, squared cutoff,
// acceptance threshold and the draw tag (counter word 3).
struct RuleX {
  RuleD r;
  float rc2;
  uint32_t tag;
  unsigned long long thresh;
};

// Particle arrays of one storage set, slot order.  Positions have two
// buffers: a step reads parity p and writes the jittered positions to p ^ 1.
struct Arr {
  float *x[2], *y[2], *z[2];
  int32_t *typ, *st, *adj, *id;  // id == nullptr: slot == id
  uint8_t* role;                 // kRoleT / kRoleA / 0 from (type, state) and the rule
  float *vx, *vy, *vz;           // velocities (bonded-force coupling only; else null)
};

enum Role : uint8_t { kRoleNone = 0, kRoleT = 1, kRoleA = 2 };
// With several rules the role byte is a mask: bit r = T of rule r, bit 4 + r =
// A of rule r.
constexpr uint8_t kMaskT = 0x0F, kMaskA = 0xF0;

// Everything a kernel needs, passed by value as the kernel argument.
struct Dev {
  Arr set[2];           // storage sets (the sort writes the other one)
  // A grid: per-cell counts by parity; bucket records (x, y, z, id), the
  // A's slot and (rows of width <= kAdjStage) its adjacency row; overflow
  // records and slots
  uint32_t* cnt[2];
  float4 *rec, *ovf[2];
  int32_t *rsa, *ovf_sa[2];
  int4* radj;
  // selection: per-id minimum key (w1, id_T) of the A side; the resolve
  // empties the key it reads back as its own
  unsigned long long* slotA;
  // per sweep workgroup, by parity: counters and retained pairs
  // (id_A, slot_A, slot_T, id_T) with their w2 words
  int32_t* wgo[2];
  int4* wge[2];
  uint32_t* wgk[2];
  uint8_t* tflag;       // per slot: this T has a retained pair in the current step
  int2* tnear;          // nearest policy, per T id: (id of its closest A, the T's slot),
                        // written in the step for every T with a candidate
  int2* wgw[2];         // staged bonds (id_A, id_T), kWinCap per workgroup, by parity
  int2* wov[2];         // staged bonds beyond kWinCap (capacity n/2 + 1 each)
  int32_t* abst[2];     // per prep workgroup: A's binned, by parity
  // spatial sort: bricks, and within a brick its A's, then its (bs + 1)^3
  // "dual cells" (nd bins per brick): per-bin counts, offsets within the
  // brick, and the rank of every particle within its bin
  int32_t* bstart;      // nbricks + 1 slot offsets
  uint32_t* bcnt;
  uint32_t *dcnt, *dloc;
  int32_t* rank;
  // outputs
  int32_t* bonds;       // stateless step: (id_A, id_T) in id_A order
  int64_t bonds_cap;
  int32_t bonds_rule;   // stateless step: rows (id_A, id_T, rule) instead
  int32_t* log;         // (step, id_A, id_T) rows
  int64_t log_cap;
  int32_t* part;        // per step and closing group: kPart partial counters
  int64_t part_cap;     // steps the partial-counter log holds
  unsigned long long* sortbuf;  // stateless step: bonds beyond LDS
  Ctl* ctl;
  // geometry, rule, draws
  int32_t n, B, nc, ncell, nwg_sweep, nwg_prep, ngroups;
  int32_t bs, nb, nbricks, sorted;  // brick edge (cells), bricks per side, total, storage sorted
  int32_t nd;                        // sort bins per brick, (bs + 1)^3 + 1
  uint32_t nb_m;                     // floor(2^32 / nb): brick coordinates by multiplication
  int32_t jitter;       // 1: resident system (positions ping-pong, re-jitter by jit_c)
                        // 0: caller's arrays, read only
  int32_t adj_staged;   // B <= kAdjStage: records carry the adjacency row
  // batched launches only: steps of the current block this system takes part
  // in (0 .. k_limit - 1) and the reaction step of the block's first step
  int32_t k_limit;
  uint32_t first_step;
  float L, halfL, rc2, inv_w, jit_c;
  unsigned long long thresh, seed;
  RuleD rule;
  // several concurrent rules (nrules > 1; then rc2 is the largest cutoff's)
  int32_t nrules;
  RuleX mr[kMaxRules];
  uint8_t *wfa, *wft;   // per slot: won as an A / as a T in this step (one writer each)
  // fused binning (fuse = 1: sorted storage, one rule, random selection, no
  // MD): the sweep of step k bins the A records of step k + 1 itself, so no
  // binning kernel runs.  Counts by step mod 3 (read in step k, filled for
  // k + 1, cleared for k + 2), bucket records and overflow by step parity;
  // apos[slot]: where the A's record of the next step went (bucket index, or
  // -1 - overflow index), for the resolve to drop it if the A's role ends
  int32_t fuse;
  // resident systems: the control block's parity origin (par0) as the host
  // keeps it, so that the resolve addresses its lists without reading the
  // control block first
  uint32_t kpar0;
  uint32_t* fcnt[3];
  float4* frec[2];
  int32_t* fsa[2];
  float4* fovf[2];
  int32_t* fovf_sa[2];
  int32_t* apos;
  // a resident system's sweep stores the re-jittered positions
  // non-temporally: set when one parity's positions (12 bytes per particle)
  // take at most half of the L2s, where they would otherwise still sit,
  // dirty, when the kernel ends and delay the next kernel's start
  int32_t nt_pos;
  // bonded-force coupling (md_theta > 0): md_theta velocity-Verlet steps with
  // the mirror-LJ bond force before each reaction step, instead of the
  // re-jitter; slot_of maps ids to slots of the current storage set
  int32_t md_theta;
  float md_dt, md_h, md_sc2, md_two_sc, md_sig, md_e24;
  int32_t* slot_of;
  int4 *wina, *wint;    // per slot, the winning pair as A / as T:
                        // (partner id, partner slot, rule, 0)
};

// A batch of independent systems stepped in lockstep: their Devs in device
// memory and, per kernel, the map of grid blocks to (replica, local block,
// blocks of that replica).
struct BatchLaunch {
  const Dev* ds;
  int nrep;
  const int4 *prep0, *prepk, *sweep, *close, *part;  // prep at k == 0 / k > 0, sweep and
  int n_prep0, n_prepk, n_sweep, n_close, n_part;     // resolve, closing, particle blocks
  int n_sortl;          // blocks of the per-brick sort scan of the largest replica
  const int4* res;      // resolve: four bricks per block (one per wavefront)
  int n_res;
  int two;              // some replica's brick edge exceeds kOneCellBrick
  int any_random, any_nearest;  // some replica selects with that policy
  int fuse;             // every replica bins its next step's A's in its sweep
};

}  // namespace pr
