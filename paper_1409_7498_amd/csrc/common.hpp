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
constexpr int kTailThreads = 1024;  // one workgroup resolves and applies
constexpr int kSortLds = 4096;      // bonds per step sorted in LDS (else in HBM)
constexpr int kSweepThreads = 256;
constexpr int kStatsPerStep = 9;    // pr_stats fields
constexpr int kWgStats = 4;         // per sweep workgroup: t_elig, in_rc, drawn, excluded
// Spatially sorted storage: particles are kept ordered by "brick" (a block of
// bs^3 coarse cells); one sweep workgroup owns a brick and stages the A
// records of the brick plus one halo cell layer in LDS.
constexpr int kMaxBrick = 4;
constexpr int kStageCells = (kMaxBrick + 2) * (kMaxBrick + 2) * (kMaxBrick + 2);
constexpr int kStageRecs = 1024;

// Device control block: every count whose value is data dependent lives here,
// so a step needs no host round trip and a captured graph can replay it.
struct Ctl {
  uint32_t step;      // current reaction step (draw counter word 0)
  int32_t err;        // first device-detected error (0 = none)
  uint32_t par;       // buffer parity of this step (flips every step)
  uint32_t pad0;
  uint32_t na[2];     // A-list lengths, indexed by parity
  uint32_t ovf_n;     // A records beyond their cell bucket this step
  uint32_t nprop;     // A's with a retained candidate this step
  uint32_t nwin;      // bonds created by the last step
  uint32_t stats_n;   // records in the per-step counter log
  uint64_t log_n;     // rows appended to the bond log (may exceed capacity)
};

struct RuleD {
  int32_t type_a, a_min, a_max, d_a;
  int32_t type_t, t_min, t_max, d_t;
  int32_t exclude;
};

// Everything a kernel needs, passed by value as the kernel argument.
struct Dev {
  // particle storage, slot order (slot == id unless id/slot_of are set)
  float *x, *y, *z;
  int32_t *typ, *st, *adj;
  int32_t *id, *slot_of;
  // A list (slots), by parity
  int32_t* alist[2];
  // A grid: per-cell counts by parity, bucket records, overflow records
  uint32_t* cnt[2];
  float4 *rec, *ovf;
  // selection: per-id minimum keys of the A side and the T side
  unsigned long long *slotA, *slotT;
  int32_t* propA;       // ids of A's with a retained candidate
  // spatial sort: brick offsets of the storage, counters, ranks, second buffers
  int32_t* bstart;      // nbricks + 1 slot offsets (valid when sorted)
  uint32_t* bcnt;
  int32_t* rank;
  float *x2, *y2, *z2;
  int32_t *typ2, *st2, *adj2, *id2;
  int32_t* wgst;        // sweep workgroup counters
  unsigned long long* sortbuf;  // bonds of one step when they exceed LDS
  // outputs
  int32_t* bonds;       // per-step (id_A, id_T), may be null
  int64_t bonds_cap;
  int32_t* log;         // (step, id_A, id_T) rows, may be null
  int64_t log_cap;
  long long* slog;      // kStatsPerStep counters per step, may be null
  int64_t slog_cap;
  Ctl* ctl;
  // geometry, rule, draws
  int32_t n, B, nc, ncell, nwg_sweep;
  int32_t bs, nb, nbricks, sorted;  // brick edge (cells), bricks per side, total, storage sorted
  float L, halfL, rc2, inv_w, jit_c;
  unsigned long long thresh, seed;
  RuleD rule;
};

}  // namespace pr
