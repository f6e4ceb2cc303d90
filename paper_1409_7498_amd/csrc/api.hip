// api.hip -- host runtime and C ABI of the reaction-step library.
//
// Owns device memory (resident systems and the per-device workspace of the
// stateless single step), validates arguments before any launch, sizes the
// coarse A grid and the bricks, and drives the per-step kernel sequence of
// kernels.hip -- directly, or replayed from a captured HIP graph that holds a
// whole block of steps (one spatial sort followed by sort_period steps).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "../../include/polyreact.h"

namespace pr {
hipError_t launch_ctl_reset(Ctl* c, uint32_t step, int full, hipStream_t s);
hipError_t launch_classify(const Dev& d, hipStream_t s);
hipError_t launch_identity(const Dev& d, hipStream_t s);
hipError_t launch_generate(const Dev& d, int kind, unsigned long long gseed, float c0, float a,
                           int nl, unsigned long long thr, hipStream_t s);
hipError_t launch_step(const Dev& d, int k, hipStream_t s, hipEvent_t ev_sweep0,
                       hipEvent_t ev_sweep1);
hipError_t launch_block_end(const Dev& d, int K, hipStream_t s);
hipError_t launch_single_end(const Dev& d, hipStream_t s);
hipError_t launch_sort(const Dev& d, hipStream_t s);
hipError_t log_order(int32_t* log, int64_t n, hipStream_t s);
hipError_t launch_gather_out(const Dev& d, float* ox, float* oy, float* oz, int32_t* otyp,
                             int32_t* ost, int32_t* oadj, hipStream_t s);
hipError_t launch_draws(const uint32_t* ctr, long long n, unsigned long long key, uint32_t* out,
                        hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_md_init(const Dev& d, unsigned long long vseed, float cv, hipStream_t s);
hipError_t launch_sqrt_rn(const float* in, float* out, long long n, hipStream_t s);
hipError_t launch_gather_v(const Dev& d, float* ox, float* oy, float* oz, hipStream_t s);
hipError_t launch_kinetics(const Dev& d, int nstate, int nbins, const float* e2,
                           unsigned long long* pop, unsigned long long* pairs,
                           unsigned long long* hist, hipStream_t s);
hipError_t launch_jitter_only(const Dev& d, int n_steps, hipStream_t s, hipEvent_t ev0,
                              hipEvent_t ev1);
hipError_t launch_stream_copy(const void* src, void* dst, long long bytes, int width,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
}  // namespace pr

using namespace pr;

namespace {

thread_local std::string g_err = "";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(PR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int validate_rule(const pr_rule* r, float L) {
  if (!r) return fail(PR_EINVAL, "rule is NULL");
  if (!(r->rc > 0.0f) || !std::isfinite(r->rc)) return fail(PR_EINVAL, "rc must be > 0");
  if (!std::isfinite(L) || !(L > 2.0f * r->rc))
    return fail(PR_EINVAL, "box L=%g must exceed 2*rc=%g", (double)L, 2.0 * r->rc);
  if (!(r->p >= 0.0 && r->p <= 1.0)) return fail(PR_EINVAL, "p=%g outside [0, 1]", r->p);
  if (r->type_a == r->type_t && r->a_min <= r->t_max && r->t_min <= r->a_max)
    return fail(PR_ERULE_AMBIGUOUS, "type_a == type_t and the A/T state windows overlap");
  if (r->policy != PR_POLICY_RANDOM && r->policy != PR_POLICY_NEAREST)
    return fail(PR_EINVAL, "policy=%d (PR_POLICY_RANDOM or PR_POLICY_NEAREST)", r->policy);
  return PR_OK;
}

// pr_stats from the kPart partial counters of a step (layout: a_elig, t_elig,
// in_rc, drawn, excluded, proposals, bonds, lost).  Random selection: the
// accepted candidates are the drawn pairs less the excluded ones; nearest:
// every tested pair that passes bonds.
pr_stats stats_of(const long long h[kPart], int32_t policy) {
  const long long accepted = policy == PR_POLICY_NEAREST ? h[6] : h[3] - h[4];
  return pr_stats{h[0], h[1], h[2], h[3], h[4], accepted, h[5], h[6], h[7]};
}

unsigned long long threshold(double p) {
  double t = std::ceil(p * 4294967296.0);
  if (t < 0.0) t = 0.0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (unsigned long long)t;
}

// The store policy of a resident system's sweep for the re-jittered
// positions (Dev::nt_pos): one parity of n particles' positions against half
// of the L2s (8 XCDs x 4 MiB).  Measured with non-temporal stores: 1M
// particles 30.9 -> 30.45 us per step, the gap between the sweep and the next
// kernel 2.8 -> 2.0 us; 4M particles, and the 4.5M of a 256-replica batch,
// 2-3% slower (their positions leave the L2s during the kernel anyway).
// Batches keep plain stores.
constexpr int64_t kNtPosBytes = 16ll << 20;
int32_t nt_positions(int64_t n) { return 12 * n <= kNtPosBytes ? 1 : 0; }

int sweep_blocks(int32_t n) { return std::max(1, (n + kThreads - 1) / kThreads); }
int prep_blocks(int32_t n) {
  return std::max(1, (int)(((int64_t)n + kThreads * kPrepRoles - 1) / (kThreads * kPrepRoles)));
}

// Coarse A grid: nc cells per side of width L/nc >= 2 rc (1 + 2^-10); the
// margin keeps the 2x2x2 block exact under FP32 rounding of the cell index.
// Bricks of bs^3 cells; the staged region (bs + 2 cells per side) must not
// wrap onto itself, so bs <= nc - 2, else one brick covers the whole grid.
void set_geometry(Dev& d, int32_t n, float L, int32_t B, const pr_rule* r, uint64_t seed,
                  int brick_pref) {
  d.n = n;
  d.B = B;
  d.L = L;
  d.halfL = 0.5f * L;
  d.rc2 = r->rc * r->rc;
  long long nc = (long long)std::floor((double)L / (2.0 * (double)r->rc * (1.0 + 1.0 / 1024.0)));
  if (nc < 1) nc = 1;
  const long long cell_cap = std::max<long long>(2LL * n, 4096LL);
  while (nc > 1 && nc * nc * nc > cell_cap) --nc;
  d.nc = (int32_t)nc;
  d.ncell = (int32_t)(nc * nc * nc);
  d.inv_w = (float)((double)nc / (double)L);
  d.thresh = threshold(r->p);
  d.seed = seed;
  d.rule = RuleD{r->type_a, r->a_min, r->a_max, r->d_a, r->type_t, r->t_min, r->t_max, r->d_t,
                 r->exclude_bonded, r->policy};
  d.nrules = 1;
  d.mr[0] = RuleX{d.rule, d.rc2, 0u, d.thresh};
  d.nwg_sweep = sweep_blocks(n);
  d.nwg_prep = prep_blocks(n);
  d.adj_staged = B <= kAdjStage ? 1 : 0;
  d.nt_pos = nt_positions(n);
  d.k_limit = INT32_MAX;
  d.first_step = 0;
  d.jit_c = 0.0f;
  d.part = nullptr;
  d.part_cap = 0;
  const int bs = std::min<int>(std::max(1, std::min(brick_pref, kMaxBrick)), (int)nc - 2);
  if (bs >= 1) {
    d.bs = bs;
    d.nb = (int32_t)((nc + bs - 1) / bs);
  } else {
    d.bs = (int32_t)nc;
    d.nb = 1;
  }
  d.nbricks = d.nb * d.nb * d.nb;
  d.nd = (d.bs + 1) * (d.bs + 1) * (d.bs + 1) + 1;  // the brick's A's, then its dual cells
  d.nb_m = (uint32_t)((1ull << 32) / (unsigned long long)d.nb);  // nb >= 1; nb = 1 gives 0
  d.sorted = 0;
  // closing groups cover the larger of the two sweep grids (dense, bricks)
  d.ngroups = (std::max(d.nwg_sweep, d.nbricks) + kGroup - 1) / kGroup;
}

// Validation of a set of concurrent rules (each as validate_rule; several
// rules use the random selection).
int validate_rules(const pr_rule* rules, int32_t nrules, float L) {
  if (!rules || nrules < 1 || nrules > kMaxRules)
    return fail(PR_EINVAL, "nrules=%d (1..%d)", nrules, kMaxRules);
  for (int32_t r = 0; r < nrules; ++r) {
    int e = validate_rule(&rules[r], L);
    if (e) return e;
    if (nrules > 1 && rules[r].policy != PR_POLICY_RANDOM)
      return fail(PR_EINVAL, "several rules use the random selection (rule %d)", r);
  }
  return PR_OK;
}

// Geometry of a system of nrules concurrent rules: the A grid is sized for
// the largest cutoff; each rule keeps its own cutoff, threshold and tag.
void set_geometry_rules(Dev& d, int32_t n, float L, int32_t B, const pr_rule* rules,
                        int32_t nrules, uint64_t seed, int brick_pref) {
  pr_rule big = rules[0];
  for (int32_t r = 1; r < nrules; ++r) big.rc = std::max(big.rc, rules[r].rc);
  set_geometry(d, n, L, B, &big, seed, brick_pref);
  d.rule.d_a = rules[0].d_a;
  if (nrules == 1) {
    d.rc2 = rules[0].rc * rules[0].rc;
    d.mr[0].rc2 = d.rc2;
    return;
  }
  d.nrules = nrules;
  for (int32_t r = 0; r < nrules; ++r) {
    const pr_rule& q = rules[r];
    d.mr[r] = RuleX{RuleD{q.type_a, q.a_min, q.a_max, q.d_a, q.type_t, q.t_min, q.t_max, q.d_t,
                          q.exclude_bonded, q.policy},
                    q.rc * q.rc, r == 0 ? 0u : 0x100u + (uint32_t)r, threshold(q.p)};
  }
}

// Device allocations of one handle.  dry = true only adds up the bytes (the
// footprint of a system before it is created: the same allocation code runs).
// async = true: stream-ordered allocation on astream (hipMallocAsync /
// hipFreeAsync), so that freeing does not wait for unrelated device work.
struct Arena {
  std::vector<void*> ptrs;
  bool dry = false, async = false;
  hipStream_t astream = nullptr;
  hipMemPool_t pool = nullptr;  // async: the pool to draw from (null: the device's default)
  size_t bytes = 0;
  // carve mode (base != null): every allocation is the next 256-byte aligned
  // piece of the caller's region [base, base + cap); nothing is allocated or
  // freed, and running past cap fails with PR_ECAP
  char* base = nullptr;
  size_t cap = 0;
  ~Arena() { release(); }
  void release() {
    for (void* p : ptrs) (void)(async ? hipFreeAsync(p, astream) : hipFree(p));
    ptrs.clear();
  }
  template <typename T>
  int alloc(T** out, size_t count) {
    if (count == 0) count = 1;
    const size_t nb = count * sizeof(T);
    const size_t at = bytes;
    bytes += (nb + 255) & ~(size_t)255;
    if (dry) {
      *out = nullptr;
      return PR_OK;
    }
    if (base) {
      if (bytes > cap)
        return fail(PR_ECAP, "scratch needs more than its %zu bytes", cap);
      *out = (T*)(base + at);
      return PR_OK;
    }
    void* p = nullptr;
    const hipError_t he = !async ? hipMalloc(&p, nb)
                          : pool ? hipMallocFromPoolAsync(&p, nb, pool, astream)
                                 : hipMallocAsync(&p, nb, astream);
    if (he != hipSuccess) return fail(PR_ENOMEM, "hipMalloc of %zu bytes failed", nb);
    ptrs.push_back(p);
    *out = (T*)p;
    return PR_OK;
  }
};

// Scratch of one step (everything but the particle arrays and the logs).
// nwg: sweep workgroups to provide for (the larger of the two sweep grids).
int alloc_scratch(Arena& a, Dev& d, int32_t n, int32_t nwg, hipStream_t s) {
  int e;
  if ((e = a.alloc(&d.tflag, n)))
    return e;
  if ((e = a.alloc(&d.cnt[0], d.ncell)) || (e = a.alloc(&d.cnt[1], d.ncell))) return e;
  const size_t nrec = (size_t)d.ncell * kCellCap;
  if ((e = a.alloc(&d.rec, nrec)) || (e = a.alloc(&d.rsa, nrec)) ||
      (e = a.alloc(&d.radj, nrec)))
    return e;
  if ((e = a.alloc(&d.slotA, n)) || (e = a.alloc(&d.tnear, n))) return e;
  for (int p = 0; p < 2; ++p) {
    if ((e = a.alloc(&d.ovf[p], n)) || (e = a.alloc(&d.ovf_sa[p], n)) ||
        (e = a.alloc(&d.wgo[p], (size_t)nwg * kWgOut)) ||
        (e = a.alloc(&d.wge[p], (size_t)nwg * kRetCap)) ||
        (e = a.alloc(&d.wgk[p], (size_t)nwg * kRetCap)) ||
        (e = a.alloc(&d.wgw[p], (size_t)nwg * kWinCap)) || (e = a.alloc(&d.wov[p], n / 2 + 1)) ||
        (e = a.alloc(&d.abst[p], (size_t)sweep_blocks(n))))
      return e;
  }
  if ((e = a.alloc(&d.ctl, 1))) return e;
  if (d.nrules > 1 && ((e = a.alloc(&d.wfa, n)) || (e = a.alloc(&d.wft, n)) ||
                       (e = a.alloc(&d.wina, n)) || (e = a.alloc(&d.wint, n))))
    return e;
  if (a.dry || a.base) return PR_OK;  // a carved region is cleared by its user
  HIP_TRY(hipMemsetAsync(d.cnt[0], 0, sizeof(uint32_t) * std::max(1, d.ncell), s));
  HIP_TRY(hipMemsetAsync(d.cnt[1], 0, sizeof(uint32_t) * std::max(1, d.ncell), s));
  HIP_TRY(hipMemsetAsync(d.slotA, 0xFF, sizeof(unsigned long long) * std::max(1, n), s));
  HIP_TRY(hipMemsetAsync(d.tflag, 0, std::max(1, n), s));
  HIP_TRY(hipMemsetAsync(d.ctl, 0, sizeof(Ctl), s));
  return PR_OK;
}

// Per-device workspace of the stateless single step, grown on demand.
struct Workspace {
  Arena arena;
  Dev d{};
  int32_t n = -1, ncell = -1;
  int32_t* part = nullptr;
  int32_t ngroups = 0;
  int32_t* log = nullptr;
  uint8_t* role = nullptr;
  unsigned long long* sortbuf = nullptr;
  Ctl* hctl = nullptr;  // pinned host copies
  int32_t* hpart = nullptr;
  bool multi = false;   // holds the arrays of several concurrent rules
  ~Workspace() {
    if (hctl) (void)hipHostFree(hctl);
    if (hpart) (void)hipHostFree(hpart);
  }
};

std::mutex g_ws_mu;
std::vector<Workspace*> g_ws;  // indexed by device

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pr_last_error(void) { return g_err.c_str(); }

const char* pr_version(void) { return "polyreact 0.2 (gfx950)"; }

double pr_p_from_rate(double k, double dt, double theta, int32_t* warn) {
  if (warn) *warn = 0;
  if (!(k >= 0.0) || !(dt >= 0.0) || !(theta >= 0.0) || !std::isfinite(k * dt * theta))
    return -1.0;
  const double p = k * dt * theta;
  if (warn && p > 0.1) *warn = 1;
  return p;
}

int pr_draws(const uint32_t* ctr, int64_t n, uint64_t key, uint32_t* out, void* stream) {
  if (n < 0 || n > (int64_t)kMaxParticles) return fail(PR_EINVAL, "n=%lld", (long long)n);
  if (n == 0) return PR_OK;
  if (!ctr || !out) return fail(PR_EINVAL, "NULL array");
  HIP_TRY(launch_draws(ctr, (long long)n, (unsigned long long)key, out, (hipStream_t)stream));
  return PR_OK;
}

}  // extern "C"

namespace {

// Validation shared by the stateless single-step entry points.
int check_single(int32_t n, float L, const float* x, const float* y, const float* z,
                 const int32_t* type, const int32_t* state, const int32_t* adj, int32_t B,
                 const pr_rule* rule, const int32_t* bonds, int32_t cap, const int32_t* n_bonds) {
  if (n < 0 || n > kMaxParticles || B < 1) return fail(PR_EINVAL, "n=%d B=%d", n, B);
  int e = validate_rule(rule, L);
  if (e) return e;
  if (!n_bonds) return fail(PR_EINVAL, "n_bonds is NULL");
  if ((int64_t)cap < (int64_t)n / 2) return fail(PR_ECAP, "cap=%d < n/2=%d", cap, n / 2);
  if (n > 0 && (!x || !y || !z || !type || !state || !adj || !bonds))
    return fail(PR_EINVAL, "NULL device array");
  return PR_OK;
}

// Points d (scratch pointers already set) at the caller's arrays with the
// geometry of this call (the scratch may be sized for a larger one).
void bind_single(Dev& d, const Dev& geo, float* x, float* y, float* z, int32_t* type,
                 int32_t* state, int32_t* adj, uint8_t* role, int32_t* bonds, int32_t cap) {
  d.n = geo.n;
  d.B = geo.B;
  d.L = geo.L;
  d.halfL = geo.halfL;
  d.rc2 = geo.rc2;
  d.nc = geo.nc;
  d.ncell = geo.ncell;
  d.inv_w = geo.inv_w;
  d.thresh = geo.thresh;
  d.seed = geo.seed;
  d.rule = geo.rule;
  d.nrules = geo.nrules;
  for (int r = 0; r < kMaxRules; ++r) d.mr[r] = geo.mr[r];
  d.adj_staged = geo.adj_staged;
  d.nwg_sweep = geo.nwg_sweep;
  d.nwg_prep = geo.nwg_prep;
  d.jitter = 0;
  d.nt_pos = 0;
  d.sorted = 0;
  const Arr caller{{x, x}, {y, y}, {z, z}, type, state, adj, nullptr, role};
  d.set[0] = d.set[1] = caller;
  d.bonds = bonds;
  d.bonds_cap = cap;
  d.bonds_rule = 0;
  d.log_cap = (int64_t)geo.n / 2 + 1;
  d.part_cap = 1;
  d.ngroups = (d.nwg_sweep + kGroup - 1) / kGroup;
}

// The launches of one stateless step (count buffers already cleared), the
// read-back of its control block and counters into hctl / hpart (host
// memory of d.ngroups * kPart words) and the results.
int single_step(const Dev& d, uint32_t step, hipStream_t s, Ctl* hctl, int32_t* hpart,
                int32_t* n_bonds, pr_stats* st) {
  HIP_TRY(launch_ctl_reset(d.ctl, step, 1, s));
  HIP_TRY(launch_classify(d, s));
  HIP_TRY(launch_step(d, 0, s, nullptr, nullptr));
  HIP_TRY(launch_single_end(d, s));
  HIP_TRY(hipMemcpyAsync(hctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hpart, d.part, sizeof(int32_t) * d.ngroups * kPart,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const Ctl c = *hctl;
  if (c.err) return fail(c.err, "invalid particle position (NaN or outside [0, L))");
  *n_bonds = (int32_t)c.log_n;
  long long h[kPart] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int g = 0; g < d.ngroups; ++g)
    for (int q = 0; q < kPart; ++q) h[q] += hpart[g * kPart + q];
  if (st) *st = stats_of(h, d.rule.policy);
  if (h[7] > 0) return fail(PR_ECAP, "%lld adjacency appends found a full row", h[7]);
  return PR_OK;
}

// Scratch of the allocation-free single step: one region per device, the
// file-scope array below.  Host code never passes the array's name to a
// kernel (on the host it only stands for the symbol); it uses the device
// address hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kScratchBytes = (size_t)24 << 20;
constexpr int32_t kScratchMaxN = 32768;
constexpr int kScratchMaxDev = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu[kScratchMaxDev];  // one call at a time per device
char* g_scratch_ptr[kScratchMaxDev] = {};
std::mutex g_scratch_init_mu;

// Carves the scratch of a single step of up to n particles and ncell cells
// out of arena a (the same buffers pr_react_step's workspace allocates).
int carve_single(Arena& a, Dev& d, int32_t n, uint8_t** role) {
  int e = alloc_scratch(a, d, n, sweep_blocks(n), nullptr);
  if (e) return e;
  size_t n2 = 1;
  while (n2 < (size_t)n / 2 + 1) n2 <<= 1;
  const int ngroups = (sweep_blocks(n) + kGroup - 1) / kGroup;
  if ((e = a.alloc(&d.part, (size_t)ngroups * kPart)) ||
      (e = a.alloc(&d.log, 3 * ((size_t)n / 2 + 1))) || (e = a.alloc(role, (size_t)n)) ||
      (e = a.alloc(&d.sortbuf, n2)))
    return e;
  return PR_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// The stateless step with nrules concurrent rules (nrules == 1: the single
// rule of pr_react_step) on the per-device workspace.
int react_step_impl(int32_t n, float L, const float* x, const float* y, const float* z,
                    const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                    const pr_rule* rules, int32_t nrules, uint64_t seed, uint32_t step,
                    int32_t* bonds, int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream,
                    bool triples) {
  int e = validate_rules(rules, nrules, L);
  if (e) return e;
  if ((e = check_single(n, L, x, y, z, type, state, adj, B, rules, bonds, cap, n_bonds))) return e;
  *n_bonds = 0;
  if (st) std::memset(st, 0, sizeof *st);
  if (n == 0) return PR_OK;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_ws_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1, nullptr);
  Workspace*& ws = g_ws[dev];
  Dev geo{};
  set_geometry_rules(geo, n, L, B, rules, nrules, seed, kDefaultBrick);
  if (!ws || ws->n < n || ws->ncell < geo.ncell || (nrules > 1 && !ws->multi)) {
    const bool multi = nrules > 1 || (ws && ws->multi);
    delete ws;
    ws = new Workspace();
    ws->d = geo;
    ws->d.nrules = multi ? 2 : 1;  // allocation of the several-rule arrays
    const int32_t n_alloc = std::max(n, 1024);
    if ((e = alloc_scratch(ws->arena, ws->d, n_alloc, sweep_blocks(n_alloc), s))) {
      delete ws;
      ws = nullptr;
      return e;
    }
    ws->multi = multi;
    size_t n2 = 1;
    while (n2 < (size_t)n_alloc / 2 + 1) n2 <<= 1;
    ws->ngroups = (sweep_blocks(n_alloc) + kGroup - 1) / kGroup;
    if ((e = ws->arena.alloc(&ws->part, (size_t)ws->ngroups * kPart)) ||
        (e = ws->arena.alloc(&ws->log, 3 * ((size_t)n_alloc / 2 + 1))) ||
        (e = ws->arena.alloc(&ws->role, (size_t)n_alloc)) ||
        (e = ws->arena.alloc(&ws->sortbuf, n2)))
      return e;
    HIP_TRY(hipHostMalloc((void**)&ws->hctl, sizeof(Ctl)));
    HIP_TRY(hipHostMalloc((void**)&ws->hpart, sizeof(int32_t) * ws->ngroups * kPart));
    ws->n = n_alloc;
    ws->ncell = geo.ncell;
  }
  Dev d = ws->d;  // scratch pointers
  d.log = ws->log;
  d.sortbuf = ws->sortbuf;
  d.part = ws->part;
  bind_single(d, geo, const_cast<float*>(x), const_cast<float*>(y), const_cast<float*>(z),
              const_cast<int32_t*>(type), state, adj, ws->role, bonds, cap);
  d.bonds_rule = triples ? 1 : 0;
  // The workspace serves calls of any box size: a previous call may have left
  // counts in cells beyond this call's grid, so both count buffers are cleared
  // over their whole allocation (each step only clears the cells it uses).
  HIP_TRY(hipMemsetAsync(d.cnt[0], 0, sizeof(uint32_t) * (size_t)ws->ncell, s));
  HIP_TRY(hipMemsetAsync(d.cnt[1], 0, sizeof(uint32_t) * (size_t)ws->ncell, s));
  return single_step(d, step, s, ws->hctl, ws->hpart, n_bonds, st);
}

}  // namespace

extern "C" {

int pr_react_step(int32_t n, float L, const float* x, const float* y, const float* z,
                  const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                  const pr_rule* rule, uint64_t seed, uint32_t step, int32_t* bonds,
                  int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream) {
  return react_step_impl(n, L, x, y, z, type, state, adj, B, rule, 1, seed, step, bonds, cap,
                         n_bonds, st, stream, false);
}

int pr_react_step_multi(int32_t n, float L, const float* x, const float* y, const float* z,
                        const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                        const pr_rule* rules, int32_t nrules, uint64_t seed, uint32_t step,
                        int32_t* bonds, int32_t cap, int32_t* n_bonds, pr_stats* st,
                        void* stream) {
  return react_step_impl(n, L, x, y, z, type, state, adj, B, rules, nrules, seed, step, bonds,
                         cap, n_bonds, st, stream, true);
}

int pr_react_step_noalloc(int32_t n, float L, const float* x, const float* y, const float* z,
                          const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                          const pr_rule* rule, uint64_t seed, uint32_t step, int32_t* bonds,
                          int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream) {
  int e = check_single(n, L, x, y, z, type, state, adj, B, rule, bonds, cap, n_bonds);
  if (e) return e;
  if (n > kScratchMaxN)
    return fail(PR_EINVAL, "n=%d: the allocation-free step takes at most %d particles", n,
                kScratchMaxN);
  Dev geo{};
  set_geometry(geo, n, L, B, rule, seed, kDefaultBrick);
  Arena dry;
  dry.dry = true;
  uint8_t* role = nullptr;
  Dev dd = geo;
  if ((e = carve_single(dry, dd, std::max(n, 1), &role))) return e;
  if (dry.bytes > kScratchBytes)
    return fail(PR_EINVAL, "n=%d, %d cells: %zu bytes of scratch, the allocation-free step "
                "holds %zu", n, geo.ncell, dry.bytes, kScratchBytes);
  *n_bonds = 0;
  if (st) std::memset(st, 0, sizeof *st);
  if (n == 0) return PR_OK;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchMaxDev) return fail(PR_EINVAL, "device %d", dev);
  {
    std::lock_guard<std::mutex> lk(g_scratch_init_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      g_scratch_ptr[dev] = (char*)ptr;
    }
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
  Arena carve;
  carve.base = g_scratch_ptr[dev];
  carve.cap = kScratchBytes;
  Dev d = geo;
  if ((e = carve_single(carve, d, n, &role))) return e;
  bind_single(d, geo, const_cast<float*>(x), const_cast<float*>(y), const_cast<float*>(z),
              const_cast<int32_t*>(type), state, adj, role, bonds, cap);
  // the region keeps the previous call's contents: clear what the kernels
  // expect empty (cell counts, A keys, T flags) with fill kernels
  HIP_TRY(launch_fill_u32(d.cnt[0], d.ncell, 0u, s));
  HIP_TRY(launch_fill_u32(d.cnt[1], d.ncell, 0u, s));
  HIP_TRY(launch_fill_u32((uint32_t*)d.slotA, 2LL * n, 0xFFFFFFFFu, s));
  HIP_TRY(launch_fill_u32((uint32_t*)d.tflag, ((long long)n + 3) / 4, 0u, s));
  Ctl hctl{};
  int32_t hpart[((kScratchMaxN + kThreads - 1) / kThreads + kGroup - 1) / kGroup * kPart];
  return single_step(d, step, s, &hctl, hpart, n_bonds, st);
}

}  // extern "C"

// ===========================================================================
// Resident systems
// ===========================================================================
struct pr_sys {
  int dev = 0;
  hipStream_t stream = nullptr;   // the caller's stream: every launch goes here
  hipStream_t cap = nullptr;      // private stream, used only to capture graphs
  Arena arena;
  Dev d{};
  pr_rule rule{};
  int64_t log_cap = 0;
  int64_t part_cap = 0;
  int64_t steps_since_load = 0;
  int64_t steps_since_sort = 0;
  bool loaded = false;
  bool poisoned = false;
  int32_t sort_period = 0;
  int32_t use_graphs = 1;
  // fused binning: allowed (pr_sys_set_fused_binning), and the step and
  // jitter scale the device's next-step A records were written for (rec_ok:
  // they exist)
  int32_t allow_fuse = 1;
  bool rec_ok = false;
  uint32_t rec_step = 0;
  float rec_jit = 0.0f;
  // captured segments of steps: (a sort when one is due and) K steps and the
  // block end, keyed by what the captured kernels hold
  struct Seg {
    hipGraphExec_t gexec = nullptr;
    int32_t steps = 0;
    bool sort = false;
    float jit = -1.0f;
    long long part = 0;
    int32_t fuse = 0;
    uint32_t kpar0 = 0;  // parity origin the segment was captured at
    uint64_t used = 0;
  };
  std::vector<Seg> segs;
  uint64_t seg_clock = 0;
  float *rx = nullptr, *ry = nullptr, *rz = nullptr;  // id-order read buffers
  int32_t *rtyp = nullptr, *rst = nullptr, *radj = nullptr;
  Ctl* hctl = nullptr;
  bool own_hctl = true;  // false: the pinned word belongs to a server's pool
  // kinetics counters (allocated on first use): pop, pairs, hist, bin edges
  unsigned long long* kin = nullptr;
  float* kin_e2 = nullptr;
  ~pr_sys() {
    for (Seg& g : segs)
      if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
    if (cap) (void)hipStreamDestroy(cap);
    if (hctl && own_hctl) (void)hipHostFree(hctl);
  }
};

namespace {

int check_sys(pr_sys* s, bool need_loaded) {
  if (!s) return fail(PR_EINVAL, "NULL system handle");
  if (s->poisoned) return fail(PR_EHIP, "system handle unusable after a HIP error");
  if (need_loaded && !s->loaded) return fail(PR_EINVAL, "system holds no valid configuration");
  return PR_OK;
}

int sync_ctl(pr_sys* s) {
  HIP_TRY(hipMemcpyAsync(s->hctl, s->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return PR_OK;
}

void drop_graph(pr_sys* s) {
  for (pr_sys::Seg& g : s->segs)
    if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
  s->segs.clear();
}

// The partial-counter log holds `need` steps (grown by doubling; a copy keeps
// the steps already logged).
int grow_part(pr_sys* s, int64_t need) {
  if (need <= s->part_cap) return PR_OK;
  const int64_t cap = std::max<int64_t>(need, 2 * s->part_cap);
  const size_t row = (size_t)s->d.ngroups * kPart;
  int32_t* nb = nullptr;
  int e = s->arena.alloc(&nb, (size_t)cap * row);
  if (e) return e;
  if (s->d.part && s->part_cap > 0)
    HIP_TRY(hipMemcpyAsync(nb, s->d.part, sizeof(int32_t) * row * s->part_cap,
                           hipMemcpyDeviceToDevice, s->stream));
  s->d.part = nb;  // the old block stays in the arena until destroy
  s->part_cap = cap;
  s->d.part_cap = cap;
  drop_graph(s);  // the captured kernels hold the old pointer
  return PR_OK;
}

// Unsorted storage until the first sort: sweep workgroups take consecutive slots.
void set_dense(pr_sys* s) {
  s->d.sorted = 0;
  s->d.fuse = 0;
  s->d.nwg_sweep = sweep_blocks(s->d.n);
  s->rec_ok = false;
}

// Whether the sweeps of a sorted system can bin the next step's A's
// themselves: one rule with the random selection, no MD (the MD moves the
// particles between steps), the buckets allocated.
bool fuse_eligible(const pr_sys* s) {
  const Dev& d = s->d;
  return s->allow_fuse && d.nrules == 1 && d.rule.policy == PR_POLICY_RANDOM && d.md_theta == 0 &&
         d.fcnt[0] != nullptr;
}

// The fused-binning buckets, allocated on the first run that can use them.
int alloc_fused(pr_sys* s) {
  Dev& d = s->d;
  if (d.fcnt[0] || !s->allow_fuse || d.nrules != 1 || d.rule.policy != PR_POLICY_RANDOM)
    return PR_OK;
  Dev t = d;
  const size_t n = (size_t)d.n, nrec = (size_t)d.ncell * kCellCap;
  int e = 0;
  for (int q = 0; q < 3 && !e; ++q) e = s->arena.alloc(&t.fcnt[q], (size_t)d.ncell);
  for (int p = 0; p < 2 && !e; ++p) {
    if (!e) e = s->arena.alloc(&t.frec[p], nrec);
    if (!e) e = s->arena.alloc(&t.fsa[p], nrec);
    if (!e) e = s->arena.alloc(&t.fovf[p], n);
    if (!e) e = s->arena.alloc(&t.fovf_sa[p], n);
  }
  if (!e) e = s->arena.alloc(&t.apos, n);
  if (e) return e;  // what was allocated stays in the arena until destroy
  for (int q = 0; q < 3; ++q) d.fcnt[q] = t.fcnt[q];
  for (int p = 0; p < 2; ++p) {
    d.frec[p] = t.frec[p];
    d.fsa[p] = t.fsa[p];
    d.fovf[p] = t.fovf[p];
    d.fovf_sa[p] = t.fovf_sa[p];
  }
  d.apos = t.apos;
  drop_graph(s);
  return PR_OK;
}

// A run from step first_step with jitter scale jit: with fused binning the
// device holds the A records of one step only (binned at their re-jittered
// positions), so a run that does not continue the last one sorts (and bins
// them again) first.
void fuse_check_run(pr_sys* s, uint32_t first_step) {
  if (!s->d.sorted || !s->d.fuse) return;
  if (s->rec_ok && s->rec_step == first_step && s->rec_jit == s->d.jit_c) return;
  if (s->sort_period > 0)
    s->steps_since_sort = s->sort_period;
  else
    set_dense(s);
  s->rec_ok = false;
}

void fuse_after_run(pr_sys* s, uint32_t first_step, uint32_t n_steps) {
  s->rec_ok = s->d.sorted && s->d.fuse;
  s->rec_step = first_step + n_steps;
  s->rec_jit = s->d.jit_c;
}

int after_load(pr_sys* s) {
  hipStream_t st = s->stream;
  set_dense(s);
  drop_graph(s);
  s->steps_since_sort = 0;
  // parity 0 after the reset: both cell-count buffers start cleared
  HIP_TRY(hipMemsetAsync(s->d.cnt[0], 0, sizeof(uint32_t) * (size_t)s->d.ncell, st));
  HIP_TRY(hipMemsetAsync(s->d.cnt[1], 0, sizeof(uint32_t) * (size_t)s->d.ncell, st));
  HIP_TRY(launch_ctl_reset(s->d.ctl, 0, 1, st));
  s->d.kpar0 = 0;
  HIP_TRY(launch_identity(s->d, st));
  HIP_TRY(launch_classify(s->d, st));
  int e = sync_ctl(s);
  if (e) return e;
  s->steps_since_load = 0;
  if (s->hctl->err) {
    s->loaded = false;
    return fail(s->hctl->err, "invalid particle position (NaN or outside [0, L))");
  }
  s->loaded = true;
  return PR_OK;
}

// Counting sort of the storage by brick (writes the other storage set);
// afterwards the sweep runs per brick.
int sort_storage(pr_sys* s, hipStream_t st) {
  s->d.fuse = fuse_eligible(s) ? 1 : 0;
  HIP_TRY(launch_sort(s->d, st));
  s->d.sorted = 1;
  s->d.nwg_sweep = s->d.nbricks;
  s->steps_since_sort = 0;
  return PR_OK;
}

// A block of K steps on st: a sort first when due, K steps, the block end.
// ev (timed runs, K == 1): events before the prep, before and after the sweep.
// sort_ev (may be null): events around the sort, when one runs (*sorted = 1).
int run_block(pr_sys* s, hipStream_t st, int32_t K, hipEvent_t* ev,
              hipEvent_t* sort_ev = nullptr, bool* sorted = nullptr) {
  int e;
  if (sorted) *sorted = false;
  if (s->sort_period > 0 && (!s->d.sorted || s->steps_since_sort >= s->sort_period)) {
    if (sort_ev) HIP_TRY(hipEventRecord(sort_ev[0], st));
    if ((e = sort_storage(s, st))) return e;
    if (sort_ev) HIP_TRY(hipEventRecord(sort_ev[1], st));
    if (sorted) *sorted = true;
  }
  if (ev) HIP_TRY(hipEventRecord(ev[0], st));
  for (int32_t k = 0; k < K; ++k)
    HIP_TRY(launch_step(s->d, k, st, ev ? ev[1] : nullptr, ev ? ev[2] : nullptr));
  HIP_TRY(launch_block_end(s->d, K, st));
  s->steps_since_sort += K;
  s->d.kpar0 = (s->d.kpar0 + (uint32_t)K) & 1u;
  return PR_OK;
}

// Whether the next step of a run starts with a spatial sort.
bool sort_due(const pr_sys* s) {
  return s->sort_period > 0 && (!s->d.sorted || s->steps_since_sort >= s->sort_period);
}

// The next segment of a run with `left` steps to go: a sort when one is due,
// then up to the next sort (or 32 steps without sorting).
int32_t next_segment(const pr_sys* s, uint32_t left, bool* with_sort) {
  *with_sort = sort_due(s);
  int64_t room = s->sort_period > 0
                     ? (*with_sort ? s->sort_period : s->sort_period - s->steps_since_sort)
                     : 32;
  return (int32_t)std::min<int64_t>(room, left);
}

// The host-side state a segment leaves behind (the kernels move the device
// side).
void after_segment(pr_sys* s, int32_t K, bool with_sort) {
  if (with_sort) {
    s->d.fuse = fuse_eligible(s) ? 1 : 0;
    s->d.sorted = 1;
    s->d.nwg_sweep = s->d.nbricks;
    s->steps_since_sort = K;
  } else {
    s->steps_since_sort += K;
  }
  s->d.kpar0 = (s->d.kpar0 + (uint32_t)K) & 1u;
}

// The captured graph of a segment of K steps (with a sort first when
// with_sort), capturing it on the private stream if it is not cached.
int segment_graph(pr_sys* s, int32_t K, bool with_sort, hipGraphExec_t* out) {
  const long long part = (long long)(size_t)s->d.part;
  for (pr_sys::Seg& g : s->segs)
    if (g.steps == K && g.sort == with_sort && g.jit == s->d.jit_c && g.part == part &&
        g.fuse == s->d.fuse && g.kpar0 == s->d.kpar0) {
      g.used = ++s->seg_clock;
      *out = g.gexec;
      return PR_OK;
    }
  constexpr size_t kMaxSegs = 6;
  if (s->segs.size() >= kMaxSegs) {  // drop the least recently used
    size_t lru = 0;
    for (size_t i = 1; i < s->segs.size(); ++i)
      if (s->segs[i].used < s->segs[lru].used) lru = i;
    (void)hipGraphExecDestroy(s->segs[lru].gexec);
    s->segs.erase(s->segs.begin() + (long)lru);
  }
  hipGraph_t g = nullptr;
  if (!s->cap) HIP_TRY(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
  const Dev saved_d = s->d;
  const int64_t saved_since = s->steps_since_sort;
  const int e = run_block(s, s->cap, K, nullptr);
  const hipError_t ce = hipStreamEndCapture(s->cap, &g);
  // capturing executes nothing: the host-side state moves only when the
  // graph is launched (see run_impl)
  s->d = saved_d;
  s->steps_since_sort = saved_since;
  if (e) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  if (ce != hipSuccess) return fail(PR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
  hipGraphExec_t ge = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(PR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  pr_sys::Seg seg;
  seg.gexec = ge;
  seg.steps = K;
  seg.sort = with_sort;
  seg.jit = s->d.jit_c;
  seg.part = part;
  seg.fuse = s->d.fuse;
  seg.kpar0 = s->d.kpar0;
  seg.used = ++s->seg_clock;
  s->segs.push_back(seg);
  *out = ge;
  return PR_OK;
}

}  // namespace

namespace {

// Every device allocation of a resident system but the partial-counter log
// (grown on demand) and the host-read staging buffers (on first read).
int alloc_system(Arena& A, Dev& d, int32_t n, int32_t B, int64_t log_cap, hipStream_t st) {
  int e = alloc_scratch(A, d, n, std::max(sweep_blocks(n), d.nbricks), st);
  for (int q = 0; q < 2 && !e; ++q) {
    Arr& a = d.set[q];
    for (int p = 0; p < 2 && !e; ++p) {
      if (!e) e = A.alloc(&a.x[p], n);
      if (!e) e = A.alloc(&a.y[p], n);
      if (!e) e = A.alloc(&a.z[p], n);
    }
    if (!e) e = A.alloc(&a.typ, n);
    if (!e) e = A.alloc(&a.st, n);
    if (!e) e = A.alloc(&a.id, n);
    if (!e) e = A.alloc(&a.role, n);
    if (!e) e = A.alloc(&a.adj, (size_t)n * B);
  }
  if (!e) e = A.alloc(&d.log, (size_t)log_cap * 3);
  if (!e) e = A.alloc(&d.bstart, (size_t)d.nbricks + 1);
  if (!e) e = A.alloc(&d.bcnt, (size_t)d.nbricks);
  if (!e) e = A.alloc(&d.dcnt, (size_t)d.nbricks * d.nd);
  if (!e) e = A.alloc(&d.dloc, (size_t)d.nbricks * d.nd);
  if (!e) e = A.alloc(&d.rank, n);
  if (!e && !A.dry &&
      (hipMemsetAsync(d.bcnt, 0, sizeof(uint32_t) * d.nbricks, st) != hipSuccess ||
       hipMemsetAsync(d.dcnt, 0, sizeof(uint32_t) * d.nbricks * d.nd, st) != hipSuccess))
    e = fail(PR_EHIP, "hipMemsetAsync failed");
  return e;
}

}  // namespace

extern "C" {

int pr_footprint(const pr_replica_desc* r, uint32_t n_steps, int64_t* bytes) {
  if (!r || !bytes) return fail(PR_EINVAL, "NULL argument");
  if (r->n < 1 || r->n > kMaxParticles || r->B < 1)
    return fail(PR_EINVAL, "n=%d B=%d", r->n, r->B);
  if (r->brick < 0 || r->brick > kMaxBrick) return fail(PR_EINVAL, "brick=%d", r->brick);
  int e = validate_rule(&r->rule, r->L);
  if (e) return e;
  Dev d{};
  set_geometry(d, r->n, r->L, r->B, &r->rule, r->seed, r->brick > 0 ? r->brick : kDefaultBrick);
  Arena A;
  A.dry = true;
  const int64_t log_cap = r->log_cap > 0 ? r->log_cap : r->n;
  if ((e = alloc_system(A, d, r->n, r->B, log_cap, nullptr))) return e;
  // partial counters for max(1024, n_steps) steps; host-read staging buffers
  const size_t part = (size_t)std::max<uint32_t>(1024u, n_steps) * d.ngroups * kPart * 4;
  const size_t rd = (size_t)r->n * (3 * 4 + 4 + 4 * (size_t)r->B);
  *bytes = (int64_t)(A.bytes + ((part + 255) & ~(size_t)255) + rd);
  return PR_OK;
}

}  // extern "C"

namespace {

// Resources a server lends to the systems it creates: device memory drawn in
// stream order from its pool (systems are created and retired while other
// work runs, and a plain hipFree would wait for that work) and a pinned
// control word from its own pool (hipHostFree waits for the device too).
struct SysLease {
  hipMemPool_t pool = nullptr;
  Ctl* hctl = nullptr;
};

int sys_create(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule, uint64_t seed,
               int64_t log_cap, void* stream, int32_t brick, const SysLease* lease,
               int32_t nrules = 1) {
  if (!out) return fail(PR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > kMaxParticles || B < 1) return fail(PR_EINVAL, "n=%d B=%d", n, B);
  if (brick < 0 || brick > kMaxBrick) return fail(PR_EINVAL, "brick=%d", brick);
  int e = validate_rules(rule, nrules, L);
  if (e) return e;
  pr_sys* s = new pr_sys();
  s->stream = (hipStream_t)stream;
  s->arena.async = lease != nullptr;
  s->arena.astream = s->stream;
  s->arena.pool = lease ? lease->pool : nullptr;
  s->rule = *rule;
  if (lease) {
    s->hctl = lease->hctl;
    s->own_hctl = false;
  }
  if (hipGetDevice(&s->dev) != hipSuccess) {
    delete s;
    return fail(PR_EHIP, "hipGetDevice failed");
  }
  Dev& d = s->d;
  set_geometry_rules(d, n, L, B, rule, nrules, seed, brick > 0 ? brick : kDefaultBrick);
  s->log_cap = log_cap > 0 ? log_cap : n;
  e = alloc_system(s->arena, d, n, B, s->log_cap, s->stream);
  if (!e && !s->hctl && hipHostMalloc((void**)&s->hctl, sizeof(Ctl)) != hipSuccess)
    e = fail(PR_ENOMEM, "hipHostMalloc failed");
  if (!e) e = grow_part(s, 1024);
  if (e) {
    delete s;
    return e;
  }
  d.bonds = nullptr;
  d.bonds_cap = 0;
  d.log_cap = s->log_cap;
  d.sortbuf = nullptr;
  d.jitter = 1;
  s->sort_period = 64;
  set_dense(s);
  *out = s;
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_sys_create(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule, uint64_t seed,
                  int64_t log_cap, void* stream) {
  return sys_create(out, n, L, B, rule, seed, log_cap, stream, 0, nullptr);
}

int pr_sys_create_ex(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule,
                     uint64_t seed, int64_t log_cap, void* stream, int32_t brick) {
  return sys_create(out, n, L, B, rule, seed, log_cap, stream, brick, nullptr);
}

int pr_sys_create_multi(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rules,
                        int32_t nrules, uint64_t seed, int64_t log_cap, void* stream,
                        int32_t brick) {
  return sys_create(out, n, L, B, rules, seed, log_cap, stream, brick, nullptr, nrules);
}

int pr_sys_geometry(pr_sys* s, int32_t* nc, int32_t* brick, int32_t* nbricks) {
  int e = check_sys(s, false);
  if (e) return e;
  if (nc) *nc = s->d.nc;
  if (brick) *brick = s->d.bs;
  if (nbricks) *nbricks = s->d.nbricks;
  return PR_OK;
}

void pr_sys_destroy(pr_sys* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  delete s;
}

int pr_sys_load(pr_sys* s, const float* x, const float* y, const float* z, const int32_t* type,
                const int32_t* state, const int32_t* adj, int32_t on_device) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!x || !y || !z || !type || !state || !adj) return fail(PR_EINVAL, "NULL array");
  const Arr& a = s->d.set[0];
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const size_t n = (size_t)s->d.n;
  HIP_TRY(hipMemcpyAsync(a.x[0], x, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(a.y[0], y, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(a.z[0], z, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(a.typ, type, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(a.st, state, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(a.adj, adj, n * 4 * s->d.B, k, s->stream));
  return after_load(s);
}

int pr_sys_generate(pr_sys* s, int32_t kind, uint64_t gen_seed, double sigma0) {
  int e = check_sys(s, false);
  if (e) return e;
  if (kind != 0 && kind != 1) return fail(PR_EINVAL, "kind must be 0 (step) or 1 (chain)");
  if (!(sigma0 >= 0.0) || sigma0 * 6.0 >= (double)s->d.L * 0.5)
    return fail(PR_EINVAL, "sigma0=%g", sigma0);
  const Dev& d = s->d;
  int nl = 1;
  while ((long long)nl * nl * nl < (long long)d.n) ++nl;
  const float a = (float)((double)d.L / nl);
  const float c0 = (float)(sigma0 / 256.0);
  const unsigned long long thr = threshold(kind == 0 ? 0.05 : 0.001);
  HIP_TRY(launch_generate(d, kind, gen_seed, c0, a, nl, thr, s->stream));
  return after_load(s);
}

int pr_sys_set_sort_period(pr_sys* s, int32_t sort_period) {
  int e = check_sys(s, false);
  if (e) return e;
  if (sort_period < 0) return fail(PR_EINVAL, "sort_period < 0");
  s->sort_period = sort_period;
  drop_graph(s);
  return PR_OK;
}

int pr_sys_set_fused_binning(pr_sys* s, int32_t enable) {
  int e = check_sys(s, false);
  if (e) return e;
  if (enable != 0 && enable != 1) return fail(PR_EINVAL, "enable=%d (0 or 1)", enable);
  s->allow_fuse = enable;
  drop_graph(s);
  // the next run sorts first, and takes up (or leaves) fused binning there
  if (s->d.sorted && s->sort_period > 0)
    s->steps_since_sort = s->sort_period;
  else
    set_dense(s);
  s->rec_ok = false;
  return PR_OK;
}

int pr_sys_fused_binning(pr_sys* s, int32_t* active) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!active) return fail(PR_EINVAL, "active is NULL");
  *active = s->d.sorted && s->d.fuse ? 1 : 0;
  return PR_OK;
}

static int run_impl(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma, float* ms,
                    float* ms_sort = nullptr) {
  int e = check_sys(s, true);
  if (e) return e;
  if (!(sigma >= 0.0) || sigma * 6.0 >= (double)s->d.L * 0.5)
    return fail(PR_EINVAL, "sigma=%g", sigma);
  if (s->d.md_theta > 0 && sigma != 0.0)
    return fail(PR_EINVAL, "the MD of pr_sys_set_md moves the particles: sigma must be 0");
  if ((e = grow_part(s, s->steps_since_load + n_steps))) return e;
  if ((e = alloc_fused(s))) return e;
  s->d.jit_c = (float)(sigma / std::sqrt(21845.0));  // unit-variance offsets
  fuse_check_run(s, first_step);
  hipStream_t st = s->stream;
  HIP_TRY(launch_ctl_reset(s->d.ctl, first_step, 0, st));
  if (ms) {
    // phase timing: one-step blocks launched directly, HIP events around the
    // prep (jitter + A binning), the sweep and the whole step, and around
    // the sorts that fall due
    std::vector<hipEvent_t> ev((size_t)n_steps * 5 + 1);
    for (auto& v : ev) HIP_TRY(hipEventCreate(&v));
    std::vector<char> did_sort(n_steps, 0);
    for (uint32_t k = 0; k < n_steps; ++k) {
      bool sorted = false;
      if ((e = run_block(s, st, 1, &ev[3 * k], &ev[3 * n_steps + 1 + 2 * k], &sorted))) return e;
      did_sort[k] = sorted;
    }
    HIP_TRY(hipEventRecord(ev[3 * n_steps], st));
    HIP_TRY(hipEventSynchronize(ev[3 * n_steps]));
    float tp = 0, tstep = 0, tsw = 0, tsort = 0;
    int nsort = 0;
    for (uint32_t k = 0; k < n_steps; ++k) {
      float a = 0, b = 0, c = 0, so = 0;
      HIP_TRY(hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]));
      HIP_TRY(hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]));
      const size_t next = k + 1 < n_steps ? 3 * (k + 1) : 3 * n_steps;
      if (k + 1 < n_steps && did_sort[k + 1]) {
        // the next step's sort runs between this step and the next one
        HIP_TRY(hipEventElapsedTime(&c, ev[3 * k], ev[3 * n_steps + 1 + 2 * (k + 1)]));
      } else {
        HIP_TRY(hipEventElapsedTime(&c, ev[3 * k], ev[next]));
      }
      if (did_sort[k]) {
        HIP_TRY(hipEventElapsedTime(&so, ev[3 * n_steps + 1 + 2 * k],
                                    ev[3 * n_steps + 2 + 2 * k]));
        tsort += so;
        nsort++;
      }
      tp += a;
      tsw += b;
      tstep += c;
    }
    ms[0] = tp;
    ms[1] = tstep;
    ms[2] = tsw;
    if (ms_sort) {
      ms_sort[0] = tsort;
      ms_sort[1] = (float)nsort;
    }
    for (auto& v : ev) (void)hipEventDestroy(v);
    s->steps_since_load += n_steps;
    fuse_after_run(s, first_step, n_steps);
    return PR_OK;
  }
  uint32_t left = n_steps;
  while (left > 0) {
    bool with_sort = false;
    const int32_t K = next_segment(s, left, &with_sort);
    if (s->use_graphs) {
      hipGraphExec_t ge = nullptr;
      if ((e = segment_graph(s, K, with_sort, &ge))) return e;
      HIP_TRY(hipGraphLaunch(ge, st));
      after_segment(s, K, with_sort);
    } else {
      for (int32_t k = 0; k < K; ++k)
        if ((e = run_block(s, st, 1, nullptr))) return e;
    }
    left -= (uint32_t)K;
  }
  s->steps_since_load += n_steps;
  fuse_after_run(s, first_step, n_steps);
  return PR_OK;
}

int pr_sys_run(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma) {
  return run_impl(s, first_step, n_steps, sigma, nullptr);
}

int pr_sys_run_timed(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma, float* ms) {
  if (!ms) return fail(PR_EINVAL, "ms is NULL");
  return run_impl(s, first_step, n_steps, sigma, ms, ms + 3);
}

int pr_sys_prepare(pr_sys* s, uint32_t n_steps, double sigma) {
  int e = check_sys(s, true);
  if (e) return e;
  if (!(sigma >= 0.0) || sigma * 6.0 >= (double)s->d.L * 0.5)
    return fail(PR_EINVAL, "sigma=%g", sigma);
  if (!s->use_graphs) return PR_OK;
  if ((e = grow_part(s, s->steps_since_load + n_steps))) return e;
  if ((e = alloc_fused(s))) return e;
  s->d.jit_c = (float)(sigma / std::sqrt(21845.0));
  // walk the segments the run would take, capturing each, then restore the
  // host-side state (nothing ran)
  const Dev saved_d = s->d;
  const int64_t saved_since = s->steps_since_sort;
  uint32_t left = n_steps;
  while (left > 0 && !e) {
    bool with_sort = false;
    const int32_t K = next_segment(s, left, &with_sort);
    hipGraphExec_t ge = nullptr;
    e = segment_graph(s, K, with_sort, &ge);
    after_segment(s, K, with_sort);
    left -= (uint32_t)K;
  }
  s->d = saved_d;
  s->steps_since_sort = saved_since;
  return e;
}

int pr_sys_set_md(pr_sys* s, int32_t theta, double dt, double sig, double eps, double temp,
                  uint64_t vseed) {
  int e = check_sys(s, true);
  if (e) return e;
  if (theta < 0 || theta > 100000) return fail(PR_EINVAL, "theta=%d", theta);
  drop_graph(s);
  // the next run sorts first: fused binning (the MD moves the particles
  // between reaction steps) is taken up or left there
  if (s->d.sorted && s->sort_period > 0)
    s->steps_since_sort = s->sort_period;
  else
    set_dense(s);
  s->rec_ok = false;
  Dev& d = s->d;
  if (theta == 0) {
    d.md_theta = 0;
    return PR_OK;
  }
  if (!(dt > 0.0) || !(sig > 0.0) || !(eps >= 0.0) || !(temp >= 0.0) ||
      !(2.0 * std::pow(2.0, 1.0 / 6.0) * sig < 0.5 * (double)d.L))
    return fail(PR_EINVAL, "dt=%g sig=%g eps=%g temp=%g", dt, sig, eps, temp);
  const size_t n = (size_t)d.n;
  if (!d.slot_of) {
    for (int q = 0; q < 2 && !e; ++q) {
      Arr& a = d.set[q];
      if (!e) e = s->arena.alloc(&a.vx, n);
      if (!e) e = s->arena.alloc(&a.vy, n);
      if (!e) e = s->arena.alloc(&a.vz, n);
    }
    if (!e) e = s->arena.alloc(&d.slot_of, n);
    if (e) {
      for (int q = 0; q < 2; ++q) d.set[q].vx = d.set[q].vy = d.set[q].vz = nullptr;
      d.slot_of = nullptr;
      return e;
    }
  }
  // the oracle's parameters, rounded to FP32 from double
  const double sc = std::pow(2.0, 1.0 / 6.0) * sig;
  d.md_theta = theta;
  d.md_dt = (float)dt;
  d.md_h = (float)(0.5 * dt);
  const float scf = (float)sc;
  d.md_sc2 = (float)((double)scf * (double)scf);
  d.md_two_sc = (float)(2.0 * (double)scf);
  d.md_sig = (float)sig;
  d.md_e24 = (float)(24.0 * eps);
  const float cv = (float)std::sqrt(temp / 21845.0);
  HIP_TRY(launch_md_init(d, (unsigned long long)vseed, cv, s->stream));
  return sync_ctl(s);
}

int pr_sys_read_velocities(pr_sys* s, float* vx, float* vy, float* vz) {
  int e = check_sys(s, true);
  if (e) return e;
  if (!s->d.slot_of) return fail(PR_EINVAL, "no velocities: pr_sys_set_md was not called");
  if (!vx || !vy || !vz) return fail(PR_EINVAL, "NULL output");
  const size_t n = (size_t)s->d.n;
  float* buf = nullptr;
  if ((e = s->arena.alloc(&buf, 3 * n))) return e;  // kept in the arena until destroy
  HIP_TRY(launch_gather_v(s->d, buf, buf + n, buf + 2 * n, s->stream));
  HIP_TRY(hipMemcpyAsync(vx, buf, n * 4, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(vy, buf + n, n * 4, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(vz, buf + 2 * n, n * 4, hipMemcpyDeviceToHost, s->stream));
  if ((e = sync_ctl(s))) return e;
  if (s->hctl->err) return fail(s->hctl->err, "device error during the run");
  return PR_OK;
}

int pr_sys_jitter(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma,
                  float* kernel_ms) {
  int e = check_sys(s, true);
  if (e) return e;
  if (!(sigma >= 0.0) || sigma * 6.0 >= (double)s->d.L * 0.5)
    return fail(PR_EINVAL, "sigma=%g", sigma);
  if (n_steps == 0) {
    if (kernel_ms) *kernel_ms = 0.0f;
    return PR_OK;
  }
  s->d.jit_c = (float)(sigma / std::sqrt(21845.0));
  s->rec_ok = false;  // the particles move: the next run bins again (after a sort)
  hipStream_t st = s->stream;
  HIP_TRY(launch_ctl_reset(s->d.ctl, first_step, 0, st));
  if (!kernel_ms) {
    HIP_TRY(launch_jitter_only(s->d, (int)n_steps, st, nullptr, nullptr));
    s->d.kpar0 = (s->d.kpar0 + n_steps) & 1u;
    return PR_OK;
  }
  // per-step kernel times, stamped at each kernel's own start and end
  float total = 0.0f;
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreate(&ev[0]));
  HIP_TRY(hipEventCreate(&ev[1]));
  for (uint32_t k = 0; k < n_steps && !e; ++k) {
    Dev dk = s->d;
    if (launch_jitter_only(dk, 1, st, ev[0], ev[1]) != hipSuccess ||
        hipEventSynchronize(ev[1]) != hipSuccess) {
      e = fail(PR_EHIP, "jitter-only launch failed");
      break;
    }
    s->d.kpar0 = (s->d.kpar0 + 1u) & 1u;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    total += ms;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  *kernel_ms = total;
  return e;
}

int pr_sys_kinetics(pr_sys* s, int32_t nstate, int64_t* pop, int64_t* pairs, int32_t nbins,
                    int64_t* hist) {
  int e = check_sys(s, true);
  if (e) return e;
  if (nstate < 1 || nstate > kKinMaxState || nbins < 0 || nbins > kKinMaxBins)
    return fail(PR_EINVAL, "nstate=%d (1..%d), nbins=%d (0..%d)", nstate, kKinMaxState, nbins,
                kKinMaxBins);
  if (!pop || !pairs || (nbins > 0 && !hist)) return fail(PR_EINVAL, "NULL output");
  if (s->d.nrules > 1) return fail(PR_EINVAL, "kinetics counters take one rule");
  // kKinSlices slices of counters (the kernels spread their sums over them)
  const size_t nk = (size_t)kKinStride * kKinSlices;
  if (!s->kin && ((e = s->arena.alloc(&s->kin, nk)) ||
                  (e = s->arena.alloc(&s->kin_e2, (size_t)kKinMaxBins + 1))))
    return e;
  // bin edges: e2[b] = fl32((rc b / nbins)^2), the product taken in double
  std::vector<float> e2((size_t)nbins + 1);
  for (int b = 0; b <= nbins; ++b) {
    const double r = (double)s->rule.rc * (double)b / (double)nbins;
    e2[(size_t)b] = (float)(r * r);
  }
  hipStream_t st = s->stream;
  unsigned long long *kp = s->kin, *kq = s->kin + kKinMaxState, *kh = s->kin + 2 * kKinMaxState;
  HIP_TRY(hipMemcpyAsync(s->kin_e2, e2.data(), e2.size() * sizeof(float), hipMemcpyHostToDevice,
                         st));
  HIP_TRY(launch_fill_u32((uint32_t*)s->kin, 2 * (long long)nk, 0u, st));
  HIP_TRY(launch_kinetics(s->d, nstate, nbins, s->kin_e2, kp, kq, kh, st));
  std::vector<unsigned long long> h(kKinStride);  // the first slice holds the sums
  HIP_TRY(hipMemcpyAsync(h.data(), s->kin, (size_t)kKinStride * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
  if ((e = sync_ctl(s))) return e;
  if (s->hctl->err) return fail(s->hctl->err, "device error during the run");
  for (int q = 0; q < nstate; ++q) {
    pop[q] = (int64_t)h[(size_t)q];
    pairs[q] = (int64_t)h[(size_t)(kKinMaxState + q)];
  }
  for (int b = 0; b < nbins; ++b) hist[b] = (int64_t)h[(size_t)(2 * kKinMaxState + b)];
  return PR_OK;
}

int pr_sqrt_rn(const float* in, float* out, int64_t n, void* stream) {
  if (n < 0 || n > (int64_t)kMaxParticles) return fail(PR_EINVAL, "n=%lld", (long long)n);
  if (n > 0 && (!in || !out)) return fail(PR_EINVAL, "NULL array");
  HIP_TRY(launch_sqrt_rn(in, out, (long long)n, (hipStream_t)stream));
  return PR_OK;
}

int pr_stream_copy(const void* src, void* dst, int64_t bytes, int32_t width, void* stream,
                   float* kernel_ms) {
  if (width != 4 && width != 8 && width != 16) return fail(PR_EINVAL, "width=%d", width);
  if (bytes < 0 || bytes % width) return fail(PR_EINVAL, "bytes=%lld", (long long)bytes);
  if (bytes == 0) {
    if (kernel_ms) *kernel_ms = 0.0f;
    return PR_OK;
  }
  if (!src || !dst) return fail(PR_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (kernel_ms) {
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
  }
  const hipError_t he = launch_stream_copy(src, dst, (long long)bytes, width, st, ev[0], ev[1]);
  int e = he == hipSuccess ? PR_OK : fail(PR_EHIP, "stream copy: %s", hipGetErrorString(he));
  if (kernel_ms && !e) {
    if (hipEventSynchronize(ev[1]) != hipSuccess) e = fail(PR_EHIP, "hipEventSynchronize");
    else (void)hipEventElapsedTime(kernel_ms, ev[0], ev[1]);
  }
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  return e;
}

namespace {

// The configuration in particle-id order into host or device memory (any
// pointer may be NULL); synchronises and reports a pending device error.
int sys_read(pr_sys* s, float* x, float* y, float* z, int32_t* type, int32_t* state,
             int32_t* adj, int32_t on_device) {
  int e = check_sys(s, false);
  if (e) return e;
  const Dev& d = s->d;
  const size_t n = (size_t)d.n;
  if (on_device) {
    HIP_TRY(launch_gather_out(d, x, y, z, type, state, adj, s->stream));
  } else {
    if (!s->rx) {
      if ((e = s->arena.alloc(&s->rx, n)) || (e = s->arena.alloc(&s->ry, n)) ||
          (e = s->arena.alloc(&s->rz, n)) || (e = s->arena.alloc(&s->rst, n)) ||
          (e = s->arena.alloc(&s->radj, n * d.B)))
        return e;
    }
    if (type && !s->rtyp && (e = s->arena.alloc(&s->rtyp, n))) return e;
    HIP_TRY(launch_gather_out(d, x ? s->rx : nullptr, y ? s->ry : nullptr, z ? s->rz : nullptr,
                              type ? s->rtyp : nullptr, state ? s->rst : nullptr,
                              adj ? s->radj : nullptr, s->stream));
    const hipMemcpyKind k = hipMemcpyDeviceToHost;
    if (x) HIP_TRY(hipMemcpyAsync(x, s->rx, n * 4, k, s->stream));
    if (y) HIP_TRY(hipMemcpyAsync(y, s->ry, n * 4, k, s->stream));
    if (z) HIP_TRY(hipMemcpyAsync(z, s->rz, n * 4, k, s->stream));
    if (type) HIP_TRY(hipMemcpyAsync(type, s->rtyp, n * 4, k, s->stream));
    if (state) HIP_TRY(hipMemcpyAsync(state, s->rst, n * 4, k, s->stream));
    if (adj) HIP_TRY(hipMemcpyAsync(adj, s->radj, n * 4 * d.B, k, s->stream));
  }
  if ((e = sync_ctl(s))) return e;
  if (s->hctl->err) return fail(s->hctl->err, "device error during the run");
  return PR_OK;
}

}  // namespace

int pr_sys_read(pr_sys* s, float* x, float* y, float* z, int32_t* state, int32_t* adj,
                int32_t on_device) {
  return sys_read(s, x, y, z, nullptr, state, adj, on_device);
}

}  // extern "C"

namespace {

// The bond log in (step, id_A) order.  pin (may be NULL): pinned host memory
// of pin_bytes for the device copy (the rows are ordered in place there).
int sys_bonds(pr_sys* s, int32_t* out, int64_t cap, int64_t* n, void* pin, size_t pin_bytes) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL output");
  if ((e = sync_ctl(s))) return e;
  const int64_t total = (int64_t)s->hctl->log_n;
  const int64_t have = std::min<int64_t>(total, s->log_cap);
  const int64_t m = std::min<int64_t>(have, cap);
  if (m > 0) {
    // the rows of one step were appended in workgroup order: the device
    // orders the log in place by (step, id_A) (log_order), then it is copied
    struct Row {
      int32_t step, a, t;
    };
    HIP_TRY(log_order(s->d.log, have, s->stream));
    std::vector<Row> vrows;
    Row* rows = nullptr;
    if (pin && pin_bytes >= (size_t)m * sizeof(Row)) {
      rows = (Row*)pin;
    } else {
      vrows.resize((size_t)m);
      rows = vrows.data();
    }
    HIP_TRY(hipMemcpyAsync(rows, s->d.log, (size_t)m * sizeof(Row), hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->d.nrules > 1)  // the rule of each bond rides in bits 30-31 of id_T
      for (size_t i = 0; i < (size_t)m; ++i) rows[i].t &= 0x3FFFFFFF;
    std::memcpy(out, rows, (size_t)m * sizeof(Row));
  }
  *n = total;
  if (total > s->log_cap)
    return fail(PR_ECAP, "bond log overflowed: %lld > %lld", (long long)total,
                (long long)s->log_cap);
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_sys_bonds(pr_sys* s, int32_t* out, int64_t cap, int64_t* n) {
  return sys_bonds(s, out, cap, n, nullptr, 0);
}

int pr_sys_stats(pr_sys* s, pr_stats* out, int64_t cap, int64_t* n) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL output");
  if ((e = sync_ctl(s))) return e;
  const int64_t have = std::min<int64_t>((int64_t)s->hctl->stats_n0, s->part_cap);
  const int64_t m = std::min<int64_t>(have, cap);
  if (m > 0) {
    const size_t row = (size_t)s->d.ngroups * kPart;
    std::vector<int32_t> p((size_t)m * row);
    HIP_TRY(hipMemcpyAsync(p.data(), s->d.part, p.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int64_t k = 0; k < m; ++k) {
      long long h[kPart] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int g = 0; g < s->d.ngroups; ++g)
        for (int q = 0; q < kPart; ++q) h[q] += p[(size_t)k * row + (size_t)g * kPart + q];
      out[k] = stats_of(h, s->rule.policy);
    }
  }
  *n = have;
  return PR_OK;
}

}  // extern "C"

namespace {

// Layout of a checkpoint: this header, then x, y, z, type, state (n each),
// adj (n * B), the bond-log rows (3 int32 each) and the per-step counters.
struct CkHeader {
  char magic[8];
  int32_t n, B;
  float L;
  int32_t exclude_bonded;
  uint64_t seed;
  int32_t type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t;
  float rc;
  int32_t policy;
  double p;
  int64_t rows, steps;
};
constexpr char kCkMagic[8] = {'P', 'R', 'C', 'K', 'P', 'T', '0', '1'};

int64_t ck_bytes(const Dev& d, int64_t rows, int64_t steps) {
  return (int64_t)sizeof(CkHeader) + (int64_t)d.n * (5 * 4 + 4 * (int64_t)d.B) + rows * 12 +
         steps * (int64_t)sizeof(pr_stats);
}

bool same_rule(const CkHeader& h, const pr_sys* s) {
  const pr_rule& r = s->rule;
  return h.n == s->d.n && h.B == s->d.B && h.L == s->d.L && h.seed == s->d.seed &&
         h.type_a == r.type_a && h.a_min == r.a_min && h.a_max == r.a_max && h.d_a == r.d_a &&
         h.type_t == r.type_t && h.t_min == r.t_min && h.t_max == r.t_max && h.d_t == r.d_t &&
         h.rc == r.rc && h.p == r.p && h.exclude_bonded == r.exclude_bonded &&
         h.policy == r.policy;
}

}  // namespace

extern "C" {

int pr_sys_checkpoint(pr_sys* s, void* buf, int64_t cap, int64_t* bytes) {
  int e = check_sys(s, true);
  if (e) return e;
  if (s->d.nrules > 1) return fail(PR_EINVAL, "checkpoints hold one rule");
  if (s->d.md_theta > 0) return fail(PR_EINVAL, "checkpoints hold no velocities");
  if (!bytes) return fail(PR_EINVAL, "bytes is NULL");
  if ((e = sync_ctl(s))) return e;
  if (s->hctl->err) return fail(s->hctl->err, "device error during the run");
  const int64_t rows = (int64_t)s->hctl->log_n;
  if (rows > s->log_cap)
    return fail(PR_ECAP, "bond log overflowed (%lld > %lld): no complete checkpoint",
                (long long)rows, (long long)s->log_cap);
  const int64_t steps = std::min<int64_t>((int64_t)s->hctl->stats_n0, s->part_cap);
  const Dev& d = s->d;
  const int64_t need = ck_bytes(d, rows, steps);
  *bytes = need;
  if (!buf) return PR_OK;
  if (cap < need) return fail(PR_ECAP, "checkpoint needs %lld bytes", (long long)need);
  CkHeader h{};
  std::memcpy(h.magic, kCkMagic, 8);
  const pr_rule& r = s->rule;
  h.n = d.n;
  h.B = d.B;
  h.L = d.L;
  h.exclude_bonded = r.exclude_bonded;
  h.seed = d.seed;
  h.type_a = r.type_a;
  h.a_min = r.a_min;
  h.a_max = r.a_max;
  h.d_a = r.d_a;
  h.type_t = r.type_t;
  h.t_min = r.t_min;
  h.t_max = r.t_max;
  h.d_t = r.d_t;
  h.rc = r.rc;
  h.policy = r.policy;
  h.p = r.p;
  h.rows = rows;
  h.steps = steps;
  char* q = (char*)buf;
  std::memcpy(q, &h, sizeof h);
  q += sizeof h;
  const size_t n = (size_t)d.n;
  float* x = (float*)q;
  int32_t* typ = (int32_t*)(x + 3 * n);
  int32_t* st = typ + n;
  int32_t* adj = st + n;
  int32_t* log = adj + n * d.B;
  pr_stats* stats = (pr_stats*)(log + 3 * rows);
  if ((e = sys_read(s, x, x + n, x + 2 * n, typ, st, adj, 0))) return e;
  int64_t got = 0;
  if ((e = sys_bonds(s, log, rows, &got, nullptr, 0))) return e;
  if ((e = pr_sys_stats(s, stats, steps, &got))) return e;
  return PR_OK;
}

int pr_sys_restore(pr_sys* s, const void* buf, int64_t bytes) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!buf || bytes < (int64_t)sizeof(CkHeader)) return fail(PR_EINVAL, "no checkpoint");
  CkHeader h;
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, kCkMagic, 8) != 0) return fail(PR_EINVAL, "not a checkpoint");
  if (!same_rule(h, s)) return fail(PR_EINVAL, "checkpoint of another system (n, B, L, rule, seed)");
  if (h.rows < 0 || h.steps < 0 || bytes != ck_bytes(s->d, h.rows, h.steps))
    return fail(PR_EINVAL, "malformed checkpoint");
  if (h.rows > s->log_cap)
    return fail(PR_ECAP, "checkpoint holds %lld bonds, log capacity %lld", (long long)h.rows,
                (long long)s->log_cap);
  const Dev& d0 = s->d;
  const size_t n = (size_t)d0.n, row = (size_t)d0.ngroups * kPart;
  const char* q = (const char*)buf + sizeof h;
  const float* x = (const float*)q;
  const int32_t* typ = (const int32_t*)(x + 3 * n);
  const int32_t* st = typ + n;
  const int32_t* adj = st + n;
  const int32_t* log = adj + n * d0.B;
  std::vector<int32_t> part((size_t)h.steps * row, 0);
  for (int64_t k = 0; k < h.steps; ++k) {
    pr_stats t;
    std::memcpy(&t, (const char*)(log + 3 * h.rows) + k * sizeof(pr_stats), sizeof t);
    // partial layout: a_elig, t_elig, in_rc, drawn, excluded, proposals, bonds, lost
    const int64_t v[kPart] = {t.a_elig,   t.t_elig,    t.in_rc, t.drawn,
                              t.excluded, t.proposals, t.bonds, t.adj_overflow};
    for (int c = 0; c < kPart; ++c) {
      int64_t left = v[c];
      if (left < 0) return fail(PR_EINVAL, "malformed checkpoint (negative counter)");
      for (int g = 0; g < d0.ngroups && left > 0; ++g) {
        const int64_t put = std::min<int64_t>(left, INT32_MAX);
        part[(size_t)k * row + (size_t)g * kPart + c] = (int32_t)put;
        left -= put;
      }
      if (left > 0) return fail(PR_EINVAL, "counter too large for the counter log");
    }
  }
  // the configuration (validated on the device), then the logs
  if ((e = pr_sys_load(s, x, x + n, x + 2 * n, typ, st, adj, 0))) return e;
  if ((e = grow_part(s, h.steps))) return e;
  const Dev& d = s->d;
  if (h.rows > 0)
    HIP_TRY(hipMemcpyAsync(d.log, log, (size_t)h.rows * 12, hipMemcpyHostToDevice, s->stream));
  if (h.steps > 0)
    HIP_TRY(hipMemcpyAsync(d.part, part.data(), part.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s->stream));
  const uint32_t n0 = (uint32_t)h.steps;
  const uint64_t ln = (uint64_t)h.rows;
  HIP_TRY(hipMemcpyAsync(&d.ctl->stats_n0, &n0, sizeof n0, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(&d.ctl->log_n, &ln, sizeof ln, hipMemcpyHostToDevice, s->stream));
  s->steps_since_load = h.steps;
  return sync_ctl(s);
}

int pr_autotune(const pr_replica_desc* r, uint32_t n_steps, double sigma, int32_t copies,
                void* stream, int32_t* best, float* us) {
  if (!r || !best) return fail(PR_EINVAL, "NULL argument");
  if (n_steps < 1 || copies < 1) return fail(PR_EINVAL, "n_steps=%u copies=%d", n_steps, copies);
  *best = 0;
  if (us)
    for (int b = 0; b < kMaxBrick; ++b) us[b] = -1.0f;
  int64_t bytes = 0;
  int e = pr_footprint(r, n_steps + 64, &bytes);  // validates the description
  if (e) return e;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    for (hipEvent_t v : ev)
      if (v) (void)hipEventDestroy(v);
    return fail(PR_EHIP, "hipEventCreate failed");
  }
  float best_us = 0.0f;
  std::vector<int32_t> tried;  // brick counts already timed (clamped requests repeat one)
  for (int b = 1; b <= kMaxBrick && !e; ++b) {
    Dev g{};
    set_geometry(g, r->n, r->L, r->B, &r->rule, r->seed, b);
    if (std::find(tried.begin(), tried.end(), g.nbricks) != tried.end()) continue;
    tried.push_back(g.nbricks);
    // one system, or `copies` identical replicas stepped as one batch; one
    // untimed block (first sort, graph capture), then n_steps timed
    pr_replica_desc q = *r;
    q.brick = b;
    pr_sys* s = nullptr;
    pr_batch* bt = nullptr;
    if (copies == 1) {
      e = sys_create(&s, q.n, q.L, q.B, &q.rule, q.seed, q.log_cap, stream, b, nullptr);
      if (!e) e = pr_sys_generate(s, q.gen_kind, q.gen_seed, q.gen_sigma0);
      if (!e) e = pr_sys_run(s, 1, 64, sigma);
    } else {
      std::vector<pr_replica_desc> qs((size_t)copies, q);
      e = pr_batch_create(&bt, qs.data(), copies, stream);
      if (!e) e = pr_batch_run(bt, 1, 64, sigma);
    }
    float ms = 0.0f;
    if (!e) {
      if (hipEventRecord(ev[0], st) != hipSuccess) e = fail(PR_EHIP, "hipEventRecord failed");
      if (!e) e = s ? pr_sys_run(s, 65, n_steps, sigma) : pr_batch_run(bt, 65, n_steps, sigma);
      if (!e && (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                 hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
        e = fail(PR_EHIP, "timing events failed");
    }
    if (s) pr_sys_destroy(s);
    if (bt) pr_batch_destroy(bt);
    if (e) break;
    const float t = ms * 1000.0f / ((float)n_steps * (float)copies);
    if (us) us[g.bs - 1] = t;
    if (*best == 0 || t < best_us) {
      *best = g.bs;
      best_us = t;
    }
  }
  for (hipEvent_t v : ev) (void)hipEventDestroy(v);
  return e;
}

int pr_autotune_cached(const pr_replica_desc* r, uint32_t n_steps, double sigma, int32_t copies,
                       void* stream, const char* cache_path, int32_t* best, float* us) {
  if (!cache_path) return pr_autotune(r, n_steps, sigma, copies, stream, best, us);
  if (!r || !best) return fail(PR_EINVAL, "NULL argument");
  if (copies < 1) return fail(PR_EINVAL, "copies=%d", copies);
  int64_t bytes = 0;
  int e = pr_footprint(r, n_steps + 64, &bytes);  // validates the description
  if (e) return e;
  Dev g{};
  set_geometry(g, r->n, r->L, r->B, &r->rule, r->seed, kDefaultBrick);
  // one line per tuned geometry: "pr-tune 2 <nc> <copies> <B> <best> <us 1..kMaxBrick>"
  static_assert(kMaxBrick == 6, "the cache line holds six times");
  if (FILE* f = std::fopen(cache_path, "r")) {
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
      int ver = 0, nc = 0, cp = 0, bw = 0, b = 0;
      float t[kMaxBrick] = {-1.0f, -1.0f, -1.0f, -1.0f, -1.0f, -1.0f};
      if (std::sscanf(line, "pr-tune %d %d %d %d %d %f %f %f %f %f %f", &ver, &nc, &cp, &bw, &b,
                      &t[0], &t[1], &t[2], &t[3], &t[4], &t[5]) == 5 + kMaxBrick &&
          ver == 2 && nc == g.nc && cp == copies && bw == r->B && b >= 1 && b <= kMaxBrick) {
        std::fclose(f);
        *best = b;
        if (us)
          for (int q = 0; q < kMaxBrick; ++q) us[q] = t[q];
        return PR_OK;
      }
    }
    std::fclose(f);
  }
  float t[kMaxBrick];
  if ((e = pr_autotune(r, n_steps, sigma, copies, stream, best, t))) return e;
  if (us)
    for (int q = 0; q < kMaxBrick; ++q) us[q] = t[q];
  FILE* f = std::fopen(cache_path, "a");
  if (!f) return fail(PR_EINVAL, "cannot append to the tuning cache %s", cache_path);
  std::fprintf(f, "pr-tune 2 %d %d %d %d %.3f %.3f %.3f %.3f %.3f %.3f\n", g.nc, copies, r->B,
               *best, t[0], t[1], t[2], t[3], t[4], t[5]);
  std::fclose(f);
  return PR_OK;
}

int pr_sys_set_graphs(pr_sys* s, int32_t on) {
  int e = check_sys(s, false);
  if (e) return e;
  s->use_graphs = on ? 1 : 0;
  drop_graph(s);
  return PR_OK;
}

}  // extern "C"

// ===========================================================================
// Batched ensembles
// ===========================================================================
namespace pr {
hipError_t launch_ctl_b(const BatchLaunch& b, int op, uint32_t arg, hipStream_t s);
hipError_t launch_step_b(const BatchLaunch& b, int k, hipStream_t s);
hipError_t launch_block_end_b(const BatchLaunch& b, int K, hipStream_t s);
hipError_t launch_sort_b(const BatchLaunch& b, hipStream_t s);
}  // namespace pr

struct pr_batch {
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  std::vector<pr_sys*> sys;
  Arena arena;
  BatchLaunch bl{};
  Dev* ds = nullptr;              // device copies of the replicas' Devs
  std::vector<Dev> hds;           // host staging of the same
  hipEvent_t copied = nullptr;    // the last upload of hds has completed
  int32_t sort_period = 64;
  hipGraphExec_t gexec = nullptr;
  int32_t g_steps = 0;
  ~pr_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (copied) (void)hipEventDestroy(copied);
    if (cap) (void)hipStreamDestroy(cap);
    for (pr_sys* s : sys) pr_sys_destroy(s);
  }
};

namespace {

int check_batch(pr_batch* b, int32_t rep) {
  if (!b) return fail(PR_EINVAL, "NULL batch handle");
  if (rep < 0 || rep >= (int32_t)b->sys.size())
    return fail(PR_EINVAL, "replica %d outside [0, %zu)", rep, b->sys.size());
  return PR_OK;
}

// Maps of grid blocks to (replica, local block, blocks of the replica) for
// the sorted-storage kernels of the batch.
int fill_maps(const std::vector<pr_sys*>& sys, Arena& arena, BatchLaunch& bl) {
  std::vector<int4> prep0, prepk, sweep, close, part, res;
  int n_sortl = 1, two = 0, any_random = 0, any_nearest = 0;
  for (int r = 0; r < (int)sys.size(); ++r) {
    const Dev& d = sys[r]->d;
    if (d.bs > kOneCellBrick && d.nbricks > 1) two = 1;
    if (d.rule.policy == PR_POLICY_NEAREST) any_nearest = 1;
    else any_random = 1;
    n_sortl = std::max(n_sortl, (d.nbricks + kThreads / 64 - 1) / (kThreads / 64));
    for (int q = 0; q < d.nwg_prep; ++q) prep0.push_back(make_int4(r, q, d.nwg_prep, 0));
    for (int q = 0; q < d.ngroups + d.nwg_prep; ++q)
      prepk.push_back(make_int4(r, q, d.ngroups + d.nwg_prep, 0));
    for (int q = 0; q < d.nbricks; ++q) sweep.push_back(make_int4(r, q, d.nbricks, 0));
    for (int q = 0; q < (d.nbricks + 3) / 4; ++q) res.push_back(make_int4(r, q, d.nbricks, 0));
    for (int q = 0; q < d.ngroups; ++q) close.push_back(make_int4(r, q, d.ngroups, 0));
    const int np = (d.n + kThreads - 1) / kThreads;
    for (int q = 0; q < np; ++q) part.push_back(make_int4(r, q, np, 0));
  }
  int4 *m0, *mk, *ms, *mc, *mp, *mr;
  int e;
  if ((e = arena.alloc(&m0, prep0.size())) || (e = arena.alloc(&mk, prepk.size())) ||
      (e = arena.alloc(&ms, sweep.size())) || (e = arena.alloc(&mc, close.size())) ||
      (e = arena.alloc(&mp, part.size())) || (e = arena.alloc(&mr, res.size())))
    return e;
  HIP_TRY(hipMemcpy(m0, prep0.data(), prep0.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(mk, prepk.data(), prepk.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ms, sweep.data(), sweep.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(mc, close.data(), close.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(mp, part.data(), part.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(mr, res.data(), res.size() * sizeof(int4), hipMemcpyHostToDevice));
  bl.prep0 = m0;
  bl.prepk = mk;
  bl.sweep = ms;
  bl.close = mc;
  bl.part = mp;
  bl.n_prep0 = (int)prep0.size();
  bl.n_prepk = (int)prepk.size();
  bl.n_sweep = (int)sweep.size();
  bl.n_close = (int)close.size();
  bl.n_part = (int)part.size();
  bl.n_sortl = n_sortl;
  bl.two = two;
  bl.any_random = any_random;
  bl.any_nearest = any_nearest;
  bl.fuse = 0;  // set by the batch when every replica has its fused buckets
  bl.res = mr;
  bl.n_res = (int)res.size();
  bl.nrep = (int)sys.size();
  return PR_OK;
}

// One block of K steps for every replica: a sort, the steps, the block end.
int run_block_b(const BatchLaunch& bl, hipStream_t st, int32_t K) {
  HIP_TRY(launch_sort_b(bl, st));
  for (int32_t k = 0; k < K; ++k) HIP_TRY(launch_step_b(bl, k, st));
  HIP_TRY(launch_block_end_b(bl, K, st));
  return PR_OK;
}

int capture_block_b(pr_batch* b, int32_t K) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int e = run_block_b(b->bl, b->cap, K);
  const hipError_t ce = hipStreamEndCapture(b->cap, &g);
  if (e) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  if (ce != hipSuccess) return fail(PR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
  const hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    b->gexec = nullptr;
    return fail(PR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  }
  b->g_steps = K;
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_batch_create(pr_batch** out, const pr_replica_desc* reps, int32_t n_rep, void* stream) {
  if (!out) return fail(PR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_rep < 1 || !reps) return fail(PR_EINVAL, "n_rep=%d", n_rep);
  pr_batch* b = new pr_batch();
  b->stream = (hipStream_t)stream;
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return fail(PR_EHIP, "hipStreamCreate/hipEventCreate failed");
  }
  int e = PR_OK;
  for (int32_t r = 0; r < n_rep && !e; ++r) {
    const pr_replica_desc& q = reps[r];
    pr_sys* s = nullptr;
    e = pr_sys_create_ex(&s, q.n, q.L, q.B, &q.rule, q.seed, q.log_cap, stream, q.brick);
    if (!e) {
      b->sys.push_back(s);
      e = pr_sys_generate(s, q.gen_kind, q.gen_seed, q.gen_sigma0);
    }
    if (e) {
      const std::string msg = g_err;
      fail(e, "replica %d: %s", r, msg.c_str());
    }
  }
  if (!e) e = fill_maps(b->sys, b->arena, b->bl);
  // fused binning when every replica can take it (one rule, the random
  // selection): no binning kernel in the batch's steps
  if (!e && !b->bl.any_nearest) {
    bool all = true;
    for (pr_sys* s : b->sys) {
      if (alloc_fused(s) != PR_OK || !s->d.fcnt[0]) {
        all = false;
        break;
      }
    }
    b->bl.fuse = all ? 1 : 0;
  }
  if (!e) e = b->arena.alloc(&b->ds, (size_t)n_rep);
  if (e) {
    delete b;
    return e;
  }
  b->bl.ds = b->ds;
  b->bl.nrep = n_rep;
  b->hds.resize((size_t)n_rep);
  *out = b;
  return PR_OK;
}

void pr_batch_destroy(pr_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  delete b;
}

int pr_batch_run(pr_batch* b, uint32_t first_step, uint32_t n_steps, double sigma) {
  int e = check_batch(b, 0);
  if (e) return e;
  for (pr_sys* s : b->sys) {
    if ((e = check_sys(s, true))) return e;
    if (!(sigma >= 0.0) || sigma * 6.0 >= (double)s->d.L * 0.5)
      return fail(PR_EINVAL, "sigma=%g", sigma);
  }
  if (n_steps == 0) return PR_OK;
  hipStream_t st = b->stream;
  HIP_TRY(hipEventSynchronize(b->copied));  // the staging copy of a previous run is done
  // the replicas' Devs as the batch's blocks leave them: storage sorted at
  // the start of every block, logs sized for the whole run
  for (size_t r = 0; r < b->sys.size(); ++r) {
    pr_sys* s = b->sys[r];
    if ((e = grow_part(s, s->steps_since_load + n_steps))) return e;
    s->d.jit_c = (float)(sigma / std::sqrt(21845.0));
    s->d.sorted = 1;
    s->d.fuse = b->bl.fuse;  // the batch's sweeps bin the next step's A's, or k_prep_b does
    s->rec_ok = false;
    s->d.nwg_sweep = s->d.nbricks;
    b->hds[r] = s->d;
    b->hds[r].k_limit = INT32_MAX;
    b->hds[r].first_step = first_step;
  }
  HIP_TRY(hipMemcpyAsync(b->ds, b->hds.data(), sizeof(Dev) * b->hds.size(),
                         hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(b->copied, st));
  HIP_TRY(launch_ctl_b(b->bl, 0, 0u, st));
  const int32_t K = b->sort_period;
  uint32_t left = n_steps;
  while (left > 0) {
    if (left >= (uint32_t)K) {
      if (!b->gexec || b->g_steps != K)
        if ((e = capture_block_b(b, K))) return e;
      HIP_TRY(hipGraphLaunch(b->gexec, st));
      left -= (uint32_t)K;
    } else {
      if ((e = run_block_b(b->bl, st, (int32_t)left))) return e;
      left = 0;
    }
  }
  // host-side state of every replica after the run
  for (pr_sys* s : b->sys) {
    drop_graph(s);
    s->steps_since_sort = n_steps % (uint32_t)K == 0 ? K : (int32_t)(n_steps % (uint32_t)K);
    s->steps_since_load += n_steps;
    s->d.kpar0 = (s->d.kpar0 + n_steps) & 1u;  // the batch advanced the parity origin
  }
  return PR_OK;
}

int pr_batch_run_loop(pr_batch* b, uint32_t first_step, uint32_t n_steps, double sigma) {
  int e = check_batch(b, 0);
  if (e) return e;
  for (pr_sys* s : b->sys) {
    const int32_t g = s->use_graphs;
    s->use_graphs = 0;
    drop_graph(s);
    e = pr_sys_run(s, first_step, n_steps, sigma);
    s->use_graphs = g;
    if (e) return e;
  }
  return PR_OK;
}

int pr_batch_bonds(pr_batch* b, int32_t rep, int32_t* out, int64_t cap, int64_t* n) {
  int e = check_batch(b, rep);
  return e ? e : pr_sys_bonds(b->sys[rep], out, cap, n);
}

int pr_batch_read(pr_batch* b, int32_t rep, float* x, float* y, float* z, int32_t* state,
                  int32_t* adj, int32_t on_device) {
  int e = check_batch(b, rep);
  return e ? e : pr_sys_read(b->sys[rep], x, y, z, state, adj, on_device);
}

int pr_batch_stats(pr_batch* b, int32_t rep, pr_stats* out, int64_t cap, int64_t* n) {
  int e = check_batch(b, rep);
  return e ? e : pr_sys_stats(b->sys[rep], out, cap, n);
}

int pr_batch_kinetics(pr_batch* b, int32_t rep, int32_t nstate, int64_t* pop, int64_t* pairs,
                      int32_t nbins, int64_t* hist) {
  int e = check_batch(b, rep);
  return e ? e : pr_sys_kinetics(b->sys[rep], nstate, pop, pairs, nbins, hist);
}

}  // extern "C"

// ===========================================================================
// Serving
// ===========================================================================
namespace {

using Clock = std::chrono::steady_clock;

struct SrvReq {
  uint64_t ticket = 0;
  pr_replica_desc desc{};
  uint32_t n_steps = 0, done_steps = 0, round_steps = 0;
  double sigma = 0.0;
  int64_t bytes = 0;
  Clock::time_point t_submit, t_done;
  int32_t status = 0;  // 0 queued, 1 running, 2 done, 3 failed
  int32_t code = 0;
  std::atomic<bool> cancel{false};  // admitted and cancelled: retired at the round's end
  pr_sys* sys = nullptr;
  // results, host memory
  std::vector<int32_t> bonds;
  int64_t n_bonds = 0;
  std::vector<float> x, y, z;
  std::vector<int32_t> state, adj;
  std::vector<pr_stats> stats;
};

}  // namespace

struct pr_server {
  int dev = 0;
  int64_t budget = 0, used = 0;
  int32_t max_slots = 1;
  hipStream_t stream = nullptr;    // rounds
  hipStream_t iostream = nullptr;  // admission (generation) and result copies
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SrvReq*> queue;
  std::vector<SrvReq*> active;  // worker thread only (under mu when changed)
  std::unordered_map<uint64_t, SrvReq*> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t rounds = 0, n_done = 0, n_failed = 0;
  double busy_s = 0.0, admit_s = 0.0, finish_s = 0.0, launch_s = 0.0, wait_s = 0.0;
  std::thread worker;
  // batched launch state of the active set
  Arena maps;
  BatchLaunch bl{};
  Arena dsa;
  Dev* ds = nullptr;
  size_t ds_cap = 0;
  std::vector<Dev> hds;
  bool set_changed = true;
  // what the server lends its systems: a stream-ordered device pool that
  // keeps up to the budget mapped, and pinned control words (never freed
  // while the server lives: freeing pinned memory waits for the device)
  hipMemPool_t pool = nullptr;
  // the control-word pool is shared by the worker (admission, failures) and
  // the finisher (retirement): every use holds ctl_mu
  std::mutex ctl_mu;
  std::vector<Ctl*> ctl_chunks, ctl_free;
  // retirement runs on its own thread and stream: results copied out (into
  // pinned staging, grown and never shrunk: freeing pinned memory waits for
  // the device), systems destroyed, memory handed back; the worker meanwhile
  // launches the next round
  std::thread finisher;
  std::deque<SrvReq*> fin_q;
  std::condition_variable cv_fin;
  bool fin_stop = false;
  uint64_t freed = 0;  // retirements so far (the worker waits on it when memory is short)
  hipStream_t fstream = nullptr;
  void* stage = nullptr;
  size_t stage_bytes = 0;
};

namespace {

// The worker's results copy of a finished replica, then its device memory
// freed.  Returns the error code (0 = done).
// A pinned control word from the server's pool (worker thread; the
// finisher returns words concurrently, so both hold ctl_mu).
Ctl* srv_ctl(pr_server* S) {
  std::lock_guard<std::mutex> lk(S->ctl_mu);
  if (S->ctl_free.empty()) {
    const int chunk = 64;
    Ctl* c = nullptr;
    if (hipHostMalloc((void**)&c, sizeof(Ctl) * chunk) != hipSuccess) return nullptr;
    S->ctl_chunks.push_back(c);
    for (int i = chunk - 1; i >= 0; --i) S->ctl_free.push_back(c + i);
  }
  Ctl* c = S->ctl_free.back();
  S->ctl_free.pop_back();
  return c;
}

// Returns a control word to the pool (worker or finisher thread).
void srv_put_ctl(pr_server* S, Ctl* c) {
  if (!c) return;
  std::lock_guard<std::mutex> lk(S->ctl_mu);
  S->ctl_free.push_back(c);
}

int srv_finish(pr_server* S, SrvReq* r) {
  pr_sys* s = r->sys;
  const size_t n = (size_t)r->desc.n, B = (size_t)r->desc.B;
  // the device copies land in the pinned staging (DMA at full speed), then
  // in the request's host arrays
  int64_t nb = 0;
  int e = pr_sys_bonds(s, nullptr, 0, &nb);
  const size_t need = std::max((size_t)n * (16 + 4 * B), (size_t)std::max<int64_t>(nb, 1) * 12);
  if (!e && S->stage_bytes < need) {
    const size_t grow = std::max(need, 2 * S->stage_bytes);
    if (S->stage) (void)hipHostFree(S->stage);
    S->stage = nullptr;
    S->stage_bytes = 0;
    if (hipHostMalloc(&S->stage, grow) == hipSuccess) S->stage_bytes = grow;
    else S->stage = nullptr;  // the copies then go to pageable memory
  }
  if (!e) {
    r->bonds.resize((size_t)std::max<int64_t>(nb, 1) * 3);
    e = sys_bonds(s, r->bonds.data(), nb, &nb, S->stage, S->stage_bytes);
    r->n_bonds = nb;
  }
  if (!e) {
    r->x.resize(n);
    r->y.resize(n);
    r->z.resize(n);
    r->state.resize(n);
    r->adj.resize(n * B);
    if (S->stage) {
      float* sx = (float*)S->stage;
      int32_t* ss = (int32_t*)(sx + 3 * n);
      int32_t* sa = ss + n;
      e = pr_sys_read(s, sx, sx + n, sx + 2 * n, ss, sa, 0);
      if (!e) {
        std::memcpy(r->x.data(), sx, n * 4);
        std::memcpy(r->y.data(), sx + n, n * 4);
        std::memcpy(r->z.data(), sx + 2 * n, n * 4);
        std::memcpy(r->state.data(), ss, n * 4);
        std::memcpy(r->adj.data(), sa, n * B * 4);
      }
    } else {
      e = pr_sys_read(s, r->x.data(), r->y.data(), r->z.data(), r->state.data(), r->adj.data(), 0);
    }
  }
  if (!e) {
    int64_t ns = 0;
    e = pr_sys_stats(s, nullptr, 0, &ns);
    if (!e) {
      r->stats.resize((size_t)std::max<int64_t>(ns, 1));
      e = pr_sys_stats(s, r->stats.data(), ns, &ns);
      r->stats.resize((size_t)ns);
    }
  }
  Ctl* c = s->hctl;
  pr_sys_destroy(s);
  srv_put_ctl(S, c);
  r->sys = nullptr;
  return e;
}

// Creates and generates an admitted replica (worker thread).
int srv_admit(pr_server* S, SrvReq* r) {
  const pr_replica_desc& q = r->desc;
  pr_sys* s = nullptr;
  SysLease lease;
  lease.pool = S->pool;
  if (!(lease.hctl = srv_ctl(S))) return fail(PR_ENOMEM, "hipHostMalloc failed");
  int e = sys_create(&s, q.n, q.L, q.B, &q.rule, q.seed, q.log_cap, S->iostream, q.brick, &lease);
  if (!e) e = pr_sys_generate(s, q.gen_kind, q.gen_seed, q.gen_sigma0);
  if (!e) e = grow_part(s, std::max<int64_t>(1024, r->n_steps));
  if (e) {
    if (s) pr_sys_destroy(s);  // a leased word is not the system's to free
    srv_put_ctl(S, lease.hctl);
    return e;
  }
  s->d.jit_c = (float)(r->sigma / std::sqrt(21845.0));
  r->sys = s;
  return PR_OK;
}

// Launches one round on the server's stream: every active replica takes
// min(64, steps left) steps in the batched launches.  Asynchronous; the
// round's end is S->ev1.
int srv_launch_round(pr_server* S) {
  const int32_t Kmax = 64;
  int e;
  if (S->set_changed) {
    std::vector<pr_sys*> sys;
    for (SrvReq* r : S->active) sys.push_back(r->sys);
    S->maps.release();
    S->maps.bytes = 0;
    if ((e = fill_maps(sys, S->maps, S->bl))) return e;
    if (S->ds_cap < sys.size()) {
      S->dsa.release();
      S->ds_cap = std::max<size_t>(sys.size(), 2 * S->ds_cap);
      if ((e = S->dsa.alloc(&S->ds, S->ds_cap))) return e;
    }
    S->bl.ds = S->ds;
    S->set_changed = false;
  }
  S->hds.resize(S->active.size());
  int32_t K = 0;
  for (size_t i = 0; i < S->active.size(); ++i) {
    SrvReq* r = S->active[i];
    pr_sys* s = r->sys;
    const int32_t kl = (int32_t)std::min<uint32_t>((uint32_t)Kmax, r->n_steps - r->done_steps);
    s->d.sorted = 1;
    s->d.fuse = 0;  // the batched kernels bin the A's every step
    s->rec_ok = false;
    s->d.nwg_sweep = s->d.nbricks;
    S->hds[i] = s->d;
    S->hds[i].k_limit = kl;
    S->hds[i].first_step = 1u + r->done_steps;
    r->round_steps = (uint32_t)kl;
    K = std::max(K, kl);
  }
  hipStream_t st = S->stream;
  HIP_TRY(hipMemcpyAsync(S->ds, S->hds.data(), sizeof(Dev) * S->hds.size(), hipMemcpyHostToDevice,
                         st));
  HIP_TRY(hipEventRecord(S->ev0, st));
  HIP_TRY(launch_ctl_b(S->bl, 0, 0u, st));
  if ((e = run_block_b(S->bl, st, K))) return e;
  HIP_TRY(hipEventRecord(S->ev1, st));
  return PR_OK;
}

// Waits for the launched round and books its steps.
int srv_end_round(pr_server* S) {
  HIP_TRY(hipEventSynchronize(S->ev1));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, S->ev0, S->ev1));
  S->busy_s += ms * 1e-3;
  S->rounds++;
  for (SrvReq* r : S->active) {
    r->done_steps += r->round_steps;
    drop_graph(r->sys);
    r->sys->steps_since_sort = (int64_t)r->round_steps;
    r->sys->steps_since_load += r->round_steps;
    r->sys->d.kpar0 = (r->sys->d.kpar0 + r->round_steps) & 1u;
  }
  return PR_OK;
}

// Takes requests off the queue while a slot and their footprint are free.
std::vector<SrvReq*> srv_take(pr_server* S, size_t resident) {
  std::vector<SrvReq*> adm;
  std::lock_guard<std::mutex> lk(S->mu);
  while (!S->queue.empty()) {  // arrival order: the head waits until it fits
    SrvReq* r = S->queue.front();
    if ((int32_t)(resident + adm.size()) >= S->max_slots || S->used + r->bytes > S->budget) break;
    S->queue.pop_front();
    S->used += r->bytes;
    r->status = 1;
    adm.push_back(r);
  }
  return adm;
}

void srv_fail(pr_server* S, SrvReq* r, int e) {
  if (r->sys) {
    Ctl* c = r->sys->hctl;
    pr_sys_destroy(r->sys);
    srv_put_ctl(S, c);
    r->sys = nullptr;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  r->t_done = Clock::now();
  r->status = 3;
  r->code = e;
  S->used -= r->bytes;
  S->n_failed++;
}

// The worker: round r + 1 is launched as soon as round r has ended; while it
// runs, the requests that finished in round r are copied out and freed and
// new requests are admitted (their generation runs on the I/O stream), to
// join round r + 2.
// The finisher: retires finished replicas in arrival order of completion.
void fin_loop(pr_server* S) {
  (void)hipSetDevice(S->dev);
  for (;;) {
    SrvReq* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_fin.wait(lk, [&] { return S->fin_stop || !S->fin_q.empty(); });
      if (S->fin_q.empty()) break;  // stopping, nothing left
      r = S->fin_q.front();
      S->fin_q.pop_front();
    }
    const auto t0 = Clock::now();
    r->sys->stream = S->fstream;  // its last round has ended: the copies and frees go here
    r->sys->arena.astream = S->fstream;
    const int fe = srv_finish(S, r);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      r->t_done = Clock::now();
      r->status = fe ? 3 : 2;
      r->code = fe;
      S->used -= r->bytes;
      S->freed++;
      if (fe) S->n_failed++;
      else S->n_done++;
      S->finish_s += std::chrono::duration<double>(Clock::now() - t0).count();
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

void srv_loop(pr_server* S) {
  (void)hipSetDevice(S->dev);
  std::vector<SrvReq*> incoming, finished;
  bool in_flight = false;
  bool short_of_memory = false;  // requests wait for memory the finisher returns
  uint64_t freed_seen = 0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop || !S->active.empty() || !incoming.empty() || in_flight ||
               (!S->queue.empty() && (!short_of_memory || S->freed != freed_seen));
      });
      if (S->stop) break;
      freed_seen = S->freed;
    }
    // the round in flight ends; finished replicas leave, admitted ones join
    if (in_flight) {
      const auto t0 = Clock::now();
      const int e = srv_end_round(S);
      S->wait_s += std::chrono::duration<double>(Clock::now() - t0).count();
      in_flight = false;
      std::vector<SrvReq*> keep;
      bool cancelled = false;
      for (SrvReq* r : S->active) {
        if (e) {
          srv_fail(S, r, e);
        } else if (r->done_steps >= r->n_steps) {
          finished.push_back(r);
        } else if (r->cancel.load()) {
          srv_fail(S, r, PR_ECANCELED);
          cancelled = true;
        } else {
          keep.push_back(r);
        }
      }
      if (cancelled) S->cv_done.notify_all();
      std::lock_guard<std::mutex> lk(S->mu);
      if (keep.size() != S->active.size()) S->set_changed = true;
      S->active.swap(keep);
    }
    if (!incoming.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (SrvReq* r : incoming) S->active.push_back(r);
      incoming.clear();
      S->set_changed = true;
    }
    if (!S->active.empty()) {
      const auto t0 = Clock::now();
      const int e = srv_launch_round(S);
      S->launch_s += std::chrono::duration<double>(Clock::now() - t0).count();
      if (e) {
        for (SrvReq* r : S->active) srv_fail(S, r, e);
        std::lock_guard<std::mutex> lk(S->mu);
        S->active.clear();
        S->set_changed = true;
      } else {
        in_flight = true;
      }
    }
    // while the round runs: finished replicas to the finisher, new requests in
    if (!finished.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (SrvReq* r : finished) S->fin_q.push_back(r);
      finished.clear();
      S->cv_fin.notify_one();
    }
    const std::vector<SrvReq*> taken = srv_take(S, S->active.size() + incoming.size());
    {
      std::lock_guard<std::mutex> lk(S->mu);
      short_of_memory = taken.empty() && !S->queue.empty();
    }
    for (SrvReq* r : taken) {
      const auto t0 = Clock::now();
      const int e = srv_admit(S, r);
      S->admit_s += std::chrono::duration<double>(Clock::now() - t0).count();
      if (e) {
        srv_fail(S, r, e);
        S->cv_done.notify_all();
      } else {
        incoming.push_back(r);
      }
    }
  }
  if (in_flight) (void)hipEventSynchronize(S->ev1);
  std::lock_guard<std::mutex> lk(S->mu);  // the destroyer frees what is still resident
  for (SrvReq* r : incoming) S->active.push_back(r);
  for (SrvReq* r : finished) S->active.push_back(r);
}

SrvReq* srv_find(pr_server* S, uint64_t t) {
  auto it = S->all.find(t);
  return it == S->all.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

int pr_server_create(pr_server** out, int64_t hbm_budget, int32_t max_slots, void* stream) {
  if (!out) return fail(PR_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget <= 0 || max_slots < 1)
    return fail(PR_EINVAL, "budget=%lld max_slots=%d", (long long)hbm_budget, max_slots);
  pr_server* S = new pr_server();
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  S->stream = (hipStream_t)stream;
  if (hipGetDevice(&S->dev) != hipSuccess ||
      (!S->stream && hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) ||
      hipStreamCreateWithFlags(&S->iostream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->fstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&S->ev0) != hipSuccess || hipEventCreate(&S->ev1) != hipSuccess) {
    delete S;
    return fail(PR_EHIP, "hipGetDevice/hipStreamCreate/hipEventCreate failed");
  }
  S->own_stream = stream == nullptr;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = S->dev;
  if (hipMemPoolCreate(&S->pool, &props) != hipSuccess) {
    S->pool = nullptr;
    pr_server_destroy(S);
    return fail(PR_EHIP, "hipMemPoolCreate failed");
  }
  uint64_t keep = (uint64_t)hbm_budget;
  (void)hipMemPoolSetAttribute(S->pool, hipMemPoolAttrReleaseThreshold, &keep);
  S->finisher = std::thread(fin_loop, S);
  S->worker = std::thread(srv_loop, S);
  *out = S;
  return PR_OK;
}

void pr_server_destroy(pr_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->fin_stop = true;  // the finisher drains its queue first
  }
  S->cv_fin.notify_all();
  if (S->finisher.joinable()) S->finisher.join();
  for (SrvReq* r : S->active)
    if (r->sys) pr_sys_destroy(r->sys);
  for (auto& kv : S->all) delete kv.second;
  (void)hipStreamSynchronize(S->stream);
  S->maps.release();
  S->dsa.release();
  if (S->iostream) (void)hipStreamSynchronize(S->iostream);
  if (S->fstream) (void)hipStreamSynchronize(S->fstream);
  if (S->pool) (void)hipMemPoolDestroy(S->pool);
  for (Ctl* c : S->ctl_chunks) (void)hipHostFree(c);
  if (S->stage) (void)hipHostFree(S->stage);
  if (S->ev0) (void)hipEventDestroy(S->ev0);
  if (S->ev1) (void)hipEventDestroy(S->ev1);
  if (S->own_stream) (void)hipStreamDestroy(S->stream);
  if (S->iostream) (void)hipStreamDestroy(S->iostream);
  if (S->fstream) (void)hipStreamDestroy(S->fstream);
  delete S;
}

int pr_server_submit(pr_server* S, const pr_replica_desc* r, uint32_t n_steps, double sigma,
                     uint64_t* ticket) {
  if (!S || !r || !ticket) return fail(PR_EINVAL, "NULL argument");
  if (n_steps < 1) return fail(PR_EINVAL, "n_steps=0");
  if (!(sigma >= 0.0) || sigma * 6.0 >= (double)r->L * 0.5) return fail(PR_EINVAL, "sigma=%g", sigma);
  if (r->gen_kind != 0 && r->gen_kind != 1) return fail(PR_EINVAL, "gen_kind=%d", r->gen_kind);
  if (!(r->gen_sigma0 >= 0.0) || r->gen_sigma0 * 6.0 >= (double)r->L * 0.5)
    return fail(PR_EINVAL, "gen_sigma0=%g", r->gen_sigma0);
  int64_t bytes = 0;
  int e = pr_footprint(r, n_steps, &bytes);
  if (e) return e;
  if (bytes > S->budget)
    return fail(PR_EBUSY, "footprint %lld B exceeds the budget %lld B", (long long)bytes,
                (long long)S->budget);
  SrvReq* q = new SrvReq();
  q->desc = *r;
  q->n_steps = n_steps;
  q->sigma = sigma;
  q->bytes = bytes;
  q->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    q->ticket = S->next_ticket++;
    S->all[q->ticket] = q;
    S->queue.push_back(q);
  }
  S->cv_work.notify_all();
  *ticket = q->ticket;
  return PR_OK;
}

int pr_server_wait(pr_server* S, uint64_t ticket, double timeout_s, int32_t* status, int32_t* code,
                   double* latency_s) {
  if (!S) return fail(PR_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  SrvReq* q = srv_find(S, ticket);
  if (!q) return fail(PR_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (timeout_s > 0.0)
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                        [&] { return q->status >= 2; });
  if (status) *status = q->status;
  if (code) *code = q->code;
  if (latency_s)
    *latency_s = q->status >= 2 ? std::chrono::duration<double>(q->t_done - q->t_submit).count() : -1.0;
  return PR_OK;
}

int pr_server_poll(pr_server* S, uint64_t ticket, int32_t* status, int32_t* code,
                   double* latency_s) {
  return pr_server_wait(S, ticket, 0.0, status, code, latency_s);
}

int pr_server_cancel(pr_server* S, uint64_t ticket) {
  if (!S) return fail(PR_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    SrvReq* q = srv_find(S, ticket);
    if (!q) return fail(PR_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (q->status >= 2)
      return fail(PR_EBUSY, "request %llu has already finished", (unsigned long long)ticket);
    const auto it = std::find(S->queue.begin(), S->queue.end(), q);
    if (it == S->queue.end()) {  // admitted: the worker retires it after its round
      q->cancel.store(true);
      return PR_OK;
    }
    S->queue.erase(it);
    q->status = 3;
    q->code = PR_ECANCELED;
    q->t_done = Clock::now();
    S->n_failed++;
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
  return PR_OK;
}

static SrvReq* srv_done(pr_server* S, uint64_t ticket, int* e) {
  SrvReq* q = srv_find(S, ticket);
  if (!q) {
    *e = fail(PR_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    return nullptr;
  }
  if (q->status != 2) {
    *e = fail(q->status == 3 ? q->code : PR_EBUSY, "request %llu is not done",
              (unsigned long long)ticket);
    return nullptr;
  }
  *e = PR_OK;
  return q;
}

int pr_server_bonds(pr_server* S, uint64_t ticket, int32_t* out, int64_t cap, int64_t* n) {
  if (!S || !n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int e;
  SrvReq* q = srv_done(S, ticket, &e);
  if (!q) return e;
  const int64_t m = std::min<int64_t>(cap, q->n_bonds);
  if (m > 0) std::memcpy(out, q->bonds.data(), (size_t)m * 3 * sizeof(int32_t));
  *n = q->n_bonds;
  return PR_OK;
}

int pr_server_read(pr_server* S, uint64_t ticket, float* x, float* y, float* z, int32_t* state,
                   int32_t* adj) {
  if (!S) return fail(PR_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  int e;
  SrvReq* q = srv_done(S, ticket, &e);
  if (!q) return e;
  const size_t n = (size_t)q->desc.n;
  if (x) std::memcpy(x, q->x.data(), n * 4);
  if (y) std::memcpy(y, q->y.data(), n * 4);
  if (z) std::memcpy(z, q->z.data(), n * 4);
  if (state) std::memcpy(state, q->state.data(), n * 4);
  if (adj) std::memcpy(adj, q->adj.data(), n * 4 * (size_t)q->desc.B);
  return PR_OK;
}

int pr_server_stats(pr_server* S, uint64_t ticket, pr_stats* out, int64_t cap, int64_t* n) {
  if (!S || !n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int e;
  SrvReq* q = srv_done(S, ticket, &e);
  if (!q) return e;
  const int64_t m = std::min<int64_t>(cap, (int64_t)q->stats.size());
  if (m > 0) std::memcpy(out, q->stats.data(), (size_t)m * sizeof(pr_stats));
  *n = (int64_t)q->stats.size();
  return PR_OK;
}

int pr_server_release(pr_server* S, uint64_t ticket) {
  if (!S) return fail(PR_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  SrvReq* q = srv_find(S, ticket);
  if (!q) return fail(PR_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (q->status < 2) return fail(PR_EBUSY, "request %llu is not finished", (unsigned long long)ticket);
  S->all.erase(ticket);
  delete q;
  return PR_OK;
}

int pr_server_info_get(pr_server* S, pr_server_info* out) {
  if (!S || !out) return fail(PR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out->budget = S->budget;
  out->used = S->used;
  out->queued = (int64_t)S->queue.size();
  out->active = (int64_t)S->active.size();
  out->done = S->n_done;
  out->failed = S->n_failed;
  out->rounds = S->rounds;
  out->busy_s = S->busy_s;
  out->admit_s = S->admit_s;
  out->finish_s = S->finish_s;
  out->launch_s = S->launch_s;
  out->wait_s = S->wait_s;
  return PR_OK;
}

}  // extern "C"
