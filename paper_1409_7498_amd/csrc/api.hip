// api.hip -- host runtime and C ABI of the reaction-step library.
//
// Owns device memory (resident systems and the per-device workspace of the
// stateless single step), validates arguments before any launch, sizes the
// coarse A grid, and drives the per-step kernel sequence of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
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
hipError_t launch_jitter(const Dev& d, hipStream_t s);
hipError_t launch_generate(const Dev& d, int kind, unsigned long long gseed, float c0, float a,
                           int nl, unsigned long long thr, hipStream_t s);
hipError_t launch_step(const Dev& d, int abin_grid, hipStream_t s, hipEvent_t ev_sweep0,
                       hipEvent_t ev_sweep1);
hipError_t launch_sort(const Dev& d, hipStream_t s);
hipError_t launch_alist_rebuild(const Dev& d, hipStream_t s);
hipError_t launch_identity(const Dev& d, hipStream_t s);
hipError_t launch_gather_out(const Dev& d, float* ox, float* oy, float* oz, int32_t* ost,
                             int32_t* oadj, hipStream_t s);
int abin_blocks(const Dev& d, long long na_hint);
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
  return PR_OK;
}

unsigned long long threshold(double p) {
  double t = std::ceil(p * 4294967296.0);
  if (t < 0.0) t = 0.0;
  if (t > 4294967296.0) t = 4294967296.0;
  return (unsigned long long)t;
}

// Coarse A grid: nc cells per side of width L/nc >= 2 rc (1 + 2^-10); the
// margin keeps the 2x2x2 block exact under FP32 rounding of the cell index.
void set_geometry(Dev& d, int32_t n, float L, int32_t B, const pr_rule* r, uint64_t seed) {
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
                 r->exclude_bonded};
  d.nwg_sweep = std::max(1, (n + kSweepThreads - 1) / kSweepThreads);
  d.jit_c = 0.0f;
  // bricks of bs^3 cells; the staged region (bs + 2 cells per side) must not
  // wrap onto itself, so bs <= nc - 2, else one brick covers the whole grid
  int bs = std::min<int>(kMaxBrick, (int)nc - 2);
  if (bs >= 1) {
    d.bs = bs;
    d.nb = (int32_t)((nc + bs - 1) / bs);
  } else {
    d.bs = (int32_t)nc;
    d.nb = 1;
  }
  d.nbricks = d.nb * d.nb * d.nb;
  d.sorted = 0;
}

struct Arena {
  std::vector<void*> ptrs;
  ~Arena() { release(); }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
  template <typename T>
  int alloc(T** out, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess)
      return fail(PR_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    ptrs.push_back(p);
    *out = (T*)p;
    return PR_OK;
  }
};

// Scratch of one step (everything but the particle arrays and the logs).
int alloc_scratch(Arena& a, Dev& d, int32_t n, hipStream_t s) {
  int e;
  if ((e = a.alloc(&d.alist[0], n)) || (e = a.alloc(&d.alist[1], n))) return e;
  if ((e = a.alloc(&d.cnt[0], d.ncell)) || (e = a.alloc(&d.cnt[1], d.ncell))) return e;
  if ((e = a.alloc(&d.rec, (size_t)d.ncell * kCellCap)) || (e = a.alloc(&d.ovf, n))) return e;
  if ((e = a.alloc(&d.slotA, n)) || (e = a.alloc(&d.slotT, n))) return e;
  if ((e = a.alloc(&d.propA, n)) || (e = a.alloc(&d.wgst, (size_t)d.nwg_sweep * kWgStats)))
    return e;
  size_t n2 = 1;
  while (n2 < (size_t)n / 2 + 1) n2 <<= 1;
  if ((e = a.alloc(&d.sortbuf, n2)) || (e = a.alloc(&d.ctl, 1))) return e;
  HIP_TRY(hipMemsetAsync(d.cnt[0], 0, sizeof(uint32_t) * std::max(1, d.ncell), s));
  HIP_TRY(hipMemsetAsync(d.cnt[1], 0, sizeof(uint32_t) * std::max(1, d.ncell), s));
  HIP_TRY(hipMemsetAsync(d.slotA, 0xFF, sizeof(unsigned long long) * std::max(1, n), s));
  HIP_TRY(hipMemsetAsync(d.slotT, 0xFF, sizeof(unsigned long long) * std::max(1, n), s));
  HIP_TRY(hipMemsetAsync(d.ctl, 0, sizeof(Ctl), s));
  return PR_OK;
}

// Per-device workspace of the stateless single step, grown on demand.
struct Workspace {
  Arena arena;
  Dev d{};
  int32_t n = -1, ncell = -1;
  long long* slog = nullptr;
  Ctl* hctl = nullptr;           // pinned host copies
  long long* hstats = nullptr;
  ~Workspace() {
    if (hctl) (void)hipHostFree(hctl);
    if (hstats) (void)hipHostFree(hstats);
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

const char* pr_version(void) { return "polyreact 0.1 (gfx950)"; }

int pr_react_step(int32_t n, float L, const float* x, const float* y, const float* z,
                  const int32_t* type, int32_t* state, int32_t* adj, int32_t B,
                  const pr_rule* rule, uint64_t seed, uint32_t step, int32_t* bonds,
                  int32_t cap, int32_t* n_bonds, pr_stats* st, void* stream) {
  if (n < 0 || B < 1) return fail(PR_EINVAL, "n=%d B=%d", n, B);
  int e = validate_rule(rule, L);
  if (e) return e;
  if (!n_bonds) return fail(PR_EINVAL, "n_bonds is NULL");
  if ((int64_t)cap < (int64_t)n / 2) return fail(PR_ECAP, "cap=%d < n/2=%d", cap, n / 2);
  if (n > 0 && (!x || !y || !z || !type || !state || !adj || !bonds))
    return fail(PR_EINVAL, "NULL device array");
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
  set_geometry(geo, n, L, B, rule, seed);
  if (!ws || ws->n < n || ws->ncell < geo.ncell) {
    delete ws;
    ws = new Workspace();
    ws->d = geo;
    const int32_t n_alloc = std::max(n, 1024);
    ws->d.nwg_sweep = (n_alloc + kSweepThreads - 1) / kSweepThreads;
    if ((e = alloc_scratch(ws->arena, ws->d, n_alloc, s))) {
      delete ws;
      ws = nullptr;
      return e;
    }
    if ((e = ws->arena.alloc(&ws->slog, kStatsPerStep))) return e;
    HIP_TRY(hipHostMalloc((void**)&ws->hctl, sizeof(Ctl)));
    HIP_TRY(hipHostMalloc((void**)&ws->hstats, sizeof(long long) * kStatsPerStep));
    ws->n = std::max(n, 1024);
    ws->ncell = geo.ncell;
  }
  Dev d = ws->d;  // scratch pointers
  // geometry of this call (the A grid may be smaller than the allocation)
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
  d.nwg_sweep = geo.nwg_sweep;
  d.x = const_cast<float*>(x);
  d.y = const_cast<float*>(y);
  d.z = const_cast<float*>(z);
  d.typ = const_cast<int32_t*>(type);
  d.st = state;
  d.adj = adj;
  d.id = d.slot_of = nullptr;
  d.bonds = bonds;
  d.bonds_cap = cap;
  d.log = nullptr;
  d.log_cap = 0;
  d.slog = ws->slog;
  d.slog_cap = 1;
  // The workspace serves calls of any box size: a previous call may have left
  // counts in cells beyond this call's grid, so both count buffers are cleared
  // over their whole allocation (each step only clears the cells it uses).
  HIP_TRY(hipMemsetAsync(d.cnt[0], 0, sizeof(uint32_t) * (size_t)ws->ncell, s));
  HIP_TRY(hipMemsetAsync(d.cnt[1], 0, sizeof(uint32_t) * (size_t)ws->ncell, s));
  HIP_TRY(launch_ctl_reset(d.ctl, step, 1, s));
  HIP_TRY(launch_classify(d, s));
  HIP_TRY(launch_step(d, abin_blocks(d, n / 8), s, nullptr, nullptr));
  HIP_TRY(hipMemcpyAsync(ws->hctl, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ws->hstats, ws->slog, sizeof(long long) * kStatsPerStep,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const Ctl c = *ws->hctl;
  if (c.err) return fail(c.err, "invalid particle position (NaN or outside [0, L))");
  *n_bonds = (int32_t)c.nwin;
  const long long* h = ws->hstats;
  if (st) *st = pr_stats{h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7], h[8]};
  if (h[8] > 0) return fail(PR_ECAP, "%lld adjacency appends found a full row", h[8]);
  return PR_OK;
}

}  // extern "C"

// ===========================================================================
// Resident systems
// ===========================================================================
struct pr_sys {
  int dev = 0;
  hipStream_t stream = nullptr;
  Arena arena;
  Dev d{};
  pr_rule rule{};
  int64_t log_cap = 0;
  int64_t slog_cap = 0;
  int64_t steps_since_load = 0;
  long long na_hint = 0;
  bool loaded = false;
  bool poisoned = false;
  int32_t sort_period = 0;
  int64_t steps_since_sort = 0;
  float *rx = nullptr, *ry = nullptr, *rz = nullptr;  // id-order read buffers
  int32_t *rst = nullptr, *radj = nullptr;
  Ctl* hctl = nullptr;
  ~pr_sys() {
    if (hctl) (void)hipHostFree(hctl);
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

int grow_slog(pr_sys* s, int64_t need) {
  if (need <= s->slog_cap) return PR_OK;
  int64_t cap = std::max<int64_t>(need, 2 * s->slog_cap);
  long long* nb = nullptr;
  int e = s->arena.alloc(&nb, (size_t)cap * kStatsPerStep);
  if (e) return e;
  if (s->d.slog && s->slog_cap > 0)
    HIP_TRY(hipMemcpyAsync(nb, s->d.slog, sizeof(long long) * kStatsPerStep * s->slog_cap,
                           hipMemcpyDeviceToDevice, s->stream));
  s->d.slog = nb;  // the old block stays in the arena until destroy
  s->slog_cap = cap;
  s->d.slog_cap = cap;
  return PR_OK;
}

int after_load(pr_sys* s) {
  hipStream_t st = s->stream;
  s->d.sorted = 0;
  s->d.nwg_sweep = std::max(1, (s->d.n + kSweepThreads - 1) / kSweepThreads);
  s->steps_since_sort = 0;
  HIP_TRY(launch_identity(s->d, st));
  HIP_TRY(launch_ctl_reset(s->d.ctl, 0, 1, st));
  HIP_TRY(launch_classify(s->d, st));
  int e = sync_ctl(s);
  if (e) return e;
  s->steps_since_load = 0;
  if (s->hctl->err) {
    s->loaded = false;
    return fail(s->hctl->err, "invalid particle position (NaN or outside [0, L))");
  }
  s->na_hint = s->hctl->na[0];
  s->loaded = true;
  return PR_OK;
}

}  // namespace

extern "C" {

int pr_sys_create(pr_sys** out, int32_t n, float L, int32_t B, const pr_rule* rule, uint64_t seed,
                  int64_t log_cap, void* stream) {
  if (!out) return fail(PR_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || B < 1) return fail(PR_EINVAL, "n=%d B=%d", n, B);
  int e = validate_rule(rule, L);
  if (e) return e;
  pr_sys* s = new pr_sys();
  s->stream = (hipStream_t)stream;
  s->rule = *rule;
  if (hipGetDevice(&s->dev) != hipSuccess) {
    delete s;
    return fail(PR_EHIP, "hipGetDevice failed");
  }
  Dev& d = s->d;
  set_geometry(d, n, L, B, rule, seed);
  s->log_cap = log_cap > 0 ? log_cap : n;
  e = alloc_scratch(s->arena, d, n, s->stream);
  if (!e) e = s->arena.alloc(&d.x, n);
  if (!e) e = s->arena.alloc(&d.y, n);
  if (!e) e = s->arena.alloc(&d.z, n);
  if (!e) e = s->arena.alloc(&d.typ, n);
  if (!e) e = s->arena.alloc(&d.st, n);
  if (!e) e = s->arena.alloc(&d.adj, (size_t)n * B);
  if (!e) e = s->arena.alloc(&d.log, (size_t)s->log_cap * 3);
  if (!e) e = s->arena.alloc(&d.id, n);
  if (!e) e = s->arena.alloc(&d.slot_of, n);
  if (!e) e = s->arena.alloc(&d.bstart, (size_t)d.nbricks + 1);
  if (!e) e = s->arena.alloc(&d.bcnt, (size_t)d.nbricks);
  if (!e) e = s->arena.alloc(&d.rank, n);
  if (!e) e = s->arena.alloc(&d.x2, n);
  if (!e) e = s->arena.alloc(&d.y2, n);
  if (!e) e = s->arena.alloc(&d.z2, n);
  if (!e) e = s->arena.alloc(&d.typ2, n);
  if (!e) e = s->arena.alloc(&d.st2, n);
  if (!e) e = s->arena.alloc(&d.id2, n);
  if (!e) e = s->arena.alloc(&d.adj2, (size_t)n * B);
  if (!e && d.nbricks > d.nwg_sweep) {
    // sweep counters for the brick grid as well
    e = s->arena.alloc(&d.wgst, (size_t)d.nbricks * kWgStats);
  }
  if (!e && hipMemsetAsync(d.bcnt, 0, sizeof(uint32_t) * d.nbricks, s->stream) != hipSuccess)
    e = fail(PR_EHIP, "hipMemsetAsync failed");
  if (!e && hipHostMalloc((void**)&s->hctl, sizeof(Ctl)) != hipSuccess)
    e = fail(PR_ENOMEM, "hipHostMalloc failed");
  if (e) {
    delete s;
    return e;
  }
  d.bonds = nullptr;
  d.bonds_cap = 0;
  d.log_cap = s->log_cap;
  s->sort_period = 64;
  if ((e = grow_slog(s, 1024))) {
    delete s;
    return e;
  }
  *out = s;
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
  const Dev& d = s->d;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const size_t n = (size_t)d.n;
  HIP_TRY(hipMemcpyAsync(d.x, x, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(d.y, y, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(d.z, z, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(d.typ, type, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(d.st, state, n * 4, k, s->stream));
  HIP_TRY(hipMemcpyAsync(d.adj, adj, n * 4 * d.B, k, s->stream));
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
  return PR_OK;
}

// Counting sort of the storage by brick, then the A list in the new order.
static int sort_storage(pr_sys* s) {
  Dev& d = s->d;
  HIP_TRY(launch_sort(d, s->stream));
  std::swap(d.x, d.x2);
  std::swap(d.y, d.y2);
  std::swap(d.z, d.z2);
  std::swap(d.typ, d.typ2);
  std::swap(d.st, d.st2);
  std::swap(d.adj, d.adj2);
  std::swap(d.id, d.id2);
  d.sorted = 1;
  d.nwg_sweep = d.nbricks;
  HIP_TRY(launch_alist_rebuild(d, s->stream));
  s->steps_since_sort = 0;
  return PR_OK;
}

static int run_impl(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma, float* ms) {
  int e = check_sys(s, true);
  if (e) return e;
  if (!(sigma >= 0.0) || sigma * 6.0 >= (double)s->d.L * 0.5)
    return fail(PR_EINVAL, "sigma=%g", sigma);
  if ((e = grow_slog(s, s->steps_since_load + n_steps))) return e;
  s->d.jit_c = (float)(sigma / 256.0);
  const int abin_grid = abin_blocks(s->d, s->na_hint);
  hipStream_t st = s->stream;
  HIP_TRY(launch_ctl_reset(s->d.ctl, first_step, 0, st));
  std::vector<hipEvent_t> ev;
  if (ms) {
    ev.resize((size_t)n_steps * 4);
    for (auto& v : ev) HIP_TRY(hipEventCreate(&v));
  }
  for (uint32_t k = 0; k < n_steps; ++k) {
    if (s->sort_period > 0 && (!s->d.sorted || s->steps_since_sort >= s->sort_period))
      if ((e = sort_storage(s))) return e;
    s->steps_since_sort++;
    const Dev& d = s->d;
    if (ms) HIP_TRY(hipEventRecord(ev[4 * k], st));
    if (sigma > 0.0) HIP_TRY(launch_jitter(d, st));
    if (ms) HIP_TRY(hipEventRecord(ev[4 * k + 1], st));
    HIP_TRY(launch_step(d, abin_grid, st, ms ? ev[4 * k + 2] : nullptr,
                        ms ? ev[4 * k + 3] : nullptr));
  }
  s->steps_since_load += n_steps;
  if (ms) {
    hipEvent_t end;
    HIP_TRY(hipEventCreate(&end));
    HIP_TRY(hipEventRecord(end, st));
    HIP_TRY(hipEventSynchronize(end));
    float tj = 0, tr = 0, tsw = 0;
    for (uint32_t k = 0; k < n_steps; ++k) {
      float a = 0, b = 0, c = 0;
      hipEvent_t stop = (k + 1 < n_steps) ? ev[4 * (k + 1)] : end;
      HIP_TRY(hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]));
      HIP_TRY(hipEventElapsedTime(&b, ev[4 * k + 1], stop));
      HIP_TRY(hipEventElapsedTime(&c, ev[4 * k + 2], ev[4 * k + 3]));
      tj += a;
      tr += b;
      tsw += c;
    }
    ms[0] = tj;
    ms[1] = tr;
    ms[2] = tsw;
    for (auto& v : ev) (void)hipEventDestroy(v);
    (void)hipEventDestroy(end);
  }
  return PR_OK;
}

int pr_sys_run(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma) {
  return run_impl(s, first_step, n_steps, sigma, nullptr);
}

int pr_sys_run_timed(pr_sys* s, uint32_t first_step, uint32_t n_steps, double sigma, float* ms) {
  if (!ms) return fail(PR_EINVAL, "ms is NULL");
  return run_impl(s, first_step, n_steps, sigma, ms);
}

int pr_sys_read(pr_sys* s, float* x, float* y, float* z, int32_t* state, int32_t* adj,
                int32_t on_device) {
  int e = check_sys(s, false);
  if (e) return e;
  const Dev& d = s->d;
  const size_t n = (size_t)d.n;
  if (on_device) {
    HIP_TRY(launch_gather_out(d, x, y, z, state, adj, s->stream));
  } else {
    if (!s->rx) {
      if ((e = s->arena.alloc(&s->rx, n)) || (e = s->arena.alloc(&s->ry, n)) ||
          (e = s->arena.alloc(&s->rz, n)) || (e = s->arena.alloc(&s->rst, n)) ||
          (e = s->arena.alloc(&s->radj, n * d.B)))
        return e;
    }
    HIP_TRY(launch_gather_out(d, x ? s->rx : nullptr, y ? s->ry : nullptr, z ? s->rz : nullptr,
                              state ? s->rst : nullptr, adj ? s->radj : nullptr, s->stream));
    const hipMemcpyKind k = hipMemcpyDeviceToHost;
    if (x) HIP_TRY(hipMemcpyAsync(x, s->rx, n * 4, k, s->stream));
    if (y) HIP_TRY(hipMemcpyAsync(y, s->ry, n * 4, k, s->stream));
    if (z) HIP_TRY(hipMemcpyAsync(z, s->rz, n * 4, k, s->stream));
    if (state) HIP_TRY(hipMemcpyAsync(state, s->rst, n * 4, k, s->stream));
    if (adj) HIP_TRY(hipMemcpyAsync(adj, s->radj, n * 4 * d.B, k, s->stream));
  }
  if ((e = sync_ctl(s))) return e;
  if (s->hctl->err) return fail(s->hctl->err, "device error during the run");
  return PR_OK;
}

int pr_sys_bonds(pr_sys* s, int32_t* out, int64_t cap, int64_t* n) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL output");
  if ((e = sync_ctl(s))) return e;
  const int64_t total = (int64_t)s->hctl->log_n;
  const int64_t have = std::min<int64_t>(total, s->log_cap);
  const int64_t m = std::min<int64_t>(have, cap);
  if (m > 0) HIP_TRY(hipMemcpy(out, s->d.log, (size_t)m * 12, hipMemcpyDeviceToHost));
  *n = total;
  if (total > s->log_cap) return fail(PR_ECAP, "bond log overflowed: %lld > %lld", (long long)total,
                                      (long long)s->log_cap);
  return PR_OK;
}

int pr_sys_stats(pr_sys* s, pr_stats* out, int64_t cap, int64_t* n) {
  int e = check_sys(s, false);
  if (e) return e;
  if (!n || (cap > 0 && !out)) return fail(PR_EINVAL, "NULL output");
  if ((e = sync_ctl(s))) return e;
  const int64_t have = std::min<int64_t>((int64_t)s->hctl->stats_n, s->slog_cap);
  const int64_t m = std::min<int64_t>(have, cap);
  if (m > 0)
    HIP_TRY(hipMemcpy(out, s->d.slog, (size_t)m * sizeof(pr_stats), hipMemcpyDeviceToHost));
  *n = have;
  return PR_OK;
}

}  // extern "C"
