// kernels.hip -- HIP kernels of the reaction step for gfx950 (CDNA4, wave64).
//
// One reaction step (Table I of the paper, steps 1-9, on one GPU; the
// communication steps 4, 6 and 8 have nothing to exchange):
//   k_abin    A-role particles (a sparse list) -> coarse cell buckets
//   k_sweep   every particle streams once (coalesced SoA loads); each
//             T-eligible one tests the A records of its 2x2x2 cell block:
//             cutoff (step 1), keyed Philox draw (step 2), bonded exclusion,
//             A-side choice by 64-bit atomicMin of (w1, id_T) (steps 3-5)
//   k_tail    one workgroup: T-side choice by atomicMin of (w2, id_A) (steps
//             6-7), bonds sorted by id_A, states and adjacency (step 9)
// plus k_jitter (the MD stand-in between steps), k_generate (synthetic
// initial configuration) and k_classify (A list from scratch, validation).
//
// Arithmetic follows the contract of include/polyreact.h: FP32 min-image
// distance with explicitly rounded operations (no contraction), Philox4x32-10
// per pair keyed by (step, id_A, id_T), integer threshold on word 0.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/polyreact.h"

namespace pr {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies (hi/lo) and xors, the 64-bit key bumped by the Weyl increments
// after each round.
// ---------------------------------------------------------------------------
struct W4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     unsigned long long key) {
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t byte_sum(uint32_t v, uint32_t acc) {
  return __builtin_amdgcn_sad_u8(v, 0u, acc);  // |bytes - 0| summed, plus acc
}

// Irwin-Hall(12) offsets of the jitter: S_d = (12 bytes) - 1530, bytes of
// words 3d..3d+2 of the blocks (step, id, 0..2, tag).
__device__ __forceinline__ void ih12(uint32_t step, uint32_t id, uint32_t tag,
                                     unsigned long long key, int32_t S[3]) {
  const W4 a = philox(step, id, 0u, tag, key);
  const W4 b = philox(step, id, 1u, tag, key);
  const W4 c = philox(step, id, 2u, tag, key);
  S[0] = (int32_t)byte_sum(a.w2, byte_sum(a.w1, byte_sum(a.w0, 0u))) - 1530;
  S[1] = (int32_t)byte_sum(b.w1, byte_sum(b.w0, byte_sum(a.w3, 0u))) - 1530;
  S[2] = (int32_t)byte_sum(c.w0, byte_sum(b.w3, byte_sum(b.w2, 0u))) - 1530;
}

__device__ __forceinline__ float wrap_box(float v, float L) {
  if (v < 0.0f) v = __fadd_rn(v, L);
  if (v >= L) v = __fsub_rn(v, L);
  return v;
}

__device__ __forceinline__ float min_image(float d, float L, float halfL) {
  if (d > halfL) d = __fsub_rn(d, L);
  else if (d < -halfL) d = __fadd_rn(d, L);
  return d;
}

__device__ __forceinline__ bool in_window(int32_t t, int32_t s, int32_t type, int32_t lo,
                                          int32_t hi) {
  return t == type && s >= lo && s <= hi;
}

__device__ __forceinline__ int cell1(float u, int nc) {
  int c = (int)floorf(u);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Wave-aggregated append: one atomic per wavefront, lane order inside it.
__device__ __forceinline__ void wave_append(bool pred, int32_t value, int32_t* list,
                                            uint32_t* counter) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = value;
}

// Exclusive prefix sum over the workgroup (wave64 shuffles, then wave
// totals in LDS).  Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* s_wave,
                                                    uint32_t& total) {
  const int lane = __lane_id(), w = threadIdx.x / 64, nw = blockDim.x / 64;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < nw; ++i) {
      const uint32_t t = s_wave[i];
      s_wave[i] = acc;
      acc += t;
    }
    s_wave[nw] = acc;
  }
  __syncthreads();
  total = s_wave[nw];
  const uint32_t r = s_wave[w] + x - v;
  __syncthreads();
  return r;
}

__device__ __forceinline__ void set_err(Ctl* c, int code) { atomicCAS(&c->err, 0, code); }

__device__ __forceinline__ int32_t read_err(const Ctl* c) {
  return __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Control block set-up (a kernel rather than a memset/memcpy so that a
// captured graph may hold it).
// ---------------------------------------------------------------------------
__global__ void k_ctl_reset(Ctl* c, uint32_t step, int full) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->step = step;
    if (full) {  // par is kept: the cell counts of parity par are the cleared ones
      c->err = 0;
      c->na[0] = c->na[1] = 0;
      c->ovf_n = 0;
      c->nprop = 0;
      c->nwin = 0;
      c->stats_n = 0;
      c->log_n = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Validation and A list from scratch (after a load, and for the stateless
// single step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_classify(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cur = d.ctl->par;
  bool isA = false;
  if (k < d.n) {
    const float x = d.x[k], y = d.y[k], z = d.z[k];
    const bool ok = (x >= 0.0f && x < d.L) && (y >= 0.0f && y < d.L) && (z >= 0.0f && z < d.L);
    if (!ok) set_err(d.ctl, PR_EINVAL);
    isA = in_window(d.typ[k], d.st[k], d.rule.type_a, d.rule.a_min, d.rule.a_max);
  }
  wave_append(isA, k, d.alist[cur], &d.ctl->na[cur]);
}

// ---------------------------------------------------------------------------
// Re-jitter (stand-in for MD between reaction steps).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_jitter(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  if (read_err(d.ctl)) return;
  const uint32_t step = d.ctl->step;
  const uint32_t id = d.id ? (uint32_t)d.id[k] : (uint32_t)k;
  int32_t S[3];
  ih12(step, id, 1u, d.seed, S);
  d.x[k] = wrap_box(__fadd_rn(d.x[k], __fmul_rn((float)S[0], d.jit_c)), d.L);
  d.y[k] = wrap_box(__fadd_rn(d.y[k], __fmul_rn((float)S[1], d.jit_c)), d.L);
  d.z[k] = wrap_box(__fadd_rn(d.z[k], __fmul_rn((float)S[2], d.jit_c)), d.L);
}

// ---------------------------------------------------------------------------
// Synthetic jittered-lattice initial configuration (slot == id).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_generate(Dev d, int kind, unsigned long long gseed,
                                                  float c0, float a, int nl,
                                                  unsigned long long thr_x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const unsigned long long n3 = (unsigned long long)nl * nl * nl;
  const unsigned long long s = ((unsigned long long)k * 2147483647ull) % n3;
  const int ix = (int)(s % nl), iy = (int)((s / nl) % nl), iz = (int)(s / ((unsigned long long)nl * nl));
  int32_t S[3];
  ih12(0u, (uint32_t)k, 2u, gseed, S);
  const float px = __fmul_rn(__fadd_rn((float)ix, 0.5f), a);
  const float py = __fmul_rn(__fadd_rn((float)iy, 0.5f), a);
  const float pz = __fmul_rn(__fadd_rn((float)iz, 0.5f), a);
  d.x[k] = wrap_box(__fadd_rn(px, __fmul_rn((float)S[0], c0)), d.L);
  d.y[k] = wrap_box(__fadd_rn(py, __fmul_rn((float)S[1], c0)), d.L);
  d.z[k] = wrap_box(__fadd_rn(pz, __fmul_rn((float)S[2], c0)), d.L);
  const W4 w = philox(0u, (uint32_t)k, 0u, 3u, gseed);
  const bool pick = (unsigned long long)w.w0 < thr_x;
  if (kind == 0) {
    d.typ[k] = pick ? 1 : 0;
    d.st[k] = pick ? 4 : 2;
  } else {
    d.typ[k] = 0;
    d.st[k] = pick ? 2 : 0;
  }
  for (int b = 0; b < d.B; ++b) d.adj[(size_t)k * d.B + b] = -1;
}

// ---------------------------------------------------------------------------
// A list -> cell buckets.  Drops A's whose state left the A window, keeps the
// rest in the list of the next parity, and records (x, y, z, id) per cell.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_abin(Dev d) {
  if (read_err(d.ctl)) return;
  const uint32_t cur = d.ctl->par, nxt = cur ^ 1u;
  const uint32_t na = d.ctl->na[cur];
  const int nc = d.nc;
  for (uint32_t base = blockIdx.x * blockDim.x; base < na; base += gridDim.x * blockDim.x) {
    const uint32_t k = base + threadIdx.x;
    int slot = -1;
    bool keep = false;
    if (k < na) {
      slot = d.alist[cur][k];
      keep = in_window(d.typ[slot], d.st[slot], d.rule.type_a, d.rule.a_min, d.rule.a_max);
    }
    wave_append(keep, slot, d.alist[nxt], &d.ctl->na[nxt]);
    if (keep) {
      const float x = d.x[slot], y = d.y[slot], z = d.z[slot];
      const int id = d.id ? d.id[slot] : slot;
      const int cx = cell1(__fmul_rn(x, d.inv_w), nc);
      const int cy = cell1(__fmul_rn(y, d.inv_w), nc);
      const int cz = cell1(__fmul_rn(z, d.inv_w), nc);
      const int c = (cz * nc + cy) * nc + cx;
      const uint32_t r = atomicAdd(&d.cnt[cur][c], 1u);
      const float4 rec = make_float4(x, y, z, __int_as_float(id));
      if (r < (uint32_t)kCellCap) {
        d.rec[(size_t)c * kCellCap + r] = rec;
      } else {
        const uint32_t o = atomicAdd(&d.ctl->ovf_n, 1u);
        d.ovf[o] = rec;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dense sweep: every particle once.  T-eligible particles test the A records
// of the 2x2x2 cells around them (cell width >= 2 rc) and the overflow list.
// ---------------------------------------------------------------------------
struct SweepCtx {
  float xj, yj, zj;
  uint32_t idj, step;
  int in_rc, drawn, excl;
};

__device__ __forceinline__ void test_pair(const Dev& d, SweepCtx& t, float4 a) {
  const int ida = __float_as_int(a.w);
  const float dx = min_image(__fsub_rn(t.xj, a.x), d.L, d.halfL);
  const float dy = min_image(__fsub_rn(t.yj, a.y), d.L, d.halfL);
  const float dz = min_image(__fsub_rn(t.zj, a.z), d.L, d.halfL);
  const float r2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
  if (!(r2 < d.rc2)) return;
  t.in_rc++;
  const W4 w = philox(t.step, (uint32_t)ida, t.idj, 0u, d.seed);
  if (!((unsigned long long)w.w0 < d.thresh)) return;
  t.drawn++;
  if (d.rule.exclude) {
    const int sa = d.slot_of ? d.slot_of[ida] : ida;
    const int32_t* row = d.adj + (size_t)sa * d.B;
    for (int b = 0; b < d.B; ++b)
      if (row[b] == (int32_t)t.idj) {
        t.excl++;
        return;
      }
  }
  const unsigned long long key = ((unsigned long long)w.w1 << 32) | (unsigned long long)t.idj;
  const unsigned long long old = atomicMin(&d.slotA[ida], key);
  if (old == kEmpty) {
    const uint32_t p = atomicAdd(&d.ctl->nprop, 1u);
    d.propA[p] = ida;
  }
}

// The 2x2x2 block of coarse cells around a particle: per dimension the cells
// floor(u - 1/2) and floor(u - 1/2) + 1 (periodic), u = x / cell width.
// Cell width >= 2 rc (1 + 2^-10) puts every partner within rc in this block.
struct Block2 {
  int cx[2], cy[2], cz[2], m;
};

__device__ __forceinline__ void lo_hi(float v, float inv_w, int nc, int out[2]) {
  const int l = (int)floorf(__fsub_rn(__fmul_rn(v, inv_w), 0.5f));
  out[0] = l < 0 ? l + nc : l;
  out[1] = l + 1 >= nc ? l + 1 - nc : l + 1;
  if (nc == 1) out[0] = out[1] = 0;
}

__device__ __forceinline__ Block2 block_of(const Dev& d, float x, float y, float z) {
  Block2 b;
  lo_hi(x, d.inv_w, d.nc, b.cx);
  lo_hi(y, d.inv_w, d.nc, b.cy);
  lo_hi(z, d.inv_w, d.nc, b.cz);
  b.m = d.nc > 1 ? 2 : 1;
  return b;
}

// One T particle against the global cell buckets.
__device__ __forceinline__ void sweep_global(const Dev& d, SweepCtx& t, const Block2& bk,
                                             uint32_t cur) {
  const int nc = d.nc;
  for (int a = 0; a < bk.m; ++a)
    for (int b = 0; b < bk.m; ++b)
      for (int e = 0; e < bk.m; ++e) {
        const int c = (bk.cz[a] * nc + bk.cy[b]) * nc + bk.cx[e];
        uint32_t nr = d.cnt[cur][c];
        nr = nr < (uint32_t)kCellCap ? nr : (uint32_t)kCellCap;
        const float4* rec = d.rec + (size_t)c * kCellCap;
        for (uint32_t r = 0; r < nr; ++r) test_pair(d, t, rec[r]);
      }
}

__device__ __forceinline__ void wg_stats_out(const Dev& d, int* s_cnt, int t_elig,
                                             const SweepCtx& t) {
  if (t_elig) atomicAdd(&s_cnt[0], t_elig);
  if (t.in_rc) atomicAdd(&s_cnt[1], t.in_rc);
  if (t.drawn) atomicAdd(&s_cnt[2], t.drawn);
  if (t.excl) atomicAdd(&s_cnt[3], t.excl);
  __syncthreads();
  if (threadIdx.x < kWgStats) d.wgst[blockIdx.x * kWgStats + threadIdx.x] = s_cnt[threadIdx.x];
}

// Unsorted storage (and the stateless step): one thread per particle.
__global__ __launch_bounds__(kSweepThreads) void k_sweep(Dev d) {
  __shared__ int s_cnt[kWgStats];
  if (threadIdx.x < kWgStats) s_cnt[threadIdx.x] = 0;
  const bool dead = read_err(d.ctl) != 0;
  const uint32_t step = d.ctl->step, cur = d.ctl->par, nxt = cur ^ 1u;
  const uint32_t novf = d.ctl->ovf_n;
  // clear the bucket counts of the next step's parity
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d.ncell; c += gridDim.x * blockDim.x)
    d.cnt[nxt][c] = 0u;
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int t_elig = 0;
  SweepCtx t;
  t.in_rc = t.drawn = t.excl = 0;
  if (!dead && k < d.n &&
      in_window(d.typ[k], d.st[k], d.rule.type_t, d.rule.t_min, d.rule.t_max)) {
    t_elig = 1;
    t.xj = d.x[k];
    t.yj = d.y[k];
    t.zj = d.z[k];
    t.idj = d.id ? (uint32_t)d.id[k] : (uint32_t)k;
    t.step = step;
    sweep_global(d, t, block_of(d, t.xj, t.yj, t.zj), cur);
    for (uint32_t r = 0; r < novf; ++r) test_pair(d, t, d.ovf[r]);
  }
  wg_stats_out(d, s_cnt, t_elig, t);
}

// Brick geometry: staged region = brick cells plus one halo layer per side
// (or the whole grid in single-brick mode, bs == nc).
struct Region {
  int base[3], ext[3];
};

__device__ __forceinline__ Region region_of(const Dev& d, int b) {
  Region g;
  const int nb = d.nb;
  const int bc[3] = {b % nb, (b / nb) % nb, b / (nb * nb)};
  for (int q = 0; q < 3; ++q) {
    if (d.nbricks == 1) {
      g.base[q] = 0;
      g.ext[q] = d.nc;
    } else {
      const int lo = bc[q] * d.bs;
      const int sz = min(d.bs, d.nc - lo);
      g.base[q] = lo == 0 ? d.nc - 1 : lo - 1;
      g.ext[q] = sz + 2;
    }
  }
  return g;
}

__device__ __forceinline__ int local_of(int c, int base, int nc) {
  int l = c - base;
  return l < 0 ? l + nc : l;
}

// Sorted storage: one workgroup per brick; A records of the staged region
// in LDS; particles that drifted out of reach of the region since the last
// sort (and bricks whose region holds too many records) use the global path.
__global__ __launch_bounds__(kSweepThreads) void k_sweep_brick(Dev d) {
  __shared__ int s_cnt[kWgStats];
  __shared__ uint32_t s_off[kStageCells + 1];
  __shared__ uint32_t s_wave[kSweepThreads / 64 + 1];
  __shared__ float4 s_rec[kStageRecs];
  if (threadIdx.x < kWgStats) s_cnt[threadIdx.x] = 0;
  const bool dead = read_err(d.ctl) != 0;
  const uint32_t step = d.ctl->step, cur = d.ctl->par, nxt = cur ^ 1u;
  const uint32_t novf = d.ctl->ovf_n;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d.ncell; c += gridDim.x * blockDim.x)
    d.cnt[nxt][c] = 0u;
  const Region g = region_of(d, blockIdx.x);
  const int ncs = g.ext[0] * g.ext[1] * g.ext[2];
  const int nc = d.nc;
  // counts of the staged cells -> exclusive offsets
  uint32_t mine = 0;
  int myc = 0;
  if ((int)threadIdx.x < ncs) {
    const int l = threadIdx.x;
    const int lx = l % g.ext[0], ly = (l / g.ext[0]) % g.ext[1], lz = l / (g.ext[0] * g.ext[1]);
    int cx = g.base[0] + lx, cy = g.base[1] + ly, cz = g.base[2] + lz;
    cx -= cx >= nc ? nc : 0;
    cy -= cy >= nc ? nc : 0;
    cz -= cz >= nc ? nc : 0;
    myc = (cz * nc + cy) * nc + cx;
    mine = dead ? 0u : d.cnt[cur][myc];
    mine = mine < (uint32_t)kCellCap ? mine : (uint32_t)kCellCap;
  }
  uint32_t total = 0;
  const uint32_t off = block_scan_excl(mine, s_wave, total);
  if ((int)threadIdx.x < ncs) s_off[threadIdx.x] = off;
  if (threadIdx.x == 0) s_off[ncs] = total;
  const bool staged = total <= (uint32_t)kStageRecs;
  if (staged && (int)threadIdx.x < ncs)
    for (uint32_t r = 0; r < mine; ++r) s_rec[off + r] = d.rec[(size_t)myc * kCellCap + r];
  __syncthreads();
  int t_elig = 0;
  SweepCtx t;
  t.in_rc = t.drawn = t.excl = 0;
  t.step = step;
  const int s0 = d.bstart[blockIdx.x], s1 = d.bstart[blockIdx.x + 1];
  for (int k = s0 + threadIdx.x; !dead && k < s1; k += blockDim.x) {
    if (!in_window(d.typ[k], d.st[k], d.rule.type_t, d.rule.t_min, d.rule.t_max)) continue;
    t_elig++;
    t.xj = d.x[k];
    t.yj = d.y[k];
    t.zj = d.z[k];
    t.idj = (uint32_t)d.id[k];
    const Block2 bk = block_of(d, t.xj, t.yj, t.zj);
    int lx[2], ly[2], lz[2];
    bool inside = staged;
    for (int q = 0; q < bk.m; ++q) {
      lx[q] = local_of(bk.cx[q], g.base[0], nc);
      ly[q] = local_of(bk.cy[q], g.base[1], nc);
      lz[q] = local_of(bk.cz[q], g.base[2], nc);
      inside = inside && lx[q] < g.ext[0] && ly[q] < g.ext[1] && lz[q] < g.ext[2];
    }
    if (inside) {
      for (int a = 0; a < bk.m; ++a)
        for (int b = 0; b < bk.m; ++b)
          for (int e = 0; e < bk.m; ++e) {
            const int l = (lz[a] * g.ext[1] + ly[b]) * g.ext[0] + lx[e];
            const uint32_t q1 = s_off[l + 1];
            for (uint32_t q = s_off[l]; q < q1; ++q) test_pair(d, t, s_rec[q]);
          }
    } else {
      sweep_global(d, t, bk, cur);
    }
    for (uint32_t r = 0; r < novf; ++r) test_pair(d, t, d.ovf[r]);
  }
  wg_stats_out(d, s_cnt, t_elig, t);
}

// ---------------------------------------------------------------------------
// Spatial sort of the storage by brick (counting sort: count, scan, scatter).
// Results never depend on the storage order; the sort only gives each sweep
// workgroup a compact region of space.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int brick_of(const Dev& d, float x, float y, float z) {
  if (d.nbricks == 1) return 0;
  const int cx = cell1(__fmul_rn(x, d.inv_w), d.nc) / d.bs;
  const int cy = cell1(__fmul_rn(y, d.inv_w), d.nc) / d.bs;
  const int cz = cell1(__fmul_rn(z, d.inv_w), d.nc) / d.bs;
  return (cz * d.nb + cy) * d.nb + cx;
}

__global__ __launch_bounds__(256) void k_sort_count(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const int b = brick_of(d, d.x[k], d.y[k], d.z[k]);
  d.rank[k] = (int32_t)atomicAdd(&d.bcnt[b], 1u);
}

__global__ __launch_bounds__(1024) void k_sort_scan(Dev d) {
  __shared__ uint32_t s_wave[1024 / 64 + 1];
  uint32_t carry = 0;
  for (int base = 0; base < d.nbricks; base += blockDim.x) {
    const int b = base + threadIdx.x;
    const uint32_t v = b < d.nbricks ? d.bcnt[b] : 0u;
    uint32_t total = 0;
    const uint32_t ex = block_scan_excl(v, s_wave, total);
    if (b < d.nbricks) {
      d.bstart[b] = (int32_t)(carry + ex);
      d.bcnt[b] = 0u;
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    d.bstart[d.nbricks] = (int32_t)carry;
    d.ctl->na[d.ctl->par] = 0;  // the A list is rebuilt in the new order
  }
}

__global__ __launch_bounds__(256) void k_sort_scatter(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const float x = d.x[k], y = d.y[k], z = d.z[k];
  const int ns = d.bstart[brick_of(d, x, y, z)] + d.rank[k];
  d.x2[ns] = x;
  d.y2[ns] = y;
  d.z2[ns] = z;
  d.typ2[ns] = d.typ[k];
  d.st2[ns] = d.st[k];
  const int id = d.id[k];
  d.id2[ns] = id;
  d.slot_of[id] = ns;
  for (int b = 0; b < d.B; ++b) d.adj2[(size_t)ns * d.B + b] = d.adj[(size_t)k * d.B + b];
}

// A list from scratch in storage order (after a sort), no validation.
__global__ __launch_bounds__(256) void k_alist_rebuild(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cur = d.ctl->par;
  const bool isA =
      k < d.n && in_window(d.typ[k], d.st[k], d.rule.type_a, d.rule.a_min, d.rule.a_max);
  wave_append(isA, k, d.alist[cur], &d.ctl->na[cur]);
}

__global__ __launch_bounds__(256) void k_identity(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  d.id[k] = k;
  d.slot_of[k] = k;
}

// Storage order -> particle-id order.
__global__ __launch_bounds__(256) void k_gather_out(Dev d, float* ox, float* oy, float* oz,
                                                    int32_t* ost, int32_t* oadj) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const int id = d.id[k];
  if (ox) ox[id] = d.x[k];
  if (oy) oy[id] = d.y[k];
  if (oz) oz[id] = d.z[k];
  if (ost) ost[id] = d.st[k];
  if (oadj)
    for (int b = 0; b < d.B; ++b) oadj[(size_t)id * d.B + b] = d.adj[(size_t)k * d.B + b];
}

// ---------------------------------------------------------------------------
// Resolution and application, one workgroup.
// ---------------------------------------------------------------------------
__device__ void bitonic_sort(unsigned long long* buf, int n2) {
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < n2; t += blockDim.x) {
        const int ixj = t ^ j;
        if (ixj > t) {
          const unsigned long long a = buf[t], b = buf[ixj];
          const bool up = (t & k) == 0;
          if ((a > b) == up) {
            buf[t] = b;
            buf[ixj] = a;
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
}

__device__ __forceinline__ bool adj_append(int32_t* row, int B, int32_t v) {
  for (int b = 0; b < B; ++b)
    if (row[b] < 0) {
      row[b] = v;
      return true;
    }
  return false;
}

__global__ __launch_bounds__(kTailThreads) void k_tail(Dev d) {
  __shared__ unsigned long long wins[kSortLds];
  __shared__ uint32_t s_nwin, s_ovf;
  __shared__ long long s_sum[kWgStats];
  Ctl* c = d.ctl;
  if (read_err(c)) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const uint32_t step = c->step, cur = c->par, nxt = cur ^ 1u;
  const uint32_t nprop = c->nprop;
  const uint32_t a_elig = c->na[nxt];
  if (tid == 0) {
    s_nwin = 0;
    s_ovf = 0;
  }
  if (tid < kWgStats) s_sum[tid] = 0;
  __syncthreads();
  // steps 6-7: every proposal bids for its T with (w2, id_A)
  for (uint32_t k = tid; k < nprop; k += bs) {
    const int i = d.propA[k];
    const unsigned long long key =
        __hip_atomic_load(&d.slotA[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t j = (uint32_t)key;
    const W4 w = philox(step, (uint32_t)i, j, 0u, d.seed);
    atomicMin(&d.slotT[j], ((unsigned long long)w.w2 << 32) | (uint32_t)i);
  }
  __threadfence();
  __syncthreads();
  for (uint32_t k = tid; k < nprop; k += bs) {
    const int i = d.propA[k];
    const unsigned long long key =
        __hip_atomic_load(&d.slotA[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t j = (uint32_t)key;
    const W4 w = philox(step, (uint32_t)i, j, 0u, d.seed);
    const unsigned long long bid = ((unsigned long long)w.w2 << 32) | (uint32_t)i;
    const unsigned long long best =
        __hip_atomic_load(&d.slotT[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (best == bid) {
      const uint32_t pos = atomicAdd(&s_nwin, 1u);
      const unsigned long long v = ((unsigned long long)(uint32_t)i << 32) | j;
      if (pos < (uint32_t)kSortLds) wins[pos] = v;
      d.sortbuf[pos] = v;
    }
  }
  __threadfence();
  __syncthreads();
  const uint32_t nwin = s_nwin;
  int n2 = 1;
  while (n2 < (int)nwin) n2 <<= 1;
  unsigned long long* buf = (n2 <= kSortLds) ? wins : d.sortbuf;
  for (int t = (int)nwin + tid; t < n2; t += bs) buf[t] = kEmpty;
  __threadfence_block();
  __syncthreads();
  if (nwin > 1) bitonic_sort(buf, n2);
  // step 9: bonds in id_A order, states, adjacency, A-list additions
  const uint64_t log0 = c->log_n;
  for (uint32_t k = tid; k < nwin; k += bs) {
    const unsigned long long v = buf[k];
    const int i = (int)(v >> 32), j = (int)(uint32_t)v;
    const int si = d.slot_of ? d.slot_of[i] : i;
    const int sj = d.slot_of ? d.slot_of[j] : j;
    d.st[si] += d.rule.d_a;
    const int32_t nt = d.st[sj] + d.rule.d_t;
    d.st[sj] = nt;
    uint32_t lost = 0;
    if (!adj_append(d.adj + (size_t)si * d.B, d.B, j)) lost++;
    if (!adj_append(d.adj + (size_t)sj * d.B, d.B, i)) lost++;
    if (lost) atomicAdd(&s_ovf, lost);
    if (in_window(d.typ[sj], nt, d.rule.type_a, d.rule.a_min, d.rule.a_max)) {
      const uint32_t p = atomicAdd(&c->na[nxt], 1u);
      d.alist[nxt][p] = sj;
    }
    if (d.bonds && (int64_t)k < d.bonds_cap) {
      d.bonds[2 * (size_t)k] = i;
      d.bonds[2 * (size_t)k + 1] = j;
    }
    if (d.log) {
      const uint64_t row = log0 + k;
      if ((int64_t)row < d.log_cap) {
        d.log[3 * row] = (int32_t)step;
        d.log[3 * row + 1] = i;
        d.log[3 * row + 2] = j;
      }
    }
  }
  // reset every touched selection slot
  for (uint32_t k = tid; k < nprop; k += bs) {
    const int i = d.propA[k];
    const unsigned long long key = d.slotA[i];
    d.slotT[(uint32_t)key] = kEmpty;
    d.slotA[i] = kEmpty;
  }
  // counters of the sweep workgroups
  long long acc[kWgStats] = {0, 0, 0, 0};
  for (int g = tid; g < d.nwg_sweep; g += bs)
    for (int q = 0; q < kWgStats; ++q) acc[q] += d.wgst[g * kWgStats + q];
  for (int q = 0; q < kWgStats; ++q)
    if (acc[q]) atomicAdd((unsigned long long*)&s_sum[q], (unsigned long long)acc[q]);
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const uint32_t sn = c->stats_n;
    if (d.slog && (int64_t)sn < d.slog_cap) {
      long long* r = d.slog + (size_t)sn * kStatsPerStep;
      r[0] = a_elig;
      r[1] = s_sum[0];
      r[2] = s_sum[1];
      r[3] = s_sum[2];
      r[4] = s_sum[3];
      r[5] = s_sum[2] - s_sum[3];
      r[6] = nprop;
      r[7] = nwin;
      r[8] = s_ovf;
    }
    c->stats_n = sn + 1;
    c->log_n = log0 + nwin;
    c->nwin = nwin;
    c->na[cur] = 0;
    c->nprop = 0;
    c->ovf_n = 0;
    c->par = nxt;
    c->step = step + 1;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static inline int blocks_for(long long n, int t) { return (int)((n + t - 1) / t); }

hipError_t launch_ctl_reset(Ctl* c, uint32_t step, int full, hipStream_t s) {
  k_ctl_reset<<<1, 64, 0, s>>>(c, step, full);
  return hipGetLastError();
}

hipError_t launch_classify(const Dev& d, hipStream_t s) {
  if (d.n > 0) k_classify<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_jitter(const Dev& d, hipStream_t s) {
  if (d.n > 0) k_jitter<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_generate(const Dev& d, int kind, unsigned long long gseed, float c0, float a,
                           int nl, unsigned long long thr, hipStream_t s) {
  if (d.n > 0) k_generate<<<blocks_for(d.n, 256), 256, 0, s>>>(d, kind, gseed, c0, a, nl, thr);
  return hipGetLastError();
}

int abin_blocks(const Dev& d, long long na_hint) {
  long long b = blocks_for(na_hint > 0 ? na_hint : 1, 256);
  if (b < 64) b = 64;
  if (b > 4096) b = 4096;
  (void)d;
  return (int)b;
}

hipError_t launch_step(const Dev& d, int abin_grid, hipStream_t s, hipEvent_t ev_sweep0,
                       hipEvent_t ev_sweep1) {
  k_abin<<<abin_grid, 256, 0, s>>>(d);
  if (ev_sweep0) (void)hipEventRecord(ev_sweep0, s);
  if (d.sorted)
    k_sweep_brick<<<d.nbricks, kSweepThreads, 0, s>>>(d);
  else
    k_sweep<<<blocks_for(d.n, kSweepThreads), kSweepThreads, 0, s>>>(d);
  if (ev_sweep1) (void)hipEventRecord(ev_sweep1, s);
  k_tail<<<1, kTailThreads, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_sort(const Dev& d, hipStream_t s) {
  k_sort_count<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  k_sort_scan<<<1, 1024, 0, s>>>(d);
  k_sort_scatter<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

// after the caller swapped the primary and secondary buffers
hipError_t launch_alist_rebuild(const Dev& d, hipStream_t s) {
  k_alist_rebuild<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_identity(const Dev& d, hipStream_t s) {
  k_identity<<<blocks_for(d.n, 256), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_gather_out(const Dev& d, float* ox, float* oy, float* oz, int32_t* ost,
                             int32_t* oadj, hipStream_t s) {
  k_gather_out<<<blocks_for(d.n, 256), 256, 0, s>>>(d, ox, oy, oz, ost, oadj);
  return hipGetLastError();
}

}  // namespace pr
