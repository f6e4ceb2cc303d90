// kernels.hip -- HIP kernels of the reaction step for gfx950 (CDNA4, wave64).
//
// One reaction step is three kernels (Table I of the paper, steps 1-9, on one
// GPU; the communication steps 4, 6 and 8 have nothing to exchange):
//   k_prep     closes the previous step (counters, bond rows), bins the
//              A-role particles into coarse cells of width >= 2 rc (record:
//              jittered position, id, slot, adjacency row) and re-jitters every
//              particle (the MD stand-in between steps; positions ping-pong
//              between two buffers)
//   k_sweep    every particle streams once with coalesced SoA loads (in brick
//              order once the storage is sorted, the A records of the brick and
//              its halo staged in LDS); in-range pairs (step 1) go to an LDS
//              queue so that the keyed Philox draws (step 2) run on full
//              wavefronts; each retained pair lowers its A's key (w1, id_T) by
//              a 64-bit atomicMin (steps 3-5) and joins the workgroup's list
//   k_resolve  per sweep workgroup (one wavefront each), the listed pairs
//              whose A chose their T; of those the smallest (w2, id_A) per T
//              is bonded, states and adjacency updated (steps 6-9)
// plus the counting sort of the storage by brick (within a brick its A's,
// then the rest by dual cell), the synthetic generator and the helpers of the
// runtime.
//
// Arithmetic follows the contract of include/polyreact.h: FP32 min-image
// distance with explicitly rounded operations (no contraction), Philox4x32-10
// per pair keyed by (step, id_A, id_T), integer threshold on word 0.  Every
// selection is a minimum over 64-bit keys, so no result depends on thread or
// atomic order, nor on the storage order of the particles.
#include <hip/hip_ext.h>
#include <algorithm>
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

// a ^ b ^ c in one instruction (gfx950's three-input bitwise op; 0x96 is the
// truth table of the three-way exclusive or)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     unsigned long long key) {
  // the key (the seed) is uniform in every caller
  uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)key);
  uint32_t k1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(key >> 32));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product each (a single v_mad_u64_u32)
    const unsigned long long p0 = 0xD2511F53ull * c0, p1 = 0xCD9E8D57ull * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = xor3(hi1, c1, k0);
    const uint32_t n2 = xor3(hi0, c3, k1);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // the round keys are bumped on the scalar unit each round rather than
    // precomputed: twenty live key registers would spill to vector lanes
    asm volatile("" : "+s"(k0), "+s"(k1));
  }
  return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t byte_sum(uint32_t v, uint32_t acc) {
  return __builtin_amdgcn_sad_u8(v, 0u, acc);  // |bytes - 0| summed, plus acc
}

// Irwin-Hall(12) offsets of the synthetic initial configuration:
// S_d = (12 bytes) - 1530, bytes of words 3d..3d+2 of the blocks
// (step, id, 0..2, tag).
__device__ __forceinline__ void ih12(uint32_t step, uint32_t id, uint32_t tag,
                                     unsigned long long key, int32_t S[3]) {
  const W4 a = philox(step, id, 0u, tag, key);
  const W4 b = philox(step, id, 1u, tag, key);
  const W4 c = philox(step, id, 2u, tag, key);
  S[0] = (int32_t)byte_sum(a.w2, byte_sum(a.w1, byte_sum(a.w0, 0u))) - 1530;
  S[1] = (int32_t)byte_sum(b.w1, byte_sum(b.w0, byte_sum(a.w3, 0u))) - 1530;
  S[2] = (int32_t)byte_sum(c.w0, byte_sum(b.w3, byte_sum(b.w2, 0u))) - 1530;
}

// Irwin-Hall(4) offsets of the re-jitter between reaction steps (the stand-in
// for the MD): S_d = (the 4 bytes of word d) - 510, block (step, id, 0, tag).
__device__ __forceinline__ void ih4(uint32_t step, uint32_t id, uint32_t tag,
                                    unsigned long long key, int32_t S[3]) {
  const W4 a = philox(step, id, 0u, tag, key);
  // the -510 rides in the accumulator (32-bit wrap: the sum is in [0, 1020])
  constexpr uint32_t kMinus510 = 0u - 510u;
  S[0] = (int32_t)byte_sum(a.w0, kMinus510);
  S[1] = (int32_t)byte_sum(a.w1, kMinus510);
  S[2] = (int32_t)byte_sum(a.w2, kMinus510);
}

// Correctly rounded FP32 square root of a positive normal x: the hardware
// estimate (within one ulp) is moved one ulp down or up when x lies beyond
// the midpoint to that neighbour; the residuals x - s_dn * s and x - s_up * s
// are each rounded once by the fused multiply-add, and their signs decide
// exactly (s_dn * s and s_up * s are the midpoints' squares up to a term below
// the rounding of x).
__device__ __forceinline__ float sqrt_rn(float x) {
  float s = __builtin_amdgcn_sqrtf(x);
  const float s_dn = __uint_as_float(__float_as_uint(s) - 1u);
  const float s_up = __uint_as_float(__float_as_uint(s) + 1u);
  const float v_dn = __builtin_fmaf(-s_dn, s, x);
  const float v_up = __builtin_fmaf(-s_up, s, x);
  s = v_dn <= 0.0f ? s_dn : s;
  s = v_up > 0.0f ? s_up : s;
  return s;
}

__device__ __forceinline__ float wrap_box(float v, float L) {
  if (v < 0.0f) v = __fadd_rn(v, L);
  if (v >= L) v = __fsub_rn(v, L);
  return v;
}

// Single conditional wrap of a difference (selects, no branches).
__device__ __forceinline__ float min_image(float d, float L, float halfL) {
  const float dn = __fsub_rn(d, L), up = __fadd_rn(d, L);
  return d > halfL ? dn : (d < -halfL ? up : d);
}

__device__ __forceinline__ bool in_window(int32_t t, int32_t s, int32_t type, int32_t lo,
                                          int32_t hi) {
  return t == type && s >= lo && s <= hi;
}

__device__ __forceinline__ bool is_a(const Dev& d, int32_t t, int32_t s) {
  return in_window(t, s, d.rule.type_a, d.rule.a_min, d.rule.a_max);
}

__device__ __forceinline__ bool is_t(const Dev& d, int32_t t, int32_t s) {
  return in_window(t, s, d.rule.type_t, d.rule.t_min, d.rule.t_max);
}

__device__ __forceinline__ uint8_t role_of(const Dev& d, int32_t t, int32_t s) {
  if (d.nrules > 1) {  // a mask over the rules: T bits 0-3, A bits 4-7
    uint32_t m = 0;
    for (int r = 0; r < d.nrules; ++r) {
      const RuleD& q = d.mr[r].r;
      if (in_window(t, s, q.type_t, q.t_min, q.t_max)) m |= 1u << r;
      if (in_window(t, s, q.type_a, q.a_min, q.a_max)) m |= 16u << r;
    }
    return (uint8_t)m;
  }
  return is_t(d, t, s) ? kRoleT : (is_a(d, t, s) ? kRoleA : kRoleNone);
}

// Whether a role byte makes its particle an A (of some rule).
__device__ __forceinline__ bool role_is_a(uint32_t b, bool multi) {
  return multi ? (b & kMaskA) != 0u : b == kRoleA;
}

__device__ __forceinline__ int cell1(float u, int nc) {
  int c = (int)floorf(u);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ int cell_of(const Dev& d, float x, float y, float z) {
  const int nc = d.nc;
  const int cx = cell1(__fmul_rn(x, d.inv_w), nc);
  const int cy = cell1(__fmul_rn(y, d.inv_w), nc);
  const int cz = cell1(__fmul_rn(z, d.inv_w), nc);
  return (cz * nc + cy) * nc + cx;
}

__device__ __forceinline__ void set_err(Ctl* c, int code) { atomicCAS(&c->err, 0, code); }

__device__ __forceinline__ int32_t read_err(const Ctl* c) {
  return __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element p (0 or 1) of a two-element array held in the kernel argument:
// both pointers are read and one selected, without dynamic indexing (which
// would copy the argument to scratch); the select keeps the pointers in the
// global address space.
template <typename T>
__device__ __forceinline__ T* pick(T* const (&v)[2], uint32_t p) {
  T* const a = v[0];
  T* const b = v[1];
  return (p & 1u) ? b : a;
}

// Storage set s, member by member (a select of the whole aggregate would be
// built in scratch memory).
__device__ __forceinline__ Arr pick_set(const Dev& d, uint32_t s) {
  // s is uniform: a scalar select keeps the pointers in scalar registers
  s = (uint32_t)__builtin_amdgcn_readfirstlane((int)s);
  const Arr &u = d.set[0], &v = d.set[1];
  Arr r;
  for (int q = 0; q < 2; ++q) {
    r.x[q] = pick({u.x[q], v.x[q]}, s);
    r.y[q] = pick({u.y[q], v.y[q]}, s);
    r.z[q] = pick({u.z[q], v.z[q]}, s);
  }
  r.typ = pick({u.typ, v.typ}, s);
  r.st = pick({u.st, v.st}, s);
  r.adj = pick({u.adj, v.adj}, s);
  r.id = pick({u.id, v.id}, s);
  r.role = pick({u.role, v.role}, s);
  r.vx = pick({u.vx, v.vx}, s);
  r.vy = pick({u.vy, v.vy}, s);
  r.vz = pick({u.vz, v.vz}, s);
  return r;
}

// Step k of the current block: reaction step number and buffer parity.
struct StepInfo {
  uint32_t step, par;
};

__device__ __forceinline__ StepInfo step_info(const Ctl* c, int k) {
  // uniform over the launch (scalar registers, scalar selects of buffers)
  const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c->step0);
  const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c->par0);
  return StepInfo{s0 + (uint32_t)k, (p0 + (uint32_t)k) & 1u};
}

// Buffers kept by step mod 3 (fused binning).
__device__ __forceinline__ uint32_t mod3(uint32_t step) { return step % 3u; }

// Inclusive prefix sum over the wavefront with DPP: shifts by 1, 2, 4 and 8
// lanes within each row of 16, then the row broadcasts of lanes 15 and 31
// (lanes without a source add 0).  Every lane of the wavefront must be
// active.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// Exclusive prefix sum over the workgroup (wavefront scans, then the
// wavefront totals through LDS, read by every thread).  Every thread of the
// block must call it, with every lane active.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* s_wave,
                                                    uint32_t& total) {
  const int lane = __lane_id(), w = threadIdx.x / 64, nw = blockDim.x / 64;
  const uint32_t x = wave_scan_incl(v);
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  uint32_t below = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    const uint32_t t = s_wave[i];
    below += i < w ? t : 0u;
    all += t;
  }
  total = all;
  __syncthreads();  // s_wave is free for the next call
  return below + x - v;
}

// Adds v of every lane to *dst with one LDS atomic per wavefront (every lane
// of the wave must call it, with every lane active).
__device__ __forceinline__ void wave_add(int* dst, int v) {
  const int t = (int)wave_scan_incl((uint32_t)v);  // lane 63: the wavefront's sum
  if (__lane_id() == 63 && t) atomicAdd(dst, t);
}

// ---------------------------------------------------------------------------
// Control block set-up (a kernel rather than a memset/memcpy so that a
// captured graph may hold it).  A full reset selects storage set 0 and
// parity 0 (the caller clears both cell-count buffers with it).
// ---------------------------------------------------------------------------
__global__ void k_ctl_reset(Ctl* c, uint32_t step, int full) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->step0 = step;
    if (full) {
      c->par0 = 0;
      c->err = 0;
      c->set = 0;
      for (int p = 0; p < 2; ++p) {
        c->ovf_n[p] = 0;
        c->ret_ovf[p] = 0;
        c->nwin_ovf[p] = 0;
      }
      c->stats_n0 = 0;
      c->log_n = 0;
    }
  }
}

// Position validation and the roles (after a load, and for the stateless
// single step).
__global__ __launch_bounds__(kThreads) void k_classify(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const Arr a = pick_set(d, 0);
  const float x = pick(a.x, 0)[k], y = pick(a.y, 0)[k], z = pick(a.z, 0)[k];
  const bool ok = (x >= 0.0f && x < d.L) && (y >= 0.0f && y < d.L) && (z >= 0.0f && z < d.L);
  if (!ok) set_err(d.ctl, PR_EINVAL);
  a.role[k] = role_of(d, a.typ[k], a.st[k]);
}

// Identity storage order after a load (slot == id), cleared T flags.
__global__ __launch_bounds__(kThreads) void k_identity(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  if (pick_set(d, 0).id) pick_set(d, 0).id[k] = k;
  if (d.slot_of) d.slot_of[k] = k;
  d.tflag[k] = 0;
}

// ---------------------------------------------------------------------------
// Synthetic jittered-lattice initial configuration (storage set 0, parity 0,
// slot == id).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_generate(Dev d, int kind, unsigned long long gseed,
                                                       float c0, float a, int nl,
                                                       unsigned long long thr_x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const Arr o = pick_set(d, 0);
  const unsigned long long n3 = (unsigned long long)nl * nl * nl;
  const unsigned long long s = ((unsigned long long)k * 2147483647ull) % n3;
  const int ix = (int)(s % nl), iy = (int)((s / nl) % nl),
            iz = (int)(s / ((unsigned long long)nl * nl));
  int32_t S[3];
  ih12(0u, (uint32_t)k, 2u, gseed, S);
  const float px = __fmul_rn(__fadd_rn((float)ix, 0.5f), a);
  const float py = __fmul_rn(__fadd_rn((float)iy, 0.5f), a);
  const float pz = __fmul_rn(__fadd_rn((float)iz, 0.5f), a);
  pick(o.x, 0)[k] = wrap_box(__fadd_rn(px, __fmul_rn((float)S[0], c0)), d.L);
  pick(o.y, 0)[k] = wrap_box(__fadd_rn(py, __fmul_rn((float)S[1], c0)), d.L);
  pick(o.z, 0)[k] = wrap_box(__fadd_rn(pz, __fmul_rn((float)S[2], c0)), d.L);
  const W4 w = philox(0u, (uint32_t)k, 0u, 3u, gseed);
  const bool pick = (unsigned long long)w.w0 < thr_x;
  if (kind == 0) {
    o.typ[k] = pick ? 1 : 0;
    o.st[k] = pick ? 4 : 2;
  } else {
    o.typ[k] = 0;
    o.st[k] = pick ? 2 : 0;
  }
  for (int b = 0; b < d.B; ++b) o.adj[(size_t)k * d.B + b] = -1;
}

// ---------------------------------------------------------------------------
// Closing a step, group g (one workgroup of kThreads): the counters of sweep
// workgroups g*kGroup .. +kGroup summed into the step's partial record and
// their staged bonds appended to the bond log (one reservation per group; rows
// of a step end up in group order and readers order them by id_A).  Group 0
// also takes the bonds beyond the staging windows and resets the step's
// per-parity counters.
// ---------------------------------------------------------------------------
static_assert(kWinCap >= 2, "the closing reads two staged bonds ahead");
__device__ void close_group(const Dev& d, uint32_t par, uint32_t step, uint32_t sidx, int g,
                            uint32_t* s_wave) {
  __shared__ int s_sum[kPart];
  __shared__ uint64_t s_row;
  Ctl* c = d.ctl;
  const int tid = threadIdx.x;
  if (tid < kPart) s_sum[tid] = 0;
  const int w = g * kGroup + tid;
  const int2* staged = pick(d.wgw, par) + w * kWinCap;
  int o[kWgOut] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // a workgroup stages 0.3 bonds per step on average: its first two are read
  // with its counters, before their number is known (a window holds
  // kWinCap >= 2), which saves a dependent round trip in the common case
  int2 pre[2] = {make_int2(0, 0), make_int2(0, 0)};
  if (w < d.nwg_sweep) {
    const int32_t* src = pick(d.wgo, par) + w * kWgOut;
#pragma unroll
    for (int q = 0; q < kWgOut; ++q) o[q] = src[q];
    pre[0] = staged[0];
    pre[1] = staged[1];
  }
  // the A's of the step: counted by the sweep workgroups (fused binning), else
  // by the binning workgroups (strided over the groups)
  int a_elig = d.fuse ? o[kOutAElig] : 0;
  for (int q = w; !d.fuse && q < d.nwg_prep; q += d.ngroups * kGroup)
    a_elig += pick(d.abst, par)[q];
  const uint32_t nw = (uint32_t)min(o[kOutBonds], kWinCap);
  uint32_t tot = 0;
  const uint32_t off = block_scan_excl(nw, s_wave, tot);
  const uint32_t nwov = g == 0 ? c->nwin_ovf[par] : 0u;
  if (tid == 0 && tot + nwov > 0) s_row = atomicAdd((unsigned long long*)&c->log_n,
                                                    (unsigned long long)(tot + nwov));
  // partial layout: a_elig, t_elig, in_rc, drawn, excluded, proposals, bonds, lost
  const int v[kPart] = {a_elig,         o[kOutTElig], o[kOutInRc], o[kOutDrawn],
                        o[kOutExcl],    o[kOutProp],  o[kOutBonds], o[kOutLost]};
#pragma unroll
  for (int q = 0; q < kPart; ++q) wave_add(&s_sum[q], v[q]);
  __syncthreads();
  const uint64_t row0 = s_row;
  for (uint32_t e = 0; e < nw; ++e) {
    const uint64_t row = row0 + off + e;
    const int2 b = e < 2 ? pre[e] : staged[e];
    if ((int64_t)row < d.log_cap) {
      d.log[3 * row] = (int32_t)step;
      d.log[3 * row + 1] = b.x;
      d.log[3 * row + 2] = b.y;
    }
  }
  if (g == 0) {
    for (uint32_t e = tid; e < nwov; e += blockDim.x) {
      const uint64_t row = row0 + tot + e;
      const int2 b = pick(d.wov, par)[e];
      if ((int64_t)row < d.log_cap) {
        d.log[3 * row] = (int32_t)step;
        d.log[3 * row + 1] = b.x;
        d.log[3 * row + 2] = b.y;
      }
    }
  }
  __syncthreads();
  if (tid < kPart && (int64_t)sidx < d.part_cap)
    d.part[((size_t)sidx * d.ngroups + g) * kPart + tid] = s_sum[tid];
  if (g == 0 && tid == 0) {
    c->ovf_n[par] = 0;
    c->ret_ovf[par] = 0;
    c->nwin_ovf[par] = 0;
  }
}

// ---------------------------------------------------------------------------
// k_prep: [closing groups of step k - 1 when k > 0][binning of the A-role
// particles, kThreads * kPrepRoles slots per block].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_body(const Dev& d, int k, int blk) {
  __shared__ int s_na;
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  const StepInfo si = step_info(d.ctl, k);
  const Arr a = pick_set(d, d.ctl->set & 1u);
  const int ncl = k > 0 ? d.ngroups : 0;
  int b = blk;
  if (b < ncl) {  // closing groups of the previous step of the block
    close_group(d, si.par ^ 1u, si.step - 1u, d.ctl->stats_n0 + (uint32_t)k - 1u, b, s_wave);
    return;
  }
  b -= ncl;
  // binning of the A's: each lane scans kPrepRoles role bytes, the slots of
  // the wavefront's A's are compacted into LDS (ballot-free: a wave prefix
  // sum of the per-lane counts) and handled one per lane.  An A's record
  // holds its re-jittered position (the same draws as the sweep's), id, slot
  // and adjacency row.
  __shared__ int32_t s_list[kThreads / 64][kPrepRoles * 64];
  if (threadIdx.x == 0) s_na = 0;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int i0 = (b * kThreads + threadIdx.x) * kPrepRoles;
  const bool ok = read_err(d.ctl) == 0;
  uint32_t rw[kPrepRoles / 4] = {0u, 0u, 0u, 0u};
  if (ok && i0 + kPrepRoles <= d.n) {
    const uint4 v = *(const uint4*)(a.role + i0);
    rw[0] = v.x;
    rw[1] = v.y;
    rw[2] = v.z;
    rw[3] = v.w;
  } else if (ok && i0 < d.n) {
#pragma unroll
    for (int q = 0; q < kPrepRoles / 4; ++q)
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + 4 * q + e;
        if (i < d.n) rw[q] |= (uint32_t)a.role[i] << (8 * e);
      }
  }
  int na = 0;
  const bool multi = d.nrules > 1;
#pragma unroll
  for (int q = 0; q < kPrepRoles / 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) na += role_is_a((rw[q] >> (8 * e)) & 0xFFu, multi);
  const uint32_t incl = wave_scan_incl((uint32_t)na);
  const int wtot = __builtin_amdgcn_readlane((int)incl, 63);
  int at = (int)incl - na;
#pragma unroll
  for (int q = 0; q < kPrepRoles / 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (role_is_a((rw[q] >> (8 * e)) & 0xFFu, multi)) s_list[wv][at++] = i0 + 4 * q + e;
  __syncthreads();
  for (int e = lane; e < wtot; e += 64) {
    const int i = s_list[wv][e];
    float x = pick(a.x, si.par)[i], y = pick(a.y, si.par)[i], z = pick(a.z, si.par)[i];
    const int id = a.id ? a.id[i] : i;
    int4 q4 = make_int4(-1, -1, -1, -1);
    if (d.adj_staged) {
      const int32_t* row = a.adj + (size_t)i * d.B;
      q4.x = row[0];
      if (d.B > 1) q4.y = row[1];
      if (d.B > 2) q4.z = row[2];
      if (d.B > 3) q4.w = row[3];
    }
    if (d.jitter && d.jit_c != 0.0f) {
      int32_t S[3];
      ih4(si.step, (uint32_t)id, 1u, d.seed, S);
      x = wrap_box(__fadd_rn(x, __fmul_rn((float)S[0], d.jit_c)), d.L);
      y = wrap_box(__fadd_rn(y, __fmul_rn((float)S[1], d.jit_c)), d.L);
      z = wrap_box(__fadd_rn(z, __fmul_rn((float)S[2], d.jit_c)), d.L);
    }
    const int c = cell_of(d, x, y, z);
    const uint32_t r = atomicAdd(&pick(d.cnt, si.par)[c], 1u);
    const float4 rec = make_float4(x, y, z, __int_as_float(id));
    if (r < (uint32_t)kCellCap) {
      const size_t ri = (size_t)c * kCellCap + r;
      d.rec[ri] = rec;
      d.rsa[ri] = i;
      if (d.adj_staged) d.radj[ri] = q4;
    } else {
      const uint32_t o = atomicAdd(&d.ctl->ovf_n[si.par], 1u);
      pick(d.ovf, si.par)[o] = rec;
      pick(d.ovf_sa, si.par)[o] = i;
    }
  }
  if (lane == 0 && wtot) atomicAdd(&s_na, wtot);
  __syncthreads();
  if (threadIdx.x == 0) pick(d.abst, si.par)[b] = s_na;
}

// Closes step k of the block (one workgroup per closing group).
__device__ __forceinline__ void close_body(const Dev& d, int k, int g) {
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  const StepInfo si = step_info(d.ctl, k);
  close_group(d, si.par, si.step, d.ctl->stats_n0 + (uint32_t)k, g, s_wave);
}

// Advances the block origin by K steps (after the block's last step closed).
__device__ __forceinline__ void advance_ctl(Ctl* c, int K) {
  c->step0 += (uint32_t)K;
  c->par0 = (c->par0 + (uint32_t)K) & 1u;
  c->stats_n0 += (uint32_t)K;
}

// ---------------------------------------------------------------------------
// Pair tests shared by the sweep and the resolution.
// ---------------------------------------------------------------------------
// The 2x2x2 block of coarse cells around a particle: per dimension the cells
// floor(u - 1/2) and floor(u - 1/2) + 1 (periodic), u = x / cell width.
__device__ __forceinline__ void lo_hi(float v, float inv_w, int nc, int& c0, int& c1) {
  const int l = (int)floorf(__fsub_rn(__fmul_rn(v, inv_w), 0.5f));
  c0 = l < 0 ? l + nc : l;
  c1 = l + 1 >= nc ? l + 1 - nc : l + 1;
  if (nc == 1) c0 = c1 = 0;
}

// floor(v) as an integer in one instruction (v is a finite coordinate in
// cell units, far inside the int range): identical to (int)floorf(v)
__device__ __forceinline__ int floor_int(float v) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

// Local coordinate, in a staged region whose first cell is `base`, of the
// lower cell floor(u - 1/2) of a particle's 2x2x2 block (u = v / width; the
// cell index, in [-1, nc - 1], is taken mod nc): in [0, nc - 1].
__device__ __forceinline__ int local_lo(float v, float inv_w, int base, int nc) {
  const int l = floor_int(__fsub_rn(__fmul_rn(v, inv_w), 0.5f)) - base;
  return l < 0 ? l + nc : l;
}

__device__ __forceinline__ float dist2(const Dev& d, float xj, float yj, float zj, float4 a) {
  const float dx = min_image(__fsub_rn(xj, a.x), d.L, d.halfL);
  const float dy = min_image(__fsub_rn(yj, a.y), d.L, d.halfL);
  const float dz = min_image(__fsub_rn(zj, a.z), d.L, d.halfL);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// dist2 of two positions whose difference is known to lie within
// (-L/2, L/2) in every component (the minimum image is the identity there).
__device__ __forceinline__ float dist2_plain(float xj, float yj, float zj, float4 a) {
  const float dx = __fsub_rn(xj, a.x), dy = __fsub_rn(yj, a.y), dz = __fsub_rn(zj, a.z);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// dist2 of two positions whose differences lie within (-L/2, L/2) in every
// component but axis kAxis (there the minimum image is taken as in dist2):
// the same value as dist2.
template <int kAxis>
__device__ __forceinline__ float dist2_axis(const Dev& d, float xj, float yj, float zj, float4 a) {
  float dx = __fsub_rn(xj, a.x), dy = __fsub_rn(yj, a.y), dz = __fsub_rn(zj, a.z);
  if (kAxis == 0) dx = min_image(dx, d.L, d.halfL);
  if (kAxis == 1) dy = min_image(dy, d.L, d.halfL);
  if (kAxis == 2) dz = min_image(dz, d.L, d.halfL);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

__device__ __forceinline__ bool row_has(const int32_t* row, int B, int32_t v) {
  for (int b = 0; b < B; ++b)
    if (row[b] == v) return true;
  return false;
}

// The A records of a step: per-cell counts and bucket records with the A's
// slots, then the overflow list.
struct Buckets {
  const uint32_t* cnt;
  const float4* rec;
  const int32_t* sa;
  const float4* ovf;
  const int32_t* osa;
  uint32_t novf;
};

// Those of step `step` (parity par): filled by the binning kernel (kF =
// false), or with fused binning by the previous step's sweep.
template <bool kF>
__device__ __forceinline__ Buckets step_buckets(const Dev& d, uint32_t par, uint32_t step) {
  if (kF) {
    const uint32_t q = mod3(step);
    return Buckets{d.fcnt[q], pick(d.frec, par), pick(d.fsa, par), pick(d.fovf, par),
                   pick(d.fovf_sa, par), d.ctl->fovf_n[q]};
  }
  return Buckets{pick(d.cnt, par), d.rec, d.rsa, pick(d.ovf, par), pick(d.ovf_sa, par),
                 d.ctl->ovf_n[par]};
}

// Visits the A records (record, slot of the A) of the 2x2x2 cell block around
// (x, y, z) in the buckets, then the overflow list.
template <typename F>
__device__ __forceinline__ void for_global_records(const Dev& d, const Buckets& bk, float x,
                                                   float y, float z, F f) {
  const int nc = d.nc;
  int cx0, cx1, cy0, cy1, cz0, cz1;
  lo_hi(x, d.inv_w, nc, cx0, cx1);
  lo_hi(y, d.inv_w, nc, cy0, cy1);
  lo_hi(z, d.inv_w, nc, cz0, cz1);
  const int m = nc > 1 ? 2 : 1;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ia = q >> 2, ib = (q >> 1) & 1, ie = q & 1;
    if (ia >= m || ib >= m || ie >= m) continue;
    const int c = ((ia ? cz1 : cz0) * nc + (ib ? cy1 : cy0)) * nc + (ie ? cx1 : cx0);
    uint32_t nr = bk.cnt[c];
    nr = nr < (uint32_t)kCellCap ? nr : (uint32_t)kCellCap;
    const size_t r0 = (size_t)c * kCellCap;
    for (uint32_t r = 0; r < nr; ++r) f(bk.rec[r0 + r], bk.sa[r0 + r]);
  }
  for (uint32_t r = 0; r < bk.novf; ++r) f(bk.ovf[r], bk.osa[r]);
}

// Staged region of a brick along one dimension: the brick's cells plus one
// halo cell per side (the whole grid in single-brick mode).
__device__ __forceinline__ void region_dim(const Dev& d, int bc, int& base, int& ext) {
  if (d.nbricks == 1) {
    base = 0;
    ext = d.nc;
  } else {
    const int lo = bc * d.bs;
    const int sz = min(d.bs, d.nc - lo);
    base = lo == 0 ? d.nc - 1 : lo - 1;
    ext = sz + 2;
  }
}

// q = w / nb and r = w mod nb for a brick index: a high multiply by
// floor(2^32 / nb) is below the quotient by at most one.
__device__ __forceinline__ int div_nb(const Dev& d, int w, int& r) {
  uint32_t q = __umulhi((uint32_t)w, d.nb_m);
  int rr = w - (int)q * d.nb;
  if (rr >= d.nb) {
    q++;
    rr -= d.nb;
  }
  r = rr;
  return (int)q;
}

// x / d for the small operands of a staged region (x < 1024, d <= 64) as
// (x * m) >> 16 with m = ceil(2^16 / d): exact there, and two instructions
// instead of an integer division.
__device__ __forceinline__ uint32_t recip16(uint32_t d) { return (65536u + d - 1u) / d; }
__device__ __forceinline__ int div_small(int x, uint32_t m) { return (int)(((uint32_t)x * m) >> 16); }

__device__ __forceinline__ int local_of(int c, int base, int nc) {
  const int l = c - base;
  return l < 0 ? l + nc : l;
}

// ---------------------------------------------------------------------------
// Fused binning.  The sweep of step k writes the A records of step k + 1 into
// cell buckets of their own (counts by step mod 3, records by step parity):
// each A's own sweep workgroup re-jitters it once more and appends it to the
// bucket of its cell.  The resolve of step k then drops the record of an A
// whose bond ends its A role (its x becomes NaN: no distance test with it
// passes) and appends a T that takes the A role.
// ---------------------------------------------------------------------------
// Appends the record of A (slot, id) at (x, y, z) to the buckets of step
// `step` (parity par) and notes where it went.
__device__ __forceinline__ void fuse_bin(const Dev& d, uint32_t par, uint32_t step, int slot,
                                         uint32_t id, float x, float y, float z) {
  const int c = cell_of(d, x, y, z);
  const uint32_t r = atomicAdd(&d.fcnt[mod3(step)][c], 1u);
  const float4 rec = make_float4(x, y, z, __uint_as_float(id));
  if (r < (uint32_t)kCellCap) {
    const int q = c * kCellCap + (int)r;
    pick(d.frec, par)[q] = rec;
    pick(d.fsa, par)[q] = slot;
    d.apos[slot] = q;
  } else {
    const uint32_t o = atomicAdd(&d.ctl->fovf_n[mod3(step)], 1u);
    pick(d.fovf, par)[o] = rec;
    pick(d.fovf_sa, par)[o] = slot;
    d.apos[slot] = -1 - (int)o;
  }
}

// Drops the record of the next step (parity par) at q (a bucket record, or
// overflow entry -1 - q), or that of the A in `slot`.
__device__ __forceinline__ void fuse_drop_at(const Dev& d, uint32_t par, int q) {
  float* x = q >= 0 ? &pick(d.frec, par)[q].x : &pick(d.fovf, par)[-1 - q].x;
  *x = __int_as_float(0x7FC00000);  // quiet NaN
}
__device__ __forceinline__ void fuse_drop(const Dev& d, uint32_t par, int slot) {
  fuse_drop_at(d, par, d.apos[slot]);
}

// Slot range of sweep/resolve workgroup w.
template <bool kBrick>
__device__ __forceinline__ void range_of(const Dev& d, int w, int& s0, int& s1) {
  if (kBrick) {
    s0 = d.bstart[w];
    s1 = d.bstart[w + 1];
  } else {
    s0 = w * kThreads;
    s1 = min(d.n, s0 + kThreads);
  }
}

// Draw, exclusion and A-side choice of an in-range pair (steps 2-5).  A
// retained pair lowers the A's key (w1, id_T) with a 64-bit atomicMin whose
// result is not needed, flags its T and is handed to the resolve in the
// workgroup's list.  arow: the A's adjacency row staged with its record
// (nullptr: the row is read from the particle arrays).
struct SweepAcc {
  int t_elig, in_rc, drawn, excl, a_elig;
};

struct RetList {
  int* n;
  int4* ent;
  uint32_t* w2;
};

__device__ __forceinline__ void retain(const Dev& d, const Arr& a, uint32_t step, int ida,
                                       int sa, uint32_t idj, int sj, const int4* arow,
                                       SweepAcc& n, const RetList& l) {
  const W4 r = philox(step, (uint32_t)ida, idj, 0u, d.seed);
  if (!((unsigned long long)r.w0 < d.thresh)) return;
  n.drawn++;
  if (d.rule.exclude) {
    bool b;
    if (arow) {
      const int4 q = *arow;
      const int v = (int)idj;
      b = q.x == v || q.y == v || q.z == v || q.w == v;
    } else {
      b = row_has(a.adj + (size_t)sa * d.B, d.B, (int32_t)idj);
    }
    if (b) {
      n.excl++;
      return;
    }
  }
  d.tflag[sj] = 1;
  atomicMin(&d.slotA[ida], ((unsigned long long)r.w1 << 32) | (unsigned long long)idj);
  const int p = atomicAdd(l.n, 1);
  if (p < kRetCap) {
    l.ent[p] = make_int4(ida, sa, sj, (int)idj);
    l.w2[p] = r.w2;
  }
}

// ---------------------------------------------------------------------------
// k_sweep: every particle is re-jittered (resident systems) and written to
// the other position buffer; T's test the step's A records at their new
// positions.  kBrick = sorted storage: one workgroup per brick, the A records
// of the brick and its halo (positions, ids, slots, adjacency rows) staged in
// LDS, each region cell's by the thread that read its count, and the brick's
// particles handled kTPass at a time.  A T whose 2x2x2 cell block lies in the staged region scans it as four
// runs of two x-adjacent cells (contiguous in LDS) and keeps up to four
// in-range pairs in registers (one byte each); the wavefront then reserves
// queue slots for all of them at once (ballot and mbcnt over the per-lane
// counts) and the queue is drawn on full wavefronts after the pass.  Every
// other T is deferred to a list and scanned again after the queue: T's with
// more in-range pairs than the registers hold, or whose pairs find the queue
// full, in the staged records; in the global buckets particles that drifted
// out of the staged region since the last sort, bricks whose region holds
// more than kStageRecs records, steps with bucket overflow, and all T's of
// kBrick = false (kThreads consecutive slots per workgroup).  A deferred T
// enters the queue with none of its pairs, so every pair is drawn exactly
// once.
// ---------------------------------------------------------------------------
// One particle of a sweep pass, loaded with coalesced SoA reads.
struct Part {
  int role, id;
  float x, y, z;
};

// Sorted storage always carries the id array; the unsorted mode may run on
// caller arrays without one (the slot is the id).
template <bool kBrick>
__device__ __forceinline__ Part load_part(const Arr& a, const float* X, const float* Y,
                                          const float* Z, int slot, int s1) {
  Part q{kRoleNone, 0, 0.0f, 0.0f, 0.0f};
  if (slot < s1) {
    // 32-bit byte offsets (n < 2^30): the loads take the array base from
    // scalar registers and need no 64-bit address arithmetic
    const uint32_t bo = (uint32_t)slot * 4u;
    q.role = a.role[(uint32_t)slot];
    q.x = *(const float*)((const char*)X + bo);
    q.y = *(const float*)((const char*)Y + bo);
    q.z = *(const float*)((const char*)Z + bo);
    q.id = kBrick || a.id ? *(const int32_t*)((const char*)a.id + bo) : slot;
  }
  return q;
}

// The re-jittered position (identical arithmetic in k_prep and k_sweep).
__device__ __forceinline__ void rejitter(const Dev& d, uint32_t step, uint32_t id, float& x,
                                         float& y, float& z) {
  int32_t S[3];
  ih4(step, id, 1u, d.seed, S);
  x = wrap_box(__fadd_rn(x, __fmul_rn((float)S[0], d.jit_c)), d.L);
  y = wrap_box(__fadd_rn(y, __fmul_rn((float)S[1], d.jit_c)), d.L);
  z = wrap_box(__fadd_rn(z, __fmul_rn((float)S[2], d.jit_c)), d.L);
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long b) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

// kTwo: two region cells per thread while staging (brick edges above
// kOneCellBrick); else one, with the smaller tables.
// kF: fused binning (the sweep bins the next step's A records; sorted storage).
// kNt: the re-jittered positions stored non-temporally (Dev::nt_pos).
template <bool kBrick, bool kTwo, bool kF = false, bool kNt = false>
__device__ __forceinline__ void sweep_body(const Dev& d, int k, int w, int nwg) {
  static_assert(!kF || kBrick, "fused binning runs on sorted storage");
  constexpr int kCells = kTwo ? kStageCells : kStageCells1;  // region cells at most
  constexpr int kPer = kBrick ? kTPass / kThreads : 1;
  constexpr int kTP = kPer * kThreads;
  constexpr uint32_t kQEmpty = 0xFFFFFFFFu;
  __shared__ float4 s_rec[kBrick ? kStageRecs : 1];
  __shared__ int4 s_radj[kBrick ? kStageRecs : 1];
  __shared__ int32_t s_rsa[kBrick ? kStageRecs : 1];
  __shared__ uint16_t s_off[kBrick ? kCells + 1 : 1];  // first record of a region cell
  __shared__ uint32_t s_q[kBrick ? kQueue : 1];  // queued pair: local T | staged record << 16
  __shared__ int32_t s_tid[kBrick ? kTP : 1];    // ids of the pass's T's
  __shared__ uint16_t s_def[kTP];            // deferred T's (local index in the pass)
  __shared__ int4 s_ent[kRetCap];
  __shared__ uint32_t s_ew2[kRetCap];
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  __shared__ int s_cnt[5];
  __shared__ int s_qn, s_ndef, s_ne, s_dead;
  const int tid = threadIdx.x;
  if (tid < 5) s_cnt[tid] = 0;
  if (tid == 0) {
    s_qn = 0;
    s_ndef = 0;
    s_ne = 0;
    s_dead = read_err(d.ctl) != 0;
  }
  // staging at the top wave priority: the workgroups dispatched last stage
  // while the compute units already run the pass loops of the others, and
  // below those waves' priority their staging waits for issue slots
  if (kBrick) __builtin_amdgcn_s_setprio(3);
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  // positions of the previous step (parity par); the re-jittered ones are
  // written to parity par ^ 1
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const bool jit = d.jitter && d.jit_c != 0.0f;
  const Buckets bk = step_buckets<kF>(d, par, step);
  const RetList rl{&s_ne, s_ent, s_ew2};
  int s0, s1;
  range_of<kBrick>(d, w, s0, s1);
  int bx = 0, ex = 0, by = 0, ey = 0, bz = 0, ez = 0;
  bool staged = false, nowrap = false, plain_x = false, plain_y = false, plain_z = false;
  const int nc = d.nc;
  int ncs = 0;
  uint32_t mine = 0, mine2 = 0, m_exy = 0, m_ex = 0;
  int gc = 0, gc2 = 0;  // global cells of this thread's region cells
  // global cell of region cell cl (region cells in z, y, x order)
  auto region_cell = [&](int cl) {
    const int lz = div_small(cl, m_exy), rem = cl - lz * ex * ey;
    const int ly = div_small(rem, m_ex), lx = rem - ly * ex;
    int cx = bx + lx, cy = by + ly, cz = bz + lz;
    cx -= cx >= nc ? nc : 0;
    cy -= cy >= nc ? nc : 0;
    cz -= cz >= nc ? nc : 0;
    return (cz * nc + cy) * nc + cx;
  };
  if (kBrick) {
    int bxc, byc;
    const int bzc = div_nb(d, div_nb(d, w, bxc), byc);
    region_dim(d, bxc, bx, ex);
    region_dim(d, byc, by, ey);
    region_dim(d, bzc, bz, ez);
    // a region that does not wrap around the box and spans less than half of
    // it: a difference of two positions in it is below L/2 in magnitude, and
    // the minimum image leaves it unchanged
    plain_x = d.nbricks > 1 && bx + ex <= nc && 2 * ex + 1 <= nc;
    plain_y = d.nbricks > 1 && by + ey <= nc && 2 * ey + 1 <= nc;
    plain_z = d.nbricks > 1 && bz + ez <= nc && 2 * ez + 1 <= nc;
    nowrap = plain_x && plain_y && plain_z;
    ncs = ex * ey * ez;
    m_exy = recip16((uint32_t)(ex * ey));
    m_ex = recip16((uint32_t)ex);
    // the record counts of this thread's region cells (2 tid and 2 tid + 1,
    // or tid), issued first
#pragma unroll
    for (int h = 0; h < (kTwo ? 2 : 1); ++h) {
      const int cl = kTwo ? 2 * tid + h : tid;
      if (cl < ncs) {
        const int gcl = region_cell(cl);
        (h ? gc2 : gc) = gcl;
        (h ? mine2 : mine) = bk.cnt[gcl];
      }
    }
  }
  // the first particle of the first pass, issued behind the record counts
  // (memory operations complete in issue order)
  Part cur = load_part<kBrick>(a, X, Y, Z, s0 + tid, s1);
  if (kBrick) {
    mine = mine < (uint32_t)kCellCap ? mine : (uint32_t)kCellCap;
    mine2 = mine2 < (uint32_t)kCellCap ? mine2 : (uint32_t)kCellCap;
    uint32_t total = 0;
    const uint32_t off = block_scan_excl(mine + mine2, s_wave, total);
    staged = total <= (uint32_t)kStageRecs && bk.novf == 0;
    // each thread stages the records of its own region cells: the first
    // kFirst of a cell loaded together, the rare rest one after another
    constexpr int kFirst = kTwo ? 2 : 4;
#pragma unroll
    for (int h = 0; h < (kTwo ? 2 : 1); ++h) {
      const int cl = kTwo ? 2 * tid + h : tid;
      const uint32_t o = h ? off + mine : off, m = h ? mine2 : mine;
      if (cl < ncs) {
        s_off[cl] = (uint16_t)o;
        if (staged) {
          const size_t r0 = (size_t)(h ? gc2 : gc) * kCellCap;
          // the first records in registers (named, so that none of them
          // lives in scratch), loaded together, then written to LDS
          float4 rv0 = make_float4(0.f, 0.f, 0.f, 0.f), rv1 = rv0, rv2 = rv0, rv3 = rv0;
          int32_t sv0 = 0, sv1 = 0, sv2 = 0, sv3 = 0;
          if (m > 0u) { rv0 = bk.rec[r0]; sv0 = bk.sa[r0]; }
          if (m > 1u) { rv1 = bk.rec[r0 + 1]; sv1 = bk.sa[r0 + 1]; }
          if (kFirst > 2 && m > 2u) { rv2 = bk.rec[r0 + 2]; sv2 = bk.sa[r0 + 2]; }
          if (kFirst > 3 && m > 3u) { rv3 = bk.rec[r0 + 3]; sv3 = bk.sa[r0 + 3]; }
          if (m > 0u) { s_rec[o] = rv0; s_rsa[o] = sv0; }
          if (m > 1u) { s_rec[o + 1] = rv1; s_rsa[o + 1] = sv1; }
          if (kFirst > 2 && m > 2u) { s_rec[o + 2] = rv2; s_rsa[o + 2] = sv2; }
          if (kFirst > 3 && m > 3u) { s_rec[o + 3] = rv3; s_rsa[o + 3] = sv3; }
          if (!kF && d.adj_staged)
            for (uint32_t j = 0; j < m && j < (uint32_t)kFirst; ++j) s_radj[o + j] = d.radj[r0 + j];
          for (uint32_t j = kFirst; j < m; ++j) {
            s_rec[o + j] = bk.rec[r0 + j];
            s_rsa[o + j] = bk.sa[r0 + j];
            if (!kF && d.adj_staged) s_radj[o + j] = d.radj[r0 + j];
          }
        }
      }
    }
    if (tid == 0) s_off[ncs] = (uint16_t)total;
  }
  __syncthreads();
  const bool dead = s_dead != 0;
  // the workgroup-uniform switches of the pass loop, one scalar register
  // whose bits are tested where they are used (kept as separate booleans
  // they would each occupy a 64-bit lane mask)
  // kFWrapX/Y/Z: only that axis of the region needs the minimum image
  constexpr uint32_t kFJit = 1u, kFMove = 2u, kFStaged = 4u, kFNowrap = 8u;
  constexpr uint32_t kFWrapX = 16u, kFWrapY = 32u, kFWrapZ = 64u;
  const uint32_t flags0 = (uint32_t)__builtin_amdgcn_readfirstlane(
      (jit ? kFJit : 0u) | (d.jitter ? kFMove : 0u) | (staged ? kFStaged : 0u) |
      (nowrap ? kFNowrap : 0u) | (!plain_x && plain_y && plain_z ? kFWrapX : 0u) |
      (plain_x && !plain_y && plain_z ? kFWrapY : 0u) |
      (plain_x && plain_y && !plain_z ? kFWrapZ : 0u));
  SweepAcc n = {0, 0, 0, 0, 0};
  for (int base = s0; base < s1 && !dead; base += kTP) {
    if (base != s0) cur = load_part<kBrick>(a, X, Y, Z, base + tid, s1);
#pragma unroll 1
    for (int u = 0; u < kPer; ++u) {
      const int lt = u * kThreads + tid;
      const int slot = base + lt;
      uint32_t fl = flags0;
      asm volatile("" : "+s"(fl));
      // wave priority by progress: the arbiter otherwise favours the oldest
      // waves, so the workgroups dispatched first race ahead and the last
      // ones end up running nearly alone on their compute units at the end
      if (kBrick) {
        if (u == 0) __builtin_amdgcn_s_setprio(3);
        else if (u == 1) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(1);
      }
      // the next particle's loads are in flight while this one is handled
      Part nxt = cur;
      if (u + 1 < kPer) nxt = load_part<kBrick>(a, X, Y, Z, slot + kThreads, s1);
      const uint32_t idj = (uint32_t)cur.id;
      if (slot < s1 && (fl & kFMove)) {  // the re-jitter (stand-in for the MD between steps)
        if (fl & kFJit) rejitter(d, step, idj, cur.x, cur.y, cur.z);
        const uint32_t bo = (uint32_t)slot * 4u;  // 32-bit byte offsets: scalar-base stores
        if (kNt) {
          __builtin_nontemporal_store(cur.x, (float*)((char*)XW + bo));
          __builtin_nontemporal_store(cur.y, (float*)((char*)YW + bo));
          __builtin_nontemporal_store(cur.z, (float*)((char*)ZW + bo));
        } else {
          *(float*)((char*)XW + bo) = cur.x;
          *(float*)((char*)YW + bo) = cur.y;
          *(float*)((char*)ZW + bo) = cur.z;
        }
      }
      if (kF && slot < s1 && cur.role == kRoleA) {
        // fused binning: the A's record of the next step, re-jittered once
        // more (its bucket's returning atomic completes behind the rest of
        // the pass)
        n.a_elig++;
        float nx = cur.x, ny = cur.y, nz = cur.z;
        if (fl & kFJit) rejitter(d, step + 1u, idj, nx, ny, nz);
        fuse_bin(d, par ^ 1u, step + 1u, slot, idj, nx, ny, nz);
      }
      // in-range staged records of this T: nh counts them all, hits keeps the
      // first four, one byte each (a T with more is deferred)
      int nh = 0;
      uint32_t hits = 0;
      bool defer = false;
      if (slot < s1 && cur.role == kRoleT) {
        n.t_elig++;
        defer = true;
        if (kBrick && (fl & kFStaged)) {
          if (kBrick) s_tid[lt] = (int)idj;
          const float px = cur.x, py = cur.y, pz = cur.z;
          // local coordinates (in the staged region) of the lower corner of
          // the T's 2x2x2 cell block: floor(u - 1/2) - base, taken mod nc
          const int lx0 = local_lo(px, d.inv_w, bx, nc), ly0 = local_lo(py, d.inv_w, by, nc),
                    lz0 = local_lo(pz, d.inv_w, bz, nc);
          if ((uint32_t)lx0 < (uint32_t)(ex - 1) && (uint32_t)ly0 < (uint32_t)(ey - 1) &&
              (uint32_t)lz0 < (uint32_t)(ez - 1)) {
            // runs (dy, dz) = (0,0), (1,0), (0,1), (1,1): cells lx0 and lx0 + 1
            const int l0 = (int)__umul24(__umul24(lz0, ey) + ly0, ex) + lx0;  // small operands
            const int l1 = l0 + ex, l2 = l0 + ex * ey, l3 = l2 + ex;
            const int b0 = (int)s_off[l0], b1 = (int)s_off[l1], b2 = (int)s_off[l2],
                      b3 = (int)s_off[l3];
            const int p1 = (int)s_off[l0 + 2] - b0;
            const int p2 = p1 + (int)s_off[l1 + 2] - b1;
            const int p3 = p2 + (int)s_off[l2 + 2] - b2;
            const int tot = p3 + (int)s_off[l3 + 2] - b3;
            const int o1 = b1 - p1, o2 = b2 - p2, o3 = b3 - p3;
            // the four runs, with the distance of the region's kind
            auto scan = [&](auto dist) {
              for (int q = 0; q < tot; ++q) {
                const int r = q + (q < p1 ? b0 : (q < p2 ? o1 : (q < p3 ? o2 : o3)));
                if (dist(s_rec[r]) < d.rc2) {
                  hits |= (uint32_t)r << ((8 * nh) & 31);
                  nh++;
                }
              }
            };
            if (fl & kFNowrap) {  // no difference can reach L/2 in this region
              scan([&](float4 a) { return dist2_plain(px, py, pz, a); });
            } else if (fl & kFWrapX) {  // the region wraps (or spans half the box) in x only
              scan([&](float4 a) { return dist2_axis<0>(d, px, py, pz, a); });
            } else if (fl & kFWrapY) {
              scan([&](float4 a) { return dist2_axis<1>(d, px, py, pz, a); });
            } else if (fl & kFWrapZ) {
              scan([&](float4 a) { return dist2_axis<2>(d, px, py, pz, a); });
            } else {
              scan([&](float4 a) { return dist2(d, px, py, pz, a); });
            }
            defer = nh > 4;
          }
        }
      }
      if (defer) nh = 0;
      if (kBrick) {
        // queue slots for the wavefront's held pairs: lane j's pairs go after
        // those of the lower lanes (counts from four ballots)
        const unsigned long long g1 = __ballot(nh >= 1), g2 = __ballot(nh >= 2),
                                 g3 = __ballot(nh >= 3), g4 = __ballot(nh >= 4);
        const uint32_t wtot =
            (uint32_t)(__popcll(g1) + __popcll(g2) + __popcll(g3) + __popcll(g4));
        if (wtot) {
          uint32_t qb = 0;
          if (__lane_id() == 0) qb = (uint32_t)atomicAdd(&s_qn, (int)wtot);
          qb = (uint32_t)__builtin_amdgcn_readlane((int)qb, 0);
          const uint32_t p =
              qb + lanes_below(g1) + lanes_below(g2) + lanes_below(g3) + lanes_below(g4);
          if (nh > 0) {
            if (p + (uint32_t)nh <= (uint32_t)kQueue) {
              n.in_rc += nh;
              for (int j = 0; j < nh; ++j)
                s_q[p + j] = (uint32_t)lt | (((hits >> (8 * j)) & 0xFFu) << 16);
            } else {
              // the pairs do not all fit: the T is deferred and the slots it
              // reserved below kQueue are marked empty
              for (int j = 0; j < nh; ++j)
                if (p + j < (uint32_t)kQueue) s_q[p + j] = kQEmpty;
              defer = true;
            }
          }
        }
      }
      if (defer) s_def[atomicAdd(&s_ndef, 1)] = (uint16_t)lt;
      cur = nxt;
    }
    __syncthreads();
    if (kBrick) {
      // the pass's queued pairs: draws on full wavefronts
      const int qn = min(s_qn, kQueue);
      for (int e = tid; e < qn; e += kThreads) {
        const uint32_t q = s_q[e];
        if (q == kQEmpty) continue;
        const uint32_t lt = q & 0xFFFFu, r = q >> 16;
        retain(d, a, step, __float_as_int(s_rec[r].w), s_rsa[r], (uint32_t)s_tid[lt],
               base + (int)lt, d.adj_staged && !kF ? &s_radj[r] : nullptr, n, rl);
      }
    }
    // the deferred T's, re-jittered again from the previous positions: in the
    // staged records when the block lies in a staged region (T's with more
    // pairs than the registers hold, or whose pairs found the queue full),
    // else in the buckets (cells 0-7 of the block, then the overflow list)
    const int ndef = s_ndef;
    for (int e = tid; e < ndef; e += kThreads) {
      const int slot = base + (int)s_def[e];
      float px = X[slot], py = Y[slot], pz = Z[slot];
      const uint32_t idj = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
      if (jit) rejitter(d, step, idj, px, py, pz);
      if (kBrick && staged) {
        const int lx0 = local_lo(px, d.inv_w, bx, nc), ly0 = local_lo(py, d.inv_w, by, nc),
                  lz0 = local_lo(pz, d.inv_w, bz, nc);
        if ((uint32_t)lx0 < (uint32_t)(ex - 1) && (uint32_t)ly0 < (uint32_t)(ey - 1) &&
            (uint32_t)lz0 < (uint32_t)(ez - 1)) {
          const int l0 = (lz0 * ey + ly0) * ex + lx0;
#pragma unroll 1
          for (int run = 0; run < 4; ++run) {
            const int lr = l0 + ((run & 1) ? ex : 0) + ((run & 2) ? ex * ey : 0);
            const int r1 = (int)s_off[lr + 2];
            for (int r = (int)s_off[lr]; r < r1; ++r) {
              if (!(dist2(d, px, py, pz, s_rec[r]) < d.rc2)) continue;
              n.in_rc++;
              retain(d, a, step, __float_as_int(s_rec[r].w), s_rsa[r], idj, slot,
                     d.adj_staged && !kF ? &s_radj[r] : nullptr, n, rl);
            }
          }
          continue;
        }
      }
      int cx0, cx1, cy0, cy1, cz0, cz1;
      lo_hi(px, d.inv_w, nc, cx0, cx1);
      lo_hi(py, d.inv_w, nc, cy0, cy1);
      lo_hi(pz, d.inv_w, nc, cz0, cz1);
      const int m = nc > 1 ? 2 : 1;
      for (int q = 0; q < 9; ++q) {
        const float4* rp;
        const int32_t* sp;
        uint32_t nr;
        if (q < 8) {
          const int ia = q >> 2, ib = (q >> 1) & 1, ie = q & 1;
          if (ia >= m || ib >= m || ie >= m) continue;
          const int cc = ((ia ? cz1 : cz0) * nc + (ib ? cy1 : cy0)) * nc + (ie ? cx1 : cx0);
          nr = bk.cnt[cc];
          nr = nr < (uint32_t)kCellCap ? nr : (uint32_t)kCellCap;
          rp = bk.rec + (size_t)cc * kCellCap;
          sp = bk.sa + (size_t)cc * kCellCap;
        } else {
          nr = bk.novf;
          rp = bk.ovf;
          sp = bk.osa;
        }
        for (uint32_t r = 0; r < nr; ++r) {
          const float4 A = rp[r];
          if (!(dist2(d, px, py, pz, A) < d.rc2)) continue;
          n.in_rc++;
          retain(d, a, step, __float_as_int(A.w), sp[r], idj, slot, nullptr, n, rl);
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      s_qn = 0;
      s_ndef = 0;
    }
    __syncthreads();
  }
  if (kF && !dead) {
    // fused binning: the counts two steps ahead (last read in the previous
    // step) are cleared for the next step's sweep
    for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads) d.fcnt[mod3(step + 2u)][q] = 0u;
    if (w == 0 && tid == 0) d.ctl->fovf_n[mod3(step + 2u)] = 0u;
  }
  // clear the bucket counts of the next step's parity (no workgroup of this
  // step reads them; with fused binning too, so that they are clear whenever
  // a step with the binning kernel follows)
  for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads)
    pick(d.cnt, par ^ 1u)[q] = 0u;
  wave_add(&s_cnt[kOutTElig], n.t_elig);
  wave_add(&s_cnt[kOutInRc], n.in_rc);
  wave_add(&s_cnt[kOutDrawn], n.drawn);
  wave_add(&s_cnt[kOutExcl], n.excl);
  if (kF) wave_add(&s_cnt[4], n.a_elig);
  __syncthreads();
  const int ne = s_ne;
  const int nk = ne < kRetCap ? ne : kRetCap;
  if (tid < nk) {
    pick(d.wge, par)[w * kRetCap + tid] = s_ent[tid];
    pick(d.wgk, par)[w * kRetCap + tid] = s_ew2[tid];
  }
  int32_t* out = pick(d.wgo, par) + w * kWgOut;
  if (tid < 4) out[tid] = s_cnt[tid];
  if (tid == 0) {
    out[kOutRet] = nk;
    if (kF) out[kOutAElig] = s_cnt[4];
    if (ne > kRetCap) atomicAdd(&d.ctl->ret_ovf[par], (uint32_t)(ne - kRetCap));
  }
}

// ---------------------------------------------------------------------------
// k_resolve: the T side (steps 6-7) and the bonds (step 9).  Every retained
// pair belongs to the workgroup that owns its T's slot.  Normally the pairs
// come from the sweep workgroup's list: a pair whose A's final key names its
// T is a proposal (the A's key is emptied for the next step), and of the
// proposals to one T the smallest (w2, id_A) is bonded.  If any list
// overflowed in this step, every flagged T enumerates its pairs again (same
// cells, same draws) instead.  An A chose exactly one T and a T bonds at most
// one A, so every state and adjacency row has one writer.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool adj_append(int32_t* row, int B, int32_t v) {
  for (int b = 0; b < B; ++b)
    if (row[b] < 0) {
      row[b] = v;
      return true;
    }
  return false;
}

struct BondCtx {
  int* nw;
  int* lost;
  uint32_t step;
};

// Fused binning after a bond of step `step`: the A's record of the next step
// is dropped when the bond ends its A role, and a T that takes the A role
// (chain growth) is binned for the next step at its re-jittered position.
__device__ void fuse_after_bond(const Dev& d, const Arr& a, uint32_t par, uint32_t step, int sa,
                                int sj, uint32_t idj, uint8_t ra, uint8_t rt) {
  if (ra != kRoleA) fuse_drop(d, par ^ 1u, sa);
  if (rt != kRoleA) return;
  float x = pick(a.x, par ^ 1u)[sj], y = pick(a.y, par ^ 1u)[sj], z = pick(a.z, par ^ 1u)[sj];
  if (d.jitter && d.jit_c != 0.0f) rejitter(d, step + 1u, idj, x, y, z);
  fuse_bin(d, par ^ 1u, step + 1u, sj, idj, x, y, z);
}

// A bond (step 9): states, roles, adjacency rows, and the staged (id_A, id_T)
// row for the log; tagged_t: id_T with the rule of a system of several rules
// in bits 30-31 (plain id_T otherwise).
__device__ __forceinline__ void make_bond_d(const Dev& d, const Arr& a, uint32_t par, int w,
                                            int ida, int sa, int sj, int idj, int32_t da,
                                            int32_t dt, int tagged_t, const BondCtx& b) {
  const int32_t na = a.st[sa] + da, nt = a.st[sj] + dt;
  a.st[sa] = na;
  a.st[sj] = nt;
  a.role[sa] = role_of(d, a.typ[sa], na);
  a.role[sj] = role_of(d, a.typ[sj], nt);
  int lost = 0;
  if (!adj_append(a.adj + (size_t)sa * d.B, d.B, (int32_t)idj)) lost++;
  if (!adj_append(a.adj + (size_t)sj * d.B, d.B, (int32_t)ida)) lost++;
  if (lost) atomicAdd(b.lost, lost);
  const int p = atomicAdd(b.nw, 1);
  if (p < kWinCap) {
    pick(d.wgw, par)[w * kWinCap + p] = make_int2(ida, tagged_t);
  } else {
    const uint32_t o = atomicAdd(&d.ctl->nwin_ovf[par], 1u);
    pick(d.wov, par)[o] = make_int2(ida, tagged_t);
  }
}

__device__ __forceinline__ void make_bond(const Dev& d, const Arr& a, uint32_t par, int w,
                                          int ida, int sa, int sj, int idj, const BondCtx& b) {
  const int32_t na = a.st[sa] + d.rule.d_a, nt = a.st[sj] + d.rule.d_t;
  a.st[sa] = na;
  a.st[sj] = nt;
  const uint8_t ra = role_of(d, a.typ[sa], na), rt = role_of(d, a.typ[sj], nt);
  a.role[sa] = ra;
  a.role[sj] = rt;
  if (d.fuse) fuse_after_bond(d, a, par, b.step, sa, sj, (uint32_t)idj, ra, rt);
  int lost = 0;
  if (!adj_append(a.adj + (size_t)sa * d.B, d.B, (int32_t)idj)) lost++;
  if (!adj_append(a.adj + (size_t)sj * d.B, d.B, (int32_t)ida)) lost++;
  if (lost) atomicAdd(b.lost, lost);
  const int p = atomicAdd(b.nw, 1);
  if (p < kWinCap) {
    pick(d.wgw, par)[w * kWinCap + p] = make_int2(ida, idj);
  } else {
    const uint32_t o = atomicAdd(&d.ctl->nwin_ovf[par], 1u);
    pick(d.wov, par)[o] = make_int2(ida, idj);
  }
}

// The operands of a bond read ahead of the decision, together with the A's
// key: both states and types and (rows of width B <= kAdjStage) both
// adjacency rows.  Every particle takes at most one bond per step, and only
// that bond writes its state and row (and, with fused binning, the bucket
// position of an A's record or a T's binned record; positions are final after
// the sweep), so values read ahead are the ones a bond made after the
// decision would read.
struct BondOps {
  int32_t sta, stt, tya, tyt;
  int4 rowa, rowt;
  // fused binning: where the A's next-step record is, and the T's position
  // of this step (binned if the bond gives the T the A role)
  int32_t apa;
  float tx, ty, tz;
};

__device__ __forceinline__ int4 load_row4(const int32_t* row, int B) {
  int4 r = make_int4(0, 0, 0, 0);  // entries beyond B are not used
  r.x = row[0];
  if (B > 1) r.y = row[1];
  if (B > 2) r.z = row[2];
  if (B > 3) r.w = row[3];
  return r;
}

// The slot adj_append would fill in a row read ahead (B when it is full).
__device__ __forceinline__ int first_empty(int4 r, int B) {
  if (r.x < 0) return 0;
  if (B > 1 && r.y < 0) return 1;
  if (B > 2 && r.z < 0) return 2;
  if (B > 3 && r.w < 0) return 3;
  return B;
}

// make_bond with its operands read ahead (rows of width B <= kAdjStage).
__device__ __forceinline__ void make_bond_ahead(const Dev& d, const Arr& a, uint32_t par, int w,
                                                int ida, int sa, int sj, int idj,
                                                const BondOps& o, const BondCtx& b) {
  const int32_t na = o.sta + d.rule.d_a, nt = o.stt + d.rule.d_t;
  a.st[sa] = na;
  a.st[sj] = nt;
  const uint8_t ra = role_of(d, o.tya, na), rt = role_of(d, o.tyt, nt);
  a.role[sa] = ra;
  a.role[sj] = rt;
  if (d.fuse) {  // fuse_after_bond with the operands read ahead
    if (ra != kRoleA) fuse_drop_at(d, par ^ 1u, o.apa);
    if (rt == kRoleA) {
      float x = o.tx, y = o.ty, z = o.tz;
      if (d.jitter && d.jit_c != 0.0f) rejitter(d, b.step + 1u, (uint32_t)idj, x, y, z);
      fuse_bin(d, par ^ 1u, b.step + 1u, sj, (uint32_t)idj, x, y, z);
    }
  }
  int lost = 0;
  const int fa = first_empty(o.rowa, d.B), ft = first_empty(o.rowt, d.B);
  if (fa < d.B) a.adj[(size_t)sa * d.B + fa] = (int32_t)idj;
  else lost++;
  if (ft < d.B) a.adj[(size_t)sj * d.B + ft] = (int32_t)ida;
  else lost++;
  if (lost) atomicAdd(b.lost, lost);
  const int p = atomicAdd(b.nw, 1);
  if (p < kWinCap) {
    pick(d.wgw, par)[w * kWinCap + p] = make_int2(ida, idj);
  } else {
    const uint32_t q = atomicAdd(&d.ctl->nwin_ovf[par], 1u);
    pick(d.wov, par)[q] = make_int2(ida, idj);
  }
}

// kWave: one wavefront per unit (four units per workgroup, unit = blockIdx.x
// * 4 + wavefront); else the whole workgroup handles unit w.  Every barrier
// is taken by the whole workgroup (mode is the same for all its units).
// kHostPar: the step's parity from Dev::kpar0 (resident systems), else from
// the control block.
template <bool kBrick, bool kWave, bool kHostPar = false>
__device__ __forceinline__ void resolve_body(const Dev& d, int k, int w, int nunits) {
  constexpr int kG = kWave ? kThreads / 64 : 1;  // units per workgroup
  constexpr int kL = kWave ? 64 : kThreads;      // lanes per unit
  __shared__ int s_nw[kG], s_lost[kG], s_prop[kG];
  __shared__ int s_mode;
  __shared__ unsigned long long s_key[kG][kRetCap];
  __shared__ int32_t s_sj[kG][kRetCap];
  const int g = kWave ? (int)(threadIdx.x >> 6) : 0;
  const int tid = kWave ? (int)__lane_id() : (int)threadIdx.x;
  if (kWave) w = w * kG + g;
  const bool live = !kWave || w < nunits;  // the last workgroup's spare wavefronts
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = kHostPar ? (d.kpar0 + (uint32_t)k) & 1u : si.par, step = si.step;
  if (tid == 0) {
    s_nw[g] = 0;
    s_lost[g] = 0;
    s_prop[g] = 0;
  }
  if (threadIdx.x == 0) s_mode = read_err(c) ? 0 : (c->ret_ovf[par] ? 2 : 1);
  // the list's length and its entries in one round trip, issued before the
  // mode is known (read but not used in the other modes, as are entries past
  // the length), then the A keys with the bonds' operands in a second one
  int ne = 0;
  int4 e = make_int4(0, 0, 0, 0);
  uint32_t w2 = 0;
  if (live) {
    ne = pick(d.wgo, par)[w * kWgOut + kOutRet];
    if (tid < kRetCap) {
      e = pick(d.wge, par)[w * kRetCap + tid];
      w2 = pick(d.wgk, par)[w * kRetCap + tid];
    }
  }
  __syncthreads();
  const int mode = s_mode;
  const Arr a = pick_set(d, c->set & 1u);
  const BondCtx bc{&s_nw[g], &s_lost[g], step};
  if (mode == 1) {
    const bool ahead = d.adj_staged != 0;
    bool chosen = false;
    unsigned long long key = kEmpty;
    BondOps ops{0, 0, 0, 0, make_int4(0, 0, 0, 0), make_int4(0, 0, 0, 0), 0, 0.0f, 0.0f, 0.0f};
    if (tid < ne) {
      const unsigned long long ka = d.slotA[e.x];
      if (ahead) {
        ops.sta = a.st[e.y];
        ops.stt = a.st[e.z];
        ops.tya = a.typ[e.y];
        ops.tyt = a.typ[e.z];
        ops.rowa = load_row4(a.adj + (size_t)e.y * d.B, d.B);
        ops.rowt = load_row4(a.adj + (size_t)e.z * d.B, d.B);
        if (d.fuse) {
          ops.apa = d.apos[e.y];
          ops.tx = pick(a.x, par ^ 1u)[e.z];
          ops.ty = pick(a.y, par ^ 1u)[e.z];
          ops.tz = pick(a.z, par ^ 1u)[e.z];
        }
      }
      d.tflag[e.z] = 0;
      chosen = (uint32_t)ka == (uint32_t)e.w;
      if (chosen) {
        d.slotA[e.x] = kEmpty;
        key = ((unsigned long long)w2 << 32) | (uint32_t)e.x;
        atomicAdd(&s_prop[g], 1);
      }
      s_key[g][tid] = key;
      s_sj[g][tid] = e.z;
    }
    __syncthreads();
    if (chosen) {
      bool win = true;
      for (int f = 0; f < ne; ++f)
        if (s_sj[g][f] == e.z && s_key[g][f] < key) win = false;
      if (win) {
        if (ahead) make_bond_ahead(d, a, par, w, e.x, e.y, e.z, e.w, ops, bc);
        else make_bond(d, a, par, w, e.x, e.y, e.z, e.w, bc);
      }
    }
  } else if (mode == 2 && live) {
    const float *X = pick(a.x, par ^ 1u), *Y = pick(a.y, par ^ 1u), *Z = pick(a.z, par ^ 1u);
    const Buckets bk = d.fuse ? step_buckets<true>(d, par, step) : step_buckets<false>(d, par, step);
    int s0, s1;
    range_of<kBrick>(d, w, s0, s1);
    for (int base = s0; base < s1; base += kL) {
      const int slot = base + tid;
      if (slot < s1 && d.tflag[slot]) {
        d.tflag[slot] = 0;
        const float xj = X[slot], yj = Y[slot], zj = Z[slot];
        const uint32_t idj = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
        unsigned long long best = kEmpty;
        int best_sa = 0, np = 0;
        for_global_records(d, bk, xj, yj, zj, [&](float4 A, int sa) {
          if (!(dist2(d, xj, yj, zj, A) < d.rc2)) return;
          const int ida = __float_as_int(A.w);
          if ((uint32_t)d.slotA[ida] != idj) return;  // not retained, or the A chose another T
          const W4 r = philox(step, (uint32_t)ida, idj, 0u, d.seed);
          d.slotA[ida] = kEmpty;
          np++;
          const unsigned long long bid = ((unsigned long long)r.w2 << 32) | (uint32_t)ida;
          if (bid < best) {
            best = bid;
            best_sa = sa;
          }
        });
        if (np) atomicAdd(&s_prop[g], np);
        if (best != kEmpty) make_bond(d, a, par, w, (int)(uint32_t)best, best_sa, slot, (int)idj, bc);
      }
    }
  }
  __syncthreads();
  if (tid == 0 && live) {
    int32_t* out = pick(d.wgo, par) + w * kWgOut;
    out[kOutProp] = s_prop[g];
    out[kOutBonds] = s_nw[g];
    out[kOutLost] = s_lost[g];
  }
}

// ---------------------------------------------------------------------------
// The "nearest" selection (LAMMPS fix bond/create, Sec. IV A of the paper):
// every candidate pair -- eligible, in range, not already bonded when the
// rule excludes bonded pairs -- is visited once, from its T, which keeps its
// closest A in registers (key (r2 bits, id_A): r2 >= 0 orders like its bits,
// equal distances go to the lower id) and lowers the A's key (r2 bits, id_T)
// with a 64-bit atomicMin.  A T with a candidate leaves (its closest A, its
// slot) in tnear[id_T].  Then each A whose closest T keeps it in return is
// tested once, with the pair's draw (word 0 of the counter (step, id_A, id_T,
// 0)), and bonds when it passes.
// ---------------------------------------------------------------------------
template <bool kBrick>
__device__ __forceinline__ void near_sweep_body(const Dev& d, int k, int w, int nwg) {
  __shared__ int s_cnt[4];
  const int tid = threadIdx.x;
  if (tid < 4) s_cnt[tid] = 0;
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const bool jit = d.jitter && d.jit_c != 0.0f;
  const Buckets bk = step_buckets<false>(d, par, step);
  const bool dead = read_err(c) != 0;
  int s0, s1;
  range_of<kBrick>(d, w, s0, s1);
  __syncthreads();
  int t_elig = 0, in_rc = 0, excl = 0;
  for (int slot = s0 + tid; slot < s1 && !dead; slot += kThreads) {
    float x = X[slot], y = Y[slot], z = Z[slot];
    const uint32_t id = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
    if (d.jitter) {  // the re-jitter, as in the random selection's sweep
      if (jit) rejitter(d, step, id, x, y, z);
      XW[slot] = x;
      YW[slot] = y;
      ZW[slot] = z;
    }
    if (a.role[slot] != kRoleT) continue;
    t_elig++;
    unsigned long long best = kEmpty;
    for_global_records(d, bk, x, y, z, [&](float4 A, int sa) {
      const float r2 = dist2(d, x, y, z, A);
      if (!(r2 < d.rc2)) return;
      in_rc++;
      if (d.rule.exclude && row_has(a.adj + (size_t)sa * d.B, d.B, (int32_t)id)) {
        excl++;
        return;
      }
      const unsigned long long rb = (unsigned long long)__float_as_uint(r2) << 32;
      const uint32_t ida = (uint32_t)__float_as_int(A.w);
      atomicMin(&d.slotA[ida], rb | id);
      const unsigned long long kt = rb | ida;
      best = kt < best ? kt : best;
    });
    if (best != kEmpty) d.tnear[id] = make_int2((int)(uint32_t)best, slot);
  }
  wave_add(&s_cnt[0], t_elig);
  wave_add(&s_cnt[1], in_rc);
  wave_add(&s_cnt[2], excl);
  // clear the bucket counts of the next step's parity (as the other sweep)
  for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads)
    pick(d.cnt, par ^ 1u)[q] = 0u;
  __syncthreads();
  int32_t* out = pick(d.wgo, par) + w * kWgOut;
  if (tid == 0) {
    out[kOutTElig] = s_cnt[0];
    out[kOutInRc] = s_cnt[1];
    out[kOutDrawn] = 0;
    out[kOutExcl] = s_cnt[2];
    out[kOutRet] = 0;
  }
}

// The brick of sweep workgroup g.  Workgroups are dispatched to the eight
// XCDs in turn (g mod 8), each XCD with an L2 of its own; XCD x takes the
// contiguous run of bricks x * q + min(x, r) .. (q or q + 1 of them, q =
// nbricks / 8, r = nbricks mod 8), a slab of neighbouring bricks, so that
// the A records a brick's neighbours stage again are in the same L2.
__device__ __forceinline__ int xcd_brick(int g, int nbricks) {
  constexpr int kXcd = 8;
  const int q = nbricks / kXcd, r = nbricks - q * kXcd;
  const int x = g % kXcd, i = g / kXcd;
  return x * q + min(x, r) + i;
}

// The A records of a brick's region staged in LDS (sorted storage, brick
// edges up to kOneCellBrick: one region cell per thread), as the random
// selection's sweep stages them, for the kernels that visit every in-range
// (A, T) pair of a T: the sweeps of the nearest selection and of several
// rules, and the kinetics counters.  A T whose 2x2x2 block leaves the staged
// region, and every T of
// a brick whose region holds more than kStageRecs records or of a step with
// bucket overflow, scans the global buckets instead; either way a T visits
// the same pairs.
struct StagedRegion {
  float4* rec;    // records (x, y, z, id_A)
  int4* radj;     // the A's adjacency rows (rows of width <= kAdjStage)
  int32_t* rsa;   // the A's slots
  uint16_t* off;  // first record of each region cell (one more entry: the total)
  int bx, ex, by, ey, bz, ez;
  bool staged, nowrap;
};

__device__ __forceinline__ void stage_region(const Dev& d, const Buckets& bk, int w,
                                             StagedRegion& g, uint32_t* s_wave) {
  const int tid = threadIdx.x, nc = d.nc;
  int bxc, byc;
  const int bzc = div_nb(d, div_nb(d, w, bxc), byc);
  region_dim(d, bxc, g.bx, g.ex);
  region_dim(d, byc, g.by, g.ey);
  region_dim(d, bzc, g.bz, g.ez);
  const int ex = g.ex, ey = g.ey, ncs = ex * ey * g.ez;
  // a region that does not wrap around the box and spans less than half of
  // it: the minimum image leaves every difference in it unchanged
  g.nowrap = d.nbricks > 1 && g.bx + ex <= nc && 2 * ex + 1 <= nc && g.by + ey <= nc &&
             2 * ey + 1 <= nc && g.bz + g.ez <= nc && 2 * g.ez + 1 <= nc;
  uint32_t mine = 0;
  int gc = 0;
  if (tid < ncs) {
    const int lz = div_small(tid, recip16((uint32_t)(ex * ey))), rem = tid - lz * ex * ey;
    const int ly = div_small(rem, recip16((uint32_t)ex)), lx = rem - ly * ex;
    int cx = g.bx + lx, cy = g.by + ly, cz = g.bz + lz;
    cx -= cx >= nc ? nc : 0;
    cy -= cy >= nc ? nc : 0;
    cz -= cz >= nc ? nc : 0;
    gc = (cz * nc + cy) * nc + cx;
    mine = bk.cnt[gc];
    mine = mine < (uint32_t)kCellCap ? mine : (uint32_t)kCellCap;
  }
  uint32_t total = 0;
  const uint32_t off = block_scan_excl(mine, s_wave, total);
  g.staged = total <= (uint32_t)kStageRecs && bk.novf == 0;
  if (tid < ncs) {
    g.off[tid] = (uint16_t)off;
    if (g.staged) {
      const size_t r0 = (size_t)gc * kCellCap;
      // the first two records loaded together, the rare rest one by one
      float4 rv0 = make_float4(0.f, 0.f, 0.f, 0.f), rv1 = rv0;
      int32_t sv0 = 0, sv1 = 0;
      int4 av0 = make_int4(-1, -1, -1, -1), av1 = av0;
      if (mine > 0u) {
        rv0 = bk.rec[r0];
        sv0 = bk.sa[r0];
        if (d.adj_staged) av0 = d.radj[r0];
      }
      if (mine > 1u) {
        rv1 = bk.rec[r0 + 1];
        sv1 = bk.sa[r0 + 1];
        if (d.adj_staged) av1 = d.radj[r0 + 1];
      }
      if (mine > 0u) {
        g.rec[off] = rv0;
        g.rsa[off] = sv0;
        g.radj[off] = av0;
      }
      if (mine > 1u) {
        g.rec[off + 1] = rv1;
        g.rsa[off + 1] = sv1;
        g.radj[off + 1] = av1;
      }
      for (uint32_t j = 2; j < mine; ++j) {
        g.rec[off + j] = bk.rec[r0 + j];
        g.rsa[off + j] = bk.sa[r0 + j];
        if (d.adj_staged) g.radj[off + j] = d.radj[r0 + j];
      }
    }
  }
  if (tid == 0) g.off[ncs] = (uint16_t)total;
  __syncthreads();
}

// Every in-range pair of the T (id_T) at (x, y, z): f(record, r2, excluded,
// slot_A, staged index or -1), the exclusion tested on the A's staged row (or its row in the
// particle arrays) when the rule excludes bonded pairs.  The staged records
// when the T's block lies in the staged region, else the global buckets.
template <bool kExcl = true, typename F>
__device__ __forceinline__ void visit_pairs(const Dev& d, const Arr& a, const Buckets& bk,
                                            const StagedRegion& g, float x, float y, float z,
                                            uint32_t id, F f) {
  const int nc = d.nc;
  if (g.staged) {
    const int lx0 = local_lo(x, d.inv_w, g.bx, nc), ly0 = local_lo(y, d.inv_w, g.by, nc),
              lz0 = local_lo(z, d.inv_w, g.bz, nc);
    if ((uint32_t)lx0 < (uint32_t)(g.ex - 1) && (uint32_t)ly0 < (uint32_t)(g.ey - 1) &&
        (uint32_t)lz0 < (uint32_t)(g.ez - 1)) {
      const int l0 = (lz0 * g.ey + ly0) * g.ex + lx0;
      auto scan = [&](auto dist) {
        for (int run = 0; run < 4; ++run) {
          const int lr = l0 + ((run & 1) ? g.ex : 0) + ((run & 2) ? g.ex * g.ey : 0);
          const int r1 = (int)g.off[lr + 2];
          for (int r = (int)g.off[lr]; r < r1; ++r) {
            const float4 A = g.rec[r];
            const float r2 = dist(A);
            if (!(r2 < d.rc2)) continue;
            bool ex_b = false;
            if (kExcl && d.rule.exclude) {
              if (d.adj_staged) {
                const int4 q = g.radj[r];
                const int v = (int)id;
                ex_b = q.x == v || q.y == v || q.z == v || q.w == v;
              } else {
                ex_b = row_has(a.adj + (size_t)g.rsa[r] * d.B, d.B, (int32_t)id);
              }
            }
            f(A, r2, ex_b, g.rsa[r], r);
          }
        }
      };
      if (g.nowrap)
        scan([&](float4 A) { return dist2_plain(x, y, z, A); });
      else
        scan([&](float4 A) { return dist2(d, x, y, z, A); });
      return;
    }
  }
  for_global_records(d, bk, x, y, z, [&](float4 A, int sa) {
    const float r2 = dist2(d, x, y, z, A);
    if (!(r2 < d.rc2)) return;
    f(A, r2, kExcl && d.rule.exclude && row_has(a.adj + (size_t)sa * d.B, d.B, (int32_t)id), sa,
      -1);
  });
}

// near_sweep_body on sorted storage with the region staged (StagedRegion):
// the same pairs get the same keys, so the outcome is that of near_sweep_body.
__device__ __forceinline__ void near_sweep_staged_body(const Dev& d, int k, int w, int nwg) {
  __shared__ float4 s_rec[kStageRecs];
  __shared__ int4 s_radj[kStageRecs];
  __shared__ int32_t s_rsa[kStageRecs];
  __shared__ uint16_t s_off[kStageCells1 + 1];
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  __shared__ int s_cnt[4];
  const int tid = threadIdx.x;
  if (tid < 4) s_cnt[tid] = 0;
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const bool jit = d.jitter && d.jit_c != 0.0f;
  const Buckets bk = step_buckets<false>(d, par, step);
  const bool dead = read_err(c) != 0;
  int s0, s1;
  range_of<true>(d, w, s0, s1);
  StagedRegion g;
  g.rec = s_rec;
  g.radj = s_radj;
  g.rsa = s_rsa;
  g.off = s_off;
  stage_region(d, bk, w, g, s_wave);
  int t_elig = 0, in_rc = 0, excl = 0;
  // one particle per thread and pass; the next pass's particle is loaded
  // while this one is handled
  float nx = 0.f, ny = 0.f, nz = 0.f;
  int32_t nid = 0;
  uint8_t nrole = kRoleNone;
  if (s0 + tid < s1) {
    nx = X[s0 + tid];
    ny = Y[s0 + tid];
    nz = Z[s0 + tid];
    nid = a.id[s0 + tid];
    nrole = a.role[s0 + tid];
  }
  for (int slot = s0 + tid; slot < s1 && !dead; slot += kThreads) {
    float x = nx, y = ny, z = nz;
    const uint32_t id = (uint32_t)nid;
    const uint8_t role = nrole;
    if (slot + kThreads < s1) {
      nx = X[slot + kThreads];
      ny = Y[slot + kThreads];
      nz = Z[slot + kThreads];
      nid = a.id[slot + kThreads];
      nrole = a.role[slot + kThreads];
    }
    if (d.jitter) {  // the re-jitter, as in the random selection's sweep
      if (jit) rejitter(d, step, id, x, y, z);
      XW[slot] = x;
      YW[slot] = y;
      ZW[slot] = z;
    }
    if (role != kRoleT) continue;
    t_elig++;
    // each candidate lowers the A's key to (r2 bits, id_T); the T keeps its
    // own closest as (r2 bits, id_A)
    unsigned long long best = kEmpty;
    visit_pairs(d, a, bk, g, x, y, z, id, [&](float4 A, float r2, bool excluded, int, int) {
      in_rc++;
      if (excluded) {
        excl++;
        return;
      }
      const unsigned long long rb = (unsigned long long)__float_as_uint(r2) << 32;
      const uint32_t ida = (uint32_t)__float_as_int(A.w);
      atomicMin(&d.slotA[ida], rb | id);
      const unsigned long long kt = rb | ida;
      best = kt < best ? kt : best;
    });
    if (best != kEmpty) d.tnear[id] = make_int2((int)(uint32_t)best, slot);
  }
  wave_add(&s_cnt[0], t_elig);
  wave_add(&s_cnt[1], in_rc);
  wave_add(&s_cnt[2], excl);
  // clear the bucket counts of the next step's parity (as the other sweep)
  for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads)
    pick(d.cnt, par ^ 1u)[q] = 0u;
  __syncthreads();
  int32_t* out = pick(d.wgo, par) + w * kWgOut;
  if (tid == 0) {
    out[kOutTElig] = s_cnt[0];
    out[kOutInRc] = s_cnt[1];
    out[kOutDrawn] = 0;
    out[kOutExcl] = s_cnt[2];
    out[kOutRet] = 0;
  }
}

// The A side of the nearest selection and the bonds: unit w (of nunits, the
// sweep's workgroup count, whose staging windows and counters it fills)
// takes the A records of a contiguous range of cells, unit 0 also the
// overflow list.  Every A record appears once, so every A key is read and
// emptied by exactly one thread.
__device__ __forceinline__ void near_resolve_body(const Dev& d, int k, int w, int nunits) {
  __shared__ int s_nw, s_lost, s_cnt[2];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_nw = 0;
    s_lost = 0;
    s_cnt[0] = 0;
    s_cnt[1] = 0;
  }
  __syncthreads();
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const BondCtx bc{&s_nw, &s_lost};
  int prop = 0, mutual = 0;
  auto visit = [&](float4 A, int sa) {
    const int ida = __float_as_int(A.w);
    const unsigned long long key = d.slotA[ida];
    if (key == kEmpty) return;
    d.slotA[ida] = kEmpty;
    prop++;
    const uint32_t idj = (uint32_t)key;
    const int2 t = d.tnear[idj];
    if (t.x != ida) return;  // the T's closest A is another one
    mutual++;
    const W4 r = philox(step, (uint32_t)ida, idj, 0u, d.seed);
    if ((unsigned long long)r.w0 < d.thresh) make_bond(d, a, par, w, ida, sa, t.y, (int)idj, bc);
  };
  if (read_err(c) == 0) {
    const int per = (d.ncell + nunits - 1) / nunits;
    const int c0 = w * per, c1 = min(d.ncell, c0 + per);
    for (int cc = c0 + tid; cc < c1; cc += kThreads) {
      uint32_t nr = pick(d.cnt, par)[cc];
      nr = nr < (uint32_t)kCellCap ? nr : (uint32_t)kCellCap;
      const size_t r0 = (size_t)cc * kCellCap;
      for (uint32_t r = 0; r < nr; ++r) visit(d.rec[r0 + r], d.rsa[r0 + r]);
    }
    if (w == 0) {
      const uint32_t novf = c->ovf_n[par];
      for (uint32_t r = tid; r < novf; r += kThreads)
        visit(pick(d.ovf, par)[r], pick(d.ovf_sa, par)[r]);
    }
  }
  wave_add(&s_cnt[0], prop);
  wave_add(&s_cnt[1], mutual);
  __syncthreads();
  if (tid == 0) {
    int32_t* out = pick(d.wgo, par) + w * kWgOut;
    out[kOutDrawn] = s_cnt[1];
    out[kOutProp] = s_cnt[0];
    out[kOutBonds] = s_nw;
    out[kOutLost] = s_lost;
  }
}

// ---------------------------------------------------------------------------
// Several concurrent rules (nrules > 1): Table I generalised over the rules.
// Every rule contributes candidates with its own draw (counter word 3 = the
// rule's tag); each A picks among its accepted candidates of all rules the
// smallest (w1, id_T), the lower rule on a tie; each T keeps the smallest
// (w2, id_A) of the pairs that picked it; a particle that wins both as an A
// and as a T keeps the pair with the smaller (w3, partner id, rule) and a
// pair is bonded only if both of its particles keep it.  Three kernels after
// the binning: the sweep (draws, A-side picks by 64-bit atomicMin, T flags),
// the T-side choice (re-enumerates the flagged T's candidates) and the final
// choice with the bonds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rule_tag(const Dev& d, int r) {
  uint32_t t = d.mr[0].tag;
#pragma unroll
  for (int q = 1; q < kMaxRules; ++q)
    if (r == q) t = d.mr[q].tag;
  return t;
}

__device__ __forceinline__ void rule_deltas(const Dev& d, int r, int32_t& da, int32_t& dt) {
  da = d.mr[0].r.d_a;
  dt = d.mr[0].r.d_t;
#pragma unroll
  for (int q = 1; q < kMaxRules; ++q)
    if (r == q) {
      da = d.mr[q].r.d_a;
      dt = d.mr[q].r.d_t;
    }
}

__device__ __forceinline__ bool key_less(unsigned long long k1, int r1, unsigned long long k2,
                                         int r2) {
  return k1 < k2 || (k1 == k2 && r1 < r2);
}

// Visits the rules r under which the pair (A record at slot sa, T of role
// mask rt) is a candidate at squared distance r2, in increasing r:
// f(r, draw words, excluded as bonded).
template <typename F>
__device__ __forceinline__ void multi_candidates(const Dev& d, const Arr& a, uint32_t step,
                                                 uint32_t rt, int sa, int ida, uint32_t idj,
                                                 float r2, F f, int arole = -1,
                                                 const int4* arow = nullptr) {
  const uint32_t both = rt & ((uint32_t)(arole >= 0 ? arole : a.role[sa]) >> 4);
  if (!both) return;
  int bonded = -1;
#pragma unroll
  for (int r = 0; r < kMaxRules; ++r) {
    if (r >= d.nrules || !((both >> r) & 1u) || !(r2 < d.mr[r].rc2)) continue;
    if (bonded < 0) {
      if (arow) {
        const int4 q = *arow;
        const int v = (int)idj;
        bonded = q.x == v || q.y == v || q.z == v || q.w == v;
      } else {
        bonded = row_has(a.adj + (size_t)sa * d.B, d.B, (int32_t)idj) ? 1 : 0;
      }
    }
    const W4 w = philox(step, (uint32_t)ida, idj, d.mr[r].tag, d.seed);
    f(r, w, d.mr[r].r.exclude && bonded > 0, w.w0 < d.mr[r].thresh);
  }
}

template <bool kBrick>
__device__ __forceinline__ void multi_sweep_body(const Dev& d, int k, int w, int nwg) {
  __shared__ int s_cnt[4];
  const int tid = threadIdx.x;
  if (tid < 4) s_cnt[tid] = 0;
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const bool jit = d.jitter && d.jit_c != 0.0f;
  const Buckets bk = step_buckets<false>(d, par, step);
  const bool dead = read_err(c) != 0;
  int s0, s1;
  range_of<kBrick>(d, w, s0, s1);
  __syncthreads();
  int t_elig = 0, in_rc = 0, drawn = 0, excl = 0;
  for (int slot = s0 + tid; slot < s1 && !dead; slot += kThreads) {
    float x = X[slot], y = Y[slot], z = Z[slot];
    const uint32_t id = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
    if (d.jitter) {
      if (jit) rejitter(d, step, id, x, y, z);
      XW[slot] = x;
      YW[slot] = y;
      ZW[slot] = z;
    }
    d.wfa[slot] = 0;
    d.wft[slot] = 0;
    const uint32_t rt = a.role[slot] & kMaskT;
    if (!rt) continue;
    t_elig++;
    bool any = false;
    for_global_records(d, bk, x, y, z, [&](float4 A, int sa) {
      const int ida = __float_as_int(A.w);
      if ((uint32_t)ida == id) return;
      const float r2 = dist2(d, x, y, z, A);
      if (!(r2 < d.rc2)) return;
      multi_candidates(d, a, step, rt, sa, ida, id, r2, [&](int, W4 wd, bool ex, bool acc) {
        in_rc++;
        if (!acc) return;
        drawn++;
        if (ex) {
          excl++;
          return;
        }
        any = true;
        atomicMin(&d.slotA[ida], ((unsigned long long)wd.w1 << 32) | id);
      });
    });
    if (any) d.tflag[slot] = 1;
  }
  wave_add(&s_cnt[0], t_elig);
  wave_add(&s_cnt[1], in_rc);
  wave_add(&s_cnt[2], drawn);
  wave_add(&s_cnt[3], excl);
  for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads)
    pick(d.cnt, par ^ 1u)[q] = 0u;
  __syncthreads();
  int32_t* out = pick(d.wgo, par) + w * kWgOut;
  if (tid == 0) {
    out[kOutTElig] = s_cnt[0];
    out[kOutInRc] = s_cnt[1];
    out[kOutDrawn] = s_cnt[2];
    out[kOutExcl] = s_cnt[3];
    out[kOutRet] = 0;
  }
}

// multi_sweep_body on sorted storage with the region staged (StagedRegion,
// with the A's role bytes): the same candidates, draws and keys.
__device__ __forceinline__ void multi_sweep_staged_body(const Dev& d, int k, int w, int nwg) {
  __shared__ float4 s_rec[kStageRecs];
  __shared__ int4 s_radj[kStageRecs];
  __shared__ int32_t s_rsa[kStageRecs];
  __shared__ uint8_t s_arole[kStageRecs];
  __shared__ uint16_t s_off[kStageCells1 + 1];
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  __shared__ int s_cnt[4];
  const int tid = threadIdx.x;
  if (tid < 4) s_cnt[tid] = 0;
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const bool jit = d.jitter && d.jit_c != 0.0f;
  const Buckets bk = step_buckets<false>(d, par, step);
  const bool dead = read_err(c) != 0;
  int s0, s1;
  range_of<true>(d, w, s0, s1);
  StagedRegion g;
  g.rec = s_rec;
  g.radj = s_radj;
  g.rsa = s_rsa;
  g.off = s_off;
  stage_region(d, bk, w, g, s_wave);
  // the staged A's role bytes (the roles of the step: nothing changes them
  // before the resolve)
  if (g.staged) {
    const int nrec = (int)s_off[g.ex * g.ey * g.ez];
    for (int r = tid; r < nrec; r += kThreads) s_arole[r] = a.role[s_rsa[r]];
    __syncthreads();
  }
  int t_elig = 0, in_rc = 0, drawn = 0, excl = 0;
  for (int slot = s0 + tid; slot < s1 && !dead; slot += kThreads) {
    float x = X[slot], y = Y[slot], z = Z[slot];
    const uint32_t id = (uint32_t)a.id[slot];
    const uint32_t rt = a.role[slot] & kMaskT;
    if (d.jitter) {
      if (jit) rejitter(d, step, id, x, y, z);
      XW[slot] = x;
      YW[slot] = y;
      ZW[slot] = z;
    }
    d.wfa[slot] = 0;
    d.wft[slot] = 0;
    if (!rt) continue;
    t_elig++;
    bool any = false;
    visit_pairs<false>(d, a, bk, g, x, y, z, id, [&](float4 A, float r2, bool, int sa, int r) {
      const int ida = __float_as_int(A.w);
      if ((uint32_t)ida == id) return;
      multi_candidates(d, a, step, rt, sa, ida, id, r2, [&](int, W4 wd, bool ex, bool acc) {
        in_rc++;
        if (!acc) return;
        drawn++;
        if (ex) {
          excl++;
          return;
        }
        any = true;
        atomicMin(&d.slotA[ida], ((unsigned long long)wd.w1 << 32) | id);
      }, r >= 0 ? (int)s_arole[r] : -1, r >= 0 && d.adj_staged ? &s_radj[r] : nullptr);
    });
    if (any) d.tflag[slot] = 1;
  }
  wave_add(&s_cnt[0], t_elig);
  wave_add(&s_cnt[1], in_rc);
  wave_add(&s_cnt[2], drawn);
  wave_add(&s_cnt[3], excl);
  for (int q = w * kThreads + tid; q < d.ncell; q += nwg * kThreads)
    pick(d.cnt, par ^ 1u)[q] = 0u;
  __syncthreads();
  int32_t* out = pick(d.wgo, par) + w * kWgOut;
  if (tid == 0) {
    out[kOutTElig] = s_cnt[0];
    out[kOutInRc] = s_cnt[1];
    out[kOutDrawn] = s_cnt[2];
    out[kOutExcl] = s_cnt[3];
    out[kOutRet] = 0;
  }
}

// The T side: every T with an accepted candidate finds the A's whose pick
// names it (the lowest rule whose accepted candidate gives the A's key) and
// keeps the smallest (w2, id_A); the pair is recorded at both slots.
template <bool kBrick>
__device__ __forceinline__ void multi_resolve_body(const Dev& d, int k, int w) {
  __shared__ int s_prop;
  const int tid = threadIdx.x;
  if (tid == 0) s_prop = 0;
  __syncthreads();
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par ^ 1u), *Y = pick(a.y, par ^ 1u), *Z = pick(a.z, par ^ 1u);
  const Buckets bk = step_buckets<false>(d, par, step);
  int s0, s1;
  range_of<kBrick>(d, w, s0, s1);
  int prop = 0;
  for (int slot = s0 + tid; slot < s1; slot += kThreads) {
    if (d.tflag[slot] != 1) continue;
    d.tflag[slot] = 0;
    const float x = X[slot], y = Y[slot], z = Z[slot];
    const uint32_t id = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
    const uint32_t rt = a.role[slot] & kMaskT;
    unsigned long long best = kEmpty;
    int best_sa = 0, best_r = 0;
    for_global_records(d, bk, x, y, z, [&](float4 A, int sa) {
      const int ida = __float_as_int(A.w);
      if ((uint32_t)ida == id) return;
      const float r2 = dist2(d, x, y, z, A);
      if (!(r2 < d.rc2)) return;
      const unsigned long long key = d.slotA[ida];
      if (key == kEmpty || (uint32_t)key != id) return;  // the A picked another T
      int got = -1;
      W4 wg{0, 0, 0, 0};
      multi_candidates(d, a, step, rt, sa, ida, id, r2, [&](int r, W4 wd, bool ex, bool acc) {
        if (got < 0 && acc && !ex && wd.w1 == (uint32_t)(key >> 32)) {
          got = r;
          wg = wd;
        }
      });
      if (got < 0) return;
      d.slotA[ida] = kEmpty;  // only this T's thread reads the key that names it
      prop++;
      const unsigned long long k2 = ((unsigned long long)wg.w2 << 32) | (uint32_t)ida;
      if (k2 < best) {
        best = k2;
        best_sa = sa;
        best_r = got;
      }
    });
    if (best != kEmpty) {
      const int ida = (int)(uint32_t)best;
      d.wint[slot] = make_int4(ida, best_sa, best_r, 0);
      d.wina[best_sa] = make_int4((int)id, slot, best_r, 0);
      d.wft[slot] = 1;
      d.wfa[best_sa] = 1;  // one writer: the A picked one T
    }
  }
  atomicAdd(&s_prop, prop);
  __syncthreads();
  if (tid == 0) pick(d.wgo, par)[w * kWgOut + kOutProp] = s_prop;
}

// Step 8 and the bonds, from the T of every winning pair.
template <bool kBrick>
__device__ __forceinline__ void multi_final_body(const Dev& d, int k, int w) {
  __shared__ int s_nw, s_lost;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_nw = 0;
    s_lost = 0;
  }
  __syncthreads();
  const Ctl* c = d.ctl;
  const StepInfo si = step_info(c, k);
  const uint32_t par = si.par, step = si.step;
  const Arr a = pick_set(d, c->set & 1u);
  const BondCtx bc{&s_nw, &s_lost};
  int s0, s1;
  range_of<kBrick>(d, w, s0, s1);
  for (int slot = s0 + tid; slot < s1; slot += kThreads) {
    if (!d.wft[slot]) continue;
    const uint32_t id = a.id ? (uint32_t)a.id[slot] : (uint32_t)slot;
    const int4 t = d.wint[slot];
    const int ida = t.x, sa = t.y, r = t.z;
    const W4 wd = philox(step, (uint32_t)ida, id, rule_tag(d, r), d.seed);
    bool keep = true;
    if (d.wfa[slot]) {  // this T also won as the A of another pair
      const int4 o = d.wina[slot];
      const W4 wo = philox(step, id, (uint32_t)o.x, rule_tag(d, o.z), d.seed);
      keep = key_less(((unsigned long long)wd.w3 << 32) | (uint32_t)ida, r,
                      ((unsigned long long)wo.w3 << 32) | (uint32_t)o.x, o.z);
    }
    if (keep && d.wft[sa]) {  // the A also won as the T of another pair
      const int4 o = d.wint[sa];
      const W4 wo = philox(step, (uint32_t)o.x, (uint32_t)ida, rule_tag(d, o.z), d.seed);
      keep = key_less(((unsigned long long)wd.w3 << 32) | id, r,
                      ((unsigned long long)wo.w3 << 32) | (uint32_t)o.x, o.z);
    }
    if (keep) {
      int32_t da, dt;
      rule_deltas(d, r, da, dt);
      make_bond_d(d, a, par, w, ida, sa, slot, (int)id, da, dt, (int)(id | ((uint32_t)r << 30)),
                  bc);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int32_t* out = pick(d.wgo, par) + w * kWgOut;
    out[kOutBonds] = s_nw;
    out[kOutLost] = s_lost;
  }
}

// ---------------------------------------------------------------------------
// Bonded-force coupling: velocity Verlet with the mirror-LJ bond force over
// the adjacency table (Sec. II D, Eq. (mirror LJ)), md_theta steps before each
// reaction step.  Kernel m = 0 .. theta of reaction step k of a block: the
// forces at the positions of parity (par0 + k + m) (partners found through
// slot_of); m = 0 kicks half a step and drifts, 0 < m < theta completes the
// previous step's second half kick, kicks and drifts, m = theta completes
// the last one.  Drifted positions go to the other parity; for odd theta the
// last kernel copies the positions over once more, so that every MD block
// flips the buffers an even number of times and the reaction step finds them
// in the parity its step number gives.  Every operation is FP32, rounded on
// its own, in the order the oracle uses.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_md(Dev d, int k, int m) {
  const Ctl* c = d.ctl;
  const uint32_t par = (c->par0 + (uint32_t)k + (uint32_t)m) & 1u;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n || read_err(c)) return;
  const float xi = X[i], yi = Y[i], zi = Z[i];
  float fx = 0.0f, fy = 0.0f, fz = 0.0f;
  bool torn = false;
  const int32_t* row = a.adj + (size_t)i * d.B;
  for (int b = 0; b < d.B; ++b) {
    const int32_t j = row[b];
    if (j < 0) continue;
    const int sj = d.slot_of[j];
    const float dx = min_image(__fsub_rn(X[sj], xi), d.L, d.halfL);
    const float dy = min_image(__fsub_rn(Y[sj], yi), d.L, d.halfL);
    const float dz = min_image(__fsub_rn(Z[sj], zi), d.L, d.halfL);
    const float r2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
    if (!(r2 > d.md_sc2)) continue;  // no force up to sigma_c
    const float r = sqrt_rn(r2);
    const float sgap = __fsub_rn(d.md_two_sc, r);
    if (!(sgap > 0.0f)) {
      torn = true;
      continue;
    }
    const float q = __fdiv_rn(d.md_sig, sgap);
    const float q2 = __fmul_rn(q, q);
    const float q6 = __fmul_rn(__fmul_rn(q2, q2), q2);
    const float q12 = __fmul_rn(q6, q6);
    const float cf =
        __fdiv_rn(__fdiv_rn(__fmul_rn(d.md_e24, __fsub_rn(__fadd_rn(q12, q12), q6)), sgap), r);
    fx = __fadd_rn(fx, __fmul_rn(cf, dx));
    fy = __fadd_rn(fy, __fmul_rn(cf, dy));
    fz = __fadd_rn(fz, __fmul_rn(cf, dz));
  }
  if (torn) set_err(d.ctl, PR_EINVAL);
  float vx = a.vx[i], vy = a.vy[i], vz = a.vz[i];
  const float h = d.md_h;
  if (m > 0) {  // the second half kick of the previous MD step
    vx = __fadd_rn(vx, __fmul_rn(h, fx));
    vy = __fadd_rn(vy, __fmul_rn(h, fy));
    vz = __fadd_rn(vz, __fmul_rn(h, fz));
  }
  if (m < d.md_theta) {  // the first half kick and the drift of MD step m
    vx = __fadd_rn(vx, __fmul_rn(h, fx));
    vy = __fadd_rn(vy, __fmul_rn(h, fy));
    vz = __fadd_rn(vz, __fmul_rn(h, fz));
    XW[i] = wrap_box(__fadd_rn(xi, __fmul_rn(d.md_dt, vx)), d.L);
    YW[i] = wrap_box(__fadd_rn(yi, __fmul_rn(d.md_dt, vy)), d.L);
    ZW[i] = wrap_box(__fadd_rn(zi, __fmul_rn(d.md_dt, vz)), d.L);
  } else if (d.md_theta & 1) {  // odd theta: one more flip of the buffers
    XW[i] = xi;
    YW[i] = yi;
    ZW[i] = zi;
  }
  a.vx[i] = vx;
  a.vy[i] = vy;
  a.vz[i] = vz;
}

// Initial velocities: per component the Irwin-Hall(4) offset of the bytes of
// word d of the Philox block (0, id, 0, 6) times cv = fl32(sqrt(T / 21845)).
__global__ __launch_bounds__(kThreads) void k_md_init(Dev d, unsigned long long vseed, float cv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const Arr a = pick_set(d, d.ctl->set & 1u);
  int32_t S[3];
  ih4(0u, a.id ? (uint32_t)a.id[i] : (uint32_t)i, 6u, vseed, S);
  a.vx[i] = __fmul_rn((float)S[0], cv);
  a.vy[i] = __fmul_rn((float)S[1], cv);
  a.vz[i] = __fmul_rn((float)S[2], cv);
}

// The id -> slot map of the current storage set.
__global__ __launch_bounds__(kThreads) void k_slot_of(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const Arr a = pick_set(d, d.ctl->set & 1u);
  d.slot_of[a.id ? a.id[i] : i] = i;
}

// Velocities in particle-id order.
__global__ __launch_bounds__(kThreads) void k_gather_v(Dev d, float* ox, float* oy, float* oz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const Arr a = pick_set(d, d.ctl->set & 1u);
  const int id = a.id ? a.id[i] : i;
  ox[id] = a.vx[i];
  oy[id] = a.vy[i];
  oz[id] = a.vz[i];
}

// ---------------------------------------------------------------------------
// Kinetics counters of the current configuration (the quantities of the
// paper's rate equations, Sec. II B-C): populations of the A type by state,
// and, per state of the A-eligible particles, their T-eligible partners
// within the cutoff (not bonded to them when the rule excludes bonded pairs)
// with a histogram of those pairs by distance.  The A records come from the
// binning kernel run on the current positions (no re-jitter); each pair is
// found once, from its T, as in the sweep.  Counts go to LDS, then one
// global atomic per workgroup and counter.
// ---------------------------------------------------------------------------
// The distance bin of an in-range pair: the b with e2[b] <= r2 < e2[b + 1]
// (the last bin ends at the cutoff), found from a guess by the uniform bin
// width in r and moved by the exact edges, so that no pair walks every bin.
__device__ __forceinline__ int kin_bin(float r2, const float* e2, int nbins, float scale) {
  int b = (int)(__fsqrt_rn(r2) * scale);
  b = b < 0 ? 0 : (b > nbins - 1 ? nbins - 1 : b);
  while (b > 0 && r2 < e2[b]) --b;
  while (b + 1 < nbins && !(r2 < e2[b + 1])) ++b;
  return b;
}

__global__ __launch_bounds__(kThreads) void k_kin_pop(Dev d, int nstate,
                                                      unsigned long long* __restrict__ pop) {
  __shared__ uint32_t s_pop[kKinMaxState];
  for (int q = threadIdx.x; q < nstate; q += blockDim.x) s_pop[q] = 0u;
  __syncthreads();
  const Arr a = pick_set(d, d.ctl->set & 1u);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += gridDim.x * blockDim.x) {
    const int32_t st = a.st[i];
    if (a.typ[i] == d.rule.type_a && st >= 0 && st < nstate) atomicAdd(&s_pop[st], 1u);
  }
  __syncthreads();
  const size_t so = (size_t)(blockIdx.x % kKinSlices) * kKinStride;
  for (int q = threadIdx.x; q < nstate; q += blockDim.x)
    if (s_pop[q]) atomicAdd(&pop[so + q], (unsigned long long)s_pop[q]);
}

__global__ __launch_bounds__(kThreads) void k_kin_pairs(Dev d, int nstate, int nbins,
                                                        const float* __restrict__ e2,
                                                        unsigned long long* __restrict__ pairs,
                                                        unsigned long long* __restrict__ hist) {
  __shared__ uint32_t s_pairs[kKinMaxState], s_hist[kKinMaxBins];
  __shared__ float s_e2[kKinMaxBins + 1];
  for (int q = threadIdx.x; q < nstate; q += blockDim.x) s_pairs[q] = 0u;
  for (int q = threadIdx.x; q < nbins; q += blockDim.x) s_hist[q] = 0u;
  for (int q = threadIdx.x; q <= nbins; q += blockDim.x) s_e2[q] = e2[q];
  __syncthreads();
  const float scale = nbins > 0 ? (float)nbins / __fsqrt_rn(d.rc2) : 0.0f;
  const Ctl* c = d.ctl;
  const uint32_t par = c->par0;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  const Buckets bk{pick(d.cnt, par), d.rec, d.rsa, pick(d.ovf, par), pick(d.ovf_sa, par),
                   c->ovf_n[par]};
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < d.n;
       slot += gridDim.x * blockDim.x) {
    if (a.role[slot] != kRoleT) continue;
    const float x = X[slot], y = Y[slot], z = Z[slot];
    const int32_t id = a.id ? a.id[slot] : slot;
    for_global_records(d, bk, x, y, z, [&](float4 A, int sa) {
      const float r2 = dist2(d, x, y, z, A);
      if (!(r2 < d.rc2)) return;
      if (d.rule.exclude && row_has(a.adj + (size_t)sa * d.B, d.B, id)) return;
      const int32_t st = a.st[sa];
      if (st >= 0 && st < nstate) atomicAdd(&s_pairs[st], 1u);
      if (nbins > 0) atomicAdd(&s_hist[kin_bin(r2, s_e2, nbins, scale)], 1u);
    });
  }
  __syncthreads();
  // the workgroup's sums go to its slice (kKinSlices of them, summed on the
  // host): few workgroups share an address
  const size_t so = (size_t)(blockIdx.x % kKinSlices) * kKinStride;
  for (int q = threadIdx.x; q < nstate; q += blockDim.x)
    if (s_pairs[q]) atomicAdd(&pairs[so + q], (unsigned long long)s_pairs[q]);
  for (int q = threadIdx.x; q < nbins; q += blockDim.x)
    if (s_hist[q]) atomicAdd(&hist[so + q], (unsigned long long)s_hist[q]);
}

// k_kin_pairs on sorted storage (brick edges up to kOneCellBrick), one
// workgroup per brick with its region's A records staged (StagedRegion): the
// same pairs, the same counts.
__global__ __launch_bounds__(kThreads) void k_kin_pairs_staged(Dev d, int nstate, int nbins,
                                                               const float* __restrict__ e2,
                                                               unsigned long long* __restrict__ pairs,
                                                               unsigned long long* __restrict__ hist) {
  __shared__ float4 s_rec[kStageRecs];
  __shared__ int4 s_radj[kStageRecs];
  __shared__ int32_t s_rsa[kStageRecs];
  __shared__ uint16_t s_off[kStageCells1 + 1];
  __shared__ uint32_t s_wave[kThreads / 64 + 1];
  __shared__ int32_t s_ast[kStageRecs];
  __shared__ uint32_t s_pairs[kKinMaxState], s_hist[kKinMaxBins];
  __shared__ float s_e2[kKinMaxBins + 1];
  for (int q = threadIdx.x; q < nstate; q += blockDim.x) s_pairs[q] = 0u;
  for (int q = threadIdx.x; q < nbins; q += blockDim.x) s_hist[q] = 0u;
  for (int q = threadIdx.x; q <= nbins; q += blockDim.x) s_e2[q] = e2[q];
  const float scale = nbins > 0 ? (float)nbins / __fsqrt_rn(d.rc2) : 0.0f;
  const Ctl* c = d.ctl;
  const uint32_t par = c->par0;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  const Buckets bk{pick(d.cnt, par), d.rec, d.rsa, pick(d.ovf, par), pick(d.ovf_sa, par),
                   c->ovf_n[par]};
  const int w = xcd_brick(blockIdx.x, gridDim.x);
  int s0, s1;
  range_of<true>(d, w, s0, s1);
  StagedRegion g;
  g.rec = s_rec;
  g.radj = s_radj;
  g.rsa = s_rsa;
  g.off = s_off;
  stage_region(d, bk, w, g, s_wave);  // ends with a barrier (the tables above too)
  // the staged A's states, so that no pair waits for a global load
  if (g.staged) {
    const int nrec = (int)s_off[g.ex * g.ey * g.ez];
    for (int r = threadIdx.x; r < nrec; r += kThreads) s_ast[r] = a.st[s_rsa[r]];
    __syncthreads();
  }
  for (int slot = s0 + threadIdx.x; slot < s1; slot += kThreads) {
    if (a.role[slot] != kRoleT) continue;
    const float x = X[slot], y = Y[slot], z = Z[slot];
    visit_pairs(d, a, bk, g, x, y, z, (uint32_t)a.id[slot],
                [&](float4, float r2, bool excluded, int sa, int r) {
                  if (excluded) return;
                  const int32_t st = r >= 0 ? s_ast[r] : a.st[sa];
                  if (st >= 0 && st < nstate) atomicAdd(&s_pairs[st], 1u);
                  if (nbins > 0) atomicAdd(&s_hist[kin_bin(r2, s_e2, nbins, scale)], 1u);
                });
  }
  __syncthreads();
  // the workgroup's sums go to its slice (kKinSlices of them, summed on the
  // host): few workgroups share an address
  const size_t so = (size_t)(blockIdx.x % kKinSlices) * kKinStride;
  for (int q = threadIdx.x; q < nstate; q += blockDim.x)
    if (s_pairs[q]) atomicAdd(&pairs[so + q], (unsigned long long)s_pairs[q]);
  for (int q = threadIdx.x; q < nbins; q += blockDim.x)
    if (s_hist[q]) atomicAdd(&hist[so + q], (unsigned long long)s_hist[q]);
}

// Sums the kKinSlices slices of the kinetics counters into the first.
__global__ void k_kin_sum(unsigned long long* kin) {
  for (int q = threadIdx.x; q < kKinStride; q += blockDim.x) {
    unsigned long long v = 0;
    for (int j = 1; j < kKinSlices; ++j) v += kin[(size_t)j * kKinStride + q];
    kin[q] += v;
  }
}

// Leaves the A grid of the current parity as a step expects to find it
// (no records, no overflow).
__global__ __launch_bounds__(kThreads) void k_kin_reset(Dev d) {
  const uint32_t par = d.ctl->par0;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < d.ncell; q += gridDim.x * blockDim.x)
    pick(d.cnt, par)[q] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.ctl->ovf_n[par] = 0u;
}

// ---------------------------------------------------------------------------
// Stateless single step: close it and sort its bonds by id_A into the
// caller's buffer (one workgroup).
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

// After k_close and k_advance of the single step: its bonds (the whole log)
// sorted by id_A into the caller's buffer.
__global__ __launch_bounds__(kFinThreads) void k_single_sort(Dev d) {
  __shared__ unsigned long long s_b[kSortLds];
  const Ctl* c = d.ctl;
  if (read_err(c)) return;
  const int64_t nb = (int64_t)c->log_n;
  const int64_t m = nb < d.log_cap ? nb : d.log_cap;
  int n2 = 1;
  while (n2 < m) n2 <<= 1;
  unsigned long long* buf = n2 <= kSortLds ? s_b : d.sortbuf;
  for (int t = threadIdx.x; t < n2; t += blockDim.x)
    buf[t] = t < m ? (((unsigned long long)(uint32_t)d.log[3 * t + 1] << 32) |
                      (uint32_t)d.log[3 * t + 2])
                   : kEmpty;
  __threadfence_block();
  __syncthreads();
  if (m > 1) bitonic_sort(buf, n2);
  for (int t = threadIdx.x; t < m && t < d.bonds_cap; t += blockDim.x) {
    if (d.bonds_rule) {  // (id_A, id_T, rule): the rule rides in bits 30-31 of id_T
      const uint32_t tt = (uint32_t)buf[t];
      d.bonds[3 * t] = (int32_t)(buf[t] >> 32);
      d.bonds[3 * t + 1] = (int32_t)(d.nrules > 1 ? tt & 0x3FFFFFFFu : tt);
      d.bonds[3 * t + 2] = (int32_t)(d.nrules > 1 ? tt >> 30 : 0u);
    } else {
      d.bonds[2 * t] = (int32_t)(buf[t] >> 32);
      d.bonds[2 * t + 1] = (int32_t)(uint32_t)buf[t];
    }
  }
}

// ---------------------------------------------------------------------------
// Spatial sort of the storage by brick, within a brick its A's first and the
// rest by dual cell (counting sort: count, per-brick scan, scan over bricks,
// scatter).  Results never depend on the storage order; the sort only gives
// each sweep workgroup a compact region and its wavefronts similar blocks.
// ---------------------------------------------------------------------------
// The sort bin of a particle: its brick b and, within it, bin 0 for an A
// (the brick's few A's then share a handful of cache lines, which the binning
// of every step reads), else 1 + its dual cell floor(u - 1/2) (u = position /
// cell width; bs + 1 values per dimension from the brick's first cell - 1).
// All T's of one dual cell have the same 2x2x2 partner block, so a wavefront
// of them scans runs of equal length.
__device__ __forceinline__ int sort_bin(const Dev& d, float x, float y, float z, uint8_t role,
                                        int& b) {
  const float ux = __fmul_rn(x, d.inv_w), uy = __fmul_rn(y, d.inv_w), uz = __fmul_rn(z, d.inv_w);
  const int nc = d.nc, bs = d.bs, e = bs + 1;
  int bx = 0, by = 0, bz = 0;
  if (d.nbricks > 1) {
    bx = cell1(ux, nc) / bs;
    by = cell1(uy, nc) / bs;
    bz = cell1(uz, nc) / bs;
  }
  b = (bz * d.nb + by) * d.nb + bx;
  const int lx = min(max((int)floorf(__fsub_rn(ux, 0.5f)) - (bx * bs - 1), 0), bs);
  const int ly = min(max((int)floorf(__fsub_rn(uy, 0.5f)) - (by * bs - 1), 0), bs);
  const int lz = min(max((int)floorf(__fsub_rn(uz, 0.5f)) - (bz * bs - 1), 0), bs);
  return b * d.nd + (role_is_a(role, d.nrules > 1) ? 0 : 1 + (lz * e + ly) * e + lx);
}

// Ranks within sort bins.  The storage is in bin order from the previous
// sort, so the 64 particles of a wavefront fall into few bins: the lowest lane
// of each bin reserves the ranks of all its lanes with one returning atomic.
__device__ __forceinline__ void sort_count_body(const Dev& d, int k) {
  const bool valid = k < d.n;
  const Arr a = pick_set(d, d.ctl->set & 1u);
  const uint32_t par = d.ctl->par0;
  int b, bin = -1;
  if (valid)
    bin = sort_bin(d, pick(a.x, par)[k], pick(a.y, par)[k], pick(a.z, par)[k], a.role[k], b);
  // group the lanes by bin: each round takes the lowest ungrouped lane's bin
  int leader = 0;
  unsigned long long peers = 0ull;
  unsigned long long todo = __ballot(valid);
  while (todo) {
    const int ld = (int)__builtin_ctzll(todo);
    const int lb = __builtin_amdgcn_readlane(bin, ld);
    const bool mine = valid && bin == lb;
    const unsigned long long m = __ballot(mine);
    if (mine) {
      leader = ld;
      peers = m;
    }
    todo &= ~m;
  }
  uint32_t r = 0u;
  if (valid && __lane_id() == (unsigned)leader)
    r = atomicAdd(&d.dcnt[bin], (uint32_t)__popcll(peers));
  r = (uint32_t)__shfl((int)r, leader);
  if (valid) d.rank[k] = (int32_t)(r + lanes_below(peers));
}

// Offsets of the bins within brick b (one wavefront, up to six consecutive
// bins per lane: nd = (bs + 1)^3 + 1 <= 344), the brick's total for the scan
// over bricks; the counts are cleared for the next sort.
__device__ __forceinline__ void sort_local_body(const Dev& d, int b) {
  if (b >= d.nbricks) return;
  constexpr int kPerLane = 6;
  const int lane = __lane_id(), nd = d.nd, per = (nd + 63) / 64;
  uint32_t* c = d.dcnt + (size_t)b * nd;
  uint32_t* o = d.dloc + (size_t)b * nd;
  const int j0 = lane * per;
  uint32_t v[kPerLane], sum = 0u;
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {
    v[q] = q < per && j0 + q < nd ? c[j0 + q] : 0u;
    sum += v[q];
  }
  const uint32_t x = wave_scan_incl(sum);
  uint32_t run = x - sum;
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {
    if (q < per && j0 + q < nd) {
      o[j0 + q] = run;
      c[j0 + q] = 0u;
    }
    run += v[q];
  }
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
  if (lane == 0) d.bcnt[b] = total;
}

__device__ __forceinline__ void sort_scan_body(const Dev& d) {
  __shared__ uint32_t s_wave[kFinThreads / 64 + 1];
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
    if (d.fuse) {  // overflow of the first two steps after the sort
      const uint32_t s0 = d.ctl->step0;
      d.ctl->fovf_n[mod3(s0)] = 0u;
      d.ctl->fovf_n[mod3(s0 + 1u)] = 0u;
    }
  }
}

__device__ __forceinline__ void sort_scatter_body(const Dev& d, int k) {
  if (k >= d.n) return;
  const uint32_t s = d.ctl->set & 1u, par = d.ctl->par0;
  const Arr a = pick_set(d, s), o = pick_set(d, s ^ 1u);
  const float x = pick(a.x, par)[k], y = pick(a.y, par)[k], z = pick(a.z, par)[k];
  const uint8_t role = a.role[k];
  int b;
  const int bin = sort_bin(d, x, y, z, role, b);
  const int ns = d.bstart[b] + (int)d.dloc[bin] + d.rank[k];
  pick(o.x, par)[ns] = x;
  pick(o.y, par)[ns] = y;
  pick(o.z, par)[ns] = z;
  o.typ[ns] = a.typ[k];
  o.st[ns] = a.st[k];
  o.role[ns] = role;
  const int id = a.id[k];
  o.id[ns] = id;
  if (a.vx) {
    o.vx[ns] = a.vx[k];
    o.vy[ns] = a.vy[k];
    o.vz[ns] = a.vz[k];
  }
  if (d.slot_of) d.slot_of[id] = ns;
  if (d.fuse && role == kRoleA) {  // the A's record of the block's first step
    float rx = x, ry = y, rz = z;
    if (d.jitter && d.jit_c != 0.0f) rejitter(d, d.ctl->step0, (uint32_t)id, rx, ry, rz);
    fuse_bin(d, par, d.ctl->step0, ns, (uint32_t)id, rx, ry, rz);
  }
  // rows of width 4 or 2 move as one vector when both arrays are aligned
  const bool vec = (((uintptr_t)a.adj | (uintptr_t)o.adj) & 15u) == 0u;
  if (vec && d.B == 4) {
    ((int4*)o.adj)[ns] = ((const int4*)a.adj)[k];
  } else if (vec && d.B == 2) {
    ((int2*)o.adj)[ns] = ((const int2*)a.adj)[k];
  } else {
    for (int q = 0; q < d.B; ++q) o.adj[(size_t)ns * d.B + q] = a.adj[(size_t)k * d.B + q];
  }
}

// ---------------------------------------------------------------------------
// Entry points.  One system: the kernel argument is its Dev and the grid is
// its own.  A batch of systems (independent replicas stepping in lockstep):
// the Devs live in device memory and map[blockIdx.x] = (replica, local block,
// blocks of that replica) spreads one grid over all of them.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_prep(Dev d, int k) { prep_body(d, k, blockIdx.x); }
__global__ __launch_bounds__(kThreads) void k_close(Dev d, int k) { close_body(d, k, blockIdx.x); }
__global__ void k_advance(Ctl* c, int K) {
  if (threadIdx.x == 0 && blockIdx.x == 0) advance_ctl(c, K);
}

// With fused binning there is no prep kernel: the closing groups of step
// k - 1 trail the sweep of step k (workgroups nwg_sweep and up when k > 0).
// Nothing the sweep reads or writes is theirs (the counters, staged bonds and
// overflow words of step k - 1's parity, the log), and they are dispatched
// with the sweep's workgroups, so their chain of round trips (with the
// returning atomic that reserves log rows) runs beside the sweep instead of
// lengthening the resolve.
template <bool kBrick, bool kTwo, bool kF, bool kNt = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_sweep(Dev d, int k) {
  if (kF && (int)blockIdx.x >= d.nwg_sweep) {
    __shared__ uint32_t s_wave[kThreads / 64 + 1];
    const StepInfo si = step_info(d.ctl, k);
    close_group(d, si.par ^ 1u, si.step - 1u, d.ctl->stats_n0 + (uint32_t)k - 1u,
                (int)blockIdx.x - d.nwg_sweep, s_wave);
    return;
  }
  const int w = kBrick ? xcd_brick(blockIdx.x, d.nwg_sweep) : (int)blockIdx.x;
  sweep_body<kBrick, kTwo, kF, kNt>(d, k, w, d.nwg_sweep);
}
template <bool kBrick>
__global__ __launch_bounds__(kThreads) void k_resolve(Dev d, int k) {
  resolve_body<kBrick, true, true>(d, k, blockIdx.x, d.nwg_sweep);
}
template <bool kBrick>
__global__ __launch_bounds__(kThreads) void k_near_sweep(Dev d, int k) {
  if (kBrick && d.bs <= kOneCellBrick)
    near_sweep_staged_body(d, k, xcd_brick(blockIdx.x, gridDim.x), gridDim.x);
  else
    near_sweep_body<kBrick>(d, k, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kThreads) void k_near_resolve(Dev d, int k) {
  near_resolve_body(d, k, blockIdx.x, gridDim.x);
}
template <bool kBrick>
__global__ __launch_bounds__(kThreads) void k_multi_sweep(Dev d, int k) {
  if (kBrick && d.bs <= kOneCellBrick)
    multi_sweep_staged_body(d, k, xcd_brick(blockIdx.x, gridDim.x), gridDim.x);
  else
    multi_sweep_body<kBrick>(d, k, blockIdx.x, gridDim.x);
}
template <bool kBrick>
__global__ __launch_bounds__(kThreads) void k_multi_resolve(Dev d, int k) {
  multi_resolve_body<kBrick>(d, k, blockIdx.x);
}
template <bool kBrick>
__global__ __launch_bounds__(kThreads) void k_multi_final(Dev d, int k) {
  multi_final_body<kBrick>(d, k, blockIdx.x);
}
__global__ __launch_bounds__(kThreads) void k_sort_count(Dev d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  sort_count_body(d, k);
  if (d.fuse) {  // fused binning: the scatter bins the first step after the sort
    const uint32_t s0 = d.ctl->step0;
    for (int q = k; q < d.ncell; q += gridDim.x * blockDim.x) {
      d.fcnt[mod3(s0)][q] = 0u;
      d.fcnt[mod3(s0 + 1u)][q] = 0u;
    }
  }
}
__global__ __launch_bounds__(kThreads) void k_sort_local(Dev d) {
  sort_local_body(d, blockIdx.x * (kThreads / 64) + (int)(threadIdx.x / 64));
}
__global__ __launch_bounds__(kFinThreads) void k_sort_scan(Dev d) { sort_scan_body(d); }
__global__ __launch_bounds__(kThreads) void k_sort_scatter(Dev d) {
  sort_scatter_body(d, blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void k_sort_flip(Ctl* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c->set ^= 1u;
}

// The block's map entry, made wavefront-uniform (scalar registers) so that
// the replica's Dev is read with scalar loads.
__device__ __forceinline__ int4 uniform_map(const int4* __restrict__ map) {
  const int4 m = map[blockIdx.x];
  return make_int4(__builtin_amdgcn_readfirstlane(m.x), __builtin_amdgcn_readfirstlane(m.y),
                   __builtin_amdgcn_readfirstlane(m.z), 0);
}

// A replica takes part in steps k < k_limit of a block; its workgroups of
// later steps return at once (uniformly: the whole block belongs to it).
__global__ __launch_bounds__(kThreads) void k_prep_b(const Dev* __restrict__ ds,
                                                     const int4* __restrict__ map, int k) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (k >= d.k_limit) return;
  prep_body(d, k, m.y);
}
template <bool kTwo, bool kF>
// With fused binning, workgroups nsw and up close step k - 1 of each replica
// (closing map cmap), as the trailing workgroups of k_sweep do.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_sweep_b(
    const Dev* __restrict__ ds, const int4* __restrict__ map, int nsw,
    const int4* __restrict__ cmap, int k) {
  if (kF && (int)blockIdx.x >= nsw) {
    const int4 c = cmap[__builtin_amdgcn_readfirstlane((int)blockIdx.x - nsw)];
    const Dev& d = ds[__builtin_amdgcn_readfirstlane(c.x)];
    if (k >= d.k_limit) return;  // the block end closes the replica's last step
    __shared__ uint32_t s_wave[kThreads / 64 + 1];
    const StepInfo si = step_info(d.ctl, k);
    close_group(d, si.par ^ 1u, si.step - 1u, d.ctl->stats_n0 + (uint32_t)k - 1u,
                __builtin_amdgcn_readfirstlane(c.y), s_wave);
    return;
  }
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (k >= d.k_limit || d.rule.policy != PR_POLICY_RANDOM) return;
  sweep_body<true, kTwo, kF>(d, k, m.y, m.z);
}
__global__ __launch_bounds__(kThreads) void k_near_sweep_b(const Dev* __restrict__ ds,
                                                           const int4* __restrict__ map, int k) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (k >= d.k_limit || d.rule.policy != PR_POLICY_NEAREST) return;
  if (d.bs <= kOneCellBrick)
    near_sweep_staged_body(d, k, m.y, m.z);
  else
    near_sweep_body<true>(d, k, m.y, m.z);
}
__global__ __launch_bounds__(kThreads) void k_near_resolve_b(const Dev* __restrict__ ds,
                                                             const int4* __restrict__ map, int k) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (k >= d.k_limit || d.rule.policy != PR_POLICY_NEAREST) return;
  near_resolve_body(d, k, m.y, m.z);
}
__global__ __launch_bounds__(kThreads) void k_resolve_b(const Dev* __restrict__ ds,
                                                        const int4* __restrict__ map, int k) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (k >= d.k_limit || d.rule.policy != PR_POLICY_RANDOM) return;
  resolve_body<true, true>(d, k, m.y, m.z);
}
__global__ __launch_bounds__(kThreads) void k_close_b(const Dev* __restrict__ ds,
                                                      const int4* __restrict__ map, int k) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  if (d.k_limit < 1) return;
  close_body(d, k < d.k_limit - 1 ? k : d.k_limit - 1, m.y);  // the replica's last step
}
// one thread per replica
__global__ void k_ctl_b(const Dev* __restrict__ ds, int nrep, int op, uint32_t arg) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrep) return;
  const Dev& d = ds[r];
  Ctl* c = d.ctl;
  if (op == 0) {
    c->step0 = d.first_step;                 // start of a block
  } else if (op == 1) {                      // end of a block of arg steps
    const int kk = d.k_limit < (int)arg ? d.k_limit : (int)arg;
    if (kk > 0) advance_ctl(c, kk);
  } else {
    c->set ^= 1u;                            // after a sort
  }
}
__global__ __launch_bounds__(kThreads) void k_sort_count_b(const Dev* __restrict__ ds,
                                                           const int4* __restrict__ map) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  sort_count_body(d, m.y * kThreads + threadIdx.x);
  if (d.fuse) {  // fused binning: the scatter bins the block's first step
    const uint32_t s0 = d.ctl->step0;
    for (int q = m.y * kThreads + threadIdx.x; q < d.ncell; q += m.z * kThreads) {
      d.fcnt[mod3(s0)][q] = 0u;
      d.fcnt[mod3(s0 + 1u)][q] = 0u;
    }
  }
}
// ngrp blocks per replica (the brick groups of the largest one)
__global__ __launch_bounds__(kThreads) void k_sort_local_b(const Dev* __restrict__ ds, int ngrp) {
  const int r = __builtin_amdgcn_readfirstlane((int)(blockIdx.x / (unsigned)ngrp));
  const int g = (int)blockIdx.x - r * ngrp;
  sort_local_body(ds[r], g * (kThreads / 64) + (int)(threadIdx.x / 64));
}
__global__ __launch_bounds__(kFinThreads) void k_sort_scan_b(const Dev* __restrict__ ds) {
  const Dev& d = ds[__builtin_amdgcn_readfirstlane((int)blockIdx.x)];
  sort_scan_body(d);
}
__global__ __launch_bounds__(kThreads) void k_sort_scatter_b(const Dev* __restrict__ ds,
                                                             const int4* __restrict__ map) {
  const int4 m = uniform_map(map);
  const Dev& d = ds[m.x];
  sort_scatter_body(d, m.y * kThreads + threadIdx.x);
}

// Storage order -> particle-id order (positions of the current parity).
__global__ __launch_bounds__(kThreads) void k_gather_out(Dev d, float* ox, float* oy, float* oz,
                                                         int32_t* otyp, int32_t* ost,
                                                         int32_t* oadj) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const Arr a = pick_set(d, d.ctl->set & 1u);
  const uint32_t par = d.ctl->par0;
  const int id = a.id[k];
  if (ox) ox[id] = pick(a.x, par)[k];
  if (oy) oy[id] = pick(a.y, par)[k];
  if (oz) oz[id] = pick(a.z, par)[k];
  if (otyp) otyp[id] = a.typ[k];
  if (ost) ost[id] = a.st[k];
  if (oadj)
    for (int b = 0; b < d.B; ++b) oadj[(size_t)id * d.B + b] = a.adj[(size_t)k * d.B + b];
}

// The re-jitter alone (the stand-in for the MD between reaction steps),
// step k of a block: every particle's position of parity par moves by the
// step's offsets into parity par ^ 1, exactly as the sweep of a reaction
// step moves it, and the cell counts of the next parity are cleared as the
// sweep clears them.  No reaction happens.
template <bool kNt>
__global__ __launch_bounds__(kThreads) void k_jitter_only(Dev d, int k) {
  const Ctl* c = d.ctl;
  const uint32_t par = (c->par0 + (uint32_t)k) & 1u, step = c->step0 + (uint32_t)k;
  const Arr a = pick_set(d, c->set & 1u);
  const float *X = pick(a.x, par), *Y = pick(a.y, par), *Z = pick(a.z, par);
  float *XW = pick(a.x, par ^ 1u), *YW = pick(a.y, par ^ 1u), *ZW = pick(a.z, par ^ 1u);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n) {
    float x = X[i], y = Y[i], z = Z[i];
    if (d.jit_c != 0.0f) rejitter(d, step, a.id ? (uint32_t)a.id[i] : (uint32_t)i, x, y, z);
    if (kNt) {  // the sweep's store policy
      __builtin_nontemporal_store(x, &XW[i]);
      __builtin_nontemporal_store(y, &YW[i]);
      __builtin_nontemporal_store(z, &ZW[i]);
    } else {
      XW[i] = x;
      YW[i] = y;
      ZW[i] = z;
    }
  }
  for (int q = i; q < d.ncell; q += gridDim.x * blockDim.x) pick(d.cnt, par ^ 1u)[q] = 0u;
}

// Moves the block origin by K steps of the re-jitter alone: the draw step
// and the position parity advance, the counter log does not (nothing was
// logged).
__global__ void k_advance_jitter(Ctl* c, int K) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->step0 += (uint32_t)K;
    c->par0 = (c->par0 + (uint32_t)K) & 1u;
  }
}

// Plain device copy of n elements of T (one element per lane and
// iteration, grid-stride): the project's own bandwidth probe, with a known
// request shape per wavefront (64 lanes x sizeof(T) contiguous bytes).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_stream_copy(const T* __restrict__ src,
                                                          T* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Fills n 32-bit words with v (clears scratch inside code a caller may
// capture into a graph, where memset nodes are avoided).
__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t* __restrict__ p, long long n,
                                                       uint32_t v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// The bonded-force kernel's square root on caller data (n values > 0, normal).
__global__ __launch_bounds__(kThreads) void k_sqrt_rn(const float* __restrict__ in,
                                                      float* __restrict__ out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt_rn(in[i]);
}

// The generator's words for caller counters (4 uint32 per counter).
__global__ __launch_bounds__(kThreads) void k_draws(const uint4* __restrict__ ctr, long long n,
                                                    unsigned long long key, uint4* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = ctr[i];
  const W4 w = philox(c.x, c.y, c.z, c.w, key);
  out[i] = make_uint4(w.w0, w.w1, w.w2, w.w3);
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
  if (d.n > 0) k_classify<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_identity(const Dev& d, hipStream_t s) {
  if (d.n > 0) k_identity<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_generate(const Dev& d, int kind, unsigned long long gseed, float c0, float a,
                           int nl, unsigned long long thr, hipStream_t s) {
  if (d.n > 0)
    k_generate<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d, kind, gseed, c0, a, nl, thr);
  return hipGetLastError();
}

// Step k of a block: prep (with the closing of step k - 1), sweep, resolve.
// ev_sweep0/1 (timed runs): the sweep is launched with hipExtLaunchKernel,
// which stamps the two events at the kernel's own start and end.
hipError_t launch_step(const Dev& d, int k, hipStream_t s, hipEvent_t ev_sweep0,
                       hipEvent_t ev_sweep1) {
  for (int m = 0; d.md_theta > 0 && m <= d.md_theta; ++m)
    k_md<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d, k, m);
  if (d.fuse) {  // two kernels: the sweep (with the closing of step k - 1), the resolve
    // the sweep, with the closing of step k - 1 in trailing workgroups (edges
    // above kOneCellBrick stage two region cells per thread)
    const dim3 g(d.nwg_sweep + (k > 0 ? d.ngroups : 0)), b(kThreads);
    auto kern = d.bs > kOneCellBrick ? (d.nt_pos ? k_sweep<true, true, true, true>
                                                 : k_sweep<true, true, true, false>)
                                     : (d.nt_pos ? k_sweep<true, false, true, true>
                                                 : k_sweep<true, false, true, false>);
    if (ev_sweep0) hipExtLaunchKernelGGL(kern, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
    else kern<<<g, b, 0, s>>>(d, k);
    k_resolve<true><<<(d.nwg_sweep + 3) / 4, kThreads, 0, s>>>(d, k);
    return hipGetLastError();
  }
  const int prep_blocks = d.nwg_prep + (k > 0 ? d.ngroups : 0);
  k_prep<<<prep_blocks, kThreads, 0, s>>>(d, k);
  const dim3 g(d.nwg_sweep), b(kThreads);
  if (d.nrules > 1) {
    if (d.sorted) {
      if (ev_sweep0)
        hipExtLaunchKernelGGL(k_multi_sweep<true>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
      else
        k_multi_sweep<true><<<g, b, 0, s>>>(d, k);
      k_multi_resolve<true><<<g, b, 0, s>>>(d, k);
      k_multi_final<true><<<g, b, 0, s>>>(d, k);
    } else {
      if (ev_sweep0)
        hipExtLaunchKernelGGL(k_multi_sweep<false>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
      else
        k_multi_sweep<false><<<g, b, 0, s>>>(d, k);
      k_multi_resolve<false><<<g, b, 0, s>>>(d, k);
      k_multi_final<false><<<g, b, 0, s>>>(d, k);
    }
    return hipGetLastError();
  }
  if (d.rule.policy == PR_POLICY_NEAREST) {
    if (d.sorted) {
      if (ev_sweep0)
        hipExtLaunchKernelGGL(k_near_sweep<true>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
      else
        k_near_sweep<true><<<g, b, 0, s>>>(d, k);
    } else {
      if (ev_sweep0)
        hipExtLaunchKernelGGL(k_near_sweep<false>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
      else
        k_near_sweep<false><<<g, b, 0, s>>>(d, k);
    }
    k_near_resolve<<<g, b, 0, s>>>(d, k);
    return hipGetLastError();
  }
  if (d.sorted && d.bs > kOneCellBrick) {
    if (ev_sweep0)
      hipExtLaunchKernelGGL(k_sweep<true, true, false>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
    else
      k_sweep<true, true, false><<<g, b, 0, s>>>(d, k);
  } else if (d.sorted) {
    if (ev_sweep0)
      hipExtLaunchKernelGGL(k_sweep<true, false, false>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
    else
      k_sweep<true, false, false><<<g, b, 0, s>>>(d, k);
  } else {
    if (ev_sweep0)
      hipExtLaunchKernelGGL(k_sweep<false, false, false>, g, b, 0, s, ev_sweep0, ev_sweep1, 0, d, k);
    else
      k_sweep<false, false, false><<<g, b, 0, s>>>(d, k);
  }
  if (d.sorted)
    k_resolve<true><<<(d.nwg_sweep + 3) / 4, kThreads, 0, s>>>(d, k);
  else
    k_resolve<false><<<(d.nwg_sweep + 3) / 4, kThreads, 0, s>>>(d, k);
  return hipGetLastError();
}

hipError_t launch_block_end(const Dev& d, int K, hipStream_t s) {
  k_close<<<d.ngroups, kThreads, 0, s>>>(d, K - 1);
  k_advance<<<1, 64, 0, s>>>(d.ctl, K);
  return hipGetLastError();
}

hipError_t launch_single_end(const Dev& d, hipStream_t s) {
  k_close<<<d.ngroups, kThreads, 0, s>>>(d, 0);
  k_advance<<<1, 64, 0, s>>>(d.ctl, 1);
  k_single_sort<<<1, kFinThreads, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_sort(const Dev& d, hipStream_t s) {
  k_sort_count<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d);
  k_sort_local<<<blocks_for(d.nbricks, kThreads / 64), kThreads, 0, s>>>(d);
  k_sort_scan<<<1, kFinThreads, 0, s>>>(d);
  k_sort_scatter<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d);
  k_sort_flip<<<1, 64, 0, s>>>(d.ctl);
  return hipGetLastError();
}

// Batched launches (every replica in one grid per kernel).
static inline int ctl_blocks(int nrep) { return (nrep + 63) / 64; }

hipError_t launch_ctl_b(const BatchLaunch& b, int op, uint32_t arg, hipStream_t s) {
  k_ctl_b<<<ctl_blocks(b.nrep), 64, 0, s>>>(b.ds, b.nrep, op, arg);
  return hipGetLastError();
}

hipError_t launch_step_b(const BatchLaunch& b, int k, hipStream_t s) {
  if (b.fuse) {  // every replica random and fused: sweep with the closing, then resolve
    const int ncl = k > 0 ? b.n_close : 0;
    if (b.two)
      k_sweep_b<true, true><<<b.n_sweep + ncl, kThreads, 0, s>>>(b.ds, b.sweep, b.n_sweep,
                                                                  b.close, k);
    else
      k_sweep_b<false, true><<<b.n_sweep + ncl, kThreads, 0, s>>>(b.ds, b.sweep, b.n_sweep,
                                                                   b.close, k);
    k_resolve_b<<<b.n_res, kThreads, 0, s>>>(b.ds, b.res, k);
    return hipGetLastError();
  }
  if (k > 0)
    k_prep_b<<<b.n_prepk, kThreads, 0, s>>>(b.ds, b.prepk, k);
  else
    k_prep_b<<<b.n_prep0, kThreads, 0, s>>>(b.ds, b.prep0, k);
  if (b.any_random) {
    if (b.two)
      k_sweep_b<true, false><<<b.n_sweep, kThreads, 0, s>>>(b.ds, b.sweep, b.n_sweep, b.close, k);
    else
      k_sweep_b<false, false><<<b.n_sweep, kThreads, 0, s>>>(b.ds, b.sweep, b.n_sweep, b.close,
                                                             k);
    k_resolve_b<<<b.n_res, kThreads, 0, s>>>(b.ds, b.res, k);
  }
  if (b.any_nearest) {
    k_near_sweep_b<<<b.n_sweep, kThreads, 0, s>>>(b.ds, b.sweep, k);
    k_near_resolve_b<<<b.n_sweep, kThreads, 0, s>>>(b.ds, b.sweep, k);
  }
  return hipGetLastError();
}

hipError_t launch_block_end_b(const BatchLaunch& b, int K, hipStream_t s) {
  k_close_b<<<b.n_close, kThreads, 0, s>>>(b.ds, b.close, K - 1);
  return launch_ctl_b(b, 1, (uint32_t)K, s);
}

hipError_t launch_sort_b(const BatchLaunch& b, hipStream_t s) {
  k_sort_count_b<<<b.n_part, kThreads, 0, s>>>(b.ds, b.part);
  k_sort_local_b<<<b.n_sortl * b.nrep, kThreads, 0, s>>>(b.ds, b.n_sortl);
  k_sort_scan_b<<<b.nrep, kFinThreads, 0, s>>>(b.ds);
  k_sort_scatter_b<<<b.n_part, kThreads, 0, s>>>(b.ds, b.part);
  return launch_ctl_b(b, 2, 0u, s);
}

hipError_t launch_gather_out(const Dev& d, float* ox, float* oy, float* oz, int32_t* otyp,
                             int32_t* ost, int32_t* oadj, hipStream_t s) {
  k_gather_out<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d, ox, oy, oz, otyp, ost, oadj);
  return hipGetLastError();
}

// n_steps of the re-jitter alone, then the block origin moved by them.
// ev0/ev1 (may be null): stamped at the start and end of each step's kernel.
hipError_t launch_jitter_only(const Dev& d, int n_steps, hipStream_t s, hipEvent_t ev0,
                              hipEvent_t ev1) {
  const dim3 g(blocks_for(d.n, kThreads)), b(kThreads);
  for (int k = 0; k < n_steps; ++k) {
    auto kern = d.nt_pos ? k_jitter_only<true> : k_jitter_only<false>;
    if (ev0) hipExtLaunchKernelGGL(kern, g, b, 0, s, ev0, ev1, 0, d, k);
    else kern<<<g, b, 0, s>>>(d, k);
  }
  k_advance_jitter<<<1, 64, 0, s>>>(d.ctl, n_steps);
  return hipGetLastError();
}

// bytes must be a multiple of width; width 4, 8 or 16.  The grid holds
// 2048 workgroups (8 per compute unit) and strides over the buffer.
hipError_t launch_stream_copy(const void* src, void* dst, long long bytes, int width,
                              hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 g(2048), b(kThreads);
  if (width == 16)
    hipExtLaunchKernelGGL(k_stream_copy<uint4>, g, b, 0, s, ev0, ev1, 0, (const uint4*)src,
                          (uint4*)dst, bytes / 16);
  else if (width == 8)
    hipExtLaunchKernelGGL(k_stream_copy<uint2>, g, b, 0, s, ev0, ev1, 0, (const uint2*)src,
                          (uint2*)dst, bytes / 8);
  else
    hipExtLaunchKernelGGL(k_stream_copy<uint32_t>, g, b, 0, s, ev0, ev1, 0, (const uint32_t*)src,
                          (uint32_t*)dst, bytes / 4);
  return hipGetLastError();
}

// Kinetics counters (counters zeroed by the caller): populations, the A
// binning of the current positions (a copy of d without re-jitter), pairs.
hipError_t launch_kinetics(const Dev& d, int nstate, int nbins, const float* e2,
                           unsigned long long* pop, unsigned long long* pairs,
                           unsigned long long* hist, hipStream_t s) {
  const int g = std::min(blocks_for(d.n, kThreads), 2048);
  k_kin_pop<<<g, kThreads, 0, s>>>(d, nstate, pop);
  Dev dn = d;
  dn.jit_c = 0.0f;
  dn.fuse = 0;  // binned into the plain buckets here, whatever the steps use
  k_prep<<<d.nwg_prep, kThreads, 0, s>>>(dn, 0);
  if (d.sorted && d.bs <= kOneCellBrick)
    k_kin_pairs_staged<<<d.nwg_sweep, kThreads, 0, s>>>(dn, nstate, nbins, e2, pairs, hist);
  else
    k_kin_pairs<<<g, kThreads, 0, s>>>(dn, nstate, nbins, e2, pairs, hist);
  k_kin_reset<<<std::min(blocks_for(d.ncell, kThreads), 1024), kThreads, 0, s>>>(dn);
  k_kin_sum<<<1, kThreads, 0, s>>>(pop);  // pop is the first slice's start
  return hipGetLastError();
}

hipError_t launch_md_init(const Dev& d, unsigned long long vseed, float cv, hipStream_t s) {
  if (d.n > 0) {
    k_slot_of<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d);
    if (cv >= 0.0f) k_md_init<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d, vseed, cv);
  }
  return hipGetLastError();
}

hipError_t launch_gather_v(const Dev& d, float* ox, float* oy, float* oz, hipStream_t s) {
  if (d.n > 0) k_gather_v<<<blocks_for(d.n, kThreads), kThreads, 0, s>>>(d, ox, oy, oz);
  return hipGetLastError();
}

hipError_t launch_sqrt_rn(const float* in, float* out, long long n, hipStream_t s) {
  if (n > 0) k_sqrt_rn<<<blocks_for(n, kThreads), kThreads, 0, s>>>(in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t s) {
  if (n > 0) k_fill_u32<<<(int)std::min<long long>(blocks_for(n, kThreads), 4096), kThreads, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_draws(const uint32_t* ctr, long long n, unsigned long long key, uint32_t* out,
                        hipStream_t s) {
  k_draws<<<blocks_for(n, kThreads), kThreads, 0, s>>>((const uint4*)ctr, n, key, (uint4*)out);
  return hipGetLastError();
}

}  // namespace pr
