"""Seeded synthetic workloads for the reaction step (host side, numpy only).

This module generates inputs; it holds none of the reaction step's arithmetic
(no distance test, acceptance, selection or bonding).  It is the one input
generator that both the library's tests and the CPU oracle's tests draw from.

The paper's own systems come from equilibrated MD runs (Sec. II D, Appendix A)
whose inputs are not available.  They are replaced by jittered simple-cubic
lattices at the paper's densities with the same cutoff and the same sparsity of
active particles:

* ``n`` = smallest integer with n^3 >= N, lattice constant ``a = fl32(L/n)``;
* particle ``i`` sits on site ``s = (i * (2^31 - 1)) mod n^3`` (a bijection that
  scatters ids over space), ``ix = s mod n, iy = (s / n) mod n, iz = s / n^2``;
* position ``fl32(fl32(ix + 0.5) * a)`` plus an integer Irwin-Hall(12)
  displacement with ``sigma0 = 0.1`` (Philox counter ``(0, i, blk, 2)``), wrapped
  once into ``[0, L)``;
* type/state from ``w = Philox((0, i, 0, 3)).w0``: step growth makes a
  crosslinker (type 1, state 4 = remaining valence) iff ``w < ceil(0.05 * 2^32)``,
  otherwise a monomer/end unit (type 0, state 2); chain growth makes an
  initiator (state 2 = active end) iff ``w < ceil(0.001 * 2^32)``, otherwise a free
  monomer (state 0).

Philox4x32-10 here is this module's own vectorised implementation of the
published generator (Salmon et al., SC'11); the library's device generator
implements the same recipe independently and is tested against this one.
"""
import math

import numpy as np

MASTER_SEED = 0x14097498
RC = 1.12
SIGMA_JITTER = 0.05
SIGMA_LATTICE = 0.1
DENSITY = 0.85

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, key):
    """Vectorised Philox4x32-10; counters are broadcastable uint32 arrays."""
    c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64) & _MASK
                                           for c in (c0, c1, c2, c3)))
    k0, k1 = int(key) & 0xFFFFFFFF, (int(key) >> 32) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0, k1 = (k0 + _W0) & 0xFFFFFFFF, (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0), p1 & _MASK,
                          (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1), p0 & _MASK)
    return tuple(np.asarray(c, dtype=np.uint32) for c in (c0, c1, c2, c3))


def threshold(p):
    """ceil(p * 2^32) clamped to [0, 2^32]: w < threshold  <=>  w * 2^-32 < p."""
    return int(min(max(math.ceil(p * 4294967296.0), 0), 4294967296))


def ih12(step, ids, tag, seed):
    """Integer Irwin-Hall(12) offsets S (n x 3, int32): sum of 12 bytes - 1530."""
    ids = np.asarray(ids, dtype=np.uint64)
    words = []
    for blk in range(3):
        words.extend(philox4x32_10(step, ids, blk, tag, seed))
    out = np.empty((ids.shape[0], 3), dtype=np.int32)
    for d in range(3):
        s = np.zeros(ids.shape[0], dtype=np.int64)
        for w in words[3 * d:3 * d + 3]:
            w = w.astype(np.int64)
            s += (w & 0xFF) + ((w >> 8) & 0xFF) + ((w >> 16) & 0xFF) + ((w >> 24) & 0xFF)
        out[:, d] = (s - 1530).astype(np.int32)
    return out


def _wrap(v, L):
    L = np.float32(L)
    v = np.where(v < np.float32(0), v + L, v).astype(np.float32)
    v = np.where(v >= L, v - L, v).astype(np.float32)
    return v


def lattice_sites(N, L):
    n = 1
    while n ** 3 < N:
        n += 1
    a = np.float32(float(np.float32(L)) / n)
    i = np.arange(N, dtype=np.uint64)
    s = (i * np.uint64(2 ** 31 - 1)) % np.uint64(n ** 3)
    ix, iy, iz = s % np.uint64(n), (s // np.uint64(n)) % np.uint64(n), s // np.uint64(n * n)
    half = np.float32(0.5)
    return tuple(((c.astype(np.float32) + half) * a).astype(np.float32) for c in (ix, iy, iz))


class Config:
    """One synthetic workload."""

    def __init__(self, name, N, L, kind, p, steps, seed, sigma=SIGMA_JITTER, rc=RC, gen_seed=None):
        self.name, self.N, self.L, self.kind = name, int(N), float(np.float32(L)), kind
        self.p, self.steps, self.seed, self.sigma, self.rc = float(p), int(steps), int(seed), sigma, rc
        # seed of the initial configuration (the reaction steps draw with `seed`)
        self.gen_seed = int(seed if gen_seed is None else gen_seed)

    def rule(self):
        return rule_for(self.kind, self.rc, self.p)

    @property
    def B(self):
        return 4 if self.kind == "step" else 2

    def initial(self):
        """The initial configuration (host arrays), as generate() makes it."""
        return generate(self.N, self.L, self.kind, self.gen_seed)

    def desc(self, log_cap=None):
        """Replica description (the keys of the library's replica struct)."""
        return dict(n=self.N, L=self.L, B=self.B, rule=self.rule(), seed=self.seed,
                    kind=self.kind, gen_seed=self.gen_seed, sigma0=SIGMA_LATTICE,
                    log_cap=2 * self.N if log_cap is None else log_cap)

    def __repr__(self):
        return "Config(%s, N=%d, L=%g, %s, p=%g, steps=%d)" % (self.name, self.N, self.L, self.kind,
                                                               self.p, self.steps)


def rule_for(kind, rc=RC, p=0.01, policy="random"):
    """Rule parameters as a dict (keys follow the library's rule struct).

    step growth (Sec. II C): A = crosslinker (type 1) with remaining valence in
    [1, 4], -1 per bond; T = end unit (type 0) with remaining valence in [1, 2],
    -1 per bond.  chain growth (Sec. II B): one type; free monomer 0, active end
    2, inert 1; A = active end (2 -> 1), T = free monomer (0 -> 2, becomes the
    new active end).  policy: "random" (the paper's selection) or "nearest"
    (the closest-partner selection of LAMMPS fix bond/create, Sec. IV A)."""
    if kind == "step":
        return dict(type_a=1, a_min=1, a_max=4, d_a=-1, type_t=0, t_min=1, t_max=2, d_t=-1,
                    rc=rc, p=p, exclude_bonded=1, policy=policy)
    if kind == "chain":
        return dict(type_a=0, a_min=2, a_max=2, d_a=-1, type_t=0, t_min=0, t_max=0, d_t=2,
                    rc=rc, p=p, exclude_bonded=1, policy=policy)
    raise ValueError(kind)


def generate(N, L, kind, seed, sigma0=SIGMA_LATTICE, B=None):
    """Jittered-lattice initial configuration: dict of x, y, z, type, state, adj."""
    x, y, z = lattice_sites(N, L)
    ids = np.arange(N, dtype=np.uint64)
    S = ih12(0, ids, 2, seed)
    c = np.float32(sigma0 / 256.0)
    x = _wrap((x + (S[:, 0].astype(np.float32) * c).astype(np.float32)).astype(np.float32), L)
    y = _wrap((y + (S[:, 1].astype(np.float32) * c).astype(np.float32)).astype(np.float32), L)
    z = _wrap((z + (S[:, 2].astype(np.float32) * c).astype(np.float32)).astype(np.float32), L)
    w = philox4x32_10(0, ids, 0, 3, seed)[0].astype(np.uint64)
    if kind == "step":
        cross = w < np.uint64(threshold(0.05))
        type_ = cross.astype(np.int32)
        state = np.where(cross, 4, 2).astype(np.int32)
        B = B or 4
    elif kind == "chain":
        init = w < np.uint64(threshold(0.001))
        type_ = np.zeros(N, dtype=np.int32)
        state = np.where(init, 2, 0).astype(np.int32)
        B = B or 2
    else:
        raise ValueError(kind)
    adj = np.full((N, B), -1, dtype=np.int32)
    return dict(L=float(np.float32(L)), x=x, y=y, z=z, type=type_, state=state, adj=adj)


def box_for(N, rho=DENSITY):
    return float(np.float32((N / rho) ** (1.0 / 3.0)))


CONFIGS = {
    "c1": Config("c1_step_4k", 4000, 16.75, "step", 0.01, 200, MASTER_SEED + 1),
    "c2": Config("c2_step_1m", 1048576, 105.6, "step", 0.005, 1000, MASTER_SEED + 2),
    "c3": Config("c3_chain_4m", 4194304, 167.7, "chain", 0.02, 2000, MASTER_SEED + 3),
}


def replica_configs(n_rep=256, steps=500, seed=MASTER_SEED + 4, nmin=2000, nmax=65536):
    """Batched ensemble: N log-uniform in [nmin, nmax], even r step / odd r chain
    growth, p uniform in [0.001, 0.02], density 0.85; per-replica seed from
    Philox((r, 0, 0, 4)) words 0-1, sizes and rates from Philox((r, 0, 0, 5))."""
    r = np.arange(n_rep, dtype=np.uint64)
    k = philox4x32_10(r, 0, 0, 4, seed)
    u = philox4x32_10(r, 0, 0, 5, seed)
    out = []
    for i in range(n_rep):
        u0 = float(u[0][i]) / 4294967296.0
        u1 = float(u[1][i]) / 4294967296.0
        N = int(round(math.exp(math.log(nmin) + (math.log(nmax) - math.log(nmin)) * u0)))
        kind = "step" if i % 2 == 0 else "chain"
        p = 0.001 + 0.019 * u1
        rseed = int(k[0][i]) | (int(k[1][i]) << 32)
        out.append(Config("rep%d" % i, N, box_for(N), kind, p, steps, rseed,
                          gen_seed=rseed ^ 0x5A5A))
    return out


def request_stream(n_req=10000, rate=200.0, steps=1000, seed=MASTER_SEED + 5, nmin=1000,
                   nmax=1048576):
    """Served stream: Poisson arrivals at ``rate``/s; N log-uniform in [nmin, nmax];
    step/chain 50/50; p uniform in [0.001, 0.02].  Returns (arrival_s, configs)."""
    r = np.arange(n_req, dtype=np.uint64)
    k = philox4x32_10(r, 0, 0, 4, seed)
    u = philox4x32_10(r, 0, 0, 5, seed)
    t, arrivals, cfgs = 0.0, [], []
    for i in range(n_req):
        u0, u1, u2, u3 = (float(u[j][i]) / 4294967296.0 for j in range(4))
        t += -math.log(1.0 - u3) / rate
        N = int(round(math.exp(math.log(nmin) + (math.log(nmax) - math.log(nmin)) * u0)))
        kind = "step" if u2 < 0.5 else "chain"
        p = 0.001 + 0.019 * u1
        rseed = int(k[0][i]) | (int(k[1][i]) << 32)
        arrivals.append(t)
        cfgs.append(Config("req%d" % i, N, box_for(N), kind, p, steps, rseed,
                           gen_seed=rseed ^ 0x5A5A))
    return np.array(arrivals), cfgs
