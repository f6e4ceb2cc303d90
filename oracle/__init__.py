"""ctypes wrapper of the CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP implementation.
"""
import ctypes as C

import numpy as np

from . import build as _build

_lib = None

ST_NAMES = ("a_elig", "t_elig", "in_rc", "drawn", "excluded", "accepted", "proposals", "bonds",
            "adj_overflow")
ST_COUNT = len(ST_NAMES)

OK, EINVAL, ERULE_AMBIGUOUS, ECAP, ENOMEM = 0, -1, -2, -3, -4


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def load(path=None):
    """Load (building if needed) the oracle library; ``path`` selects a variant."""
    global _lib
    if path is not None:
        return _declare(C.CDLL(path))
    if _lib is None:
        _lib = _declare(C.CDLL(_build.ensure_built()))
    return _lib


def _declare(lib):
    i32, i64, u32, u64, f32, f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float, C.c_double
    P = C.POINTER
    lib.or_philox_bulk.argtypes = [i64, P(u32), P(u64), P(u32)]
    lib.or_philox_bulk.restype = None
    lib.or_threshold.argtypes = [f64]
    lib.or_threshold.restype = u64
    rule = [i32, i32, i32, i32, i32, i32, i32, i32, f32, f64, i32]
    lib.or_react_step.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32), i32,
                                  *rule, u64, u32, P(i32), i64, P(i64), P(i64)]
    lib.or_react_step.restype = C.c_int
    lib.or_run.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32), i32,
                           *rule, u64, u32, u32, f64, P(i32), i64, P(i64), P(i64)]
    lib.or_run.restype = C.c_int
    lib.or_react_step_nearest.argtypes = lib.or_react_step.argtypes
    lib.or_react_step_nearest.restype = C.c_int
    lib.or_run_nearest.argtypes = lib.or_run.argtypes
    lib.or_run_nearest.restype = C.c_int
    lib.or_sample_bonds.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32), i32,
                                    *rule, u64, u32, P(i64), i64, P(i32)]
    lib.or_sample_bonds.restype = C.c_int
    lib.or_near_cutoff.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32),
                                   i32, i32, i32, i32, i32, i32, f32, f64, P(i64), P(i64)]
    lib.or_near_cutoff.restype = C.c_int
    lib.or_ih12_offsets.argtypes = [u32, u32, u32, u64, P(i32)]
    lib.or_ih12_offsets.restype = None
    lib.or_ih4_offsets.argtypes = [u32, u32, u32, u64, P(i32)]
    lib.or_ih4_offsets.restype = None
    lib.or_jitter_scale.argtypes = [f64]
    lib.or_jitter_scale.restype = C.c_float
    lib.or_jitter.argtypes = [i32, f32, P(f32), P(f32), P(f32), u64, u32, f64]
    lib.or_jitter.restype = None
    lib.or_react_step_multi.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32),
                                        i32, P(i32), P(f32), P(f64), i32, u64, u32, P(i32), i64,
                                        P(i64), P(i64)]
    lib.or_react_step_multi.restype = C.c_int
    lib.or_run_multi.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32), i32,
                                 P(i32), P(f32), P(f64), i32, u64, u32, u32, f64, P(i32), i64,
                                 P(i64), P(i64)]
    lib.or_run_multi.restype = C.c_int
    lib.or_rule_tag.argtypes = [i32]
    lib.or_rule_tag.restype = u32
    lib.or_md_block.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(f32), P(f32), P(f32), P(i32),
                                i32, f64, f64, f64, i32]
    lib.or_md_block.restype = C.c_int
    lib.or_md_energy.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(f32), P(f32), P(f32), P(i32),
                                 i32, f64, f64]
    lib.or_md_energy.restype = C.c_double
    lib.or_md_velocities.argtypes = [i32, P(f32), P(f32), P(f32), u64, f64]
    lib.or_md_velocities.restype = None
    lib.or_run_md.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(f32), P(f32), P(f32), P(i32),
                              P(i32), P(i32), i32, *rule, u64, u32, u32, f64, f64, f64, i32,
                              P(i32), i64, P(i64), P(i64)]
    lib.or_run_md.restype = C.c_int
    lib.or_kinetics.argtypes = [i32, f32, P(f32), P(f32), P(f32), P(i32), P(i32), P(i32), i32,
                                i32, i32, i32, i32, i32, i32, f32, i32, i32, P(i64), P(i64), i32,
                                P(i64)]
    lib.or_kinetics.restype = C.c_int
    lib.or_kin_edge2.argtypes = [f32, i32, i32]
    lib.or_kin_edge2.restype = C.c_float
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = C.c_int
    return lib


class Rule:
    """Reaction rule T^t + A^a -> T^(t+dT)-A^(a+dA) (Sec. II, Eq. (2)).

    policy: "random" (the paper's selection, Table I) or "nearest" (the
    closest-partner selection of LAMMPS fix bond/create, Sec. IV A)."""

    def __init__(self, type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t, rc, p,
                 exclude_bonded=1, policy="random"):
        self.type_a, self.a_min, self.a_max, self.d_a = type_a, a_min, a_max, d_a
        self.type_t, self.t_min, self.t_max, self.d_t = type_t, t_min, t_max, d_t
        self.rc, self.p, self.exclude_bonded = float(rc), float(p), int(exclude_bonded)
        assert policy in ("random", "nearest"), policy
        self.policy = policy

    def args(self):
        return (self.type_a, self.a_min, self.a_max, self.d_a, self.type_t, self.t_min,
                self.t_max, self.d_t, C.c_float(self.rc), self.p, self.exclude_bonded)

    def replace(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Rule(**d)


def philox(ctr, key, lib=None):
    """Philox4x32-10 of counters ``ctr`` (n x 4 uint32) under keys ``key`` (n uint64)."""
    lib = lib or load()
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(np.broadcast_to(np.asarray(key, dtype=np.uint64), (ctr.shape[0],)))
    out = np.empty_like(ctr)
    lib.or_philox_bulk(ctr.shape[0], _p(ctr, C.c_uint32), _p(key, C.c_uint64), _p(out, C.c_uint32))
    return out


def threshold(p, lib=None):
    return int((lib or load()).or_threshold(float(p)))


class System:
    """Host-side particle system: SoA arrays, mutated in place by the oracle."""

    def __init__(self, L, x, y, z, type_, state, adj):
        self.L = float(np.float32(L))
        self.x = np.ascontiguousarray(x, dtype=np.float32).copy()
        self.y = np.ascontiguousarray(y, dtype=np.float32).copy()
        self.z = np.ascontiguousarray(z, dtype=np.float32).copy()
        self.type = np.ascontiguousarray(type_, dtype=np.int32).copy()
        self.state = np.ascontiguousarray(state, dtype=np.int32).copy()
        self.adj = np.ascontiguousarray(adj, dtype=np.int32).copy()
        assert self.adj.ndim == 2 and self.adj.shape[0] == self.x.shape[0]

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def B(self):
        return self.adj.shape[1]

    def copy(self):
        return System(self.L, self.x, self.y, self.z, self.type, self.state, self.adj)


def react_step(sysm, rule, seed, step, lib=None):
    """One reaction step in place.  Returns (code, bonds[n_b, 2], stats dict)."""
    lib = lib or load()
    n = sysm.n
    cap = n // 2 + 1
    bonds = np.empty((cap, 2), dtype=np.int32)
    nb = C.c_int64(0)
    st = np.zeros(ST_COUNT, dtype=np.int64)
    fn = lib.or_react_step_nearest if rule.policy == "nearest" else lib.or_react_step
    code = fn(n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                             _p(sysm.z, C.c_float), _p(sysm.type, C.c_int32),
                             _p(sysm.state, C.c_int32), _p(sysm.adj, C.c_int32), sysm.B,
                             *rule.args(), C.c_uint64(seed), C.c_uint32(step), _p(bonds, C.c_int32),
                             cap, C.byref(nb), _p(st, C.c_int64))
    return code, bonds[: nb.value].copy(), dict(zip(ST_NAMES, st.tolist()))


def run(sysm, rule, seed, first_step, n_steps, sigma, log_cap=None, lib=None):
    """Steps first_step.. in place; each jitters (sigma > 0) then reacts.

    Returns (code, log[n, 3] of (step, id_A, id_T), stats[n_steps, ST_COUNT])."""
    lib = lib or load()
    n = sysm.n
    if log_cap is None:
        log_cap = max(16, n * 4)
    log = np.empty((log_cap, 3), dtype=np.int32)
    nl = C.c_int64(0)
    st = np.zeros((max(n_steps, 1), ST_COUNT), dtype=np.int64)
    fn = lib.or_run_nearest if rule.policy == "nearest" else lib.or_run
    code = fn(n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                      _p(sysm.z, C.c_float), _p(sysm.type, C.c_int32), _p(sysm.state, C.c_int32),
                      _p(sysm.adj, C.c_int32), sysm.B, *rule.args(), C.c_uint64(seed),
                      C.c_uint32(first_step), C.c_uint32(n_steps), float(sigma),
                      _p(log, C.c_int32), log_cap, C.byref(nl), _p(st, C.c_int64))
    return code, log[: min(nl.value, log_cap)].copy(), st[:n_steps]


def sample_bonds(sysm, rule, seed, step, ids, lib=None):
    """Partner id of each sampled particle in this step's bonds (-1: none)."""
    lib = lib or load()
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.empty(ids.shape[0], np.int32)
    code = lib.or_sample_bonds(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float),
                               _p(sysm.y, C.c_float), _p(sysm.z, C.c_float),
                               _p(sysm.type, C.c_int32), _p(sysm.state, C.c_int32),
                               _p(sysm.adj, C.c_int32), sysm.B, *rule.args(), C.c_uint64(seed),
                               C.c_uint32(step), _p(ids, C.c_int64), ids.shape[0],
                               _p(out, C.c_int32))
    assert code == 0, code
    return out


def jitter(sysm, seed, step, sigma, lib=None):
    lib = lib or load()
    lib.or_jitter(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                  _p(sysm.z, C.c_float), C.c_uint64(seed), C.c_uint32(step), float(sigma))


def ih12_offsets(step, ids, tag, seed, lib=None):
    """Integer Irwin-Hall(12) offsets S (n x 3) of the initial configuration."""
    lib = lib or load()
    out = np.empty((len(ids), 3), dtype=np.int32)
    buf = (C.c_int32 * 3)()
    for k, i in enumerate(ids):
        lib.or_ih12_offsets(C.c_uint32(step), C.c_uint32(int(i)), C.c_uint32(tag), C.c_uint64(seed), buf)
        out[k] = list(buf)
    return out


def ih4_offsets(step, ids, tag, seed, lib=None):
    """Integer Irwin-Hall(4) offsets S (n x 3) of the re-jitter for particle ``ids``."""
    lib = lib or load()
    out = np.empty((len(ids), 3), dtype=np.int32)
    buf = (C.c_int32 * 3)()
    for k, i in enumerate(ids):
        lib.or_ih4_offsets(C.c_uint32(step), C.c_uint32(int(i)), C.c_uint32(tag), C.c_uint64(seed), buf)
        out[k] = list(buf)
    return out


def jitter_scale(sigma, lib=None):
    """The FP32 displacement per unit offset of the re-jitter."""
    lib = lib or load()
    return float(lib.or_jitter_scale(float(sigma)))


def near_cutoff(sysm, rule, tol=1e-6, lib=None):
    """(count of eligible pairs with |r64 - rc| < tol, count of FP32/FP64 disagreements)."""
    lib = lib or load()
    near, dis = C.c_int64(0), C.c_int64(0)
    lib.or_near_cutoff(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                       _p(sysm.z, C.c_float), _p(sysm.type, C.c_int32), _p(sysm.state, C.c_int32),
                       rule.type_a, rule.a_min, rule.a_max, rule.type_t, rule.t_min, rule.t_max,
                       C.c_float(rule.rc), float(tol), C.byref(near), C.byref(dis))
    return near.value, dis.value


def _rule_arrays(rules):
    ri = np.zeros((len(rules), 10), np.int32)
    for k, r in enumerate(rules):
        ri[k, :9] = (r.type_a, r.a_min, r.a_max, r.d_a, r.type_t, r.t_min, r.t_max, r.d_t,
                     r.exclude_bonded)
    rc = np.array([r.rc for r in rules], np.float32)
    p = np.array([r.p for r in rules], np.float64)
    return ri, rc, p


def react_step_multi(sysm, rules, seed, step, lib=None):
    """One step with several concurrent rules, in place.  Returns (code,
    bonds[n_b, 3] of (id_A, id_T, rule), stats dict)."""
    lib = lib or load()
    ri, rc, p = _rule_arrays(rules)
    cap = sysm.n // 2 + 1
    bonds = np.empty((cap, 3), np.int32)
    nb = C.c_int64(0)
    st = np.zeros(ST_COUNT, np.int64)
    code = lib.or_react_step_multi(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float),
                                   _p(sysm.y, C.c_float), _p(sysm.z, C.c_float),
                                   _p(sysm.type, C.c_int32), _p(sysm.state, C.c_int32),
                                   _p(sysm.adj, C.c_int32), sysm.B, _p(ri, C.c_int32),
                                   _p(rc, C.c_float), _p(p, C.c_double), len(rules),
                                   C.c_uint64(seed), C.c_uint32(step), _p(bonds, C.c_int32), cap,
                                   C.byref(nb), _p(st, C.c_int64))
    return code, bonds[: nb.value].copy(), dict(zip(ST_NAMES, st.tolist()))


def run_multi(sysm, rules, seed, first_step, n_steps, sigma, log_cap=None, lib=None):
    """Steps with several rules; log rows (step, id_A, id_T, rule)."""
    lib = lib or load()
    ri, rc, p = _rule_arrays(rules)
    log_cap = log_cap or max(16, sysm.n * 4)
    log = np.empty((log_cap, 4), np.int32)
    nl = C.c_int64(0)
    st = np.zeros((max(n_steps, 1), ST_COUNT), np.int64)
    code = lib.or_run_multi(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float),
                            _p(sysm.y, C.c_float), _p(sysm.z, C.c_float), _p(sysm.type, C.c_int32),
                            _p(sysm.state, C.c_int32), _p(sysm.adj, C.c_int32), sysm.B,
                            _p(ri, C.c_int32), _p(rc, C.c_float), _p(p, C.c_double), len(rules),
                            C.c_uint64(seed), C.c_uint32(first_step), C.c_uint32(n_steps),
                            float(sigma), _p(log, C.c_int32), log_cap, C.byref(nl),
                            _p(st, C.c_int64))
    return code, log[: min(nl.value, log_cap)].copy(), st[:n_steps]


class MD:
    """Velocities of a System for the bonded-force coupling (FP32 arrays)."""

    def __init__(self, n, seed=None, temp=1.0, lib=None):
        self.vx = np.zeros(n, np.float32)
        self.vy = np.zeros(n, np.float32)
        self.vz = np.zeros(n, np.float32)
        if seed is not None:
            (lib or load()).or_md_velocities(n, _p(self.vx, C.c_float), _p(self.vy, C.c_float),
                                             _p(self.vz, C.c_float), C.c_uint64(seed), float(temp))

    def _v(self):
        return _p(self.vx, C.c_float), _p(self.vy, C.c_float), _p(self.vz, C.c_float)


def md_block(sysm, md, theta, dt=0.0025, sig=1.0, eps=1.0, lib=None):
    lib = lib or load()
    return lib.or_md_block(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                           _p(sysm.z, C.c_float), *md._v(), _p(sysm.adj, C.c_int32), sysm.B,
                           float(dt), float(sig), float(eps), int(theta))


def md_energy(sysm, md, sig=1.0, eps=1.0, lib=None):
    lib = lib or load()
    return lib.or_md_energy(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float),
                            _p(sysm.y, C.c_float), _p(sysm.z, C.c_float), *md._v(),
                            _p(sysm.adj, C.c_int32), sysm.B, float(sig), float(eps))


def run_md(sysm, md, rule, seed, first_step, n_steps, theta, dt=0.0025, sig=1.0, eps=1.0,
           log_cap=None, lib=None):
    """Reaction steps with theta MD steps before each; (code, log, stats)."""
    lib = lib or load()
    log_cap = log_cap or max(16, sysm.n * 4)
    log = np.empty((log_cap, 3), np.int32)
    nl = C.c_int64(0)
    st = np.zeros((max(n_steps, 1), ST_COUNT), np.int64)
    code = lib.or_run_md(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                         _p(sysm.z, C.c_float), *md._v(), _p(sysm.type, C.c_int32),
                         _p(sysm.state, C.c_int32), _p(sysm.adj, C.c_int32), sysm.B,
                         *rule.args(), C.c_uint64(seed), C.c_uint32(first_step),
                         C.c_uint32(n_steps), float(dt), float(sig), float(eps), int(theta),
                         _p(log, C.c_int32), log_cap, C.byref(nl), _p(st, C.c_int64))
    return code, log[: min(nl.value, log_cap)].copy(), st[:n_steps]


def kinetics(sysm, rule, nstate=8, nbins=16, lib=None):
    """Kinetics counters of the configuration: (pop[nstate], pairs[nstate],
    hist[nbins]) as numpy int64 arrays (see or_kinetics)."""
    lib = lib or load()
    pop = np.zeros(nstate, np.int64)
    pairs = np.zeros(nstate, np.int64)
    hist = np.zeros(max(nbins, 1), np.int64)
    code = lib.or_kinetics(sysm.n, C.c_float(sysm.L), _p(sysm.x, C.c_float), _p(sysm.y, C.c_float),
                           _p(sysm.z, C.c_float), _p(sysm.type, C.c_int32),
                           _p(sysm.state, C.c_int32), _p(sysm.adj, C.c_int32), sysm.B,
                           rule.type_a, rule.a_min, rule.a_max, rule.type_t, rule.t_min,
                           rule.t_max, C.c_float(rule.rc), rule.exclude_bonded, nstate,
                           _p(pop, C.c_int64), _p(pairs, C.c_int64), nbins, _p(hist, C.c_int64))
    assert code == 0, code
    return pop, pairs, hist[:nbins]


def kin_edge2(rc, b, nbins, lib=None):
    return float((lib or load()).or_kin_edge2(C.c_float(rc), b, nbins))


def num_threads(lib=None):
    return int((lib or load()).or_num_threads())


__all__ = ["Rule", "System", "react_step", "run", "jitter", "philox", "threshold", "near_cutoff",
           "kinetics", "kin_edge2", "react_step_multi", "run_multi", "MD", "md_block",
           "md_energy", "run_md",
           "sample_bonds",
           "ih12_offsets", "ih4_offsets", "jitter_scale", "ST_NAMES", "load", "num_threads"]
