"""ctypes binding of ``libpolyreact.so`` (C ABI in include/polyreact.h).

Argument marshalling only: every step of the reaction path runs in the HIP
kernels of the library.  Device arrays are torch CUDA (HIP) tensors; streams
are torch streams.  Importing this module fails loudly when the library has
not been built -- there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolyreact.so")

(PR_OK, PR_EINVAL, PR_ERULE_AMBIGUOUS, PR_ECAP, PR_ENOMEM, PR_EHIP, PR_EBUSY, PR_ENOTFOUND,
 PR_ECANCELED) = (0, -1, -2, -3, -4, -5, -6, -7, -8)
STATS_FIELDS = ("a_elig", "t_elig", "in_rc", "drawn", "excluded", "accepted", "proposals", "bonds",
                "adj_overflow")


class PrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("polyreact error %d: %s" % (code, msg))
        self.code = code


POLICIES = {"random": 0, "nearest": 1}


class Rule(C.Structure):
    _fields_ = [("type_a", C.c_int32), ("a_min", C.c_int32), ("a_max", C.c_int32),
                ("d_a", C.c_int32), ("type_t", C.c_int32), ("t_min", C.c_int32),
                ("t_max", C.c_int32), ("d_t", C.c_int32), ("rc", C.c_float),
                ("exclude_bonded", C.c_int32), ("p", C.c_double), ("policy", C.c_int32)]

    @classmethod
    def make(cls, d=None, **kw):
        """From a dict with the field names; policy may be "random" or
        "nearest" (default "random")."""
        v = dict(d or {})
        v.update(kw)
        pol = v.get("policy", "random")
        v["policy"] = POLICIES[pol] if isinstance(pol, str) else int(pol)
        return cls(**{k: v[k] for k, _ in cls._fields_})


class ReplicaDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("L", C.c_float), ("B", C.c_int32), ("rule", Rule),
                ("seed", C.c_uint64), ("gen_kind", C.c_int32), ("gen_seed", C.c_uint64),
                ("gen_sigma0", C.c_double), ("log_cap", C.c_int64), ("brick", C.c_int32)]


class ServerInfo(C.Structure):
    _fields_ = [("budget", C.c_int64), ("used", C.c_int64), ("queued", C.c_int64),
                ("active", C.c_int64), ("done", C.c_int64), ("failed", C.c_int64),
                ("rounds", C.c_int64), ("busy_s", C.c_double), ("admit_s", C.c_double),
                ("finish_s", C.c_double), ("launch_s", C.c_double), ("wait_s", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STATS_FIELDS]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in STATS_FIELDS}


def _load():
    # torch first: its HIP runtime (SONAME libamdhip64.so.7) then also serves
    # this library, so the process holds one runtime, whatever the import order
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpolyreact.so is not built (run __graft_entry__.build() or "
                          "python paper_1409_7498_amd/csrc/build.py)")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, f32, f64, vp = (C.POINTER, C.c_int32, C.c_int64, C.c_uint32,
                                           C.c_uint64, C.c_float, C.c_double, C.c_void_p)
    sig = {
        "pr_last_error": ([], C.c_char_p),
        "pr_version": ([], C.c_char_p),
        "pr_react_step": ([i32, f32, vp, vp, vp, vp, vp, vp, i32, P(Rule), u64, u32, vp, i32,
                           P(i32), P(Stats), vp], C.c_int),
        "pr_react_step_noalloc": ([i32, f32, vp, vp, vp, vp, vp, vp, i32, P(Rule), u64, u32, vp,
                                   i32, P(i32), P(Stats), vp], C.c_int),
        "pr_sys_create": ([P(vp), i32, f32, i32, P(Rule), u64, i64, vp], C.c_int),
        "pr_sys_create_ex": ([P(vp), i32, f32, i32, P(Rule), u64, i64, vp, i32], C.c_int),
        "pr_sys_geometry": ([vp, P(i32), P(i32), P(i32)], C.c_int),
        "pr_sys_destroy": ([vp], None),
        "pr_sys_load": ([vp, vp, vp, vp, vp, vp, vp, i32], C.c_int),
        "pr_sys_generate": ([vp, i32, u64, f64], C.c_int),
        "pr_sys_run": ([vp, u32, u32, f64], C.c_int),
        "pr_sys_run_timed": ([vp, u32, u32, f64, P(f32)], C.c_int),
        "pr_sys_prepare": ([vp, u32, f64], C.c_int),
        "pr_sys_jitter": ([vp, u32, u32, f64, P(f32)], C.c_int),
        "pr_stream_copy": ([vp, vp, i64, i32, vp, P(f32)], C.c_int),
        "pr_sys_kinetics": ([vp, i32, vp, vp, i32, vp], C.c_int),
        "pr_sys_set_md": ([vp, i32, f64, f64, f64, f64, u64], C.c_int),
        "pr_sys_read_velocities": ([vp, vp, vp, vp], C.c_int),
        "pr_sqrt_rn": ([vp, vp, i64, vp], C.c_int),
        "pr_react_step_multi": ([i32, f32, vp, vp, vp, vp, vp, vp, i32, vp, i32, u64, u32, vp, i32,
                                 P(i32), P(Stats), vp], C.c_int),
        "pr_sys_create_multi": ([P(vp), i32, f32, i32, vp, i32, u64, i64, vp, i32], C.c_int),
        "pr_batch_kinetics": ([vp, i32, i32, vp, vp, i32, vp], C.c_int),
        "pr_sys_read": ([vp, vp, vp, vp, vp, vp, i32], C.c_int),
        "pr_sys_checkpoint": ([vp, vp, i64, P(i64)], C.c_int),
        "pr_sys_restore": ([vp, vp, i64], C.c_int),
        "pr_p_from_rate": ([f64, f64, f64, P(i32)], C.c_double),
        "pr_draws": ([vp, i64, u64, vp, vp], C.c_int),
        "pr_server_poll": ([vp, u64, P(i32), P(i32), P(f64)], C.c_int),
        "pr_server_cancel": ([vp, u64], C.c_int),
        "pr_sys_bonds": ([vp, vp, i64, P(i64)], C.c_int),
        "pr_sys_stats": ([vp, P(Stats), i64, P(i64)], C.c_int),
        "pr_sys_set_sort_period": ([vp, i32], C.c_int),
        "pr_sys_set_graphs": ([vp, i32], C.c_int),
        "pr_sys_set_fused_binning": ([vp, i32], C.c_int),
        "pr_sys_fused_binning": ([vp, C.POINTER(i32)], C.c_int),
        "pr_batch_create": ([P(vp), P(ReplicaDesc), i32, vp], C.c_int),
        "pr_batch_destroy": ([vp], None),
        "pr_batch_run": ([vp, u32, u32, f64], C.c_int),
        "pr_batch_run_loop": ([vp, u32, u32, f64], C.c_int),
        "pr_batch_bonds": ([vp, i32, vp, i64, P(i64)], C.c_int),
        "pr_batch_read": ([vp, i32, vp, vp, vp, vp, vp, i32], C.c_int),
        "pr_batch_stats": ([vp, i32, P(Stats), i64, P(i64)], C.c_int),
        "pr_footprint": ([P(ReplicaDesc), u32, P(i64)], C.c_int),
        "pr_autotune": ([P(ReplicaDesc), u32, f64, i32, vp, P(i32), P(f32)], C.c_int),
        "pr_autotune_cached": ([P(ReplicaDesc), u32, f64, i32, vp, C.c_char_p, P(i32), P(f32)],
                               C.c_int),
        "pr_server_create": ([P(vp), i64, i32, vp], C.c_int),
        "pr_server_destroy": ([vp], None),
        "pr_server_submit": ([vp, P(ReplicaDesc), u32, f64, P(u64)], C.c_int),
        "pr_server_wait": ([vp, u64, f64, P(i32), P(i32), P(f64)], C.c_int),
        "pr_server_bonds": ([vp, u64, vp, i64, P(i64)], C.c_int),
        "pr_server_read": ([vp, u64, vp, vp, vp, vp, vp], C.c_int),
        "pr_server_stats": ([vp, u64, P(Stats), i64, P(i64)], C.c_int),
        "pr_server_release": ([vp, u64], C.c_int),
        "pr_server_info_get": ([vp, P(ServerInfo)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def exported_symbols():
    return [n for n in ("pr_last_error", "pr_version", "pr_react_step", "pr_react_step_noalloc",
                        "pr_sys_create",
                        "pr_sys_create_ex", "pr_sys_geometry", "pr_autotune",
                        "pr_sys_destroy", "pr_sys_load", "pr_sys_generate", "pr_sys_run",
                        "pr_sys_run_timed", "pr_sys_read", "pr_sys_bonds", "pr_sys_stats",
                        "pr_sys_set_sort_period", "pr_sys_set_graphs", "pr_sys_set_fused_binning",
                        "pr_sys_fused_binning", "pr_batch_create",
                        "pr_batch_destroy", "pr_batch_run", "pr_batch_run_loop", "pr_batch_bonds",
                        "pr_batch_read", "pr_batch_stats", "pr_footprint", "pr_server_create",
                        "pr_server_destroy", "pr_server_submit", "pr_server_wait",
                        "pr_server_bonds", "pr_server_read", "pr_server_stats",
                        "pr_server_release", "pr_server_info_get", "pr_sys_checkpoint",
                        "pr_sys_restore", "pr_p_from_rate", "pr_draws", "pr_server_poll",
                        "pr_server_cancel", "pr_autotune_cached", "pr_sys_prepare",
                        "pr_sys_jitter", "pr_stream_copy", "pr_sys_kinetics",
                        "pr_batch_kinetics", "pr_react_step_multi", "pr_sys_create_multi",
                        "pr_sys_set_md", "pr_sys_read_velocities", "pr_sqrt_rn")]


def _check(code):
    if code != PR_OK:
        raise PrError(code, lib.pr_last_error().decode())
    return code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def react_step(x, y, z, type_, state, adj, L, rule, seed, step, bonds=None, stream=None,
               raise_on_error=True, noalloc=False):
    """One reaction step on device tensors (state and adj updated in place).
    noalloc: through pr_react_step_noalloc (library scratch in a fixed device
    region, no allocation; n <= 32768).

    Returns (code, bonds[n_b, 2] device tensor view, stats dict)."""
    import torch
    n = x.numel()
    B = adj.shape[1] if adj.dim() == 2 else 1
    for t, dt in ((x, torch.float32), (y, torch.float32), (z, torch.float32), (type_, torch.int32),
                  (state, torch.int32), (adj, torch.int32)):
        assert t.is_cuda and t.dtype == dt and t.is_contiguous() and t.shape[0] == n
    cap = n // 2 + 1
    if bonds is None:
        bonds = torch.empty((cap, 2), dtype=torch.int32, device=x.device)
    nb = C.c_int32(0)
    st = Stats()
    r = rule if isinstance(rule, Rule) else Rule.make(rule)
    fn = lib.pr_react_step_noalloc if noalloc else lib.pr_react_step
    code = fn(n, C.c_float(L), _ptr(x), _ptr(y), _ptr(z), _ptr(type_), _ptr(state), _ptr(adj), B,
              C.byref(r), C.c_uint64(seed), C.c_uint32(step), _ptr(bonds), bonds.shape[0],
              C.byref(nb), C.byref(st), _stream(stream))
    if raise_on_error and code not in (PR_OK,):
        _check(code)
    return code, bonds[: nb.value], st.as_dict()


def _rules(rules):
    arr = (Rule * len(rules))()
    for k, r in enumerate(rules):
        arr[k] = r if isinstance(r, Rule) else Rule.make(r)
    return arr


def react_step_multi(x, y, z, type_, state, adj, L, rules, seed, step, stream=None,
                     raise_on_error=True):
    """One step with several concurrent rules on device tensors.  Returns
    (code, bonds[n_b, 3] of (id_A, id_T, rule) device tensor view, stats)."""
    import torch
    n = x.numel()
    B = adj.shape[1] if adj.dim() == 2 else 1
    cap = n // 2 + 1
    bonds = torch.empty((cap, 3), dtype=torch.int32, device=x.device)
    nb = C.c_int32(0)
    st = Stats()
    arr = _rules(rules)
    code = lib.pr_react_step_multi(n, C.c_float(L), _ptr(x), _ptr(y), _ptr(z), _ptr(type_),
                                   _ptr(state), _ptr(adj), B, arr, len(rules), C.c_uint64(seed),
                                   C.c_uint32(step), _ptr(bonds), cap, C.byref(nb), C.byref(st),
                                   _stream(stream))
    if raise_on_error and code != PR_OK:
        _check(code)
    return code, bonds[: nb.value], st.as_dict()


class System:
    """Resident particle system (pr_sys_* entry points)."""

    def __init__(self, n, L, B, rule, seed, log_cap=0, stream=None, brick=0):
        """brick: brick edge in coarse cells (1..6, 0 = 4), a tuning choice only.
        rule: one rule, or a list of several concurrent rules."""
        self._h = C.c_void_p()
        self.n, self.L, self.B = int(n), float(np.float32(L)), int(B)
        if isinstance(rule, (list, tuple)):
            arr = _rules(rule)
            _check(lib.pr_sys_create_multi(C.byref(self._h), self.n, C.c_float(L), self.B, arr,
                                           len(rule), C.c_uint64(seed), int(log_cap),
                                           _stream(stream), int(brick)))
            return
        r = rule if isinstance(rule, Rule) else Rule.make(rule)
        _check(lib.pr_sys_create_ex(C.byref(self._h), self.n, C.c_float(L), self.B, C.byref(r),
                                    C.c_uint64(seed), int(log_cap), _stream(stream), int(brick)))

    def geometry(self):
        """(coarse cells per side, effective brick edge, bricks)."""
        v = [C.c_int32(0) for _ in range(3)]
        _check(lib.pr_sys_geometry(self._h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self):
        if self._h:
            lib.pr_sys_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, cfg):
        """Load a host configuration dict (x, y, z, type, state, adj numpy arrays)."""
        arr = [np.ascontiguousarray(cfg[k], dtype=np.float32) for k in ("x", "y", "z")]
        arr += [np.ascontiguousarray(cfg[k], dtype=np.int32) for k in ("type", "state", "adj")]
        assert all(a.shape[0] == self.n for a in arr) and arr[5].shape[1] == self.B
        ptrs = [a.ctypes.data_as(C.c_void_p) for a in arr]
        _check(lib.pr_sys_load(self._h, *ptrs, 0))

    def load_device(self, x, y, z, type_, state, adj):
        _check(lib.pr_sys_load(self._h, _ptr(x), _ptr(y), _ptr(z), _ptr(type_), _ptr(state),
                               _ptr(adj), 1))

    def generate(self, kind, gen_seed, sigma0=0.1):
        _check(lib.pr_sys_generate(self._h, 0 if kind == "step" else 1, C.c_uint64(gen_seed),
                                   float(sigma0)))

    def run(self, first_step, n_steps, sigma):
        _check(lib.pr_sys_run(self._h, int(first_step), int(n_steps), float(sigma)))

    def run_timed(self, first_step, n_steps, sigma):
        ms = (C.c_float * 5)()
        _check(lib.pr_sys_run_timed(self._h, int(first_step), int(n_steps), float(sigma), ms))
        return {"prep_ms": ms[0], "step_ms": ms[1], "sweep_ms": ms[2], "sort_ms": ms[3],
                "sorts": int(ms[4])}

    def prepare(self, n_steps, sigma):
        """Capture the graphs a following run of n_steps will replay."""
        _check(lib.pr_sys_prepare(self._h, int(n_steps), float(sigma)))

    def jitter(self, first_step, n_steps, sigma, timed=False):
        """The re-jitter alone for n_steps steps; timed: returns the summed
        kernel time in ms."""
        ms = C.c_float(0.0)
        _check(lib.pr_sys_jitter(self._h, int(first_step), int(n_steps), float(sigma),
                                 C.byref(ms) if timed else None))
        return ms.value if timed else None

    def kinetics(self, nstate=8, nbins=16):
        """Kinetics counters of the current configuration: (pop, pairs, hist)
        int64 arrays (see pr_sys_kinetics)."""
        return _kinetics(lambda *a: lib.pr_sys_kinetics(self._h, *a), nstate, nbins)

    def set_md(self, theta, dt=0.0025, sig=1.0, eps=1.0, temp=1.0, vseed=0):
        """Velocity-Verlet MD with the mirror-LJ bond force, theta steps
        before each reaction step (theta = 0: back to the re-jitter)."""
        _check(lib.pr_sys_set_md(self._h, int(theta), float(dt), float(sig), float(eps),
                                 float(temp), C.c_uint64(vseed)))

    def velocities(self):
        v = [np.empty(self.n, np.float32) for _ in range(3)]
        _check(lib.pr_sys_read_velocities(self._h, *[a.ctypes.data_as(C.c_void_p) for a in v]))
        return v

    def set_sort_period(self, k):
        _check(lib.pr_sys_set_sort_period(self._h, int(k)))

    def set_graphs(self, on):
        _check(lib.pr_sys_set_graphs(self._h, 1 if on else 0))

    def set_fused_binning(self, on):
        _check(lib.pr_sys_set_fused_binning(self._h, 1 if on else 0))

    def fused_binning(self):
        v = C.c_int32(0)
        _check(lib.pr_sys_fused_binning(self._h, C.byref(v)))
        return bool(v.value)

    def read(self):
        n, B = self.n, self.B
        out = dict(x=np.empty(n, np.float32), y=np.empty(n, np.float32), z=np.empty(n, np.float32),
                   state=np.empty(n, np.int32), adj=np.empty((n, B), np.int32))
        _check(lib.pr_sys_read(self._h, *[out[k].ctypes.data_as(C.c_void_p)
                                           for k in ("x", "y", "z", "state", "adj")], 0))
        return out

    def bonds(self):
        n = C.c_int64(0)
        lib.pr_sys_bonds(self._h, None, 0, C.byref(n))
        total = n.value
        out = np.empty((max(total, 1), 3), np.int32)
        _check(lib.pr_sys_bonds(self._h, out.ctypes.data_as(C.c_void_p), total, C.byref(n)))
        return out[:total]

    def checkpoint(self):
        """The system's checkpoint (configuration, bond log, counters) as bytes."""
        n = C.c_int64(0)
        _check(lib.pr_sys_checkpoint(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib.pr_sys_checkpoint(self._h, buf, n.value, C.byref(n)))
        return buf.raw

    def restore(self, data):
        _check(lib.pr_sys_restore(self._h, data, len(data)))

    def stats(self):
        n = C.c_int64(0)
        _check(lib.pr_sys_stats(self._h, None, 0, C.byref(n)))
        arr = (Stats * max(n.value, 1))()
        _check(lib.pr_sys_stats(self._h, arr, n.value, C.byref(n)))
        return [arr[k].as_dict() for k in range(n.value)]


def _kinetics(call, nstate, nbins):
    pop, pairs = np.zeros(nstate, np.int64), np.zeros(nstate, np.int64)
    hist = np.zeros(max(nbins, 1), np.int64)
    _check(call(int(nstate), pop.ctypes.data_as(C.c_void_p), pairs.ctypes.data_as(C.c_void_p),
                int(nbins), hist.ctypes.data_as(C.c_void_p)))
    return pop, pairs, hist[:nbins]


def p_from_rate(k, dt, theta):
    """(p, warn): p = k dt Theta and whether it exceeds 0.1; ValueError on bad input."""
    w = C.c_int32(0)
    p = lib.pr_p_from_rate(float(k), float(dt), float(theta), C.byref(w))
    if p < 0.0:
        raise ValueError("k, dt and theta must be finite and >= 0")
    return p, bool(w.value)


def draws(ctr, key, stream=None):
    """Device Philox4x32-10 words of counters ctr (int32/uint32 tensor n x 4 on the device)."""
    import torch
    assert ctr.is_cuda and ctr.dtype in (torch.int32,) and ctr.dim() == 2 and ctr.shape[1] == 4
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    _check(lib.pr_draws(_ptr(ctr), ctr.shape[0], C.c_uint64(int(key)), _ptr(out),
                        _stream(stream)))
    return out


def sqrt_rn(t, stream=None):
    """The bonded-force kernel's square root of a float32 device tensor."""
    out = t.new_empty(t.shape)
    _check(lib.pr_sqrt_rn(_ptr(t), _ptr(out), t.numel(), _stream(stream)))
    return out


def stream_copy(src, dst, width=16, stream=None):
    """The library's copy kernel from tensor src to dst (same byte size);
    returns the kernel's duration in ms."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    ms = C.c_float(0.0)
    _check(lib.pr_stream_copy(_ptr(src), _ptr(dst), nbytes, int(width), _stream(stream),
                              C.byref(ms)))
    return ms.value


def replica_desc(r):
    """ReplicaDesc from a dict: n, L, B, rule, seed, kind, gen_seed, sigma0, log_cap
    and optionally brick (0 = 4)."""
    rule = r["rule"] if isinstance(r["rule"], Rule) else Rule.make(r["rule"])
    return ReplicaDesc(int(r["n"]), float(np.float32(r["L"])), int(r["B"]), rule, int(r["seed"]),
                       0 if r["kind"] == "step" else 1, int(r["gen_seed"]),
                       float(r.get("sigma0", 0.1)), int(r.get("log_cap", 0)),
                       int(r.get("brick", 0)))


def autotune(r, n_steps=128, sigma=0.05, copies=1, stream=None, cache=None):
    """Times the replica at every distinct brick edge on the device (pr_autotune),
    alone (copies = 1) or as one of `copies` identical replicas of a batch;
    with `cache` (a file path) a stored result for the same geometry is reused.
    Returns (best edge, {edge: microseconds per replica-step})."""
    d = replica_desc(r)
    best = C.c_int32(0)
    us = (C.c_float * 6)()
    if cache is None:
        _check(lib.pr_autotune(C.byref(d), int(n_steps), float(sigma), int(copies),
                               _stream(stream), C.byref(best), us))
    else:
        _check(lib.pr_autotune_cached(C.byref(d), int(n_steps), float(sigma), int(copies),
                                      _stream(stream), os.fsencode(cache), C.byref(best), us))
    return best.value, {b + 1: float(us[b]) for b in range(6) if us[b] >= 0.0}


def footprint(r, n_steps):
    b = C.c_int64(0)
    d = replica_desc(r)
    _check(lib.pr_footprint(C.byref(d), int(n_steps), C.byref(b)))
    return b.value


class Batch:
    """Batched ensemble of independent replicas (pr_batch_* entry points).

    ``reps``: list of dicts with n, L, B, rule (dict or Rule), seed, kind
    ('step' or 'chain', the synthetic start), gen_seed, sigma0 and log_cap."""

    def __init__(self, reps, stream=None):
        arr = (ReplicaDesc * len(reps))()
        for k, r in enumerate(reps):
            arr[k] = replica_desc(r)
        self.reps = [dict(r) for r in reps]
        self._h = C.c_void_p()
        _check(lib.pr_batch_create(C.byref(self._h), arr, len(reps), _stream(stream)))

    def close(self):
        if self._h:
            lib.pr_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, first_step, n_steps, sigma):
        _check(lib.pr_batch_run(self._h, int(first_step), int(n_steps), float(sigma)))

    def run_loop(self, first_step, n_steps, sigma):
        _check(lib.pr_batch_run_loop(self._h, int(first_step), int(n_steps), float(sigma)))

    def read(self, rep):
        n, B = int(self.reps[rep]["n"]), int(self.reps[rep]["B"])
        out = dict(x=np.empty(n, np.float32), y=np.empty(n, np.float32), z=np.empty(n, np.float32),
                   state=np.empty(n, np.int32), adj=np.empty((n, B), np.int32))
        _check(lib.pr_batch_read(self._h, int(rep), *[out[k].ctypes.data_as(C.c_void_p)
                                                      for k in ("x", "y", "z", "state", "adj")], 0))
        return out

    def bonds(self, rep):
        n = C.c_int64(0)
        lib.pr_batch_bonds(self._h, int(rep), None, 0, C.byref(n))
        total = n.value
        out = np.empty((max(total, 1), 3), np.int32)
        _check(lib.pr_batch_bonds(self._h, int(rep), out.ctypes.data_as(C.c_void_p), total,
                                  C.byref(n)))
        return out[:total]

    def kinetics(self, rep, nstate=8, nbins=16):
        return _kinetics(lambda *a: lib.pr_batch_kinetics(self._h, int(rep), *a), nstate, nbins)

    def stats(self, rep):
        n = C.c_int64(0)
        _check(lib.pr_batch_stats(self._h, int(rep), None, 0, C.byref(n)))
        arr = (Stats * max(n.value, 1))()
        _check(lib.pr_batch_stats(self._h, int(rep), arr, n.value, C.byref(n)))
        return [arr[k].as_dict() for k in range(n.value)]


class Server:
    """Request loop with continuous batching (pr_server_* entry points)."""

    QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, hbm_budget, max_slots, stream=None):
        self._h = C.c_void_p()
        s = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(lib.pr_server_create(C.byref(self._h), int(hbm_budget), int(max_slots), s))
        self._n = {}

    def close(self):
        if self._h:
            lib.pr_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, r, n_steps, sigma):
        d = replica_desc(r)
        t = C.c_uint64(0)
        _check(lib.pr_server_submit(self._h, C.byref(d), int(n_steps), float(sigma), C.byref(t)))
        self._n[t.value] = (int(r["n"]), int(r["B"]))
        return t.value

    def wait(self, ticket, timeout_s=0.0):
        st, code, lat = C.c_int32(0), C.c_int32(0), C.c_double(0)
        _check(lib.pr_server_wait(self._h, C.c_uint64(ticket), float(timeout_s), C.byref(st),
                                  C.byref(code), C.byref(lat)))
        return st.value, code.value, lat.value

    def poll(self, ticket):
        st, code, lat = C.c_int32(0), C.c_int32(0), C.c_double(0)
        _check(lib.pr_server_poll(self._h, C.c_uint64(ticket), C.byref(st), C.byref(code),
                                  C.byref(lat)))
        return st.value, code.value, lat.value

    def cancel(self, ticket):
        _check(lib.pr_server_cancel(self._h, C.c_uint64(ticket)))

    def bonds(self, ticket):
        n = C.c_int64(0)
        _check(lib.pr_server_bonds(self._h, C.c_uint64(ticket), None, 0, C.byref(n)))
        out = np.empty((max(n.value, 1), 3), np.int32)
        _check(lib.pr_server_bonds(self._h, C.c_uint64(ticket), out.ctypes.data_as(C.c_void_p),
                                   n.value, C.byref(n)))
        return out[: n.value]

    def read(self, ticket):
        n, B = self._n[ticket]
        out = dict(x=np.empty(n, np.float32), y=np.empty(n, np.float32), z=np.empty(n, np.float32),
                   state=np.empty(n, np.int32), adj=np.empty((n, B), np.int32))
        _check(lib.pr_server_read(self._h, C.c_uint64(ticket),
                                  *[out[k].ctypes.data_as(C.c_void_p)
                                    for k in ("x", "y", "z", "state", "adj")]))
        return out

    def stats(self, ticket):
        n = C.c_int64(0)
        _check(lib.pr_server_stats(self._h, C.c_uint64(ticket), None, 0, C.byref(n)))
        arr = (Stats * max(n.value, 1))()
        _check(lib.pr_server_stats(self._h, C.c_uint64(ticket), arr, n.value, C.byref(n)))
        return [arr[k].as_dict() for k in range(n.value)]

    def release(self, ticket):
        _check(lib.pr_server_release(self._h, C.c_uint64(ticket)))
        self._n.pop(ticket, None)

    def info(self):
        i = ServerInfo()
        _check(lib.pr_server_info_get(self._h, C.byref(i)))
        return i.as_dict()
