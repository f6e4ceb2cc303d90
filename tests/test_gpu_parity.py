"""HIP reaction step against the CPU oracle: bit-identical bonds, states,
adjacency, positions and counters on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import compare_step, gen, oracle_rule, oracle_system, random_cfg, say, to_dev
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1409_7498_amd import binding
    say("library", binding.lib.pr_version().decode())
    return binding


def _cfg_from_sys(s):
    return dict(L=s.L, x=s.x, y=s.y, z=s.z, type=s.type, state=s.state, adj=s.adj)


def _rule(kind, p, rc=1.12, excl=1):
    r = workload.rule_for(kind, rc, p)
    r["exclude_bonded"] = excl
    return r


# --- hand cases of the oracle pins, through the GPU -------------------------
HAND = [
    ("pair_in", 10.0, [(5, 5, 5), (6, 5, 5)], [1, 0], [4, 2]),
    ("pair_out", 10.0, [(5, 5, 5), (6.2, 5, 5)], [1, 0], [4, 2]),
    ("z_decides", 10.0, [(5, 5, 5), (5.7, 5.7, 5.6)], [1, 0], [4, 2]),
    ("periodic_x", 10.0, [(0.1, 5, 5), (9.5, 5, 5)], [1, 0], [4, 2]),
    ("periodic_yz", 10.0, [(5, 9.9, 0.2), (5, 0.3, 9.8)], [1, 0], [4, 2]),
    ("corner", 10.0, [(9.7, 9.7, 9.7), (0.2, 0.2, 0.2)], [1, 0], [4, 2]),
    ("two_a_one_t", 10.0, [(5, 5, 5), (6.8, 5, 5), (5.9, 5, 5)], [1, 1, 0], [4, 4, 2]),
    ("small_graph", 10.0, [(3.0, 5, 5), (4.8, 5, 5), (2.2, 5, 5), (3.9, 5, 5), (5.6, 5, 5)],
     [1, 1, 0, 0, 0], [4, 4, 2, 2, 2]),
    ("small_box", 2.3, [(0.1, 0.1, 0.1), (2.2, 0.2, 0.1), (1.1, 1.1, 1.1)], [1, 0, 0], [4, 2, 2]),
]


@pytest.mark.parametrize("case", HAND, ids=[c[0] for c in HAND])
@pytest.mark.parametrize("p", [1.0, 0.5])
def test_hand_cases(B, case, p):
    name, L, pts, types, states = case
    s = pins.mk(L, pts, types, states)
    for seed in range(20):
        compare_step(_cfg_from_sys(s), _rule("step", p), seed, 1 + seed, name)


def test_empty_and_single_particle(B):
    """No particles, and one lone A or T: no candidates, no bonds, the oracle agrees."""
    import torch
    z = torch.empty(0, dtype=torch.float32, device="cuda")
    zi = torch.empty(0, dtype=torch.int32, device="cuda")
    code, bonds, st = B.react_step(z, z, z, zi, zi, torch.empty((0, 4), dtype=torch.int32,
                                                                 device="cuda"),
                                   10.0, _rule("step", 1.0), 1, 1)
    assert code == B.PR_OK and bonds.shape[0] == 0 and all(v == 0 for v in st.values())
    for typ, state in ((1, 4), (0, 2)):
        s = pins.mk(10.0, [(5, 5, 5)], [typ], [state])
        g, st = compare_step(_cfg_from_sys(s), _rule("step", 1.0), 3, 1, "single")
        assert len(g) == 0 and st["in_rc"] == 0


def test_strict_cutoff(B):
    s = pins.mk(10.0, [(1, 1, 1), (2, 1, 1)], [1, 0], [4, 2])
    g, st = compare_step(_cfg_from_sys(s), _rule("step", 1.0, rc=1.0), 1, 1, "r2==rc2")
    assert len(g) == 0 and st["in_rc"] == 0
    rc_up = float(np.nextafter(np.float32(1.0), np.float32(2.0)))
    g, _ = compare_step(_cfg_from_sys(s), _rule("step", 1.0, rc=rc_up), 1, 1, "r2<rc2")
    assert len(g) == 1


def test_exclusion_and_overflow(B):
    adj = [[1, -1, -1, -1], [0, -1, -1, -1]]
    s = pins.mk(10.0, [(5, 5, 5), (5.8, 5, 5)], [1, 0], [3, 1], adj=adj)
    compare_step(_cfg_from_sys(s), _rule("step", 1.0, excl=1), 3, 1, "excluded")
    compare_step(_cfg_from_sys(s), _rule("step", 1.0, excl=0), 3, 1, "not excluded")
    s = pins.mk(10.0, [(5, 5, 5), (5.8, 5, 5)], [1, 0], [4, 2], B=1, adj=[[7], [-1]])
    compare_step(_cfg_from_sys(s), _rule("step", 1.0), 3, 1, "adj overflow")


def test_chain_transfer(B):
    s = pins.mk(10.0, [(2, 5, 5), (2.8, 5, 5), (3.6, 5, 5)], [0, 0, 0], [2, 0, 0], B=2)
    cfg = _cfg_from_sys(s)
    for step in (1, 2, 3):
        compare_step(cfg, _rule("chain", 1.0), 9, step, "chain%d" % step)
        o = oracle_system(cfg)
        oracle.react_step(o, oracle_rule(_rule("chain", 1.0)), 9, step)
        cfg = _cfg_from_sys(o)


# --- seeded workloads -------------------------------------------------------
@pytest.mark.parametrize("N,kind,p,seed", [
    (4000, "step", 0.01, 1), (4000, "step", 1.0, 2), (4000, "step", 0.0, 3),
    (4001, "step", 0.3, 4), (257, "step", 0.7, 5), (65, "step", 1.0, 6),
    (30000, "chain", 0.5, 7), (30011, "step", 0.05, 8), (1, "step", 1.0, 9),
])
def test_lattice_workloads(B, N, kind, p, seed):
    cfg = gen(N, workload.box_for(N) if N > 30 else 6.0, kind, seed)
    if kind == "chain" and N >= 30000:
        rng = np.random.default_rng(seed)
        cfg["state"][rng.choice(N, N // 20, replace=False)] = 2
    compare_step(cfg, _rule(kind, p), seed, 5, "lattice")


@pytest.mark.parametrize("N,kind,p,frac,seed", [
    (3000, "step", 1.0, 0.3, 11), (3000, "step", 0.2, 0.5, 12), (5000, "chain", 1.0, 0.2, 13),
    (2000, "step", 1.0, 0.05, 14),
])
def test_random_workloads(B, N, kind, p, frac, seed):
    """Uniform random positions: dense clusters, overflowing cell buckets."""
    L = workload.box_for(N)
    cfg = random_cfg(N, L, kind, seed, frac)
    compare_step(cfg, _rule(kind, p), seed, 2, "random")


def test_crowded_cell_overflow(B):
    """All A's packed into one corner: bucket overflow list and long scans."""
    rng = np.random.default_rng(5)
    N = 4000
    cfg = random_cfg(N, 20.0, "step", 5, frac=0.0)
    A = rng.choice(N, 300, replace=False)
    cfg["type"][A] = 1
    cfg["state"][A] = 4
    for v in ("x", "y", "z"):
        cfg[v][A] = rng.uniform(0.0, 2.0, A.size).astype(np.float32)
    compare_step(cfg, _rule("step", 1.0), 5, 3, "crowded")


def test_many_bonds_sort_in_hbm(B):
    """More than 4096 bonds in one step: the sort leaves LDS."""
    N = 150000
    cfg = gen(N, workload.box_for(N), "step", 21)
    g, st = compare_step(cfg, _rule("step", 1.0), 21, 1, "many bonds")
    assert st["bonds"] > 4096


def test_invalid_positions_leave_inputs(B):
    import torch
    cfg = gen(4000, 16.75, "step", 1)
    cfg["x"][17] = np.nan
    dev = to_dev(cfg)
    st0 = dev["state"].clone()
    code, bonds, _ = B.react_step(dev["x"], dev["y"], dev["z"], dev["type"], dev["state"],
                                  dev["adj"], cfg["L"], _rule("step", 1.0), 1, 1,
                                  raise_on_error=False)
    assert code == B.PR_EINVAL and bonds.shape[0] == 0
    assert torch.equal(dev["state"], st0) and bool((dev["adj"] == -1).all())
    cfg["x"][17] = np.float32(cfg["L"])
    dev = to_dev(cfg)
    code, _, _ = B.react_step(dev["x"], dev["y"], dev["z"], dev["type"], dev["state"], dev["adj"],
                              cfg["L"], _rule("step", 1.0), 1, 1, raise_on_error=False)
    assert code == B.PR_EINVAL


# --- resident system: generator, jitter and multi-step runs ------------------
def test_device_generator_matches_host(B):
    for N, L, kind, seed in ((4000, 16.75, "step", 5), (20000, workload.box_for(20000), "chain", 6),
                             (1000, workload.box_for(1000), "step", 7)):
        say("generator", N, kind)
        host = gen(N, L, kind, seed)
        r = _rule(kind, 0.01)
        s = B.System(N, L, 4 if kind == "step" else 2, r, seed)
        s.generate(kind, seed, 0.1)
        out = s.read()
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(out[k], host[k]), k
        s.close()


def _run_both(cfg, rule, seed, first, steps, sigma, sort_period=0, graphs=True):
    from paper_1409_7498_amd import binding
    n, Bw = len(cfg["x"]), cfg["adj"].shape[1]
    say("run_both", "n=%d steps=%d sort=%d graphs=%d" % (n, steps, sort_period, graphs))
    s = binding.System(n, cfg["L"], Bw, rule, seed, log_cap=8 * n)
    s.set_sort_period(sort_period)
    s.set_graphs(graphs)
    s.load(cfg)
    s.run(first, steps, sigma)
    out, log, st = s.read(), s.bonds(), s.stats()
    s.close()
    o = oracle_system(cfg)
    code, olog, ost = oracle.run(o, oracle_rule(rule), seed, first, steps, sigma)
    assert code == 0
    assert np.array_equal(log, olog), (log[:5], olog[:5])
    assert np.array_equal(out["x"], o.x) and np.array_equal(out["y"], o.y)
    assert np.array_equal(out["z"], o.z)
    assert np.array_equal(out["state"], o.state) and np.array_equal(out["adj"], o.adj)
    assert len(st) == steps
    for k, rec in enumerate(st):
        assert list(rec.values()) == ost[k].tolist(), (k, rec, ost[k])
    return log


@pytest.mark.parametrize("sort_period,graphs", [(0, False), (1, True), (16, True), (16, False),
                                               (0, True), (64, True)])
def test_c1_full_run(B, sort_period, graphs):
    c = workload.CONFIGS["c1"]
    cfg = gen(c.N, c.L, c.kind, c.seed)
    log = _run_both(cfg, c.rule(), c.seed, 1, c.steps, c.sigma, sort_period, graphs)
    assert len(log) > 200


@pytest.mark.parametrize("timed", [False, True])
@pytest.mark.parametrize("sort_period,graphs", [(64, True), (3, True), (0, False)])
def test_jitter_only_between_runs(B, timed, sort_period, graphs):
    """Reaction runs with re-jitter-only steps between them (an odd number,
    so the position parity the next run starts at flips): the same as the
    oracle taking the same steps, reaction and re-jitter alike."""
    from paper_1409_7498_amd import binding
    c = workload.CONFIGS["c1"]
    cfg = gen(c.N, c.L, c.kind, c.seed)
    rule = c.rule()
    s = binding.System(c.N, cfg["L"], cfg["adj"].shape[1], rule, c.seed, log_cap=8 * c.N)
    s.set_sort_period(sort_period)
    s.set_graphs(graphs)
    s.load(cfg)
    s.run(1, 7, c.sigma)
    s.jitter(8, 3, c.sigma, timed=timed)
    s.run(11, 9, c.sigma)
    s.jitter(20, 1, c.sigma, timed=timed)
    s.run(21, 4, c.sigma)
    out, log = s.read(), s.bonds()
    s.close()
    o = oracle_system(cfg)
    orule = oracle_rule(rule)
    logs = []
    for first, n, jit in ((1, 7, (8, 9, 10)), (11, 9, (20,)), (21, 4, ())):
        code, olog, _ = oracle.run(o, orule, c.seed, first, n, c.sigma)
        assert code == 0
        logs.append(olog)
        for step in jit:
            oracle.jitter(o, c.seed, step, c.sigma)
    olog = np.concatenate(logs)
    assert len(olog) > 20
    assert np.array_equal(log, olog), (len(log), len(olog))
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(out[k], getattr(o, k)), k


def test_log_ordered_in_place_between_runs(B):
    """Each read orders the bond log on the device, in place (Table I step 9:
    a step's bonds by id_A).  Reads between runs, whole and truncated, must
    leave the rows appended later intact: every read equals the oracle's log
    so far, and a truncated read is its prefix."""
    import ctypes as C
    c = workload.CONFIGS["c1"]
    cfg = gen(c.N, c.L, c.kind, c.seed)
    rule = _rule("step", 0.2)
    s = B.System(c.N, c.L, 4, rule, c.seed, log_cap=8 * c.N)
    s.load(cfg)
    o = oracle_system(cfg)
    orule = oracle_rule(rule)
    logs, first = [], 1
    for n in (5, 1, 9, 3):
        s.run(first, n, c.sigma)
        code, olog, _ = oracle.run(o, orule, c.seed, first, n, c.sigma)
        assert code == 0
        logs.append(olog)
        first += n
        want = np.concatenate(logs)
        half = len(want) // 2
        part = np.empty((max(half, 1), 3), np.int32)
        got_n = C.c_int64(0)
        assert B.lib.pr_sys_bonds(s._h, part.ctypes.data_as(C.c_void_p), half,
                                  C.byref(got_n)) == 0
        assert got_n.value == len(want)
        assert np.array_equal(part[:half], want[:half])
        assert np.array_equal(s.bonds(), want), (first, len(want))
    assert len(want) > 50
    s.close()


@pytest.mark.parametrize("sort_period", [1000, 5])
def test_a_list_growth_and_compaction(B, sort_period):
    """Chain growth with half the particles active and p = 1: the A list gains
    an entry per bond; with rare sorts it must be compacted in place."""
    N = 4000
    cfg = gen(N, workload.box_for(N), "chain", 61)
    cfg["state"][np.random.default_rng(61).choice(N, N // 2, replace=False)] = 2
    _run_both(cfg, _rule("chain", 1.0), 61, 1, 30, 0.05, sort_period)


@pytest.mark.parametrize("sort_period", [1000, 3, 0])
def test_window_reentry_rule(B, sort_period):
    """A rule under which particles leave and re-enter the A window between
    sorts (A: state 2 -> 1, T: state 0/1 -> +1): no duplicate A entries."""
    N = 4000
    rng = np.random.default_rng(71)
    cfg = gen(N, workload.box_for(N), "chain", 71)
    cfg["state"] = rng.integers(0, 3, N).astype(np.int32)
    cfg["adj"] = np.full((N, 32), -1, np.int32)
    rule = dict(type_a=0, a_min=2, a_max=2, d_a=-1, type_t=0, t_min=0, t_max=1, d_t=1,
                rc=1.12, p=0.5, exclude_bonded=1)
    _run_both(cfg, rule, 71, 1, 25, 0.05, sort_period)


@pytest.mark.parametrize("sort_period", [0, 10])
def test_chain_run(B, sort_period):
    N = 20000
    cfg = gen(N, workload.box_for(N), "chain", 31)
    rng = np.random.default_rng(31)
    cfg["state"][rng.choice(N, 200, replace=False)] = 2
    _run_both(cfg, _rule("chain", 0.2), 31, 1, 60, 0.05, sort_period)


@pytest.mark.parametrize("N,kind,p,period", [(65536, "step", 0.02, 8), (40000, "step", 0.3, 3),
                                             (50000, "chain", 0.5, 5)])
def test_mid_size_runs(B, N, kind, p, period):
    """Several bricks per side, ragged last brick, many sorts and drifts."""
    cfg = gen(N, workload.box_for(N), kind, 50 + N)
    if kind == "chain":
        rng = np.random.default_rng(N)
        cfg["state"][rng.choice(N, N // 50, replace=False)] = 2
    _run_both(cfg, _rule(kind, p), 50 + N, 1, 12, 0.05, period)


def test_run_resume_equals_uninterrupted(B):
    from paper_1409_7498_amd import binding
    c = workload.CONFIGS["c1"]
    cfg = gen(c.N, c.L, c.kind, c.seed)
    a = binding.System(c.N, c.L, 4, c.rule(), c.seed, log_cap=4 * c.N)
    a.load(cfg)
    a.run(1, 60, c.sigma)
    ra, la = a.read(), a.bonds()
    b = binding.System(c.N, c.L, 4, c.rule(), c.seed, log_cap=4 * c.N)
    b.load(cfg)
    b.run(1, 25, c.sigma)
    mid = b.read()
    mid["type"] = cfg["type"]
    part = b.bonds()
    b.load(mid)
    b.run(26, 35, c.sigma)
    rb, lb = b.read(), np.concatenate([part, b.bonds()])
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(ra[k], rb[k])
    assert np.array_equal(la, lb)


def test_repeat_runs_identical(B):
    c = workload.CONFIGS["c1"]
    cfg = gen(c.N, c.L, c.kind, c.seed)
    logs = []
    for _ in range(3):
        s = B.System(c.N, c.L, 4, _rule("step", 0.2), c.seed, log_cap=4 * c.N)
        s.load(cfg)
        s.run(1, 50, c.sigma)
        logs.append(s.bonds())
        s.close()
    assert all(np.array_equal(logs[0], l) for l in logs[1:])


def test_workspace_box_changes(B):
    """Stateless calls with shrinking then growing boxes share one workspace;
    cells left by a larger grid must not leak into a later call."""
    for N, seed in ((30000, 41), (2000, 42), (4000, 43), (30000, 44), (500, 45), (9000, 46)):
        cfg = gen(N, workload.box_for(N), "step", seed)
        compare_step(cfg, _rule("step", 1.0), seed, 2, "box N=%d" % N)


def test_dense_brick_queue_overflow_and_deferral(B):
    """One brick packed with four A's per cell (256 records: still staged),
    the 543 T's in it with about 1000 partners in all (the oracle counts
    them): one pass queues more pairs than the queue holds, so the surplus
    T's are deferred with none of their pairs, and 15 T's with more than four
    partners are deferred as well; the rest of the box has no A."""
    N = 40000
    cfg = gen(N, workload.box_for(N), "step", 91)
    L = cfg["L"]
    nc = int(np.floor(L / (2 * 1.12 * (1 + 1 / 1024))))
    w = L / nc
    rng = np.random.default_rng(91)
    cfg["type"][:] = 0
    cfg["state"][:] = 2
    cells = [(cx, cy, cz) for cz in range(4, 8) for cy in range(4, 8) for cx in range(4, 8)]
    A = rng.choice(N, 4 * len(cells), replace=False)
    for q, (cx, cy, cz) in enumerate(np.repeat(np.array(cells), 4, axis=0)):
        i = A[q]
        cfg["type"][i], cfg["state"][i] = 1, 4
        for v, c in (("x", cx), ("y", cy), ("z", cz)):
            cfg[v][i] = np.float32((c + rng.uniform(0.05, 0.95)) * w)
    _run_both(cfg, _rule("step", 1.0), 91, 1, 3, 0.05, 64)


@pytest.mark.parametrize("frac", [0.12, 0.2])
def test_a_rich_mixes_staged_and_unstaged_bricks(B, frac):
    """About 250 A records per brick region at 12% A's: some workgroups stage
    their region, the others scan every T in the global buckets, in one step."""
    N = 40000
    cfg = gen(N, workload.box_for(N), "step", 93)
    rng = np.random.default_rng(93)
    pick = rng.random(N) < frac
    cfg["type"] = pick.astype(np.int32)
    cfg["state"] = np.where(pick, 4, 2).astype(np.int32)
    _run_both(cfg, _rule("step", 0.3), 93, 1, 6, 0.05, 3)
