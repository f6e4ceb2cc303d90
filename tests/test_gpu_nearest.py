"""The "nearest" selection of LAMMPS fix bond/create (Sec. IV A) on the GPU
against the CPU oracle's or_react_step_nearest / or_run_nearest: bonds,
states, adjacency, positions and counters identical, for the stateless step,
resident runs (graphs, spatial sorts, re-jitter), sort-period invariance and
a batch that mixes both selection policies."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_step, gen, oracle_rule, oracle_system, random_cfg, say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _rule(kind, p):
    return workload.rule_for(kind, workload.RC, p, policy="nearest")


@pytest.mark.parametrize("kind,p,seed", [("step", 1.0, 1), ("step", 0.3, 2), ("step", 0.01, 3),
                                         ("chain", 1.0, 4), ("chain", 0.5, 5)])
def test_step_equals_oracle(kind, p, seed):
    cfg = gen(4000, 16.75, kind, seed)
    if kind == "chain":
        cfg["state"][np.random.default_rng(seed).choice(4000, 300, replace=False)] = 2
    g, st = compare_step(cfg, _rule(kind, p), seed, 3, "nearest %s p=%g" % (kind, p))
    if p >= 0.3:
        assert len(g) > 0 and st["drawn"] >= st["bonds"]


def test_step_crowded_cells():
    """Clustered random positions with 30% A's: bucket overflow lists."""
    cfg = random_cfg(6000, 9.0, "step", 21, frac=0.3)
    compare_step(cfg, _rule("step", 0.7), 21, 5, "nearest crowded")


def _run_gpu(c, rule, steps, sort_period=None):
    from paper_1409_7498_amd import binding as B
    s = B.System(c.N, c.L, c.B, rule, c.seed, log_cap=4 * c.N)
    if sort_period is not None:
        s.set_sort_period(sort_period)
    s.generate(c.kind, c.gen_seed, workload.SIGMA_LATTICE)
    s.run(1, steps, c.sigma)
    out = (s.read(), s.bonds(), s.stats())
    s.close()
    return out


def _run_oracle(c, rule, steps):
    g = c.initial()
    o = oracle_system(g)
    code, log, st = oracle.run(o, oracle_rule(rule), c.seed, 1, steps, c.sigma)
    assert code == 0
    return o, log, st


@pytest.mark.parametrize("N,kind,p,steps", [(4000, "step", 0.01, 200), (4000, "step", 0.2, 60),
                                            (65536, "step", 0.05, 40), (100000, "chain", 0.3, 50)])
def test_run_equals_oracle(N, kind, p, steps):
    c = workload.Config("near%d" % N, N, 16.75 if N == 4000 else workload.box_for(N), kind, p,
                        steps, workload.MASTER_SEED + 60 + N % 97)
    rule = _rule(kind, p)
    say("nearest run", c)
    out, log, st = _run_gpu(c, rule, steps)
    o, olog, ost = _run_oracle(c, rule, steps)
    assert np.array_equal(log, olog), (len(log), len(olog))
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(out[k], getattr(o, k)), k
    got = np.array([[r[f] for f in oracle.ST_NAMES] for r in st])
    assert np.array_equal(got, ost)
    assert len(log) > 0
    say("identical:", len(log), "bonds")


@pytest.mark.parametrize("frac,B,sort_period", [(0.3, 4, 64), (0.3, 6, 64), (0.05, 6, 5)])
def test_resident_a_rich_and_wide_rows(frac, B, sort_period):
    """Resident runs on sorted storage (the staged sweep): uniformly random
    positions with many A's (regions over the staging capacity and crowded
    cells: the global-bucket paths) and adjacency rows wider than four (the
    exclusion read from the particle arrays), against the oracle."""
    from paper_1409_7498_amd import binding as Bn
    N, L, seed, steps = 30000, 33.0, 90 + B, 24
    cfg = random_cfg(N, L, "step", seed, frac=frac)
    cfg["adj"] = np.full((N, B), -1, np.int32)
    rule = _rule("step", 0.4)
    say("nearest resident", "frac=%g B=%d sort=%d" % (frac, B, sort_period))
    s = Bn.System(N, cfg["L"], B, rule, seed, log_cap=4 * N)
    s.set_sort_period(sort_period)
    s.load(cfg)
    s.run(1, steps, 0.05)
    out, log = s.read(), s.bonds()
    s.close()
    o = oracle_system(cfg)
    code, olog, _ = oracle.run(o, oracle_rule(rule), seed, 1, steps, 0.05)
    assert code == 0
    assert len(olog) > 100
    assert np.array_equal(log, olog), (len(log), len(olog))
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(out[k], getattr(o, k)), k


def test_sort_period_invariance():
    c = workload.Config("nearsort", 262144, workload.box_for(262144), "step", 0.05, 70,
                        workload.MASTER_SEED + 70)
    rule = _rule("step", 0.05)
    ref = _run_gpu(c, rule, c.steps, sort_period=0)
    for period in (1, 7, 64):
        got = _run_gpu(c, rule, c.steps, sort_period=period)
        assert np.array_equal(got[1], ref[1]), period
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(got[0][k], ref[0][k]), (period, k)


def test_batch_mixes_policies():
    """Replicas of both policies in one batch equal each replica run alone,
    and the small ones equal the oracle."""
    from paper_1409_7498_amd import binding as B
    rng = np.random.default_rng(5)
    cfgs = []
    for r in range(8):
        N = int(rng.integers(800, 9000))
        kind = "step" if r % 2 == 0 else "chain"
        pol = "nearest" if (r // 2) % 2 == 0 else "random"
        c = workload.Config("mix%d" % r, N, workload.box_for(N), kind, float(rng.uniform(0.02, 0.4)),
                            48, workload.MASTER_SEED + 80 + r)
        cfgs.append((c, workload.rule_for(kind, workload.RC, c.p, policy=pol)))
    descs = [dict(c.desc(log_cap=4 * c.N), rule=rule) for c, rule in cfgs]
    bt = B.Batch(descs)
    bt.run(1, 48, workload.SIGMA_JITTER)
    for r, (c, rule) in enumerate(cfgs):
        log = bt.bonds(r)
        out = bt.read(r)
        o, olog, _ = _run_oracle(c, rule, 48)
        assert np.array_equal(log, olog), (r, rule["policy"])
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(out[k], getattr(o, k)), (r, k)
    bt.close()
