"""Full-size workloads in the launch configuration the benchmark times.

The oracle cannot run whole 1M/4M-particle steps in test time, so these tests
check (1) the device-generated configuration and the jittered positions
element by element, (2) the first step's bonds of a sample of active
particles one by one with the oracle's sampled form of the algorithm, and
(3) after many steps, properties that hold at any size (one bond per particle
per step, valence bookkeeping, symmetric adjacency, positions identical to the
oracle's jitter, counters consistent)."""
import numpy as np
import pytest

import oracle
from gpu_util import oracle_rule, say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _system(B, c, steps_after=0):
    s = B.System(c.N, c.L, c.B, c.rule(), c.seed, log_cap=2 * c.N)
    s.generate(c.kind, c.seed, workload.SIGMA_LATTICE)
    return s


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_first_step_sampled(name):
    from paper_1409_7498_amd import binding as B
    c = workload.CONFIGS[name]
    say("full size", c)
    s = _system(B, c)
    s.run(1, 1, c.sigma)
    out, log, st = s.read(), s.bonds(), s.stats()
    s.close()
    host = workload.generate(c.N, c.L, c.kind, c.seed)
    o = oracle.System(host["L"], host["x"], host["y"], host["z"], host["type"], host["state"],
                      host["adj"])
    oracle.jitter(o, c.seed, 1, c.sigma)
    for k in ("x", "y", "z"):
        assert np.array_equal(out[k], getattr(o, k)), k
    rule = oracle_rule(c.rule())
    isA = (o.type == rule.type_a) & (o.state >= rule.a_min) & (o.state <= rule.a_max)
    isT = (o.type == rule.type_t) & (o.state >= rule.t_min) & (o.state <= rule.t_max)
    assert st[0]["a_elig"] == int(isA.sum()) and st[0]["t_elig"] == int(isT.sum())
    assert st[0]["bonds"] == len(log) > 0
    gpu_partner = {int(i): int(j) for _, i, j in log.tolist()}
    rng = np.random.default_rng(7)
    A = np.nonzero(isA)[0]
    sample = np.unique(np.concatenate([rng.choice(A, 120, replace=False),
                                       rng.choice(log[:, 1], min(120, len(log)), replace=False)]))
    say("sampling", len(sample), "active particles with the oracle")
    ref = oracle.sample_bonds(o, rule, c.seed, 1, sample)
    got = np.array([gpu_partner.get(int(i), -1) for i in sample])
    assert np.array_equal(got, ref), np.nonzero(got != ref)
    assert (ref >= 0).sum() >= 100


@pytest.mark.parametrize("name,steps", [("c2", 200), ("c3", 100)])
def test_many_steps_invariants(name, steps):
    from paper_1409_7498_amd import binding as B
    c = workload.CONFIGS[name]
    s = _system(B, c)
    s.run(1, steps, c.sigma)
    out, log, st = s.read(), s.bonds(), s.stats()
    s.close()
    host = workload.generate(c.N, c.L, c.kind, c.seed)
    say("invariants", name, "bonds", len(log))
    assert len(st) == steps and sum(r["bonds"] for r in st) == len(log)
    # one new bond per particle per step, ids sorted by id_A within a step
    for s_ in np.unique(log[:, 0]):
        rows = log[log[:, 0] == s_]
        ids = np.concatenate([rows[:, 1], rows[:, 2]])
        assert np.unique(ids).size == ids.size
        assert np.all(np.diff(rows[:, 1]) > 0)
    deg = np.bincount(np.concatenate([log[:, 1], log[:, 2]]), minlength=c.N)
    pairs = set(map(tuple, np.sort(log[:, 1:], axis=1).tolist()))
    assert len(pairs) == len(log), "a pair bonded twice"
    if c.kind == "step":
        assert np.array_equal(host["state"] - out["state"], deg)
        assert np.all(host["type"][log[:, 1]] == 1) and np.all(host["type"][log[:, 2]] == 0)
    else:
        # chain growth: a free monomer bonds first as T (0 -> 2, one bond) then
        # as A (2 -> 1, two bonds); an initiator bonds once, as A (2 -> 1)
        st0, st1 = host["state"], out["state"]
        assert np.all(np.isin(st1, [0, 1, 2]))
        expect = np.where(st0 == 0, np.select([st1 == 0, st1 == 2, st1 == 1], [0, 1, 2]),
                          np.where(st1 == 1, 1, 0))
        assert np.all((st0 == 0) | (st1 != 0))
        assert np.array_equal(deg, expect)
    adj = out["adj"]
    assert np.array_equal((adj >= 0).sum(1), deg)
    rows = np.repeat(np.arange(c.N), adj.shape[1])
    flat = adj.ravel()
    m = flat >= 0
    fwd = set(zip(rows[m].tolist(), flat[m].tolist()))
    assert all((j, i) in fwd for i, j in fwd)
    # positions depend only on the jitter: identical to the oracle's
    o = oracle.System(host["L"], host["x"], host["y"], host["z"], host["type"], host["state"],
                      host["adj"])
    for k in range(1, steps + 1):
        oracle.jitter(o, c.seed, k, c.sigma)
    for k in ("x", "y", "z"):
        assert np.array_equal(out[k], getattr(o, k)), k


def test_storage_order_does_not_change_results():
    """Sorted storage (any period) and unsorted storage give identical runs."""
    from paper_1409_7498_amd import binding as B
    c = workload.Config("mid", 262144, workload.box_for(262144), "step", 0.02, 60,
                        workload.MASTER_SEED + 9)
    logs, outs = [], []
    for period in (0, 1, 7, 64):
        say("sort period", period)
        s = _system(B, c)
        s.set_sort_period(period)
        s.run(1, c.steps, c.sigma)
        logs.append(s.bonds())
        outs.append(s.read())
        s.close()
    for l, o in zip(logs[1:], outs[1:]):
        assert np.array_equal(l, logs[0])
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(o[k], outs[0][k])
