"""Fused binning on sorted storage (each step's sweep bins the next step's A
records, the resolve drops and adds those its bonds change): bit-identical
to the oracle, and to the same handle with the binning kernel, through drift
far beyond the staged regions, chain growth that turns T's into A's every
step, bricks and cells with more A's than a workgroup stages or a bucket
holds, every brick edge, and runs that do not continue the previous one."""
import numpy as np
import pytest

import oracle
from gpu_util import gen, oracle_rule, oracle_system, say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1409_7498_amd import binding
    return binding


def _rule(kind, p, rc=1.12):
    r = workload.rule_for(kind, rc, p)
    r["exclude_bonded"] = 1
    return r


def _chain(N, seed, active):
    cfg = gen(N, workload.box_for(N), "chain", seed)
    rng = np.random.default_rng(seed)
    cfg["state"][rng.choice(N, active, replace=False)] = 2
    return cfg


def _runs(B, cfg, rule, seed, runs, sort_period, fused=True, brick=0):
    """Runs (first, steps, sigma) one after the other on one handle and on the
    oracle; asserts identical logs, configurations and counters after each."""
    n, Bw = len(cfg["x"]), cfg["adj"].shape[1]
    s = B.System(n, cfg["L"], Bw, rule, seed, log_cap=16 * n, brick=brick)
    s.set_sort_period(sort_period)
    s.set_fused_binning(fused)
    s.load(cfg)
    o = oracle_system(cfg)
    orule = oracle_rule(rule)
    nlog = 0
    for first, steps, sigma in runs:
        say("fused-binning run n=%d first=%d steps=%d sigma=%g period=%d fused=%d brick=%d"
            % (n, first, steps, sigma, sort_period, fused, brick))
        s.run(first, steps, sigma)
        if sort_period > 0:
            assert s.fused_binning() == fused
        code, olog, ost = oracle.run(o, orule, seed, first, steps, sigma)
        assert code == 0
        log, out, st = s.bonds(), s.read(), s.stats()
        assert np.array_equal(log[nlog:], olog), (log[nlog:nlog + 5], olog[:5])
        nlog = len(log)
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(out[k], getattr(o, k)), k
        for k, rec in enumerate(st[-steps:]):
            assert list(rec.values()) == ost[k].tolist(), (k, rec, ost[k])
    s.close()
    return nlog


@pytest.mark.parametrize("fused", [True, False])
def test_drift_far_from_the_sort(B, fused):
    """sigma 0.4 per step and no sort after the first: after 40 steps the
    particles have moved about 2.5 (one cell of width 2.24 and more), so many
    T's leave their brick's staged region."""
    N = 20000
    cfg = gen(N, workload.box_for(N), "step", 201)
    _runs(B, cfg, _rule("step", 0.05), 201, [(1, 40, 0.4)], 1000, fused)


def test_chain_growth_moves_the_a_role(B):
    """Chain growth with 10% active ends and p = 1: each bond ends one A and
    makes its T the new active end, so the resolve drops and adds many A
    records every step."""
    N = 30000
    cfg = _chain(N, 203, N // 10)
    n = _runs(B, cfg, _rule("chain", 1.0), 203, [(1, 25, 0.05)], 1000)
    assert n > N // 10


def test_a_rich_bricks_fall_back(B):
    """Half the particles are A's: about 300 per brick, more than one
    workgroup stages or keeps for the next step's records, and about 5 per
    cell, so some buckets overflow."""
    N = 20000
    cfg = gen(N, workload.box_for(N), "step", 205)
    rng = np.random.default_rng(205)
    pick = rng.random(N) < 0.5
    cfg["type"] = pick.astype(np.int32)
    cfg["state"] = np.where(pick, 4, 2).astype(np.int32)
    _runs(B, cfg, _rule("step", 0.2), 205, [(1, 6, 0.05)], 3)


def test_runs_that_do_not_continue(B):
    """A run that continues the last one reuses the binned records; another
    first step or another sigma sorts first.  Every run matches the oracle."""
    N = 20000
    cfg = _chain(N, 207, 400)
    runs = [(1, 10, 0.05), (11, 7, 0.05), (40, 9, 0.05), (49, 6, 0.1), (55, 70, 0.1)]
    _runs(B, cfg, _rule("chain", 0.3), 207, runs, 16)


@pytest.mark.parametrize("brick", [1, 2, 3, 5, 6])
def test_brick_edges(B, brick):
    """N = 40000: 16 cells per side, bricks of one to six cells (the last one
    of a side ragged for edges 3 and 5)."""
    N = 40000
    cfg = gen(N, workload.box_for(N), "step", 209)
    nc = int(np.floor(cfg["L"] / (2 * 1.12 * (1 + 1 / 1024))))
    assert nc == 16
    _runs(B, cfg, _rule("step", 0.1), 209, [(1, 12, 0.1)], 5, brick=brick)


def test_few_bricks_per_side(B):
    """Two bricks per side (7 cells, edge 4) and three (5 cells, edge 2, the
    last of one cell): regions that wrap around the box."""
    for N, seed, brick in ((4000, 211, 0), (1500, 212, 2)):
        cfg = gen(N, workload.box_for(N), "step", seed)
        _runs(B, cfg, _rule("step", 0.2), seed, [(1, 30, 0.2)], 7, brick=brick)


def test_toggle_mid_run(B):
    """Fused binning switched off and on between runs of one handle."""
    N = 20000
    cfg = _chain(N, 213, 300)
    n, Bw = N, cfg["adj"].shape[1]
    rule = _rule("chain", 0.5)
    s = B.System(n, cfg["L"], Bw, rule, 213, log_cap=16 * n)
    s.set_sort_period(16)
    s.load(cfg)
    o = oracle_system(cfg)
    first = 1
    for on in (True, False, True, False):
        s.set_fused_binning(on)
        s.run(first, 20, 0.05)
        assert s.fused_binning() == on
        code, olog, _ = oracle.run(o, oracle_rule(rule), 213, first, 20, 0.05)
        first += 20
    assert np.array_equal(s.read()["adj"], o.adj)
    s.close()
