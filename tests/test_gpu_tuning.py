"""The brick edge is a tuning choice only: the storage is sorted by bricks of
brick^3 coarse cells and the sweep runs one workgroup per brick, but every
result (bonds, states, adjacency, positions, counters) must be identical for
every brick edge, alone and in a batch.  The autotuner times the distinct
edges on the device and returns the fastest."""
import time

import numpy as np
import pytest

from gpu_util import say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _desc(n, kind, p, seed, brick=0):
    return dict(n=n, L=workload.box_for(n), B=4 if kind == "step" else 2,
                rule=workload.rule_for(kind, workload.RC, p), seed=seed, kind=kind,
                gen_seed=seed + 5, sigma0=0.1, log_cap=4 * n, brick=brick)


def _run(B, d, steps, brick):
    s = B.System(d["n"], d["L"], d["B"], d["rule"], d["seed"], log_cap=d["log_cap"], brick=brick)
    s.generate(d["kind"], d["gen_seed"], d["sigma0"])
    geo = s.geometry()
    s.run(1, steps, workload.SIGMA_JITTER)
    out = (s.read(), s.bonds(), s.stats())
    s.close()
    return geo, out


def _same(a, b, label):
    assert np.array_equal(a[1], b[1]), label
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(a[0][k], b[0][k]), (label, k)
    assert a[2] == b[2], label


@pytest.mark.parametrize("kind,p", [("step", 0.05), ("chain", 0.3)])
def test_results_identical_for_every_brick(kind, p):
    from paper_1409_7498_amd import binding as B
    d = _desc(20000, kind, p, workload.MASTER_SEED + 70)
    steps = 130  # crosses the sorts at steps 65 and 129
    ref_geo, ref = _run(B, d, steps, 4)
    say("brick 4", ref_geo, "bonds", len(ref[1]))
    assert len(ref[1]) > 0
    seen = {ref_geo[:2]}
    for brick in (1, 2, 3, 5, 6):
        geo, out = _run(B, d, steps, brick)
        say("brick", brick, geo)
        assert geo[1] == brick
        seen.add(geo[:2])
        _same(out, ref, "brick %d" % brick)
    assert len(seen) == 6  # six decompositions (12 cells per side) were compared


def test_small_box_clamps_brick():
    """A box of few coarse cells clamps the brick edge to nc - 2."""
    from paper_1409_7498_amd import binding as B
    d = _desc(2000, "step", 0.05, workload.MASTER_SEED + 71)
    geo4, out4 = _run(B, d, 70, 4)
    nc = geo4[0]
    assert geo4[1] == min(4, nc - 2)
    geo1, out1 = _run(B, d, 70, 1)
    assert geo1[1] == 1
    _same(out1, out4, "clamped")


def test_autotune_and_tuned_batch():
    from paper_1409_7498_amd import binding as B
    descs = [_desc(n, kind, 0.02, workload.MASTER_SEED + 72 + i)
             for i, (n, kind) in enumerate([(3000, "step"), (12000, "chain"), (40000, "step")])]
    tuned = []
    for d in descs:
        best, us = B.autotune(d, 128, workload.SIGMA_JITTER)
        say("autotune n=%d" % d["n"], best, us)
        assert best in us and us[best] == min(us.values())
        assert all(t > 0 for t in us.values())
        bb, ub = B.autotune(d, 64, workload.SIGMA_JITTER, copies=8)
        say("autotune in a batch of 8", bb, ub)
        assert bb in ub and ub[bb] == min(ub.values())
        tuned.append(dict(d, brick=bb))
    # mixed bricks in one batch: every replica equals itself alone at the default edge
    mixed = [dict(d, brick=b) for d, b in zip(descs, (1, 2, 3))] + tuned
    bt = B.Batch(mixed)
    bt.run(1, 100, workload.SIGMA_JITTER)
    for r, d in enumerate(mixed):
        _, ref = _run(B, d, 100, 0)
        _same((bt.read(r), bt.bonds(r), bt.stats(r)), ref, "replica %d brick %d" % (r, d["brick"]))
    bt.close()


def test_autotune_cache(tmp_path):
    """A miss tunes and appends one line; a hit for the same geometry returns
    the stored choice and times without timing again; another geometry misses."""
    from paper_1409_7498_amd import binding as B
    cache = str(tmp_path / "tune.txt")
    d = _desc(20000, "step", 0.02, workload.MASTER_SEED + 80)
    best, us = B.autotune(d, 64, workload.SIGMA_JITTER, cache=cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("pr-tune 2 ")
    t0 = time.time()
    best2, us2 = B.autotune(dict(d, seed=d["seed"] + 1), 64, workload.SIGMA_JITTER, cache=cache)
    assert time.time() - t0 < 0.5
    assert best2 == best and set(us2) == set(us)
    assert all(abs(us2[b] - us[b]) < 1e-3 * max(1.0, us[b]) for b in us)
    B.autotune(_desc(3000, "step", 0.02, workload.MASTER_SEED + 81), 64, workload.SIGMA_JITTER,
               cache=cache)
    assert len(open(cache).read().splitlines()) == 2
