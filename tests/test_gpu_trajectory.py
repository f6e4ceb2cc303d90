"""Whole trajectories against stored oracle digests.

The CPU oracle is too slow to run 1M- and 4M-particle trajectories inside a
test, so tests/golden/make_digests.py ran it once, here on the CPU, and
stored per step the nine counters and the digest of the step's bond rows
(Table I, steps 1-9, iterated with the re-jitter between steps), and the
digest of the final positions, states and adjacency.  These tests run the
same workloads on the GPU in the configuration the benchmark times
(resident systems replayed from captured graphs, storage re-sorted every 64
steps; the batched ensemble; the served stream) and compare every step,
every replica and every sampled request.  Nothing here computes a reference:
the stored values come from the oracle alone."""
import os
import sys

import numpy as np
import pytest

from gpu_util import say
from paper_1409_7498_amd import workload

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import digest  # noqa: E402

pytestmark = pytest.mark.gpu


def _stat_rows(st):
    return [tuple(int(d[k]) for k in digest.STAT_NAMES) for d in st]


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_trajectory_matches_oracle(name):
    from paper_1409_7498_amd import binding as B
    header, ref, fin = digest.read_traj(os.path.join(HERE, "golden", "traj_%s.txt" % name))
    c = workload.CONFIGS[name]
    steps = max(ref)
    assert sorted(ref) == list(range(1, steps + 1))
    say("trajectory", name, c, "steps 1..%d" % steps)
    s = B.System(c.N, c.L, c.B, c.rule(), c.seed, log_cap=2 * c.N)
    s.generate(c.kind, c.gen_seed, workload.SIGMA_LATTICE)
    s.run(1, steps, c.sigma)
    log, st, out = s.bonds(), s.stats(), s.read()
    s.close()
    got = digest.step_digests(log, 1, steps)
    rows = _stat_rows(st)
    assert len(rows) == steps
    for k in range(1, steps + 1):
        want_st, want_dg = ref[k]
        assert rows[k - 1] == want_st, ("counters differ at step", k, rows[k - 1], want_st)
        assert got[k][1] == want_dg, ("bonds differ at step", k, got[k])
    f = digest.config_digests(out["x"], out["y"], out["z"], out["state"], out["adj"])
    assert f == fin, (f, fin)
    say(name, "identical to the oracle on all", steps, "steps,", len(log), "bonds")


def _read_ensemble(path):
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            rows.append(dict(index=int(p[0]), name=p[1], N=int(p[2]), kind=p[3], steps=int(p[5]),
                             bonds=int(p[6]), log=p[7], stats=p[8], pos=p[9], state=p[10],
                             adj=p[11]))
    return rows


def _replica_digests(log, st, out):
    f = digest.config_digests(out["x"], out["y"], out["z"], out["state"], out["adj"])
    return dict(bonds=len(log), log=digest.h16(np.ascontiguousarray(log, np.int32)),
                stats=digest.h16(np.asarray(_stat_rows(st), np.int64)), **f)


def _check_rows(rows, got, what):
    bad = []
    for r, g in zip(rows, got):
        want = {k: r[k] for k in ("bonds", "log", "stats", "pos", "state", "adj")}
        if g != want:
            bad.append((r["index"], r["name"], r["N"], r["kind"], g, want))
    assert not bad, (what, len(bad), bad[:3])


def test_ensemble_matches_oracle():
    """All 256 replicas of the batched ensemble, 500 steps each, in one batch."""
    from paper_1409_7498_amd import binding as B
    rows = _read_ensemble(os.path.join(HERE, "golden", "ensemble_c4.txt"))
    reps = workload.replica_configs()
    assert len(rows) == len(reps) == 256
    for r, c in zip(rows, reps):
        assert (r["name"], r["N"], r["kind"]) == (c.name, c.N, c.kind)
    steps = rows[0]["steps"]
    say("ensemble", len(reps), "replicas x", steps, "steps")
    bt = B.Batch([c.desc() for c in reps])
    bt.run(1, steps, workload.SIGMA_JITTER)
    got = [_replica_digests(bt.bonds(r), bt.stats(r), bt.read(r)) for r in range(len(reps))]
    bt.close()
    _check_rows(rows, got, "batched replicas")
    say("all", len(reps), "replicas identical to the oracle")


def test_served_sample_matches_oracle():
    """A stratified sample of the served stream, submitted together to a
    server whose slots and budget hold only part of it (continuous batching:
    replicas join and leave between rounds)."""
    from paper_1409_7498_amd import binding as B
    rows = _read_ensemble(os.path.join(HERE, "golden", "served_c5.txt"))
    _, cfgs = workload.request_stream(n_req=10000)
    picked = [cfgs[r["index"]] for r in rows]
    for r, c in zip(rows, picked):
        assert (r["name"], r["N"], r["kind"]) == (c.name, c.N, c.kind)
    say("served sample", len(picked), "requests, N", sorted(c.N for c in picked))
    big = max(B.footprint(c.desc(), c.steps) for c in picked)
    srv = B.Server(int(2.5 * big), 6)
    tickets = [srv.submit(c.desc(), c.steps, workload.SIGMA_JITTER) for c in picked]
    got = []
    for t in tickets:
        st, code, _ = srv.wait(t, 600.0)
        assert st == B.Server.DONE, (st, code)
        got.append(_replica_digests(srv.bonds(t), srv.stats(t), srv.read(t)))
    info = srv.info()
    srv.close()
    assert info["rounds"] > max(c.steps for c in picked) // 64, info
    _check_rows(rows, got, "served requests")
    say("all", len(picked), "served requests identical to the oracle")
