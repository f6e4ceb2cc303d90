"""Batched ensembles: replicas of uneven size, step and chain growth, each
with its own rule, seed and rate, stepped in lockstep by shared launches.

Every replica's run must equal (bit for bit: bonds, states, adjacency,
positions, counters) the same replica run alone as a resident system, and
the plain per-replica launch loop must give the same again; the smallest
replicas are also compared with the CPU oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import oracle_rule, say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _descs(n_rep=10, seed=workload.MASTER_SEED + 40, nmin=300, nmax=20000, pmax=0.3):
    """Small replica set: log-uniform sizes, alternating kinds, rates up to
    pmax (high rates exercise the overflow and deferral paths)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_rep):
        N = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        kind = "step" if r % 2 == 0 else "chain"
        p = float(rng.uniform(0.001, pmax))
        out.append(dict(n=N, L=workload.box_for(N), B=4 if kind == "step" else 2,
                        rule=workload.rule_for(kind, workload.RC, p), seed=int(seed + 1000 * r),
                        kind=kind, gen_seed=int(seed + 7 * r), sigma0=0.1, log_cap=4 * N))
    return out


def _alone(B, d, first, steps, sigma):
    s = B.System(d["n"], d["L"], d["B"], d["rule"], d["seed"], log_cap=d["log_cap"])
    s.generate(d["kind"], d["gen_seed"], d["sigma0"])
    s.run(first, steps, sigma)
    out = (s.read(), s.bonds(), s.stats())
    s.close()
    return out


def _same(a, b, label):
    ra, la, sa = a
    rb, lb, sb = b
    assert np.array_equal(la, lb), label
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(ra[k], rb[k]), (label, k)
    assert sa == sb, label


@pytest.mark.parametrize("steps", [150, 64, 7])
def test_batch_equals_replicas_alone(steps):
    from paper_1409_7498_amd import binding as B
    descs = _descs()
    say("batch", len(descs), "replicas, sizes", [d["n"] for d in descs], "steps", steps)
    bt = B.Batch(descs)
    bt.run(1, steps, workload.SIGMA_JITTER)
    got = [(bt.read(r), bt.bonds(r), bt.stats(r)) for r in range(len(descs))]
    bt.close()
    total = 0
    for r, d in enumerate(descs):
        say("replica", r, d["kind"], d["n"])
        ref = _alone(B, d, 1, steps, workload.SIGMA_JITTER)
        _same(got[r], ref, "replica %d" % r)
        total += len(ref[1])
    assert total > 0


def test_batch_loop_and_resume():
    """The per-replica launch loop gives the batched results; a batch run in
    two calls equals one run."""
    from paper_1409_7498_amd import binding as B
    descs = _descs(6, seed=workload.MASTER_SEED + 41)
    a = B.Batch(descs)
    a.run(1, 100, 0.05)
    b = B.Batch(descs)
    b.run_loop(1, 100, 0.05)
    c = B.Batch(descs)
    c.run(1, 37, 0.05)
    c.run(38, 63, 0.05)
    for r in range(len(descs)):
        ra = (a.read(r), a.bonds(r), a.stats(r))
        _same(ra, (b.read(r), b.bonds(r), b.stats(r)), "loop %d" % r)
        _same(ra, (c.read(r), c.bonds(r), c.stats(r)), "resume %d" % r)
    for h in (a, b, c):
        h.close()


def test_batch_against_oracle():
    from paper_1409_7498_amd import binding as B
    descs = _descs(4, seed=workload.MASTER_SEED + 42, nmin=200, nmax=1500, pmax=0.5)
    steps = 40
    bt = B.Batch(descs)
    bt.run(1, steps, 0.05)
    for r, d in enumerate(descs):
        host = workload.generate(d["n"], d["L"], d["kind"], d["gen_seed"], d["sigma0"], d["B"])
        o = oracle.System(host["L"], host["x"], host["y"], host["z"], host["type"],
                          host["state"], host["adj"])
        code, olog, ost = oracle.run(o, oracle_rule(d["rule"]), d["seed"], 1, steps, 0.05)
        assert code == 0
        out, log, st = bt.read(r), bt.bonds(r), bt.stats(r)
        say("oracle replica", r, d["kind"], d["n"], "bonds", len(olog))
        assert np.array_equal(log, olog)
        assert np.array_equal(out["state"], o.state) and np.array_equal(out["adj"], o.adj)
        assert np.array_equal(out["x"], o.x) and np.array_equal(out["z"], o.z)
        for k, rec in enumerate(st):
            assert list(rec.values()) == ost[k].tolist()
    bt.close()


def test_batch_rejects_bad_replica():
    from paper_1409_7498_amd import binding as B
    descs = _descs(3)
    descs[1] = dict(descs[1], L=1.0)  # box below 2 rc
    with pytest.raises(B.PrError) as e:
        B.Batch(descs)
    assert e.value.code == B.PR_EINVAL
