"""Bonded-force coupling on the GPU (velocity-Verlet MD with the mirror-LJ
bond potential between reaction steps, Sec. II D) against the oracle's
or_run_md: positions, velocities, bonds, states, adjacency and counters
identical; the total energy of the GPU's trajectory is conserved while bonds
form (thermoneutral bonding)."""
import numpy as np
import pytest

import oracle
from gpu_util import oracle_rule, say
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _gpu(c, theta, steps, vseed, sort_period=None):
    from paper_1409_7498_amd import binding as B
    s = B.System(c.N, c.L, c.B, c.rule(), c.seed, log_cap=4 * c.N)
    if sort_period is not None:
        s.set_sort_period(sort_period)
    s.generate(c.kind, c.gen_seed, workload.SIGMA_LATTICE)
    s.set_md(theta, 0.0025, 1.0, 1.0, 1.0, vseed)
    v0 = s.velocities()
    s.run(1, steps, 0.0)
    out = s.read()
    v = s.velocities()
    log, st = s.bonds(), s.stats()
    s.close()
    return v0, out, v, log, st


def _oracle(c, theta, steps, vseed):
    g = c.initial()
    o = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    md = oracle.MD(c.N, seed=vseed, temp=1.0)
    v0 = (md.vx.copy(), md.vy.copy(), md.vz.copy())
    code, log, st = oracle.run_md(o, md, oracle_rule(c.rule()), c.seed, 1, steps, theta)
    assert code == 0
    return v0, o, md, log, st


def test_sqrt_is_correctly_rounded():
    """The bonded force's square root against IEEE sqrt (numpy): every float
    in [1, 4) (two binades, both exponent parities) and 2^22 random normal
    floats over [2^-100, 2^100]."""
    import torch
    from paper_1409_7498_amd import binding as B
    every = np.arange(np.float32(1.0).view(np.int32), np.float32(4.0).view(np.int32),
                      dtype=np.int32).view(np.float32)
    rng = np.random.default_rng(3)
    rand = (rng.uniform(-100, 100, 1 << 22).astype(np.float64))
    rand = (np.exp2(rand) * rng.uniform(1, 2, rand.size)).astype(np.float32)
    for x in (every, rand):
        got = B.sqrt_rn(torch.from_numpy(x).cuda()).cpu().numpy()
        want = np.sqrt(x)
        bad = np.nonzero(got.view(np.int32) != want.view(np.int32))[0]
        assert bad.size == 0, (bad.size, x[bad[:5]], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("N,kind,p,theta,steps", [(4000, "step", 0.05, 25, 60),
                                                  (4000, "step", 0.05, 10, 60),
                                                  (65536, "step", 0.02, 25, 20),
                                                  (30000, "chain", 0.3, 25, 40)])
def test_md_run_equals_oracle(N, kind, p, theta, steps):
    c = workload.Config("md%d" % N, N, 16.75 if N == 4000 else workload.box_for(N), kind, p,
                        steps, workload.MASTER_SEED + 120 + theta)
    say("md run", c, "theta", theta)
    v0, out, v, log, st = _gpu(c, theta, steps, 99)
    ov0, o, md, olog, ost = _oracle(c, theta, steps, 99)
    for a, b in zip(v0, ov0):
        assert np.array_equal(a, b), "initial velocities"
    assert np.array_equal(log, olog), (len(log), len(olog))
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(out[k], getattr(o, k)), k
    for a, b in zip(v, (md.vx, md.vy, md.vz)):
        assert np.array_equal(a, b), "velocities"
    got = np.array([[r[f] for f in oracle.ST_NAMES] for r in st])
    assert np.array_equal(got, ost)
    assert len(log) > 0
    say("identical:", len(log), "bonds")


def test_md_sort_period_invariance_and_energy():
    """Results do not depend on the storage order; the energy of the GPU's
    trajectory (kinetic + mirror-LJ bonds, FP64 sum of its FP32 state) is
    conserved across 80 reaction steps that form thousands of bonds."""
    c = workload.Config("mdsort", 65536, workload.box_for(65536), "step", 0.05, 80,
                        workload.MASTER_SEED + 130)
    ref = _gpu(c, 25, c.steps, 7, sort_period=0)
    for period in (7, 64):
        got = _gpu(c, 25, c.steps, 7, sort_period=period)
        assert np.array_equal(got[3], ref[3]), period
        for k in ("x", "y", "z", "state", "adj"):
            assert np.array_equal(got[1][k], ref[1][k]), (period, k)
    g = c.initial()
    o0 = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    md0 = oracle.MD(c.N)
    md0.vx[:], md0.vy[:], md0.vz[:] = ref[0]
    e0 = oracle.md_energy(o0, md0)
    _, out, v, log, _ = ref
    o1 = oracle.System(g["L"], out["x"], out["y"], out["z"], g["type"], out["state"], out["adj"])
    md1 = oracle.MD(c.N)
    md1.vx[:], md1.vy[:], md1.vz[:] = v
    e1 = oracle.md_energy(o1, md1)
    say("energy", e0, "->", e1, "bonds", len(log))
    assert len(log) > 2000
    assert abs(e1 - e0) < 1e-3 * abs(e0), (e0, e1)
