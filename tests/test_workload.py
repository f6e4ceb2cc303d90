"""The seeded input generator: lattice bijection, fractions, box, offsets."""
import math

import numpy as np

import oracle
from paper_1409_7498_amd import workload


def test_lattice_sites_distinct_and_in_box():
    for N, L in ((4000, 16.75), (3001, 15.2), (27, 4.0)):
        x, y, z = workload.lattice_sites(N, L)
        keys = set(zip(x.tolist(), y.tolist(), z.tolist()))
        assert len(keys) == N
        for v in (x, y, z):
            assert v.min() > 0 and v.max() < np.float32(L)


def test_generate_fractions_and_box():
    for kind, frac, st_a, st_m in (("step", 0.05, 4, 2), ("chain", 0.001, 2, 0)):
        N = 200000 if kind == "chain" else 50000
        g = workload.generate(N, workload.box_for(N), kind, 99)
        L = np.float32(g["L"])
        for v in (g["x"], g["y"], g["z"]):
            assert v.dtype == np.float32 and v.min() >= 0 and v.max() < L
        active = (g["state"] == st_a) if kind == "chain" else (g["type"] == 1)
        k = int(active.sum())
        sd = math.sqrt(N * frac * (1 - frac))
        assert abs(k - N * frac) < 5 * sd
        assert np.all(g["state"][~active] == st_m)
        assert g["adj"].shape == (N, 4 if kind == "step" else 2) and np.all(g["adj"] == -1)


def test_generator_offsets_match_oracle_definition():
    ids = np.arange(0, 5000, 7)
    a = workload.ih12(0, ids, 2, 12345)
    b = oracle.ih12_offsets(0, ids, 2, 12345)
    assert np.array_equal(a, b)


def test_configs():
    c1, c2, c3 = (workload.CONFIGS[k] for k in ("c1", "c2", "c3"))
    assert (c1.N, c1.L, c1.kind, c1.p, c1.steps) == (4000, np.float32(16.75), "step", 0.01, 200)
    assert (c2.N, c3.N) == (1048576, 4194304)
    reps = workload.replica_configs()
    assert len(reps) == 256 and all(2000 <= r.N <= 65536 for r in reps)
    assert all(0.001 <= r.p <= 0.02 for r in reps)
    t, reqs = workload.request_stream(200)
    assert np.all(np.diff(t) > 0) and all(1000 <= r.N <= 1048576 for r in reqs)
