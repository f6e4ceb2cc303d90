"""Philox4x32-10 of the oracle (and of the input generator) against rocRAND.

rocRAND's header-only engine is an independent implementation of the
published generator (Salmon et al., SC'11); it is compiled here as a plain
host program and fed random counters and keys.  This pins the counter-based
generator that both the acceptance test and the jitter draw from."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1409_7498_amd import workload

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    exe = str(tmp_path_factory.mktemp("pin") / "rocrand_pin")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "golden", "rocrand_philox_pin.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def _cases(n=20000, seed=3):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n).astype(np.uint64)
    # edge counters: zeros, all ones, and the small counters the path uses
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 0], [1000, 4095, 17, 1]]
    key[:4] = [0, 2 ** 64 - 1, 0x14097498, 0x1409749A]
    return ctr, key


def test_philox_matches_rocrand(rocrand_pin):
    ctr, key = _cases()
    inp = "\n".join("%d %d %d %d %d" % (*c, k) for c, k in zip(ctr.tolist(), key.tolist()))
    out = subprocess.run([rocrand_pin], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([list(map(int, l.split())) for l in out.strip().splitlines()], dtype=np.uint64)
    got = oracle.philox(ctr, key).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_generator_philox_matches_oracle():
    ctr, key = _cases(4000, seed=5)
    got = oracle.philox(ctr, key)
    for k in range(0, 4000, 97):
        w = workload.philox4x32_10(*ctr[k].tolist(), int(key[k]))
        assert [int(v) for v in w] == got[k].tolist()


def test_threshold_exact():
    # w < ceil(p 2^32) <=> w 2^-32 < p, at the edges
    assert oracle.threshold(0.0) == 0 and oracle.threshold(1.0) == 2 ** 32
    assert oracle.threshold(0.005) == 21474837 and oracle.threshold(0.01) == 42949673
    assert oracle.threshold(2.0 ** -32) == 1 and oracle.threshold(0.5) == 2 ** 31
    for p in (0.001, 0.005, 0.01, 0.02, 0.3):
        t = oracle.threshold(p)
        assert (t - 1) / 2 ** 32 < p <= t / 2 ** 32
        assert t == workload.threshold(p)
