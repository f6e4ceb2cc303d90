"""Boundary calls beyond the step itself: the device draws against the
oracle's generator, and checkpoint / restore of a resident system."""
import numpy as np
import pytest

import oracle
from gpu_util import gen, say, to_dev
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1409_7498_amd import binding
    return binding


def test_draws_match_oracle_on_1e8_counters(B):
    """Two independent Philox4x32-10 implementations, device and oracle,
    agree word for word on 6 x 2^24 > 10^8 counters: acceptance-shaped
    counters (step, id_A, id_T, 0) and arbitrary 32-bit ones, several keys."""
    import torch
    chunk = 1 << 24
    rng = np.random.default_rng(1409)
    for c in range(6):
        key = int(rng.integers(0, 2**63)) * 2 + (c & 1)
        if c % 2 == 0:
            ids = np.arange(chunk, dtype=np.uint64)
            ctr = np.empty((chunk, 4), np.uint32)
            ctr[:, 0] = 1 + c
            ctr[:, 1] = (ids * 2654435761) & 0xFFFFFFFF
            ctr[:, 2] = (ids * 40503 + c) & 0xFFFFFFFF
            ctr[:, 3] = 0
        else:
            ctr = rng.integers(0, 2**32, size=(chunk, 4), dtype=np.uint32)
        dev = torch.from_numpy(ctr.view(np.int32)).cuda()
        got = B.draws(dev, key).cpu().numpy().view(np.uint32)
        torch.cuda.synchronize()
        want = oracle.philox(ctr, np.uint64(key))
        bad = np.flatnonzero((got != want).any(axis=1))
        say("draws chunk", c, "key", hex(key), "mismatches", bad.size)
        assert bad.size == 0, (c, bad[:4], ctr[bad[:4]])


def _sys(B, N, kind, p, seed, **kw):
    L = workload.box_for(N)
    r = workload.rule_for(kind, workload.RC, p)
    s = B.System(N, L, 4 if kind == "step" else 2, r, seed, log_cap=4 * N, **kw)
    s.generate(kind, seed + 1, 0.1)
    return s


@pytest.mark.parametrize("kind,p", [("step", 0.05), ("chain", 0.3)])
def test_checkpoint_restore_continues_identically(B, kind, p):
    """Run, checkpoint, run on; a fresh handle (another brick edge) restored
    from the checkpoint and run on gives the same bonds, counters and
    configuration as the uninterrupted run."""
    N, seed = 20000, 77
    a = _sys(B, N, kind, p, seed)
    a.run(1, 70, 0.05)
    ck = a.checkpoint()
    a.run(71, 60, 0.05)
    want = (a.bonds(), a.stats(), a.read())
    b = _sys(B, N, kind, p, seed, brick=2)
    b.run(1, 5, 0.05)  # some other state first: the restore replaces all of it
    b.restore(ck)
    assert len(b.stats()) == 70 and np.array_equal(b.bonds(), want[0][: len(b.bonds())])
    b.run(71, 60, 0.05)
    got = (b.bonds(), b.stats(), b.read())
    assert np.array_equal(got[0], want[0])
    assert got[1] == want[1]
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(got[2][k], want[2][k]), k
    say(kind, "bonds", len(want[0]), "checkpoint bytes", len(ck))
    a.close()
    b.close()


def test_restore_refuses_other_systems(B):
    """Another seed, another rule or a damaged buffer: PR_EINVAL, nothing
    changed; a log too small for the checkpoint's bonds: PR_ECAP."""
    N = 4000
    a = _sys(B, N, "step", 0.5, 5)
    a.run(1, 20, 0.05)
    ck = a.checkpoint()
    before = a.read()
    other = _sys(B, N, "step", 0.5, 6)
    with pytest.raises(B.PrError) as e:
        other.restore(ck)
    assert e.value.code == B.PR_EINVAL
    with pytest.raises(B.PrError) as e:
        a.restore(ck[:-4])
    assert e.value.code == B.PR_EINVAL
    with pytest.raises(B.PrError) as e:
        a.restore(b"XXXXXXXX" + ck[8:])
    assert e.value.code == B.PR_EINVAL
    after = a.read()
    for k in ("x", "state", "adj"):
        assert np.array_equal(after[k], before[k])
    n_b = len(a.bonds())
    assert n_b > 1
    small = B.System(N, workload.box_for(N), 4, workload.rule_for("step", workload.RC, 0.5), 5,
                     log_cap=n_b - 1)
    small.generate("step", 6, 0.1)
    with pytest.raises(B.PrError) as e:
        small.restore(ck)
    assert e.value.code == B.PR_ECAP
    for s in (a, other, small):
        s.close()
