"""The allocation-free single step (pr_react_step_noalloc) against the
allocating one (pr_react_step), through the C ABI: identical bonds, states,
adjacency and counters on consecutive calls that share the library's fixed
scratch region, the second call smaller than the first (its cells and keys
must not see the first call's leftovers), then a larger one again."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import oracle_rule, say, to_dev
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _both(cfg, rule, seed, step):
    from paper_1409_7498_amd import binding as B
    a, b = to_dev(cfg), to_dev(cfg)
    ca, ba, sa = B.react_step(a["x"], a["y"], a["z"], a["type"], a["state"], a["adj"], cfg["L"],
                              rule, seed, step, raise_on_error=False)
    cb, bb, sb = B.react_step(b["x"], b["y"], b["z"], b["type"], b["state"], b["adj"], cfg["L"],
                              rule, seed, step, raise_on_error=False, noalloc=True)
    torch.cuda.synchronize()
    assert ca == cb, (ca, cb)
    assert np.array_equal(ba.cpu().numpy(), bb.cpu().numpy())
    for k in ("state", "adj"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
    assert sa == sb, (sa, sb)
    return bb.cpu().numpy(), sb, b


def test_noalloc_equals_allocating_step():
    cases = [  # (N, kind, p, seed, step): the second call is smaller than the first
        (32768, "step", 0.3, 11, 3),
        (3000, "chain", 1.0, 12, 5),
        (20000, "step", 0.05, 13, 7),
        (1, "step", 0.5, 14, 1),
        (25000, "chain", 0.5, 15, 2),
    ]
    for N, kind, p, seed, step in cases:
        L = workload.box_for(N) if N > 100 else 10.0
        cfg = workload.generate(N, L, kind, seed)
        if kind == "chain":
            cfg["state"][np.random.default_rng(seed).choice(N, max(1, N // 20), replace=False)] = 2
        rule = workload.rule_for(kind, workload.RC, p)
        say("noalloc", N, kind, "p=%g" % p)
        bonds, st, dev = _both(cfg, rule, seed, step)
        if N <= 3000:
            s = oracle.System(cfg["L"], cfg["x"], cfg["y"], cfg["z"], cfg["type"], cfg["state"],
                              cfg["adj"])
            code, ob, ost = oracle.react_step(s, oracle_rule(rule), seed, step)
            assert np.array_equal(bonds, ob) and st == ost
            assert np.array_equal(dev["state"].cpu().numpy(), s.state)
        if N > 1000:
            assert st["bonds"] > 0


def test_noalloc_rejects_large_n():
    from paper_1409_7498_amd import binding as B
    N = 32769
    cfg = workload.generate(N, workload.box_for(N), "step", 3)
    d = to_dev(cfg)
    code, _, _ = B.react_step(d["x"], d["y"], d["z"], d["type"], d["state"], d["adj"], cfg["L"],
                              workload.rule_for("step"), 1, 1, raise_on_error=False, noalloc=True)
    assert code == B.PR_EINVAL and b"at most 32768" in B.lib.pr_last_error()
    assert np.array_equal(d["state"].cpu().numpy(), cfg["state"])
