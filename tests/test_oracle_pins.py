"""The CPU oracle against hand-derived cases, closed forms and statistics."""
import pytest

import pins


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(orc, check):
    check(orc.load())


def test_run_invariants(orc):
    pins.check_run_invariants(orc.load())


def test_step_rate_equation(orc):
    pins.check_step_rate_equation(orc.load())


def test_chain_consumption(orc):
    pins.check_chain_consumption(orc.load())


def test_sampled_bonds_equal_full_step(orc):
    """The per-particle sampled form reproduces the whole step exactly."""
    import numpy as np
    from paper_1409_7498_amd import workload
    for kind, p, seed in (("step", 0.5, 3), ("chain", 1.0, 4)):
        g = workload.generate(4000, 16.75, kind, seed)
        if kind == "chain":
            g["state"][np.random.default_rng(seed).choice(4000, 200, replace=False)] = 2
        s = orc.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
        r = orc.Rule(**workload.rule_for(kind, 1.12, p))
        ids = np.arange(4000)
        smp = orc.sample_bonds(s, r, 9, 2, ids)
        _, b, _ = orc.react_step(s.copy(), r, 9, 2)
        full = {i: j for i, j in b.tolist()}
        assert np.array_equal(smp, [full.get(int(i), -1) for i in ids])
        assert (smp >= 0).sum() == len(b) > 0
