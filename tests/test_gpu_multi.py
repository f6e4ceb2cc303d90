"""Several concurrent rules in one step (the generalisation of Table I the
library implements for the extension proposed in Sec. III B) on the GPU
against the oracle's or_react_step_multi / or_run_multi: bonds (with their
rules), states, adjacency, positions and counters identical."""
import numpy as np
import pytest

import oracle
from gpu_util import oracle_rule, say, to_dev
from paper_1409_7498_amd import workload

pytestmark = pytest.mark.gpu


def _r(type_a, a_min, a_max, d_a, type_t, t_min, t_max, d_t, p, rc=1.12):
    return dict(type_a=type_a, a_min=a_min, a_max=a_max, d_a=d_a, type_t=type_t, t_min=t_min,
                t_max=t_max, d_t=d_t, rc=rc, p=p, exclude_bonded=1, policy="random")


def chain_init_prop(p0, p1):
    """initiators (type 1, state 2) start chains; active ends (type 0, state
    2) propagate; free monomers (type 0, state 0) are the targets of both."""
    return [_r(1, 2, 2, -1, 0, 0, 0, 2, p0), _r(0, 2, 2, -1, 0, 0, 0, 2, p1)]


def cross_roles(p0, p1):
    """crosslinkers (type 1) bond end units (type 0, states 1-2); end units
    with both valences free (state 2) also bond end units with one (state 1),
    with a shorter cutoff: a state-2 end is the T of rule 0 and the A of rule 1."""
    return [_r(1, 1, 4, -1, 0, 1, 2, -1, p0), _r(0, 2, 2, -1, 0, 1, 1, -1, p1, rc=1.05)]


def chain_cfg(N, seed):
    g = workload.generate(N, workload.box_for(N), "chain", seed)
    rng = np.random.default_rng(seed)
    init = rng.choice(N, max(2, N // 200), replace=False)
    g["type"][init] = 1
    g["state"][init] = 2
    return g


def step_cfg(N, seed):
    g = workload.generate(N, workload.box_for(N), "step", seed)
    rng = np.random.default_rng(seed)
    one = rng.random(N) < 0.3
    g["state"][(g["type"] == 0) & one] = 1  # some end units with one valence left
    return g


def _orules(rules):
    return [oracle_rule(r) for r in rules]


def _compare_multi(cfg, rules, seed, step):
    from paper_1409_7498_amd import binding as B
    dev = to_dev(cfg)
    code, bonds, st = B.react_step_multi(dev["x"], dev["y"], dev["z"], dev["type"], dev["state"],
                                         dev["adj"], cfg["L"], rules, seed, step,
                                         raise_on_error=False)
    s = oracle.System(cfg["L"], cfg["x"], cfg["y"], cfg["z"], cfg["type"], cfg["state"], cfg["adj"])
    ocode, obonds, ost = oracle.react_step_multi(s, _orules(rules), seed, step)
    assert code == ocode, (code, ocode)
    assert np.array_equal(bonds.cpu().numpy(), obonds)
    assert np.array_equal(dev["state"].cpu().numpy(), s.state)
    assert np.array_equal(dev["adj"].cpu().numpy(), s.adj)
    assert st == ost, (st, ost)
    return obonds, ost


def test_one_rule_is_the_single_step():
    from paper_1409_7498_amd import binding as B
    cfg = workload.generate(4000, 16.75, "step", 5)
    rule = workload.rule_for("step", workload.RC, 0.3)
    b, st = _compare_multi(cfg, [rule], 5, 2)
    dev = to_dev(cfg)
    _, b1, st1 = B.react_step(dev["x"], dev["y"], dev["z"], dev["type"], dev["state"], dev["adj"],
                              cfg["L"], rule, 5, 2)
    assert np.array_equal(b1.cpu().numpy(), b[:, :2]) and st1 == st and len(b) > 0


@pytest.mark.parametrize("which,p0,p1,seed", [("chain", 1.0, 1.0, 1), ("chain", 0.3, 0.6, 2),
                                              ("cross", 1.0, 1.0, 3), ("cross", 0.4, 0.7, 4),
                                              ("cross", 0.05, 0.02, 5)])
def test_two_rules_step(which, p0, p1, seed):
    cfg = chain_cfg(6000, seed) if which == "chain" else step_cfg(6000, seed)
    rules = chain_init_prop(p0, p1) if which == "chain" else cross_roles(p0, p1)
    say("two rules", which, p0, p1)
    b, st = _compare_multi(cfg, rules, seed, 7)
    if p0 >= 0.3:
        assert len(b) > 0 and set(b[:, 2].tolist()) == {0, 1}, b[:20]


@pytest.mark.parametrize("which,N,steps,p0,p1", [("chain", 8000, 120, 0.2, 0.3),
                                                 ("cross", 8000, 60, 0.05, 0.05),
                                                 ("chain", 120000, 40, 0.3, 0.5)])
def test_two_rules_run(which, N, steps, p0, p1):
    from paper_1409_7498_amd import binding as B
    cfg = chain_cfg(N, 11) if which == "chain" else step_cfg(N, 12)
    rules = chain_init_prop(p0, p1) if which == "chain" else cross_roles(p0, p1)
    Bw = cfg["adj"].shape[1]
    s = B.System(N, cfg["L"], Bw, rules, 77, log_cap=4 * N)
    s.load(cfg)
    s.run(1, steps, 0.05)
    out, log, st = s.read(), s.bonds(), s.stats()
    s.close()
    o = oracle.System(cfg["L"], cfg["x"], cfg["y"], cfg["z"], cfg["type"], cfg["state"], cfg["adj"])
    code, olog, ost = oracle.run_multi(o, _orules(rules), 77, 1, steps, 0.05)
    assert code == 0
    say(which, N, "bonds", len(log), "by rule", np.bincount(olog[:, 3], minlength=2).tolist())
    assert np.array_equal(log, olog[:, :3]), (len(log), len(olog))
    for k in ("x", "y", "z", "state", "adj"):
        assert np.array_equal(out[k], getattr(o, k)), k
    got = np.array([[r[f] for f in oracle.ST_NAMES] for r in st])
    assert np.array_equal(got, ost)
    assert np.all(np.bincount(olog[:, 3], minlength=2) > 0)
