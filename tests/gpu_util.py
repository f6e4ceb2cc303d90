"""Helpers of the GPU tests: run the same seeded inputs through the HIP
library and through the CPU oracle and compare element by element."""
import sys

import numpy as np

import oracle
from paper_1409_7498_amd import workload


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(cfg):
    import torch
    d = torch.device("cuda:0")
    return dict(x=torch.from_numpy(np.ascontiguousarray(cfg["x"], np.float32)).to(d),
                y=torch.from_numpy(np.ascontiguousarray(cfg["y"], np.float32)).to(d),
                z=torch.from_numpy(np.ascontiguousarray(cfg["z"], np.float32)).to(d),
                type=torch.from_numpy(np.ascontiguousarray(cfg["type"], np.int32)).to(d),
                state=torch.from_numpy(np.ascontiguousarray(cfg["state"], np.int32)).to(d),
                adj=torch.from_numpy(np.ascontiguousarray(cfg["adj"], np.int32)).to(d))


def oracle_rule(rule):
    r = oracle.Rule(**{k: rule[k] for k in ("type_a", "a_min", "a_max", "d_a", "type_t", "t_min",
                                            "t_max", "d_t", "rc", "p", "exclude_bonded")})
    r.policy = rule.get("policy", "random")
    return r


def oracle_system(cfg):
    return oracle.System(cfg["L"], cfg["x"], cfg["y"], cfg["z"], cfg["type"], cfg["state"],
                         cfg["adj"])


def compare_step(cfg, rule, seed, step, label=""):
    """One stateless step on the GPU and in the oracle; assert identical."""
    from paper_1409_7498_amd import binding
    say("compare_step", label, "n=%d" % len(cfg["x"]), "seed=%d step=%d" % (seed, step))
    dev = to_dev(cfg)
    code, bonds, st = binding.react_step(dev["x"], dev["y"], dev["z"], dev["type"], dev["state"],
                                         dev["adj"], cfg["L"], rule, seed, step,
                                         raise_on_error=False)
    s = oracle_system(cfg)
    ocode, obonds, ost = oracle.react_step(s, oracle_rule(rule), seed, step)
    assert code == ocode, (code, ocode)
    g = bonds.cpu().numpy()
    assert np.array_equal(g, obonds), (g[:10], obonds[:10])
    assert np.array_equal(dev["state"].cpu().numpy(), s.state)
    assert np.array_equal(dev["adj"].cpu().numpy(), s.adj)
    for k in ost:
        assert st[k] == ost[k], (k, st[k], ost[k])
    return g, st


def gen(N, L, kind, seed):
    return workload.generate(N, L, kind, seed)


def random_cfg(N, L, kind, seed, frac=0.05):
    """Uniformly random positions (no lattice): clustered pairs at any distance."""
    rng = np.random.default_rng(seed)
    L = float(np.float32(L))
    x = rng.uniform(0, L, N).astype(np.float32)
    y = rng.uniform(0, L, N).astype(np.float32)
    z = rng.uniform(0, L, N).astype(np.float32)
    for v in (x, y, z):
        v[v >= np.float32(L)] = 0
    pick = rng.random(N) < frac
    if kind == "step":
        typ = pick.astype(np.int32)
        st = np.where(pick, 4, 2).astype(np.int32)
        B = 4
    else:
        typ = np.zeros(N, np.int32)
        st = np.where(pick, 2, 0).astype(np.int32)
        B = 2
    return dict(L=L, x=x, y=y, z=z, type=typ, state=st, adj=np.full((N, B), -1, np.int32))
