"""Writes the stored oracle digests of whole trajectories (tests/golden/).

Calls only the CPU oracle (oracle/) and the seeded input generator
(paper_1409_7498_amd/workload.py); nothing here runs the HIP library.  Run it
from the repository root on the CPU:

    python tests/golden/make_digests.py c1 c2 c3 c4 c5 near

Each trajectory starts from the configuration generate() makes and runs the
oracle's steps 1..S, each a re-jitter followed by the brute-force reaction
step (Table I, steps 1-9).  Files:

  traj_<cfg>.txt    per step: the nine counters and the digest of the step's
                    bond rows; the final positions, states and adjacency
  ensemble_c4.txt   per replica of the batched ensemble (256 x 500 steps):
                    bond count, digests of the whole bond log, of the counter
                    log and of the final configuration
  served_c5.txt     the same for a stratified sample of the served stream
  near_cutoff.txt   FP64 recheck of the cutoff decision (count of eligible
                    pairs with |r64 - rc| < 1e-6, and FP32/FP64 disagreements)
"""
import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import digest  # noqa: E402
from paper_1409_7498_amd import workload  # noqa: E402

TRAJ_STEPS = {"c1": 200, "c2": 200, "c3": 2000}
C5_STRATA = [(1000, 4096), (4096, 16384), (16384, 65536), (65536, 262144), (262144, 1048577)]
C5_PER = 2          # requests per (size stratum, kind)
C5_MAX_STEP_N = 300000  # step-growth requests above this are too slow for the oracle


def _oracle():
    import oracle
    oracle.load()
    return oracle


def run_config(cfg, steps):
    """Oracle run of steps 1..steps: (log, stats, final system)."""
    oracle = _oracle()
    g = cfg.initial()
    s = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    code, log, st = oracle.run(s, oracle.Rule(**cfg.rule()), cfg.seed, 1, steps, cfg.sigma,
                               log_cap=max(16, cfg.N * 4))
    assert code == 0, code
    return log, st, s


def header_of(cfg, steps, extra=()):
    return ["written by tests/golden/make_digests.py (CPU oracle only)",
            "config %s N=%d L=%r kind=%s p=%r seed=%d gen_seed=%d sigma=%r steps=1..%d"
            % (cfg.name, cfg.N, cfg.L, cfg.kind, cfg.p, cfg.seed, cfg.gen_seed, cfg.sigma, steps),
            *extra]


def do_traj(name):
    cfg = workload.CONFIGS[name]
    steps = TRAJ_STEPS[name]
    t0 = time.time()
    log, st, s = run_config(cfg, steps)
    dt = time.time() - t0
    per = digest.step_digests(log, 1, steps)
    rows = [(k + 1, tuple(st[k]), per[k + 1][1]) for k in range(steps)]
    for k in range(steps):
        assert per[k + 1][0] == st[k][7]
    fin = digest.config_digests(s.x, s.y, s.z, s.state, s.adj)
    path = os.path.join(HERE, "traj_%s.txt" % name)
    digest.write_traj(path, header_of(cfg, steps, ["bonds in total: %d; oracle wall time %.0f s"
                                                   % (len(log), dt)]), rows, fin)
    print("%s: %d steps, %d bonds, %.0f s -> %s" % (name, steps, len(log), dt, path), flush=True)


def _one_replica(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    cfg, steps = args
    log, st, s = run_config(cfg, steps)
    fin = digest.config_digests(s.x, s.y, s.z, s.state, s.adj)
    return (len(log), digest.h16(log), digest.h16(np.asarray(st, np.int64)), fin["pos"],
            fin["state"], fin["adj"])


def _single_thread():
    os.environ["OMP_NUM_THREADS"] = "1"


def _pool(jobs, workers):
    ctx = __import__("multiprocessing").get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx,
                             initializer=_single_thread) as ex:
        return list(ex.map(_one_replica, jobs, chunksize=1))


def write_ensemble(path, header, idx, cfgs, res):
    with open(path, "w") as f:
        for line in header:
            f.write("# %s\n" % line)
        f.write("# columns: index name N kind p steps bonds log_sha16 stats_sha16 pos_sha16 "
                "state_sha16 adj_sha16\n")
        for i, c, r in zip(idx, cfgs, res):
            f.write("%d %s %d %s %r %d %d %s %s %s %s %s\n"
                    % (i, c.name, c.N, c.kind, c.p, c.steps, r[0], r[1], r[2], r[3], r[4], r[5]))


def do_c4(workers):
    reps = workload.replica_configs()
    order = sorted(range(len(reps)), key=lambda k: -reps[k].N * (0.05 if reps[k].kind == "step"
                                                                 else 0.001) * reps[k].N)
    t0 = time.time()
    res = _pool([(reps[k], reps[k].steps) for k in order], workers)
    back = [None] * len(reps)
    for k, r in zip(order, res):
        back[k] = r
    path = os.path.join(HERE, "ensemble_c4.txt")
    write_ensemble(path, ["written by tests/golden/make_digests.py (CPU oracle only)",
                          "batched ensemble: workload.replica_configs() (256 replicas, "
                          "500 steps each, sigma=%r)" % workload.SIGMA_JITTER,
                          "oracle wall time %.0f s" % (time.time() - t0)],
                   list(range(len(reps))), reps, back)
    print("c4: %d replicas, %.0f s -> %s" % (len(reps), time.time() - t0, path), flush=True)


def c5_sample(n_req=10000):
    """Stratified sample of the served stream: per size stratum and kind, the
    first C5_PER requests in arrival order (step growth above C5_MAX_STEP_N
    particles: the smallest ones of the stratum instead)."""
    _, cfgs = workload.request_stream(n_req=n_req)
    pick = []
    for lo, hi in C5_STRATA:
        for kind in ("step", "chain"):
            ks = [k for k, c in enumerate(cfgs) if lo <= c.N < hi and c.kind == kind]
            if kind == "step":
                ok = [k for k in ks if cfgs[k].N <= C5_MAX_STEP_N]
                if len(ok) < len(ks):
                    ok = sorted(ok, key=lambda k: cfgs[k].N)
                ks = ok
            pick += ks[:C5_PER]
    return sorted(pick), cfgs


def do_c5(workers):
    pick, cfgs = c5_sample()
    jobs = [(cfgs[k], cfgs[k].steps) for k in pick]
    t0 = time.time()
    order = sorted(range(len(jobs)), key=lambda q: -jobs[q][0].N)
    res = _pool([jobs[q] for q in order], workers)
    back = [None] * len(jobs)
    for q, r in zip(order, res):
        back[q] = r
    path = os.path.join(HERE, "served_c5.txt")
    write_ensemble(path, ["written by tests/golden/make_digests.py (CPU oracle only)",
                          "served stream: workload.request_stream(10000); stratified sample "
                          "(c5_sample): %d per size stratum %s and kind; step-growth requests "
                          "above %d particles replaced by the stratum's smallest"
                          % (C5_PER, C5_STRATA, C5_MAX_STEP_N),
                          "oracle wall time %.0f s" % (time.time() - t0)],
                   pick, [cfgs[k] for k in pick], back)
    print("c5: %d requests, %.0f s -> %s" % (len(pick), time.time() - t0, path), flush=True)


def do_near():
    """FP64 recheck at step 1 (after the first re-jitter) of c1, c2, c3."""
    oracle = _oracle()
    lines = []
    for name in ("c1", "c2", "c3"):
        cfg = workload.CONFIGS[name]
        g = cfg.initial()
        s = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
        oracle.jitter(s, cfg.seed, 1, cfg.sigma)
        t0 = time.time()
        near, dis = oracle.near_cutoff(s, oracle.Rule(**cfg.rule()), 1e-6)
        lines.append("%s step=1 tol=1e-6 near=%d disagree=%d" % (name, near, dis))
        print(lines[-1], "(%.0f s)" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "near_cutoff.txt"), "w") as f:
        f.write("# written by tests/golden/make_digests.py (CPU oracle only): FP64 recheck of\n"
                "# the cutoff decision over all eligible (A, T) pairs after the first re-jitter\n")
        for line in lines:
            f.write(line + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="+", choices=["c1", "c2", "c3", "c4", "c5", "near"])
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    a = ap.parse_args()
    for w in a.what:
        if w in TRAJ_STEPS:
            do_traj(w)
        elif w == "c4":
            do_c4(a.workers)
        elif w == "c5":
            do_c5(a.workers)
        else:
            do_near()


if __name__ == "__main__":
    main()
