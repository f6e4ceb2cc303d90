"""Benchmark of the reaction step on one MI355X.

Workload: step growth, N = 1,048,576 particles in L = 105.6 (jittered lattice,
5% crosslinkers, r_c = 1.12, p = 0.005), generated on the device.  One step =
the re-jitter of every particle (the stand-in for the MD between reaction
steps, fused into the pair sweep) followed by the reaction step.  The storage
is re-sorted spatially every 64 steps.

Timed region: exactly --steps steps after --warmup steps, replayed from HIP
graphs captured beforehand (pr_sys_prepare), state resident in HBM, HIP
events on the system's stream.  The window holds the sorts that fall due in
it (none, or more than one per 64 steps, when --steps is not a multiple of 64
or the window is not aligned to the sort period).  ``value`` charges exactly
one sort per 64 steps: the window's time minus the sorts it held plus
steps/64 sorts, each sort timed on its own in the phase-timed run that
follows; ``window_ms`` is the raw time of the window and the JSON states the
sorts it held.

``reaction_only`` separates the reaction step from the MD stand-in: the
per-step time minus the re-jitter alone (pr_sys_jitter, its kernel's own
duration over the same number of steps).

``roofline`` covers the dominant kernel, the pair sweep: its algorithmic
bytes per launch (positions read and written, type and state) over its mean
duration, measured with events stamped at each sweep's own start and end
(hipExtLaunchKernel) on the system's stream, in a directly launched run of
the next steps.  ``copy_gbs`` is the measured ceiling of the library's own
copy kernel (pr_stream_copy, 16 bytes per lane, bytes read plus written per
second) and ``frac_of_copy`` the sweep's rate against it.  ``traffic`` is
the sweep's HBM traffic per launch from the profiler counters recorded under
profiles/ for the default workload (null when the kernel source changed
since, and for any other workload or brick edge).  ``cpu_baseline`` times
the CPU oracle on one full step of the same workload and reports the FP64
recheck of that step's cutoff decisions.

``--config c1|c3`` time the other single-system workloads, ``--config c4`` the
batched ensemble and ``--config c5`` the served stream (bench_batch, bench_serve);
``--policy nearest`` the LAMMPS selection on the default workload and ``--row
f2|f3|f4`` the other rows beyond the paper's step (bench_row).

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_B_PER_PARTICLE = 32.0   # x, y, z read (12) + type, state (8) + re-jittered x, y, z written (12)
BOND_B = 24.0                 # per new bond: the pair, two states, two adjacency entries
REACT_B_PER_PARTICLE = 20.0   # the reaction step alone: x, y, z read (12) + type, state (8)
COUNTERS = os.path.join(ROOT, "profiles", "k_sweep_step_growth_1M_counters.md")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1409_7498_amd", "csrc", f)
               for f in ("kernels.hip", "common.hpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest():
    """SHA-256 (16 hex digits) of the kernels' code: kernels.hip and common.hpp
    with line comments, trailing blanks and empty lines removed, so that an
    edit of a comment keeps a counter summary valid and an edit of code does
    not."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path) as f:
            for line in f:
                code = re.sub(r"(^|\s)//.*$", "", line.rstrip("\n")).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per sweep launch from the committed counter summary, if it was
    taken on the current kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    text = open(COUNTERS).read()
    m_d = re.search(r"kernel code digest:\s*([0-9a-f]+)", text)
    m_t = re.search(r"traffic bytes per launch:\s*([0-9.eE+]+)", text)
    if not (m_d and m_t) or m_d.group(1) != kernel_digest():
        return None
    return float(m_t.group(1))


def cpu_baseline(cfg):
    """The CPU oracle, as it is, on one full step (re-jitter + brute-force
    reaction step) of the same workload."""
    import oracle
    from paper_1409_7498_amd import workload
    g = cfg.initial()
    s = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    rule = oracle.Rule(**cfg.rule())
    t0 = time.perf_counter()
    code, _, _ = oracle.run(s, rule, cfg.seed, 1, 1, cfg.sigma)
    dt = time.perf_counter() - t0
    assert code == 0
    # FP64 recheck of the same step's cutoff decisions (after its re-jitter,
    # on the states before it), outside the timed part
    r = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    oracle.jitter(r, cfg.seed, 1, cfg.sigma)
    near, dis = oracle.near_cutoff(r, rule, 1e-6)
    return {"value": cfg.N / dt, "unit": "particles/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "one full step (re-jitter + O(N_A N) brute-force reaction step, Table I "
                      "steps 1-9) of the %d-particle workload: %.1f s wall" % (cfg.N, dt),
            "fp64_recheck": {"step": 1, "tol": 1e-6, "near": near, "disagree": dis}}


def tune_bricks(binding, descs, steps, sigma, target_wgs=4096, max_copies=256, max_brick=6):
    """Brick edge per replica from the device autotuner, one tuning per class
    of equal coarse grids (the edges a box allows depend on its cells per
    side).  Each class is timed as one of enough identical replicas of a
    batch to fill the GPU (about target_wgs sweep workgroups at the default
    edge), the context of a replica in a full ensemble."""
    import math
    from paper_1409_7498_amd import workload
    by_nc = {}
    for k, d in enumerate(descs):
        nc = int(math.floor(float(d["L"]) / (2.0 * workload.RC * (1.0 + 1.0 / 1024.0))))
        by_nc.setdefault(nc, []).append(k)
    choice, table = {}, {}
    for nc, ks in sorted(by_nc.items()):
        rep = descs[ks[len(ks) // 2]]
        bs = max(1, min(4, nc - 2))
        nb = -(-nc // bs) if nc > 2 else 1
        copies = int(min(max_copies, max(1, -(-target_wgs // nb ** 3))))
        best, us = binding.autotune(rep, steps, sigma, copies=copies)
        allowed = {b: t for b, t in us.items() if b <= max_brick}
        if allowed:
            best = min(allowed, key=allowed.get)
        table[nc] = {"brick": best, "us_per_replica_step": {b: round(t, 3) for b, t in us.items()},
                     "replicas": len(ks), "copies": copies}
        for k in ks:
            choice[k] = best
    return [dict(d, brick=choice[k]) for k, d in enumerate(descs)], table


def bench_batch(args):
    """Batched ensemble (256 replicas of uneven size, 500 steps): replicas/s of
    the batched launch against the plain per-replica launch loop, at identical
    results (bond-log and state digests compared).  Each timed region is the
    whole run of a freshly generated ensemble (graph capture included).  The
    brick edge of each replica comes from the device autotuner (untimed set-up,
    reported as autotune_s); the batch at the default edge is timed too."""
    import numpy as np
    import torch
    from paper_1409_7498_amd import binding, workload
    reps = workload.replica_configs()
    steps = args.batch_steps
    descs = [dict(n=c.N, L=c.L, B=c.B, rule=c.rule(), seed=c.seed, kind=c.kind,
                  gen_seed=c.seed ^ 0x5A5A, sigma0=workload.SIGMA_LATTICE, log_cap=2 * c.N)
             for c in reps]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    def digest(bt):
        h = hashlib.sha256()
        for r in range(len(descs)):
            h.update(bt.bonds(r).tobytes())
            h.update(bt.read(r)["state"].tobytes())
        return h.hexdigest()[:16]

    t0 = time.perf_counter()
    tuned, table = tune_bricks(binding, descs, 64, workload.SIGMA_JITTER, max_brick=args.max_brick)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    log("autotune: %.2f s, %s" % (tune_s, {nc: v["brick"] for nc, v in table.items()}))
    out = {}
    for mode, reps_ in (("batched", tuned), ("batched_default", descs), ("loop", descs)):
        bt = binding.Batch(reps_, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (bt.run_loop if mode == "loop" else bt.run)(1, steps, workload.SIGMA_JITTER)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[mode] = (dt, digest(bt))
        log("%s: %.3f s" % (mode, dt))
        bt.close()
    assert out["batched"][1] == out["loop"][1] == out["batched_default"][1], \
        "batched, default-brick and loop results differ"
    n_tot = sum(c.N for c in reps)
    res = {
        "metric": "replicas/s (batched ensemble: 256 uneven replicas)",
        "value": len(reps) / out["batched"][0],
        "unit": "replicas/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": out["batched"][0] * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic (jittered lattices, generated on device)",
        "config": {"workload": "256 replicas, N log-uniform in [2000, 65536] (total %d), "
                               "alternating step/chain growth, p in [0.001, 0.02], %d steps each"
                               % (n_tot, steps)},
        "loop_replicas_per_s": len(reps) / out["loop"][0],
        "default_brick_replicas_per_s": len(reps) / out["batched_default"][0],
        "autotune_s": tune_s,
        "autotune": {str(nc): v for nc, v in table.items()},
        "speedup_vs_loop": out["loop"][0] / out["batched"][0],
        "particle_steps_per_s": n_tot * steps / out["batched"][0],
        "results_digest": out["batched"][1],
    }
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Served stream: requests arrive as a Poisson process (200/s), each a
    replica of N log-uniform in [1000, 1,048,576] particles, step or chain
    growth, 1000 steps; a request loop with continuous batching admits them by
    HBM footprint.  Reports p50/p99 of completion minus arrival and replicas/s
    (completed requests over the time from the first arrival to the last
    completion), beside the plain per-replica launch loop on the first
    requests of the same stream (same results, digest compared)."""
    import threading
    import numpy as np
    import torch
    from paper_1409_7498_amd import binding, workload
    arrivals, cfgs = workload.request_stream(n_req=args.requests)
    descs = [dict(n=c.N, L=c.L, B=c.B, rule=c.rule(), seed=c.seed, kind=c.kind,
                  gen_seed=c.seed ^ 0x5A5A, sigma0=workload.SIGMA_LATTICE, log_cap=2 * c.N)
             for c in cfgs]
    steps = cfgs[0].steps
    torch.cuda.set_device(0)
    srv = binding.Server(int(args.budget_gb * (1 << 30)), args.slots)
    tickets = [None] * len(descs)
    t_start = time.perf_counter()

    def feed():
        for i, d in enumerate(descs):
            wait = t_start + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            tickets[i] = srv.submit(d, steps, workload.SIGMA_JITTER)

    th = threading.Thread(target=feed)
    th.start()
    lat = []
    last = 0.0
    for i in range(len(descs)):
        while tickets[i] is None:
            time.sleep(0.0005)
        st, code, l = srv.wait(tickets[i], 3600.0)
        assert st == binding.Server.DONE, (i, st, code)
        lat.append(l)
        last = max(last, arrivals[i] + l)
    th.join()
    info = srv.info()
    nb = min(args.baseline_requests, len(descs))
    h_srv = hashlib.sha256()
    for i in range(nb):
        h_srv.update(srv.bonds(tickets[i]).tobytes())
    srv.close()
    # the plain per-replica launch loop on the first nb requests (back to back)
    h_loop = hashlib.sha256()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nb):
        d = descs[i]
        s = binding.System(d["n"], d["L"], d["B"], d["rule"], d["seed"], log_cap=d["log_cap"])
        s.generate(d["kind"], d["gen_seed"], d["sigma0"])
        s.set_graphs(False)
        s.run(1, steps, workload.SIGMA_JITTER)
        h_loop.update(s.bonds().tobytes())
        s.close()
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    assert h_srv.hexdigest() == h_loop.hexdigest(), "served and loop results differ"
    lat = np.array(lat)
    n_part = float(sum(c.N for c in cfgs))
    res = {
        "metric": "served stream: replicas/s, p50/p99 completion latency",
        "value": len(descs) / last,
        "unit": "replicas/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic (jittered lattices, generated on device per request)",
        "config": {"workload": "%d requests, Poisson arrivals at 200/s, N log-uniform in "
                               "[1000, 1048576] (mean %.0f), step/chain 50/50, p in [0.001, 0.02], "
                               "%d steps each" % (len(descs), n_part / len(descs), steps),
                   "hbm_budget_gb": args.budget_gb, "slots": args.slots},
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "particle_steps_per_s": n_part * steps / last,
        "gpu_busy_fraction": info["busy_s"] / last,
        "rounds": info["rounds"],
        "worker_s": {k: round(info[k], 3) for k in ("admit_s", "finish_s", "launch_s", "wait_s")},
        "loop_replicas_per_s": nb / t_loop,
        "loop_requests": nb,
    }
    print(json.dumps(res), flush=True)


ROW_N = 1 << 20
KIN_B_PER_PARTICLE = 25.0  # type, state (8) + role (1) + x, y, z (12) + id (4)


def md_bytes(B):
    """Algorithmic bytes of one MD step per particle: positions and velocities
    read and written (48) and the adjacency row read (4 B)."""
    return 48.0 + 4.0 * B


def bench_row(args):
    """Measurement of the rows beyond the paper's step, each on a 1,048,576-
    particle system generated like the default workload:
      f2  two concurrent rules (chain initiation and propagation: initiators of
          type 1 and active ends of type 0 both bond free monomers), steps
          replayed from graphs as the default path;
      f3  the kinetics counters (pr_sys_kinetics: populations, partner counts,
          distance histogram) of the default workload after the warm-up steps,
          wall time per call (a synchronising read-out);
      f4  the bonded-force coupling: theta velocity-Verlet MD steps under the
          mirror-LJ bond force before each reaction step of the default
          workload (MD in place of the re-jitter).
    The "nearest" policy (f1) is the default path with --policy nearest."""
    import numpy as np
    import torch
    from paper_1409_7498_amd import binding, workload
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    cfg = workload.CONFIGS["c2"]
    out = {"n_gpus": 1, "steps": K, "warmup": W, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+u32", "cpu_baseline": None}

    def timed_run(s, first, sigma):
        s.prepare(K, sigma)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.run(first, K, sigma)
        e1.record(stream)
        torch.cuda.synchronize()
        st = s.stats()[-K:]
        return e0.elapsed_time(e1) / K, sum(r["bonds"] for r in st) / K

    if args.row == "f2":
        N = ROW_N
        L = workload.box_for(N)
        g = workload.generate(N, L, "chain", cfg.seed)
        init = np.random.default_rng(cfg.seed).choice(N, N // 200, replace=False)
        g["type"][init] = 1
        g["state"][init] = 2
        r = lambda ta: dict(type_a=ta, a_min=2, a_max=2, d_a=-1, type_t=0, t_min=0, t_max=0,
                            d_t=2, rc=workload.RC, p=0.02, exclude_bonded=1, policy="random")
        rules = [r(1), r(0)]
        s = binding.System(N, L, 2, rules, cfg.seed, log_cap=2 * N, stream=stream)
        s.load(g)
        s.run(1, W, cfg.sigma)
        ms, bonds = timed_run(s, 1 + W, cfg.sigma)
        s.close()
        out.update({"metric": "reaction-step particles/s, two concurrent rules",
                    "value": N / (ms * 1e-3), "unit": "particles/s", "ms_per_step": ms,
                    "bonds_per_step": bonds,
                    "data": "synthetic (jittered lattice, 0.5% initiators of type 1)",
                    "config": {"workload": "chain initiation + propagation, N=%d L=%g rc=%g "
                                           "p=0.02 each; a step = re-jitter (sigma=%g) + "
                                           "reaction step over both rules" % (N, L, workload.RC,
                                                                               cfg.sigma),
                               "row": "f2", "path": "graph replay (binning kernel, sweep, "
                                                    "resolve, final kernels per step)"}})
    elif args.row == "f3":
        s = binding.System(cfg.N, cfg.L, cfg.B, cfg.rule(), cfg.seed, log_cap=2 * cfg.N,
                           stream=stream)
        s.generate(cfg.kind, cfg.gen_seed, workload.SIGMA_LATTICE)
        s.run(1, W, cfg.sigma)
        s.kinetics(8, 16)
        torch.cuda.synchronize()
        reps = max(K // 16, 5)
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pop, pairs, hist = s.kinetics(8, 16)
            t.append(time.perf_counter() - t0)
        s.close()
        us = sorted(t)[len(t) // 2] * 1e6
        gbs = KIN_B_PER_PARTICLE * cfg.N / (us * 1e-6) / 1e9
        out.update({"metric": "kinetics counters: particles/s per read-out",
                    "value": cfg.N / (us * 1e-6), "unit": "particles/s", "ms_per_step": None,
                    "us_per_call": us, "calls": reps, "pop": pop.tolist(),
                    "pairs": pairs.tolist(), "hist_total": int(hist.sum()),
                    "data": "synthetic (jittered lattice, generated on device)",
                    "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                                 "kernel": "pr_sys_kinetics (wall time of the call)",
                                 "bytes_per_launch": KIN_B_PER_PARTICLE * cfg.N},
                    "config": {"workload": "step growth N=%d after %d steps; 8 states, 16 "
                                           "distance bins" % (cfg.N, W), "row": "f3",
                               "path": "median wall time of one call (binning, two kernels, "
                                       "copy to host)"}})
    elif args.row == "f4":
        theta = args.md_theta
        s = binding.System(cfg.N, cfg.L, cfg.B, cfg.rule(), cfg.seed, log_cap=2 * cfg.N,
                           stream=stream)
        s.generate(cfg.kind, cfg.gen_seed, workload.SIGMA_LATTICE)
        s.set_md(theta, 0.0025, 1.0, 1.0, 1.0, 7)
        s.run(1, W, 0.0)
        ms, bonds = timed_run(s, 1 + W, 0.0)
        s.close()
        out.update({"metric": "reaction steps with bonded MD: particles/s",
                    "value": cfg.N / (ms * 1e-3), "unit": "particles/s", "ms_per_step": ms,
                    "md_steps_per_reaction_step": theta, "bonds_per_step": bonds,
                    "md_bytes_per_particle_step": md_bytes(cfg.B),
                    "data": "synthetic (jittered lattice, generated on device)",
                    "config": {"workload": "step growth N=%d L=%g rc=%g p=%g; a step = %d "
                                           "velocity-Verlet steps (dt=0.0025, mirror-LJ bonds, "
                                           "sigma=eps=1, T=1) + reaction step"
                                           % (cfg.N, cfg.L, cfg.rc, cfg.p, theta),
                               "row": "f4", "path": "graph replay"}})
    else:
        raise SystemExit("--row: f2, f3 or f4 (f1 is --policy nearest)")
    print(json.dumps(out), flush=True)


def copy_bandwidth(mib=1024, reps=5, width=16):
    """Measured device copy ceiling in GB/s (bytes read plus written per
    second): the median kernel time of `reps` copies of `mib` MiB with the
    library's own copy kernel (pr_stream_copy)."""
    import torch
    from paper_1409_7498_amd import binding
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    binding.stream_copy(src, dst, width)
    times = sorted(binding.stream_copy(src, dst, width) for _ in range(reps))
    return 2 * src.numel() * 4 / (times[len(times) // 2] * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--row", default=None, choices=["f2", "f3", "f4"],
                    help="measure a row beyond the paper's step (bench_row)")
    ap.add_argument("--md-theta", type=int, default=10, help="f4: MD steps per reaction step")
    ap.add_argument("--policy", default="random", choices=["random", "nearest"],
                    help="selection: the paper's (random) or LAMMPS fix bond/create's "
                         "closest partner (nearest)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sort-period", type=int, default=-1)
    ap.add_argument("--fused-binning", type=int, default=1, choices=[0, 1],
                    help="the sweep bins the next step's A's (1) or a kernel bins them (0)")
    ap.add_argument("--brick", default="0",
                    help="brick edge in coarse cells, 1..6 (0 = the library default, 4), "
                         "or 'auto': the device autotuner's choice for the workload "
                         "(untimed set-up)")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--max-brick", type=int, default=4,
                    help="c4: largest brick edge the tuned ensemble may use (edges 5-6 "
                         "time faster per class but slow the mixed ensemble)")
    ap.add_argument("--requests", type=int, default=1000, help="c5: requests of the stream")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="c5: HBM admission budget")
    ap.add_argument("--slots", type=int, default=64, help="c5: replicas resident at once")
    ap.add_argument("--baseline-requests", type=int, default=100,
                    help="c5: requests run through the plain per-replica loop")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="MIB",
                    help="only run the library's copy kernel on MIB MiB, three times "
                         "(calibrates the HBM byte counters of the profiler), and exit")
    ap.add_argument("--probe-width", type=int, default=16,
                    help="--probe-copy: bytes per lane of the copy kernel (4, 8 or 16)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.probe_copy:
        from paper_1409_7498_amd import binding
        src = torch.ones(args.probe_copy << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        ms = [binding.stream_copy(src, dst, args.probe_width) for _ in range(3)]
        torch.cuda.synchronize()
        print(json.dumps({"probe": "pr_stream_copy", "width": args.probe_width,
                          "bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4,
                          "launches": 3, "kernel_ms": ms,
                          "gbs": 2 * src.numel() * 4 / (min(ms) * 1e-3) / 1e9}), flush=True)
        return
    from paper_1409_7498_amd import binding, workload

    if args.row:
        return bench_row(args)
    if args.config == "c4":
        return bench_batch(args)
    if args.config == "c5":
        return bench_serve(args)
    cfg = workload.CONFIGS[args.config]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.brick == "auto":
        desc = dict(n=cfg.N, L=cfg.L, B=cfg.B, rule=cfg.rule(), seed=cfg.seed, kind=cfg.kind,
                    gen_seed=cfg.seed, sigma0=workload.SIGMA_LATTICE, log_cap=2 * cfg.N)
        brick, us = binding.autotune(desc, 128, cfg.sigma, stream=stream)
        tuned = {b: round(t, 3) for b, t in sorted(us.items())}
        log("autotune: edge %d, us per step by edge %s" % (brick, tuned))
    else:
        brick = int(args.brick)
    rule = dict(cfg.rule(), policy=args.policy)
    sysm = binding.System(cfg.N, cfg.L, cfg.B, rule, cfg.seed,
                          log_cap=cfg.N * 2, stream=stream, brick=brick)
    if args.sort_period >= 0:
        sysm.set_sort_period(args.sort_period)
    sysm.set_fused_binning(bool(args.fused_binning))
    sort_period = 64 if args.sort_period < 0 else args.sort_period
    sysm.generate(cfg.kind, cfg.gen_seed, workload.SIGMA_LATTICE)
    first = 1
    sysm.run(first, args.warmup, cfg.sigma)
    first += args.warmup
    sysm.prepare(args.steps, cfg.sigma)  # the window's graphs, captured untimed
    torch.cuda.synchronize()

    # timed region: exactly K steps replayed from the captured HIP graphs,
    # events on the system's stream
    K = args.steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sysm.run(first, K, cfg.sigma)
    e1.record(stream)
    torch.cuda.synchronize()
    window_ms = e0.elapsed_time(e1)
    # sorts the window held: steps with index (from 0) a multiple of the period
    w0 = args.warmup
    sorts_in = (sum(1 for k in range(w0, w0 + K) if k % sort_period == 0)
                if sort_period > 0 else 0)
    first += K
    st = sysm.stats()[-K:]

    # kernel timing: the next steps launched directly, HIP events from each
    # step's start to its sweep (the binning kernel, when the sweep does not
    # bin), around the sweep kernel, whole steps and each sort that falls due
    # (a run of one period holds exactly one)
    KT = max(min(K, 64), sort_period if sort_period > 0 else 0)
    ph = sysm.run_timed(first, KT, cfg.sigma)
    first += KT
    sweep_ms = ph["sweep_ms"] / KT
    prep_ms = ph["prep_ms"] / KT
    sort_ms = ph["sort_ms"] / ph["sorts"] if ph["sorts"] else 0.0
    # the window with exactly K / sort_period sorts
    step_ms = (window_ms - sorts_in * sort_ms) / K + (sort_ms / sort_period if sort_period else 0)
    # the re-jitter alone over as many steps (kernel durations)
    KJ = min(K, 64)
    jit_ms = sysm.jitter(first, KJ, cfg.sigma, timed=True) / KJ
    first += KJ
    n_t = sum(r["t_elig"] for r in st) / len(st)
    bonds = sum(r["bonds"] for r in st) / len(st)
    sweep_bytes = SWEEP_B_PER_PARTICLE * cfg.N
    step_bytes = SWEEP_B_PER_PARTICLE * cfg.N + BOND_B * bonds
    react_bytes = REACT_B_PER_PARTICLE * cfg.N + BOND_B * bonds
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    react_ms = step_ms - jit_ms
    # the counters were taken on the default workload at the default edge
    profiled = (args.config == "c2" and sysm.geometry()[1] == 4 and sort_period == 64
                and args.policy == "random")
    traffic = recorded_traffic() if profiled else None
    out = {
        "metric": "reaction-step particles/s at 1M + % HBM roofline",
        "value": cfg.N / (step_ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic (jittered lattice, generated on device)",
        "config": {"workload": "%s N=%s L=%g rc=%g p=%g, %s; a step = re-jitter (sigma=%g, "
                               "fused) + reaction step"
                               % ("step growth" if cfg.kind == "step" else "chain growth",
                                  format(cfg.N, ","), cfg.L, cfg.rc, cfg.p,
                                  "5% crosslinkers" if cfg.kind == "step" else "0.1% initiators",
                                  cfg.sigma),
                   "steps_timed": K, "sort_period": sort_period,
                   "brick": sysm.geometry()[1], "brick_autotune_us": tuned,
                   "policy": args.policy, "fused_binning": sysm.fused_binning(),
                   "path": "graph replay (captured before the window)"},
        "window_ms": window_ms,
        "sorts_in_window": sorts_in,
        "sort_ms": sort_ms,
        "sort_charge": "value charges %s sorts per step (one per %d steps); the window held %d"
                       % ("1/%d" % sort_period if sort_period else "no", sort_period, sorts_in),
        "step_roofline_frac": step_bytes / (step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "reaction_only": {"ms_per_step": react_ms, "jitter_ms_per_step": jit_ms,
                          "particles_per_s": cfg.N / (react_ms * 1e-3),
                          "roofline_frac": react_bytes / (react_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                          "how": "per-step time minus the re-jitter kernel alone "
                                 "(pr_sys_jitter, same steps)"},
        "before_sweep_ms_direct": prep_ms,
        "sweep_ms_direct": sweep_ms,
        "step_ms_direct": ph["step_ms"] / KT,
        "bonds_per_step": bonds,
        "t_elig_per_step": n_t,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep" if args.policy == "random" else "k_near_sweep",
                     "bytes_per_launch": sweep_bytes},
        "cpu_baseline": None,
    }
    sysm.close()
    copy = copy_bandwidth()
    out["roofline"]["copy_gbs"] = copy
    out["roofline"]["frac_of_copy"] = achieved / copy
    if not args.no_cpu and args.policy == "random":
        log("timing the CPU oracle on one full step of the workload ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
        out["fp64_near_cutoff"] = out["cpu_baseline"]["fp64_recheck"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
