"""Benchmark of the reaction step on one MI355X.

Workload: step growth, N = 1,048,576 particles in L = 105.6 (jittered lattice,
5% crosslinkers, r_c = 1.12, p = 0.005), generated on the device.  One step =
the re-jitter (stand-in for MD between reaction steps, timed apart) followed
by one reaction step.  ``value`` is reaction-step throughput in particles/s
(N / reaction time per step), measured with HIP events around every reaction
kernel on the system's stream; the whole-loop rate is reported beside it.

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, max_steps=1):
    """The CPU oracle on a bounded sample of the same workload (first step(s))."""
    import oracle
    from paper_1409_7498_amd import workload
    g = workload.generate(cfg.N, cfg.L, cfg.kind, cfg.seed)
    s = oracle.System(g["L"], g["x"], g["y"], g["z"], g["type"], g["state"], g["adj"])
    rule = oracle.Rule(**cfg.rule())
    t0 = time.perf_counter()
    code, _, _ = oracle.run(s, rule, cfg.seed, 1, max_steps, cfg.sigma)
    dt = time.perf_counter() - t0
    assert code == 0
    return {"value": cfg.N * max_steps / dt, "unit": "particles/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d reaction step(s) (jitter + brute-force O(N_A N) step) of the full "
                      "%d-particle workload, %.1f s wall" % (max_steps, cfg.N, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sort-period", type=int, default=-1)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1409_7498_amd import binding, workload

    cfg = workload.CONFIGS[args.config]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sysm = binding.System(cfg.N, cfg.L, cfg.B, cfg.rule(), cfg.seed,
                          log_cap=cfg.N * 2, stream=stream)
    if args.sort_period >= 0:
        sysm.set_sort_period(args.sort_period)
    sysm.generate(cfg.kind, cfg.seed, workload.SIGMA_LATTICE)
    first = 1
    sysm.run(first, args.warmup, cfg.sigma)
    first += args.warmup
    torch.cuda.synchronize()

    # whole loop (jitter + reaction), events on the system's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sysm.run(first, args.steps, cfg.sigma)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    first += args.steps

    # phase timing: HIP events around the jitter, the reaction kernels and the sweep
    ph = sysm.run_timed(first, args.steps, cfg.sigma)
    st = sysm.stats()[-args.steps:]
    K = args.steps
    react_ms = ph["react_ms"] / K
    sweep_ms = ph["sweep_ms"] / K
    jitter_ms = ph["jitter_ms"] / K
    n_t = sum(r["t_elig"] for r in st) / len(st)
    bonds = sum(r["bonds"] for r in st) / len(st)
    sweep_bytes = 8.0 * cfg.N + 12.0 * n_t           # type+state of all, positions of T's
    step_bytes = 20.0 * cfg.N + 24.0 * bonds         # B_alg of one reaction step
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    out = {
        "metric": "reaction-step particles/s at 1M + % HBM roofline",
        "value": cfg.N / (react_ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": react_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic (jittered lattice, generated on device)",
        "config": {"workload": "step growth N=1,048,576 L=105.6 rc=1.12 p=0.005, 5% crosslinkers",
                   "steps_timed": K, "sigma_jitter": cfg.sigma},
        "loop_ms_per_step": loop_ms / K,
        "loop_particles_per_s": cfg.N * K / (loop_ms * 1e-3),
        "jitter_ms_per_step": jitter_ms,
        "sweep_ms_per_step": sweep_ms,
        "step_roofline_frac": step_bytes / (react_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "bonds_per_step": bonds,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep", "bytes_per_launch": sweep_bytes},
        "cpu_baseline": None,
    }
    sysm.close()
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
