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


def sysm_sort_period(args):
    return 64 if args.sort_period < 0 else args.sort_period


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sort-period", type=int, default=-1)
    ap.add_argument("--probe-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM "
                         "byte counters of the profiler) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.probe_copy:
        src = torch.ones(args.probe_copy << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": src.numel() * 4,
                          "bytes_written": dst.numel() * 4, "launches": 3}), flush=True)
        return
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

    # timed loop: K steps, each the re-jitter fused with the reaction step,
    # replayed from captured HIP graphs; events on the system's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sysm.run(first, args.steps, cfg.sigma)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    first += args.steps
    K = args.steps
    st = sysm.stats()[-K:]

    # kernel timing: the same steps launched directly, HIP events around the
    # prep kernel, the sweep kernel and whole steps
    KT = min(K, 64)
    ph = sysm.run_timed(first, KT, cfg.sigma)
    sweep_ms = ph["sweep_ms"] / KT
    prep_ms = ph["prep_ms"] / KT
    n_t = sum(r["t_elig"] for r in st) / len(st)
    bonds = sum(r["bonds"] for r in st) / len(st)
    step_ms = loop_ms / K
    sweep_bytes = 20.0 * cfg.N                     # type, state, x, y, z of every particle
    step_bytes = 32.0 * cfg.N + 24.0 * bonds       # B_alg with the re-jitter fused (+12 B)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
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
        "config": {"workload": "step growth N=1,048,576 L=105.6 rc=1.12 p=0.005, 5% crosslinkers; "
                               "a step = re-jitter (sigma=0.05) + reaction step",
                   "steps_timed": K, "sort_period": sysm_sort_period(args)},
        "step_roofline_frac": step_bytes / (step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "prep_ms_direct": prep_ms,
        "sweep_ms_direct": sweep_ms,
        "step_ms_direct": ph["step_ms"] / KT,
        "bonds_per_step": bonds,
        "t_elig_per_step": n_t,
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
