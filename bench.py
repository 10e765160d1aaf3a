"""Benchmark of the MEM integration path on one MI355X.

Workload (ttbar dilepton, 8D): 4096 seeded synthetic events (b-jet energies
with a 15 % Gaussian TF, exact leptons, two b-jet assignments), VEGAS with
65 536 points per event per iteration, FP32 matrix element / PDFs / TFs and
FP64 constraint solves and accumulation.

A step is one call of mem_integrate_events over the whole batch in
target-accuracy mode: every event runs until its MC error is below 1 % of
P (at most 64 iterations).  value = events / s to 1 %.  The fixed-budget
configuration (8 iterations x 65 536 points) is timed once for the
integrand evaluation rate and the roofline of the integrand kernel.

Prints one JSON line.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s to 1% per-event MC error (ttbar dilepton), flow vs VEGAS; integrand evals/s"
N_EVENTS = 4096
PTS = 65536
FIXED_ITERS = 8
TARGET = 0.01
MAX_ITER = 64
SEED_EVENTS = 0x14077595 + 1
PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak (packed), FLOP/s

# Algorithmic FLOP per integrand evaluation of the ttbar dilepton path,
# FP32-equivalent (an FP64 operation counts twice: the MI355X FP64 vector
# peak is half the FP32 one).  Counted by paper_1407_7595_amd/opcount.py on
# 8 events x 2 assignments x 8 VEGAS iterations x 4096 points: 2368.7 FP64 +
# 1065.3 FP32 FLOP per evaluation (profiles/flop_count_ttbar_dilepton.md).
FLOP_PER_EVAL = 2.0 * 2368.7 + 1065.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(obs, n_iters_gpu, budget_s):
    """The FP64 oracle on a bounded sample of the same workload: a few
    events, integrated with the same budget and iteration counts the GPU
    needed for them, on all host threads."""
    import numpy as np
    import oracle
    p = oracle.tt_params()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate: one event, one iteration with a small budget
    t0 = time.perf_counter()
    oracle.integrate_events(oracle.KIND_TT, p, obs[:1], SEED_EVENTS, 2048, 2)
    per_eval = (time.perf_counter() - t0) / (2 * 2048)
    evals = 0
    n = 0
    t0 = time.perf_counter()
    while n < len(obs):
        it = int(max(2, n_iters_gpu[n]))
        cost = per_eval * PTS * it / max(1, min(threads, 2))
        if n > 0 and time.perf_counter() - t0 + cost > budget_s:
            break
        oracle.integrate_events(oracle.KIND_TT, p, obs[n:n + 1], SEED_EVENTS, PTS, it)
        evals += PTS * it
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of the {len(obs)} events, each run for the iteration count the GPU needed "
                      f"to reach 1% ({PTS} points per iteration, FP64, OpenMP over the 2 assignments)",
            "evals_per_s": evals / dt, "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=N_EVENTS)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the integrals are independent, "
              "so a multi-GPU run would shard events without any exchange", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1407_7595_amd as mem
    from synth import events

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read and written")
        del src, dst
    d = events.ttbar_dilepton(args.events, SEED_EVENTS)
    comps = mem.to_components(d["obs"]).cuda()
    proc = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    n_ev = args.events
    P = torch.empty(n_ev, dtype=torch.float64, device="cuda")
    E = torch.empty_like(P)
    S = torch.empty(n_ev, dtype=torch.int32, device="cuda")
    n_used = torch.zeros(n_ev, dtype=torch.int32, device="cuda")

    # fixed budget: integrand evaluation rate and kernel timing
    log(f"fixed-budget pass: {n_ev} events x {PTS} points x {FIXED_ITERS} iterations")
    timing = (ctypes.c_double * 6)()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mem.integrate_events(comps, proc, PTS, FIXED_ITERS, outputs=(P, E, S), timing=timing)
    torch.cuda.synchronize()
    fixed_s = time.perf_counter() - t0
    kern_ms, launches, n_evals = timing[0], timing[1], timing[2]
    evals_per_s = n_evals / fixed_s
    log(f"  {fixed_s:.3f} s wall, integrand kernel {kern_ms:.1f} ms over {int(launches)} launches, "
        f"{n_evals:.3g} evaluations -> {evals_per_s:.3g} evals/s")
    fixed_rel = (E / P).cpu().numpy()

    def step():
        mem.integrate_events(comps, proc, PTS, 0, target_rel_err=TARGET, max_iter=MAX_ITER, outputs=(P, E, S),
                             n_iter_out=n_used)

    for w in range(args.warmup):
        log(f"warmup step {w}")
        step()
    torch.cuda.synchronize()
    times = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {k}: {times[-1]:.3f} s")
    total = sum(times)
    st = S.cpu().numpy()
    nu = n_used.cpu().numpy()
    conv = float(np.mean(st == 0))
    value = n_ev * args.steps / total if total > 0 else None

    roof = None
    if FLOP_PER_EVAL is not None and launches > 0:
        per_launch = FLOP_PER_EVAL * n_evals / launches
        achieved = per_launch / (kern_ms / launches * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32, "traffic": None}
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(d["obs"], nu, args.cpu_seconds)
        log(f"  {cpu}")
    out = {
        "metric": METRIC, "value": value, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps if args.steps else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"ttbar dilepton MEM, {n_ev} events, 8D VEGAS, {PTS} points/event/iteration "
                               f"to 1% per-event error (max {MAX_ITER} iterations)",
                   "events": n_ev, "points_per_iteration": PTS, "target_rel_err": TARGET,
                   "proposal": "vegas"},
        "integrand_evals_per_s": evals_per_s,
        "fixed_budget": {"iterations": FIXED_ITERS, "seconds": fixed_s, "kernel_ms": kern_ms,
                         "median_rel_err": float(np.median(fixed_rel))},
        "converged_fraction": conv, "median_iterations": float(np.median(nu)) if args.steps else None,
        "flow_vs_vegas": None,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
