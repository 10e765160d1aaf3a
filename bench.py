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
# peak is half the FP32 one).  Counted by measure/opcount.py on this
# benchmark's own fixed-budget workload: its 4096 events x 2 assignments x 8
# VEGAS iterations x 32 768 points (65 536 per event): 1160.68 FP64 + 623.83
# FP32 FLOP per evaluation (profiles/flop_count_ttbar_dilepton.md).
FLOP_PER_EVAL = 2.0 * 1160.68 + 623.83

# HBM bytes per fixed-budget launch of the integrand kernel (4096 events x
# 65 536 points), from rocprofv3 FETCH_SIZE / WRITE_SIZE passes over this
# script's fixed-budget pass, each scaled by what the counter reads for plain
# kernels of known size (profiles/hbm_counters_ttbar_dilepton_4096ev.md):
# FETCH 36 303 KiB x 2.000 + WRITE 66 532 KiB x 1.000.  Valid only for this
# workload and the kernel build the counters were taken on (set to None when
# the kernel changes, until they are taken again).
TRAFFIC_BYTES_PER_LAUNCH = (36303.2 * 2.000 + 66531.6 * 1.000) * 1024
TRAFFIC_WORKLOAD = (4096, 65536, 16384, 1)    # events, points, chunk points, waves per SIMD

# chunks of the late iterations (mem_integrate_opts.tail_chunk_points /
# tail_iter): from the eighth iteration on, when few events still run, 2048
# points per chunk spread them over more of the GPU (measured on this
# workload: 2048 from iteration 6, 8 or 10 within 0.5 % of each other; 1024
# slower than none)
TAIL = dict(tail_chunk_points=2048, tail_iter=8)

# tuned launch configurations (mem_autotune's table) shipped with the package
TUNING_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1407_7595_amd", "tuning.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(obs, n_iters_gpu, budget_s):
    """The FP64 oracle on a bounded sample of the same workload: the first
    events, each integrated with the budget and the iteration count the GPU
    needed for it to reach 1 %, in one oracle call (OpenMP over the event x
    assignment integrals on every host thread); then the oracle's rate on
    one thread over a smaller sample."""
    import numpy as np
    import oracle
    p = oracle.tt_params()
    oracle.set_threads(0)
    threads = oracle.max_threads()
    its = np.maximum(2, np.asarray(n_iters_gpu, dtype=np.int64)).astype(np.int32)
    # a first call over enough events to give every thread an integral
    # measures the rate on this workload (adapted grids cost more per
    # point than uniform ones); the second fills the rest of the budget
    n0 = min(len(obs), max(1, (threads + 1) // 2))
    t0 = time.perf_counter()
    oracle.integrate_events(oracle.KIND_TT, p, obs[:n0], SEED_EVENTS, PTS, its[:n0])
    dt0 = time.perf_counter() - t0
    rate = float(np.sum(its[:n0])) * PTS / dt0
    cum = np.cumsum(its[n0:].astype(np.int64) * PTS)
    n1 = int(np.searchsorted(cum, max(0.0, budget_s - dt0) * rate, side="right"))
    n1 = min(n1 - n1 % max(1, n0), len(obs) - n0)     # whole rounds of the thread pool
    dt1 = 0.0
    if n1 > 0:
        t1 = time.perf_counter()
        oracle.integrate_events(oracle.KIND_TT, p, obs[n0:n0 + n1], SEED_EVENTS, PTS, its[n0:n0 + n1])
        dt1 = time.perf_counter() - t1
    n = n0 + n1
    dt = dt0 + dt1
    evals = int(np.sum(its[:n].astype(np.int64))) * PTS
    used = min(threads, 2 * n)
    # one thread: the first event's two integrals at 8192 points x 2 iterations
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.integrate_events(oracle.KIND_TT, p, obs[:1], SEED_EVENTS, 8192, 2)
    one = 8192 * 2 / (time.perf_counter() - t1)
    oracle.set_threads(0)
    return {"value": n / dt, "unit": "events/s", "cores": used, "kind": "oracle",
            "sample": f"the first {n} of the {len(obs)} events in two oracle calls, each run for the iteration "
                      f"count the GPU needed to reach 1% ({PTS} points per iteration split over the 2 "
                      f"assignments, FP64, OpenMP over the {2 * n} integrals on {used} threads)",
            "evals_per_s": evals / dt, "seconds": dt, "evals_per_s_1_thread": one,
            "host_threads": threads}


# Learned proposal (the flow leg): trained on VEGAS samples of fresh events,
# then used on the benchmark events to the same accuracy.
FLOW_TRAIN_EVENTS = 50000
FLOW_TRAIN_PTS = 8192          # VEGAS points per training event per iteration
FLOW_TRAIN_ITERS = 4
FLOW_CAPTURE = 168             # samples per training integral: 100 000 x 168 ~ 2^24
FLOW_BATCH = 65536             # training minibatch
FLOW_EPOCHS = 24
FLOW_LR = (2e-3, 1e-4)         # cosine decay between these
FLOW_PTS = 16384               # flow points per event per batch
SEED_TRAIN = 0x14077595 + 4
PEAK_BF16 = 2.5e15             # MI355X dense BF16 matrix peak, FLOP/s


def flow_leg(mem, proc, comps, n_ev, args):
    """train the flow on VEGAS samples of fresh events, then integrate the
    benchmark events to 1 % with it (VEGAS fallback below ESS/N = 0.3)"""
    import numpy as np
    import torch
    from synth import events
    n_tr = args.flow_train_events
    d = events.ttbar_dilepton(n_tr, SEED_TRAIN)
    ctr = mem.to_components(d["obs"]).cuda()
    n_s = 2 * n_tr * FLOW_CAPTURE
    log(f"flow: training on {n_s} VEGAS samples of {n_tr} events, {FLOW_EPOCHS} epochs (mem_train_proposal)")
    t0 = time.perf_counter()
    f, losses = mem.train_proposal(proc, ctr, mode=mem.MEM_FLOW_BF16, vegas_points=FLOW_TRAIN_PTS,
                                   vegas_iter=FLOW_TRAIN_ITERS, capture=FLOW_CAPTURE, batch=FLOW_BATCH,
                                   epochs=FLOW_EPOCHS, lr_max=FLOW_LR[0], lr_min=FLOW_LR[1], seed=SEED_TRAIN,
                                   losses=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"flow: trained in {train_s:.1f} s, loss per integral {losses[0]:.4f} -> {losses[-1]:.4f}")
    del ctr
    torch.cuda.empty_cache()
    # the benchmark events to 1 % with the flow
    P = torch.empty(n_ev, dtype=torch.float64, device="cuda")
    E = torch.empty_like(P)
    S = torch.empty(n_ev, dtype=torch.int32, device="cuda")
    n_used = torch.zeros(n_ev, dtype=torch.int32, device="cuda")
    timing = (ctypes.c_double * 8)()

    def run(tm=None, thr=0.3):
        mem.integrate_events(comps, proc, FLOW_PTS, 0, target_rel_err=TARGET, max_iter=MAX_ITER,
                             outputs=(P, E, S), n_iter_out=n_used, flow=f, ess_threshold=thr, timing=tm,
                             allocation=mem.MEM_ALLOC_NEYMAN, **TAIL)

    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    value = n_ev * len(times) / sum(times)
    st = S.cpu().numpy()
    nu_fb = n_used.cpu().numpy()
    run(timing)                           # per-kernel times (direct launches)
    torch.cuda.synchronize()
    samp_ms, samp_n = timing[4], timing[5]
    flow_pts = timing[6]
    mfma = flow_pts * 6 * 2 * 128 * (128 + 96) / (samp_ms * 1e-3) if samp_ms > 0 else None
    # the proposal alone (no fallback), for reference
    t0 = time.perf_counter()
    run(thr=1e-12)
    torch.cuda.synchronize()
    alone_s = time.perf_counter() - t0
    st_alone = S.cpu().numpy()
    alone = {"events_per_s": n_ev / alone_s, "converged_fraction": float(np.mean(st_alone == 0)),
             "median_batches": float(np.median(n_used.cpu().numpy()))}
    # VEGAS alone with the flow leg's points per iteration (the fallback's
    # setting): the like-for-like reference for the proposal
    t0 = time.perf_counter()
    mem.integrate_events(comps, proc, FLOW_PTS, 0, target_rel_err=TARGET, max_iter=MAX_ITER,
                         outputs=(P, E, S), n_iter_out=n_used, allocation=mem.MEM_ALLOC_NEYMAN, **TAIL)
    torch.cuda.synchronize()
    v_s = time.perf_counter() - t0
    vegas_same = {"events_per_s": n_ev / v_s, "converged_fraction": float(np.mean(S.cpu().numpy() == 0)),
                  "mean_iterations": float(np.mean(n_used.cpu().numpy()))}
    # the flow seeding VEGAS's grids (MEM_FLOW_SEED_GRID) at the headline's
    # points per iteration: every iteration enters the estimate
    # (the headline's 65 536, and the flow leg's 16 384 against VEGAS at 16 384)
    def seeded_run(pts):
        def run_seeded():
            mem.integrate_events(comps, proc, pts, 0, target_rel_err=TARGET, max_iter=MAX_ITER, outputs=(P, E, S),
                                 n_iter_out=n_used, flow=f, flow_mode=mem.MEM_FLOW_SEED_GRID,
                                 allocation=mem.MEM_ALLOC_NEYMAN, **TAIL)

        run_seeded()
        torch.cuda.synchronize()
        st_times = []
        for _ in range(max(1, args.steps)):
            t0 = time.perf_counter()
            run_seeded()
            torch.cuda.synchronize()
            st_times.append(time.perf_counter() - t0)
        return {"events_per_s": n_ev * len(st_times) / sum(st_times), "points_per_iteration": pts,
                "converged_fraction": float(np.mean(S.cpu().numpy() == 0)),
                "mean_iterations": float(np.mean(n_used.cpu().numpy())),
                "median_iterations": float(np.median(n_used.cpu().numpy()))}

    seeded = seeded_run(PTS)
    log(f"flow-seeded VEGAS grids: {seeded}")
    seeded_small = seeded_run(FLOW_PTS)
    seeded_small["vs_vegas_same_points"] = seeded_small["events_per_s"] / vegas_same["events_per_s"]
    log(f"flow-seeded VEGAS grids at {FLOW_PTS} points: {seeded_small}")
    # ESS/N per integral: the untrained flow (the identity, i.e. uniform
    # sampling), the trained flow (its first batch) and the VEGAS grid after
    # three adaptations (its fourth iteration)
    n_int = 2 * n_ev

    def ess_quantiles(rec, n):
        I, var = rec[..., 0], rec[..., 1]
        den = var * (n - 1) + I * I
        e = np.where(den > 0, I * I / np.maximum(den, 1e-300), 0.0)
        return {q: float(np.quantile(e, v)) for q, v in (("p10", 0.1), ("median", 0.5), ("p90", 0.9))}

    ess = {}
    for name, fl in (("untrained_flow", mem.Flow()), ("trained_flow", f)):
        rec = torch.zeros((2, n_int, 2), dtype=torch.float64, device="cuda")
        mem.integrate_events(comps, proc, FLOW_PTS, 2, seed=SEED_TRAIN + 1, flow=fl, ess_threshold=1e-12,
                             iter_out=rec)
        torch.cuda.synchronize()
        ess[name] = ess_quantiles(rec.cpu().numpy()[0], FLOW_PTS // 2)
    rec = torch.zeros((4, n_int, 2), dtype=torch.float64, device="cuda")
    mem.integrate_events(comps, proc, FLOW_PTS, 4, seed=SEED_TRAIN + 1, iter_out=rec)
    torch.cuda.synchronize()
    ess["vegas_iteration_4"] = ess_quantiles(rec.cpu().numpy()[3], FLOW_PTS // 2)
    log(f"ESS/N quantiles over the {n_int} integrals at {FLOW_PTS // 2} points: {ess}")
    out = {"events_per_s": value, "seconds_per_step": sum(times) / len(times), "flow_alone": alone,
           "flow_seeded_grids": seeded, "flow_seeded_grids_same_points": seeded_small, "ess_over_n": ess,
           "vegas_same_points": vegas_same,
           "points_per_event_per_batch": FLOW_PTS, "fallback_fraction": float(np.mean(st == 4)),
           "converged_fraction": float(np.mean((st == 0) | (st == 4))),
           "median_batches": float(np.median(nu_fb)),
           "train": {"events": n_tr, "samples": n_s, "epochs": FLOW_EPOCHS, "seconds": train_s,
                     "loss_first": losses[0], "loss_last": losses[-1]},
           "sample_kernel": {"ms": samp_ms, "launches": samp_n, "points": flow_pts,
                             "mfma_tflops": mfma / 1e12 if mfma else None,
                             "mfma_frac": mfma / PEAK_BF16 if mfma else None},
           "integrand_kernel_ms": timing[0], "fallback_evaluations": timing[7]}
    log(f"flow: {out}")
    return out


PARTON_EVENTS = 100000
# Sec. 4's analysis: half t tbar H, half t tbar b bbar dilepton events, each
# integrated under both hypotheses at a fixed budget
F2_EVENTS = 1024
F2_PTS = 49152
F2_ITERS = 6


def parton_leg(mem, proc):
    """parton-level weights (transfer functions are delta functions: the
    matrix element x PDFs at given momenta, no integration) for 10^5 events,
    the workload of the paper's parton-level timing"""
    import numpy as np
    import torch
    from synth import events
    obs = events.ttbar_dilepton_partons(PARTON_EVENTS, SEED_EVENTS + 10)["obs"]
    comps = torch.as_tensor(np.ascontiguousarray(obs.transpose(2, 1, 0))).cuda()
    w = torch.empty(PARTON_EVENTS, dtype=torch.float64, device="cuda")
    mem.parton_weights(proc, comps, out=w)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        mem.parton_weights(proc, comps, out=w)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = {"events": PARTON_EVENTS, "assignments": 2, "ms": dt * 1e3, "events_per_s": PARTON_EVENTS / dt,
           "nonzero_fraction": float((w > 0).double().mean())}
    log(f"parton level: {out}")
    return out


def pdf_grid_leg(mem, comps, n_ev, kern_ms_toy):
    """the fixed-budget pass again with the densities interpolated from
    (ln x, ln Q) grids (the library's toy densities tabulated on 320 x 16
    nodes, x in [1e-5, 1], Q in [10, 13000] GeV): the cost of the paper's
    grid-PDF design against the closed-form toy densities"""
    import math
    import torch
    bounds = (math.log(1e-5), 0.0, math.log(10.0), math.log(13000.0))
    proc = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    proc.set_pdf_grid(mem.toy_pdf_table(320, 16, bounds), bounds)
    timing = (ctypes.c_double * 8)()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mem.integrate_events(comps, proc, PTS, FIXED_ITERS, timing=timing)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"grid": "320 x 16 nodes, 11 flavours", "kernel_ms": timing[0], "evals_per_s": timing[2] / wall,
           "kernel_time_vs_toy": timing[0] / kern_ms_toy}
    log(f"pdf grid: {out}")
    return out


def tth_vs_ttbb_leg(mem):
    """Sec. 4's analysis: the event discriminant D = log10(p_ttH / p_ttbb)
    for seeded t tbar H and t tbar b bbar dilepton events (four b-jets, 8D),
    each event integrated under both hypotheses (FP32 matrix elements,
    Neyman allocation across the assignments, a fixed budget)"""
    import numpy as np
    import torch
    from synth import events
    n_half = F2_EVENTS // 2
    obs = np.concatenate([events.ttbar_higgs_dilepton(n_half, SEED_EVENTS + 20)["obs"],
                          events.ttbar_bbbar_dilepton(n_half, SEED_EVENTS + 21)["obs"]])
    comps = mem.to_components(obs).cuda()
    out = {"events": F2_EVENTS, "signal_events": n_half, "iterations": F2_ITERS}
    res = {}
    for name, kind, pts in (("tth", mem.MEM_TTH_DILEPTON, F2_PTS), ("ttbb", mem.MEM_TTBB_DILEPTON, F2_PTS)):
        proc = mem.Process(kind, precision=mem.MEM_FP32)
        mem.integrate_events(comps[:, :, :64].contiguous(), proc, pts, 2, allocation=mem.MEM_ALLOC_NEYMAN)
        timing = (ctypes.c_double * 8)()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, E, S = mem.integrate_events(comps, proc, pts, F2_ITERS, timing=timing, allocation=mem.MEM_ALLOC_NEYMAN)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[name] = P
        p_, e_ = P.cpu().numpy(), E.cpu().numpy()
        ok = p_ > 0
        out[name] = {"points_per_iteration": pts, "seconds": wall, "events_per_s": F2_EVENTS / wall,
                     "kernel_ms": timing[0], "evals_per_s": timing[2] / wall,
                     "median_rel_err": float(np.median(e_[ok] / p_[ok])) if ok.any() else None,
                     "status_ok": float((S == 0).double().mean())}
    D = mem.discriminant(res["tth"], res["ttbb"]).cpu().numpy()
    out["D_finite_fraction"] = float(np.mean(np.isfinite(D)))
    out["events_per_s_both"] = F2_EVENTS / (out["tth"]["seconds"] + out["ttbb"]["seconds"])
    log(f"tth vs ttbb: {out}")
    return out


def f2_oracle_rates(seconds=6.0):
    """the oracle (FP64 C, one core) on the Sec. 4 workloads, bounded by
    `seconds` per measurement: parton-level weights per event and integrand
    evaluations at uniform random points"""
    import numpy as np
    import oracle
    from synth import events
    po = oracle.tt_params()
    out = {"cores": 1, "kind": "oracle"}
    rng = np.random.default_rng(5)
    for name, kind, genf, fint in (("tth", oracle.KIND_TTH_LL, events.ttbar_higgs_dilepton, oracle.tthll_integrand),
                                   ("ttbb", oracle.KIND_TTBB_LL, events.ttbar_bbbar_dilepton, oracle.ttbbll_integrand)):
        d = genf(64, SEED_EVENTS + 40)
        ev = events.four_b_partons(d, SEED_EVENTS + 41)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds / 2 and n < len(ev):
            oracle.f2_parton_weight(kind, po, ev[n])
            n += 1
        par = n / (time.perf_counter() - t0)
        n, t0 = 0, time.perf_counter()
        n_perm = 12 if name == "tth" else 24
        while time.perf_counter() - t0 < seconds / 2:
            fint(po, d["obs"][n % 64], n % n_perm, rng.random(8))
            n += 1
        out[name] = {"parton_events_per_s": par, "integrand_evals_per_s": n / (time.perf_counter() - t0)}
    log(f"tth vs ttbb oracle: {out}")
    return out


def f2_parton_leg(mem):
    """Sec. 4's parton-level timing (its Table 2): 10^5 t tbar H and 10^5
    t tbar b bbar dilepton events at parton level, every placement of the
    four b quarks summed, FP32 matrix elements"""
    import numpy as np
    import torch
    from synth import events
    out = {"events": PARTON_EVENTS}
    for name, kind, genf, seed in (("tth", mem.MEM_TTH_DILEPTON, events.ttbar_higgs_dilepton, 30),
                                   ("ttbb", mem.MEM_TTBB_DILEPTON, events.ttbar_bbbar_dilepton, 31)):
        ev = events.four_b_partons(genf(PARTON_EVENTS, SEED_EVENTS + seed), SEED_EVENTS + seed + 1)
        comps = torch.as_tensor(np.ascontiguousarray(ev.transpose(2, 1, 0))).cuda()
        proc = mem.Process(kind, precision=mem.MEM_FP32)
        w = torch.empty(PARTON_EVENTS, dtype=torch.float64, device="cuda")
        mem.parton_weights(proc, comps, out=w)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            mem.parton_weights(proc, comps, out=w)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"seconds": dt, "events_per_s": PARTON_EVENTS / dt,
                     "assignments": 12 if name == "tth" else 24, "nonzero_fraction": float((w > 0).double().mean())}
    log(f"tth vs ttbb parton level: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=N_EVENTS)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-flow", action="store_true")
    ap.add_argument("--no-grid", action="store_true", help="skip the grid-PDF pass")
    ap.add_argument("--no-f2", action="store_true", help="skip the t tbar H vs t tbar b bbar pass")
    ap.add_argument("--flow-train-events", type=int, default=FLOW_TRAIN_EVENTS)
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner on the benchmark events and write the tuning table")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB fill and a 256 MiB elementwise copy (reference for HBM byte counters)")
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
        # a fill kernel writes 256 MiB, an elementwise kernel reads them and
        # writes 256 MiB (plain kernels: hipMemcpy's blit path is only
        # partly seen by the byte counters)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: fill 268435456 bytes, then read 268435456 and write 268435456 bytes")
        del src, dst
    d = events.ttbar_dilepton(args.events, SEED_EVENTS)
    comps = mem.to_components(d["obs"]).cuda()
    proc = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    n_ev = args.events
    # launch configuration: the tuned table's entry for this device, or a
    # fresh tuning run (--tune, which rewrites the table's entry)
    launch = {"source": "default"}
    if args.tune:
        # the headline's own call: target mode to 1 %, Neyman allocation
        best, bw, rate = proc.autotune(comps, PTS, table_path=TUNING_TABLE, target_rel_err=TARGET,
                                       max_iter=MAX_ITER, allocation=mem.MEM_ALLOC_NEYMAN,
                                       candidates=[1024, 2048, 4096, 8192, 16384], **TAIL)
        launch = {"source": "tuned now", "tuner_events_per_s": rate}
        log(f"autotune: chunk {best}, {bw} waves per SIMD, {rate:.4g} events/s -> {TUNING_TABLE}")
    elif os.path.exists(TUNING_TABLE) and proc.load_tuning(TUNING_TABLE):
        launch = {"source": "table"}
    launch.update({"chunk_points": proc.chunk_points(), "waves_per_simd": proc.waves(),
                   "table": os.path.relpath(TUNING_TABLE, os.path.dirname(os.path.abspath(__file__))), **TAIL})
    log(f"launch: {launch}")
    P = torch.empty(n_ev, dtype=torch.float64, device="cuda")
    E = torch.empty_like(P)
    S = torch.empty(n_ev, dtype=torch.int32, device="cuda")
    n_used = torch.zeros(n_ev, dtype=torch.int32, device="cuda")

    # fixed budget: integrand evaluation rate and kernel timing
    log(f"fixed-budget pass: {n_ev} events x {PTS} points x {FIXED_ITERS} iterations")
    timing = (ctypes.c_double * 8)()
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

    def step(alloc=mem.MEM_ALLOC_NEYMAN):
        mem.integrate_events(comps, proc, PTS, 0, target_rel_err=TARGET, max_iter=MAX_ITER, outputs=(P, E, S),
                             n_iter_out=n_used, allocation=alloc, **TAIL)

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
    # the same step with every event's points split equally over its two
    # assignments (plain VEGAS budget split), for comparison
    equal = None
    if args.steps:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(mem.MEM_ALLOC_EQUAL)
        torch.cuda.synchronize()
        te = time.perf_counter() - t0
        equal = {"events_per_s": n_ev / te, "converged_fraction": float(np.mean(S.cpu().numpy() == 0)),
                 "median_iterations": float(np.median(n_used.cpu().numpy())),
                 "mean_iterations": float(np.mean(n_used.cpu().numpy()))}
        log(f"equal split: {equal}")
    # adaptive stratified sampling on top of the grid (equal split across
    # the assignments, which stratification requires), same target
    strat = None
    if args.steps:
        def run_strat():
            mem.integrate_events(comps, proc, PTS, 0, target_rel_err=TARGET, max_iter=MAX_ITER, outputs=(P, E, S),
                                 n_iter_out=n_used, stratify=mem.MEM_STRATIFY_ADAPTIVE)
        run_strat()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_strat()
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        strat = {"events_per_s": n_ev / ts, "converged_fraction": float(np.mean(S.cpu().numpy() == 0)),
                 "median_iterations": float(np.median(n_used.cpu().numpy())),
                 "mean_iterations": float(np.mean(n_used.cpu().numpy()))}
        log(f"stratified: {strat}")

    roof = None
    if FLOP_PER_EVAL is not None and launches > 0:
        per_launch = FLOP_PER_EVAL * n_evals / launches
        achieved = per_launch / (kern_ms / launches * 1e-3)
        traffic = (TRAFFIC_BYTES_PER_LAUNCH
                   if (n_ev, PTS, proc.chunk_points(), proc.waves()) == TRAFFIC_WORKLOAD else None)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32, "traffic": traffic}
    parton = parton_leg(mem, proc)
    grid = None if args.no_grid else pdf_grid_leg(mem, comps, n_ev, kern_ms)
    f2 = None if args.no_f2 else tth_vs_ttbb_leg(mem)
    if f2 is not None:
        f2["parton_level"] = f2_parton_leg(mem)
        if not args.no_cpu:
            f2["oracle"] = f2_oracle_rates()
    flow = None
    if not args.no_flow:
        flow = flow_leg(mem, proc, comps, n_ev, args)
        if value:
            # both uses of the trained proposal against the VEGAS headline
            # (same events, same 1 % target): sampling from it with the
            # VEGAS fallback, and seeding VEGAS's grids from it
            flow["vs_vegas"] = flow["events_per_s"] / value
            flow["flow_seeded_grids"]["vs_vegas"] = flow["flow_seeded_grids"]["events_per_s"] / value
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
                   "proposal": "vegas", "allocation": "neyman across the two assignments"},
        "integrand_evals_per_s": evals_per_s,
        "launch": launch,
        "fixed_budget": {"iterations": FIXED_ITERS, "seconds": fixed_s, "kernel_ms": kern_ms,
                         "median_rel_err": float(np.median(fixed_rel))},
        "converged_fraction": conv, "median_iterations": float(np.median(nu)) if args.steps else None,
        "mean_iterations": float(np.mean(nu)) if args.steps else None,
        "vegas_equal_split": equal,
        "vegas_stratified": strat,
        "flow_vs_vegas": flow,
        "parton_level": parton,
        "pdf_grid": grid,
        "tth_vs_ttbb": f2,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
