"""Per-configuration measurements on one GPU beside the FP64 oracle on the
host: the five workloads of the integration path (Drell-Yan 2D FP64, ttbar
dilepton 8D, the mixed persistent batch, gg -> ttbar H 9D; the learned
proposal is measured by bench.py).

For each configuration, on seeded synthetic events:
* GPU integrand evaluations/s at the configured budget (one warm-up call,
  then timed calls; kernel time from HIP events and wall time of the call);
* events/s at the configured budget, and the median relative MC error
  reached;
* FP32 vs FP64: (a) per point, the FP32 GPU integrand against the FP64
  oracle on points drawn from adapted VEGAS grids (max, 99.9 % and median
  relative error over nonzero points); (b) per integral, the first
  iteration's estimate I_0 of whole GPU integrations in both precisions:
  both run the same points on the same uniform grid, so |I_0,FP32 -
  I_0,FP64| / I_0,FP64 is the precision's effect on an estimate; (c) the
  final estimates of the two runs, |P_FP32 - P_FP64| / err (median and 99th
  percentile): after the first refinement the grids, hence the points,
  differ, so this measures statistical compatibility, not rounding;
* the oracle's evaluations/s on one host core and on all host cores
  (OpenMP over integrals), on a seeded subset of the events with a reduced
  budget (integrals are independent, so the rate carries over);
  events/s at the configured budget derived from it.

    python measure/config_table.py [--out FILE.json] [--quick]

Prints a markdown table and one JSON line.
"""
import argparse
import ctypes
import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

SEED0 = 0x14077595

CONFIGS = {
    "c0": dict(name="Drell-Yan 2D, FP64", events=64, points=4096, iters=10),
    "c1": dict(name="ttbar dilepton 8D", events=4096, points=65536, iters=8),
    "c2": dict(name="mixed batch (DY / dilepton / semileptonic)", events=20000, points=None, iters=8),
    "c3": dict(name="gg -> ttbar H 9D", events=1024, points=262144, iters=10),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ events --
def make_events(cfg, quick=False):
    """(obs list per kind, kinds per event, budgets per event, charge)"""
    import numpy as np
    from synth import events
    c = CONFIGS[cfg]
    n = c["events"] if not quick else max(8, c["events"] // 16)
    if cfg == "c0":
        return {"dy": events.drell_yan(n, SEED0 + 0)["obs"]}, ["dy"] * n, [c["points"]] * n
    if cfg == "c1":
        return {"tt": events.ttbar_dilepton(n, SEED0 + 1)["obs"]}, ["tt"] * n, [c["points"]] * n
    if cfg == "c3":
        return {"tth": events.ttbar_higgs(n, SEED0 + 3)["obs"]}, ["tth"] * n, [c["points"]] * n
    # c2: 40 % Drell-Yan, 40 % dilepton, 20 % semileptonic, shuffled; budget
    # 16384 + floor(U * 245761) points per event and iteration
    rng = np.random.default_rng(SEED0 + 2)
    n_dy, n_tt = int(0.4 * n), int(0.4 * n)
    n_sl = n - n_dy - n_tt
    kinds = ["dy"] * n_dy + ["tt"] * n_tt + ["sl"] * n_sl
    rng.shuffle(kinds)
    budgets = [int(16384 + np.floor(u * 245761)) for u in rng.random(n)]
    obs = {"dy": events.drell_yan(n_dy, SEED0 + 20)["obs"], "tt": events.ttbar_dilepton(n_tt, SEED0 + 21)["obs"],
           "sl": events.ttbar_semileptonic(n_sl, SEED0 + 22)["obs"]}
    return obs, kinds, budgets


N_OBJ = {"dy": 2, "tt": 4, "sl": 5, "tth": 7}
N_PERM = {"dy": 1, "tt": 2, "sl": 12, "tth": 24}
DIMS = {"dy": 2, "tt": 8, "sl": 7, "tth": 9}


def gpu_inputs(mem, obs, kinds):
    """components [4, n_obj, n] on the device, charges, per-event row of obs"""
    import numpy as np
    import torch
    n = len(kinds)
    n_obj = max(N_OBJ[k] for k in set(kinds))
    arr = np.zeros((n, n_obj, 4))
    charge = np.ones(n, dtype=np.int32)
    rows = []
    it = {k: iter(v) for k, v in obs.items()}
    for i, k in enumerate(kinds):
        o = next(it[k])
        rows.append(o)
        arr[i, :N_OBJ[k]] = o[:N_OBJ[k]]
        if k in ("sl", "tth"):
            charge[i] = int(o[N_OBJ[k], 0])
    comps = torch.as_tensor(np.ascontiguousarray(arr.transpose(2, 1, 0))).cuda()
    return comps, torch.as_tensor(charge).cuda(), rows


TUNING_TABLE = os.path.join(ROOT, "paper_1407_7595_amd", "tuning.txt")


def processes(mem, precision):
    """the four processes, each with its launch configuration from the
    shipped tuning table where the table has one (as the benchmark does)"""
    procs = {"dy": mem.Process(mem.MEM_DY_QQ_GAMMA_MUMU, precision=mem.MEM_FP64),
             "tt": mem.Process(mem.MEM_TT_DILEPTON, precision=precision),
             "sl": mem.Process(mem.MEM_TT_SEMILEPTON, precision=precision),
             "tth": mem.Process(mem.MEM_TTH_SEMILEPTON, precision=precision)}
    if os.path.exists(TUNING_TABLE):
        for p in procs.values():
            p.load_tuning(TUNING_TABLE)
    return procs


# --------------------------------------------------------------------- GPU --
def gpu_run(mem, comps, charge, procs, kinds, budgets, iters, seed, reps, iter_out=None):
    import numpy as np
    import torch
    plist = [procs[k] for k in kinds]
    mem.integrate_events(comps, plist, budgets, 2, seed=seed, charge=charge)     # warm-up
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        timing = (ctypes.c_double * 8)()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, E, S = mem.integrate_events(comps, plist, budgets, iters, seed=seed, charge=charge, timing=timing,
                                       iter_out=iter_out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r = {"wall_s": wall, "kernel_ms": timing[0], "launches": timing[1], "evals": timing[2]}
        if best is None or wall < best["wall_s"]:
            best = r
    P, E, S = P.cpu().numpy(), E.cpu().numpy(), S.cpu().numpy()
    stat = {}
    for k in sorted(set(kinds)):
        sel = np.array([kk == k for kk in kinds])
        vals, cnt = np.unique(S[sel], return_counts=True)
        stat[k] = {int(v): int(c) for v, c in zip(vals, cnt)}
    best["status_by_kind"] = stat
    ok = P > 0
    best.update(evals_per_s_wall=best["evals"] / best["wall_s"],
                evals_per_s_kernel=best["evals"] / (best["kernel_ms"] * 1e-3),
                events_per_s=len(kinds) / best["wall_s"],
                median_rel_err=float(np.median(E[ok] / P[ok])) if ok.any() else None,
                status_ok=float(np.mean(S == 0)))
    return best, P, E


def per_point_errors(mem, comps, charge, rows, kinds, procs32, n_events=4, n_per=128):
    """FP32 GPU integrand vs FP64 oracle on points from adapted grids"""
    import numpy as np
    import torch
    import oracle
    out = {}
    for k in sorted(set(kinds)):
        if k == "dy":
            continue
        idx = [i for i, kk in enumerate(kinds) if kk == k][:n_events]
        po = oracle.tt_params()
        fn = {"tt": lambda ev, perm, x: oracle.tt_integrand(po, ev, perm, x)[0],
              "sl": lambda ev, perm, x: oracle.sl_integrand(po, ev, perm, x)[0],
              "tth": lambda ev, perm, x: oracle.tth_integrand(po, ev, perm, x)[0]}[k]
        rel = []
        D = DIMS[k]
        for i in idx:
            sub = comps[:, :, i:i + 1].contiguous()
            ch = charge[i:i + 1].contiguous()
            n_int = N_PERM[k]
            grids = torch.empty((n_int, D, 65), dtype=torch.float64, device="cuda")
            mem.integrate_events(sub, procs32[k], 4096 * n_int, 4, seed=SEED0 + 9, grid_out=grids, charge=ch)
            ev_i = torch.zeros(n_int, dtype=torch.int32, device="cuda")
            pm_i = torch.arange(n_int, dtype=torch.int32, device="cuda")
            x = torch.empty((n_int, n_per, D), dtype=torch.float32, device="cuda")
            w = torch.empty((n_int, n_per), dtype=torch.float32, device="cuda")
            mem.vegas_capture(procs32[k], sub, ev_i, pm_i, grids, n_per, SEED0 + 9, 5, x, w, normalise=0, charge=ch)
            xd = x.double()
            for perm in range(n_int):
                f = torch.empty(n_per, dtype=torch.float64, device="cuda")
                mem.eval_points(procs32[k], sub, 0, perm, xd[perm].contiguous(), f, charge=ch)
                got = f.cpu().numpy()
                xs = xd[perm].cpu().numpy()
                for j in range(n_per):
                    want = fn(rows[i], perm, xs[j])
                    if want != 0.0 or got[j] != 0.0:
                        rel.append(abs(got[j] - want) / max(abs(want), 1e-300))
        rel = np.array(rel)
        out[k] = {"points": int(rel.size), "max": float(rel.max()), "p999": float(np.quantile(rel, 0.999)),
                  "median": float(np.median(rel))}
        log(f"  per-point FP32 vs oracle FP64 ({k}): {out[k]}")
    return out


# ------------------------------------------------------------------ oracle --
ORACLE_KIND = {"dy": "KIND_DY", "tt": "KIND_TT", "sl": "KIND_TT_SL", "tth": "KIND_TTH"}


def oracle_worker(kind, n_events, points, iters, seed):
    """(in a subprocess whose OMP_NUM_THREADS is set) evaluations / s"""
    import oracle
    from synth import events
    gen = {"dy": lambda: events.drell_yan(n_events, seed)["obs"],
           "tt": lambda: events.ttbar_dilepton(n_events, seed)["obs"],
           "sl": lambda: events.ttbar_semileptonic(n_events, seed)["obs"],
           "tth": lambda: events.ttbar_higgs(n_events, seed)["obs"]}[kind]
    obs = gen()
    p = oracle.dy_params() if kind == "dy" else oracle.tt_params()
    k = getattr(oracle, ORACLE_KIND[kind])
    oracle.integrate_events(k, p, obs[:1], seed, max(256, points // 16), 2)      # warm-up
    t0 = time.perf_counter()
    oracle.integrate_events(k, p, obs, seed, points, iters)
    dt = time.perf_counter() - t0
    print(json.dumps({"evals": n_events * points * iters, "seconds": dt}))


def oracle_rate(kind, n_events, points, iters, threads):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-worker", kind, str(n_events),
                        str(points), str(iters)], env=env, capture_output=True, text=True, check=True)
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return d["evals"] / d["seconds"]


ORACLE_SUBSET = {"dy": (64, 16384, 10), "tt": (16, 8192, 2), "sl": (2, 12 * 1024, 2), "tth": (2, 24 * 512, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out")
    ap.add_argument("--quick", action="store_true", help="a sixteenth of the events (smoke run)")
    ap.add_argument("--configs", default="c0,c1,c2,c3")
    ap.add_argument("--oracle-worker", nargs=4)
    args = ap.parse_args()
    if args.oracle_worker:
        k, n, pts, it = args.oracle_worker
        oracle_worker(k, int(n), int(pts), int(it), SEED0 + 50)
        return
    import torch
    import paper_1407_7595_amd as mem
    torch.cuda.set_device(0)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = int(os.environ.get("OMP_NUM_THREADS", cores))
    procs32 = processes(mem, mem.MEM_FP32)
    procs64 = processes(mem, mem.MEM_FP64)
    orates = {}
    res = {}
    for cfg in args.configs.split(","):
        c = CONFIGS[cfg]
        log(f"{cfg}: {c['name']}")
        obs, kinds, budgets = make_events(cfg, args.quick)
        comps, charge, rows = gpu_inputs(mem, obs, kinds)
        main_procs = procs64 if cfg == "c0" else procs32
        n_int = sum(N_PERM[k] for k in kinds)
        it32 = torch.zeros(c["iters"] * n_int * 2, dtype=torch.float64, device="cuda")
        g, P32, E32 = gpu_run(mem, comps, charge, main_procs, kinds, budgets, c["iters"], SEED0 + 7, reps=2,
                              iter_out=it32)
        r = {"name": c["name"], "events": len(kinds), "iters": c["iters"],
             "mean_points": float(sum(budgets) / len(budgets)), "gpu": g}
        log(f"  gpu: {g}")
        if cfg != "c0":
            it64 = torch.zeros_like(it32)
            _, P64, E64 = gpu_run(mem, comps, charge, procs64, kinds, budgets, c["iters"], SEED0 + 7, reps=1,
                                  iter_out=it64)
            import numpy as np
            I32 = it32.cpu().numpy().reshape(c["iters"], n_int, 2)[0, :, 0]
            I64 = it64.cpu().numpy().reshape(c["iters"], n_int, 2)[0, :, 0]
            # integrals whose first-iteration estimate is a normal FP64 number
            okI = I64 > 1e-300
            relI = np.abs(I32 - I64)[okI] / I64[okI]
            ok = (P32 > 0) & (P64 > 0) & (E64 > 0)
            d = np.abs(P32 - P64)[ok] / E64[ok]
            r["fp32_vs_fp64_estimate"] = {
                "iter0_integrals": int(okI.sum()), "iter0_rel_median": float(np.median(relI)),
                "iter0_rel_p99": float(np.quantile(relI, 0.99)), "iter0_rel_max": float(relI.max()),
                "final_dP_over_err_median": float(np.median(d)), "final_dP_over_err_p99": float(np.quantile(d, 0.99))}
            log(f"  FP32 vs FP64 estimates: {r['fp32_vs_fp64_estimate']}")
            r["fp32_vs_oracle_points"] = per_point_errors(mem, comps, charge, rows, kinds, procs32)
        # oracle rates per kind, one core and all cores
        kinds_here = sorted(set(kinds))
        for k in kinds_here:
            if k not in orates:
                n, pts, it = ORACLE_SUBSET[k]
                orates[k] = {"1": oracle_rate(k, n, pts, it, 1), str(cores): oracle_rate(k, n, pts, it, cores)}
                log(f"  oracle {k}: {orates[k]} evals/s")
        # mixture: time per evaluation weighted by the evaluations of each kind
        tot = {}
        for k, b in zip(kinds, budgets):
            tot[k] = tot.get(k, 0) + b
        evals_all = sum(tot.values())
        o = {}
        for th in ("1", str(cores)):
            t_per_eval = sum(tot[k] / evals_all / orates[k][th] for k in tot)
            o[th] = {"evals_per_s": 1.0 / t_per_eval,
                     "events_per_s": len(kinds) / (evals_all * c["iters"] * t_per_eval)}
        r["oracle"] = {"cores": cores, "rates": o,
                       "subset": {k: dict(zip(("events", "points", "iters"), ORACLE_SUBSET[k])) for k in tot}}
        res[cfg] = r
    line = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print("| config | GPU evals/s (kernel) | GPU evals/s (wall) | GPU events/s at budget | median err/P "
          "| oracle evals/s 1 core | oracle evals/s all cores | FP32 vs FP64 per point (max, p99.9) "
          "| FP32 vs FP64: I_0 same points (median, max rel); final |dP|/err (median, p99) |")
    print("|---|---|---|---|---|---|---|---|---|")
    for cfg, r in res.items():
        g, o = r["gpu"], r["oracle"]
        pp = r.get("fp32_vs_oracle_points", {})
        ppt = "; ".join(f"{k}: {v['max']:.2g}, {v['p999']:.2g}" for k, v in pp.items()) or "n/a (FP64)"
        es = r.get("fp32_vs_fp64_estimate")
        est = (f"{es['iter0_rel_median']:.2g}, {es['iter0_rel_max']:.2g}; "
               f"{es['final_dP_over_err_median']:.2g}, {es['final_dP_over_err_p99']:.2g}") if es else "n/a (FP64)"
        cores = o["cores"]
        print(f"| {cfg} {r['name']} | {g['evals_per_s_kernel']:.3g} | {g['evals_per_s_wall']:.3g} "
              f"| {g['events_per_s']:.4g} | {g['median_rel_err']:.3g} | {o['rates']['1']['evals_per_s']:.3g} "
              f"| {o['rates'][str(cores)]['evals_per_s']:.3g} ({cores}) | {ppt} | {est} |")
    print(line)


if __name__ == "__main__":
    main()
