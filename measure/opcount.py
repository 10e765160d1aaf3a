"""Algorithmic FLOP count of the ttbar dilepton integrand (GPU formulation).

Builds csrc/opcount.cpp (the device integrand headers compiled for the host
with counting scalar types) and runs it on seeded ttbar events from the
synthetic generator, through a VEGAS integration with the GPU's point
stream and grid refinement.  Prints one JSON object: operations per
evaluation by type and precision, FP32-equivalent FLOP per evaluation (an
FP64 operation counts twice), solutions per evaluation.

    python measure/opcount.py [n_points n_iter n_events [n_generated [jobs]]]

n_generated: draw that many events and count on the first n_events of
them (the generator is not prefix-stable: 32 of 4096 is a sample of the
benchmark's own 4096 events, 32 of 32 is not).
"""
import json
import os
import struct
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def run(n_points=4096, n_iter=8, n_events=8, n_generated=None, jobs=1, seed=0x14077595 + 1):
    import numpy as np
    from synth import events
    exe = os.path.join(tempfile.gettempdir(), "mem_opcount")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1407_7595_amd", "csrc"), "-o", exe,
                    os.path.join(HERE, "opcount.cpp")], check=True)
    n_gen = n_generated or n_events
    obs = events.ttbar_dilepton(n_gen, seed)["obs"][:n_events]
    # events are independent: shards of consecutive events run in parallel,
    # each told the index of its first event (the point stream's counter)
    cuts = np.linspace(0, n_events, min(jobs, n_events) + 1).astype(int)
    def shard(i0, i1):
        payload = struct.pack("<i", int(i1 - i0)) + np.ascontiguousarray(obs[i0:i1], dtype="<f8").tobytes()
        out = subprocess.run([exe, str(n_points), str(n_iter), str(i1 - i0), str(i0)], input=payload,
                             capture_output=True, check=True).stdout
        return json.loads(out), int(i1 - i0)
    with ThreadPoolExecutor(len(cuts) - 1) as pool:
        parts = list(pool.map(lambda c: shard(*c), zip(cuts[:-1], cuts[1:])))
    # per-evaluation averages, weighted by each shard's events (equal
    # evaluations per event)
    def mean(get):
        return sum(get(r) * n for r, n in parts) / n_events
    res = {"evaluations": sum(r["evaluations"] for r, _ in parts),
           "nonzero_fraction": mean(lambda r: r["nonzero_fraction"]),
           "solutions_per_eval": mean(lambda r: r["solutions_per_eval"])}
    for p in ("fp64", "fp32"):
        res[p] = {k: round(mean(lambda r: r[p][k]), 2) for k in parts[0][0][p]}
    res["flop_fp32_equivalent"] = round(2 * res["fp64"]["flop"] + res["fp32"]["flop"], 2)
    res["per_iteration_flop"] = [round(mean(lambda r: r["per_iteration_flop"][j]), 1) for j in range(n_iter)]
    res["nonzero_fraction"] = round(res["nonzero_fraction"], 6)
    res["solutions_per_eval"] = round(res["solutions_per_eval"], 6)
    res["command"] = (f"python measure/opcount.py {n_points} {n_iter} {n_events}" +
                      (f" {n_gen}" if n_generated else "") + (f" {jobs}" if jobs > 1 else ""))
    res["events"] = f"the first {n_events} of synth.events.ttbar_dilepton({n_gen}, {hex(seed)})"
    return res


if __name__ == "__main__":
    args = [int(a) for a in sys.argv[1:6]]
    print(json.dumps(run(*args), indent=1))
