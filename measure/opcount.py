"""Algorithmic FLOP count of the ttbar dilepton integrand (GPU formulation).

Builds csrc/opcount.cpp (the device integrand headers compiled for the host
with counting scalar types) and runs it on seeded ttbar events from the
synthetic generator, through a VEGAS integration with the GPU's point
stream and grid refinement.  Prints one JSON object: operations per
evaluation by type and precision, FP32-equivalent FLOP per evaluation (an
FP64 operation counts twice), solutions per evaluation.

    python measure/opcount.py [n_points n_iter n_events]
"""
import json
import os
import struct
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def run(n_points=4096, n_iter=8, n_events=8, seed=0x14077595 + 1):
    import numpy as np
    from synth import events
    exe = os.path.join(tempfile.gettempdir(), "mem_opcount")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1407_7595_amd", "csrc"), "-o", exe,
                    os.path.join(HERE, "opcount.cpp")], check=True)
    obs = events.ttbar_dilepton(n_events, seed)["obs"]
    payload = struct.pack("<i", n_events) + np.ascontiguousarray(obs, dtype="<f8").tobytes()
    out = subprocess.run([exe, str(n_points), str(n_iter), str(n_events)], input=payload, capture_output=True,
                         check=True).stdout
    res = json.loads(out)
    res["command"] = f"python measure/opcount.py {n_points} {n_iter} {n_events}"
    res["events"] = f"synth.events.ttbar_dilepton({n_events}, {hex(seed)})"
    return res


if __name__ == "__main__":
    args = [int(a) for a in sys.argv[1:4]]
    print(json.dumps(run(*args), indent=1))
