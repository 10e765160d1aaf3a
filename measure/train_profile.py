"""A short training of the dilepton proposal, for profiling the training
kernels: 2048 seeded events, VEGAS 8192 points x 3 iterations, 64 samples
captured per integral, 2 epochs of 65 536-sample batches through
mem_train_proposal.

    python measure/train_profile.py
"""
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_1407_7595_amd as mem   # noqa: E402
from synth import events            # noqa: E402


def main():
    p = mem.Process(mem.MEM_TT_DILEPTON, precision=mem.MEM_FP32)
    tr = mem.to_components(events.ttbar_dilepton(2048, 0x99)["obs"]).cuda()
    mem.train_proposal(p, tr, seed=3, vegas_points=8192, vegas_iter=3, capture=64, batch=65536, epochs=2,
                       lr_max=2e-3, lr_min=1e-4)
    torch.cuda.synchronize()
    print("done", flush=True)


if __name__ == "__main__":
    main()
